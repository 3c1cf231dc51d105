// msl_stream.hip -- storage-precision dispatch of the stream-and-collide kernels
#include "msl_internal.hpp"

template <typename S>
int msl_launch_store(msl_ctx *c, int lat, const char *in, char *out);

int msl_launch_stream_collide(msl_ctx *c, int lat, const char *in, char *out) {
  switch (c->cfg.store) {
    case MSL_FP64: return msl_launch_store<double>(c, lat, in, out);
    case MSL_FP32: return msl_launch_store<float>(c, lat, in, out);
    case MSL_FP16_DEV: return msl_launch_store<_Float16>(c, lat, in, out);
    case MSL_BF16_DEV: return msl_launch_store<bf16_t>(c, lat, in, out);
  }
  return MSL_EINVAL;
}
