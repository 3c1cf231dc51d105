// msl_stream.hip -- storage-precision dispatch of the stream-and-collide kernels
#include "msl_internal.hpp"

template <typename S, bool TH>
int msl_launch_store_th(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template <typename S, bool TH>
int msl_sc2_all_th(const msl_ctx *c);

template <typename S>
static int store_s(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  return c->cfg.thermal ? msl_launch_store_th<S, true>(c, lat, in, out, oth)
                        : msl_launch_store_th<S, false>(c, lat, in, out, oth);
}

int msl_launch_stream_collide(msl_ctx *c, int lat, const char *in, char *out, char *oth) {
  switch (c->cfg.store) {
    case MSL_FP64: return store_s<double>(c, lat, in, out, oth);
    case MSL_FP32: return store_s<float>(c, lat, in, out, oth);
    case MSL_FP16_DEV: return store_s<_Float16>(c, lat, in, out, oth);
    case MSL_BF16_DEV: return store_s<bf16_t>(c, lat, in, out, oth);
  }
  return MSL_EINVAL;
}

template <typename S>
static int sc2_all_s(const msl_ctx *c) {
  return c->cfg.thermal ? msl_sc2_all_th<S, true>(c) : msl_sc2_all_th<S, false>(c);
}

int msl_stream_sc2_all(const msl_ctx *c) {
  switch (c->cfg.store) {
    case MSL_FP64: return sc2_all_s<double>(c);
    case MSL_FP32: return sc2_all_s<float>(c);
    case MSL_FP16_DEV: return sc2_all_s<_Float16>(c);
    case MSL_BF16_DEV: return sc2_all_s<bf16_t>(c);
  }
  return 0;
}
