// msl_stream_bf16.hip -- stream-and-collide instantiations for bf16_t storage
#include "msl_stream.hpp"

template int msl_launch_store<bf16_t>(msl_ctx *c, int lat, const char *in, char *out);
