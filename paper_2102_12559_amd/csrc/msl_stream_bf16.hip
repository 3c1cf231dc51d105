// msl_stream_bf16.hip -- stream-and-collide instantiations: bf16_t storage, athermal
#include "msl_stream.hpp"

template int msl_launch_store_th<bf16_t, false>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<bf16_t, false>(const msl_ctx *c);
