// msl_stream_bf16_th.hip -- stream-and-collide instantiations: bf16_t storage, thermal (f and g)
#include "msl_stream.hpp"

template int msl_launch_store_th<bf16_t, true>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<bf16_t, true>(const msl_ctx *c);
