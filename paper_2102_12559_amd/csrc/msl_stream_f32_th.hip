// msl_stream_f32_th.hip -- stream-and-collide instantiations: float storage, thermal (f and g)
#include "msl_stream.hpp"

template int msl_launch_store_th<float, true>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<float, true>(const msl_ctx *c);
