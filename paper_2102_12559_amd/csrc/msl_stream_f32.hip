// msl_stream_f32.hip -- stream-and-collide instantiations: float storage, athermal
#include "msl_stream.hpp"

template int msl_launch_store_th<float, false>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<float, false>(const msl_ctx *c);
