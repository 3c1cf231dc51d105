// msl_stream_f64.hip -- stream-and-collide instantiations: double storage, athermal
#include "msl_stream.hpp"

template int msl_launch_store_th<double, false>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<double, false>(const msl_ctx *c);
