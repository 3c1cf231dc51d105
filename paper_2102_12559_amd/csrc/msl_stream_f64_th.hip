// msl_stream_f64_th.hip -- stream-and-collide instantiations: double storage, thermal (f and g)
#include "msl_stream.hpp"

template int msl_launch_store_th<double, true>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<double, true>(const msl_ctx *c);
