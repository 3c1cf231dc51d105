// msl_stream_f16_th.hip -- stream-and-collide instantiations: _Float16 storage, thermal (f and g)
#include "msl_stream.hpp"

template int msl_launch_store_th<_Float16, true>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<_Float16, true>(const msl_ctx *c);
