// msl_stream_f16.hip -- stream-and-collide instantiations: _Float16 storage, athermal
#include "msl_stream.hpp"

template int msl_launch_store_th<_Float16, false>(msl_ctx *c, int lat, const char *in, char *out, char *oth);
template int msl_sc2_all_th<_Float16, false>(const msl_ctx *c);
