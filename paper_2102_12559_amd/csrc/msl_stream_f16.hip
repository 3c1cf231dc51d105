// msl_stream_f16.hip -- stream-and-collide instantiations for _Float16 storage
#include "msl_stream.hpp"

template int msl_launch_store<_Float16>(msl_ctx *c, int lat, const char *in, char *out);
