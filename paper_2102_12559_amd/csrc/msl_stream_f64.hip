// msl_stream_f64.hip -- stream-and-collide instantiations for double storage
#include "msl_stream.hpp"

template int msl_launch_store<double>(msl_ctx *c, int lat, const char *in, char *out);
