// msl_stream_f32.hip -- stream-and-collide instantiations for float storage
#include "msl_stream.hpp"

template int msl_launch_store<float>(msl_ctx *c, int lat, const char *in, char *out);
