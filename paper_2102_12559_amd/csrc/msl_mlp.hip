// msl_mlp.hip -- learned lifting closure (placeholder until the MFMA kernels land)
#include "msl_device.hpp"

int msl_mlp_band_lift(msl_ctx *, char *, char *) { return MSL_OK; }
int msl_mlp_check_launch(msl_ctx *) { return MSL_OK; }

extern "C" {
int msl_mlp_dims(const msl_ctx *c, int *F, int *O, int *H, int *P) {
  if (!c) return MSL_EINVAL;
  if (F) *F = c->mlpF;
  if (O) *O = c->mlpO;
  if (H) *H = c->mlpH;
  if (P) *P = c->mlpP;
  return MSL_OK;
}
int msl_collect_snapshots(msl_ctx *, float *, float *, int, int *) { return MSL_EINVAL; }
int msl_mlp_set_weights(msl_ctx *, const float *, const float *, const float *, const float *,
                        const float *) { return MSL_EINVAL; }
int msl_mlp_get_weights(msl_ctx *, float *) { return MSL_EINVAL; }
int msl_mlp_train(msl_ctx *, const float *, const float *, int, int, int, float, float *) { return MSL_EINVAL; }
int msl_mlp_grad(msl_ctx *, const float *, const float *, int, float *, float *) { return MSL_EINVAL; }
int msl_mlp_forward(msl_ctx *, const float *, int, float *) { return MSL_EINVAL; }
int msl_mlp_get_flags(msl_ctx *, uint8_t *) { return MSL_EINVAL; }
int msl_mlp_set_flags(msl_ctx *, const uint8_t *) { return MSL_EINVAL; }
}
