// Learned path entry points (network forward/backward, learned step, rollout,
// adjoints).
#include "stage.h"

extern "C" {
int ldsv_cnn_forward(ldsv_handle*, const ldsv_net*, const float*, const float*, float*, void*) {
  ldsv_set_error("cnn_forward: not available in this build");
  return LDSV_EDTYPE;
}
int ldsv_learned_fv_step(ldsv_handle*, const ldsv_params*, const ldsv_net*, const float*,
                         const float*, float*, float*, int, float*, void*) {
  ldsv_set_error("learned_fv_step: not available in this build");
  return LDSV_EDTYPE;
}
int ldsv_rollout(ldsv_handle*, const ldsv_params*, const ldsv_net*, const void*, const void*, int,
                 int, int, void*, void*, int*, void*) {
  ldsv_set_error("rollout: not available in this build");
  return LDSV_EDTYPE;
}
int ldsv_fv_step_bwd(ldsv_handle*, const ldsv_params*, const float*, const void*, const void*,
                     const void*, const void*, void*, void*, float*, void*) {
  ldsv_set_error("fv_step_bwd: not available in this build");
  return LDSV_EDTYPE;
}
int ldsv_cnn_backward(ldsv_handle*, const ldsv_net*, const float*, const float*, const float*,
                      float*, float*, const ldsv_net_grad*, void*) {
  ldsv_set_error("cnn_backward: not available in this build");
  return LDSV_EDTYPE;
}
int ldsv_learned_fv_step_bwd(ldsv_handle*, const ldsv_params*, const ldsv_net*, const float*,
                             const float*, int, const float*, const float*, float*, float*,
                             const ldsv_net_grad*, void*) {
  ldsv_set_error("learned_fv_step_bwd: not available in this build");
  return LDSV_EDTYPE;
}
}
