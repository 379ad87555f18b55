// Host-side interface of the flux block's FNO kernels.
#pragma once

#include "internal.h"

// fields [B][8][Ny][Nx] = the two FNOs of net on (u, v); keep_pre keeps every
// layer's pre-activation in the handle's FNO workspace for the backward
int ldsv_launch_fno_forward(ldsv_handle* h, const ldsv_fluxnet* net, const float* u,
                            const float* v, float* fields, bool keep_pre, hipStream_t st);
// the handle's [B][8][Ny][Nx] field and field-gradient buffers
int ldsv_ensure_fluxblock(ldsv_handle* h);
// backward from gfields [B][8][Ny][Nx] (after a forward with the activations
// kept, run here unless forward_kept says the last forward on this handle
// kept them for the same net and input): accumulates the parameter
// gradients into gr; gu, gv (nullable) receive the input gradient, added to
// their contents when accumulate is set
int ldsv_launch_fno_backward(ldsv_handle* h, const ldsv_fluxnet* net, const ldsv_fluxnet_grad* gr,
                             const float* u, const float* v, const float* gfields, float* gu,
                             float* gv, int accumulate, hipStream_t st, bool forward_kept);
// the temporal correction FNO on the k_c history states (oldest first):
// out = (du, dv) as two [B][Ny][Nx] planes at out and out + B Ny Nx
int ldsv_launch_tc_forward(ldsv_handle* h, const ldsv_fno* tc, const float* const* hu,
                           const float* const* hv, int kc, float* out, bool keep_pre,
                           hipStream_t st);
// its backward from gout (two planes like out): ACCUMULATES the parameter
// gradients into gtc and the history-state gradients into ghu[j], ghv[j]
int ldsv_launch_tc_backward(ldsv_handle* h, const ldsv_fno* tc, const ldsv_fno_grad* gtc,
                            const float* const* hu, const float* const* hv, int kc,
                            const float* gout, float* const* ghu, float* const* ghv,
                            bool forward_kept, float* scratch_out, hipStream_t st);
