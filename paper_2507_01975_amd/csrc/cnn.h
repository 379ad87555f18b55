// Host-side interface of the network kernels.
#pragma once

#include "internal.h"

int ldsv_ensure_learned(ldsv_handle* h);
int ldsv_check_net(const ldsv_net* net);
int ldsv_launch_cnn(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                    float* out, float* const* zpre, hipStream_t st);
int ldsv_launch_cnn_backward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                             const float* gout, float* gu, float* gv, const ldsv_net_grad* dW,
                             hipStream_t st);
// launch the persistent LDS-tiled convolution (sides multiples of 16)
int ldsv_launch_conv_tile(ldsv_handle* h, int mt, int epi, const uint16_t* X, const uint16_t* W,
                          const float* bias, int cout, uint16_t* Y, float* zio, float* out,
                          hipStream_t st);
