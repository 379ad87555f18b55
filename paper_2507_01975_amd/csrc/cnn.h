// Host-side interface of the network kernels.
#pragma once

#include "internal.h"

int ldsv_ensure_learned(ldsv_handle* h);
int ldsv_check_net(const ldsv_net* net);
// forward through all layers.  Output either as float planes [B][66][Ny][Nx]
// in `out` (coefficient channels rounded to bf16 values), or, when coef16 is
// given and the grid is tiled (sides multiples of 16), as bf16 coefficients
// in blocks of 8 channels [B][8][Ny][Nx][8] in coef16 (a kind's 16 values of
// a cell are two 16-byte loads, coalesced across cells) and float correction
// planes [B][2][Ny][Nx] in tc.  Returns in *bf16_out whether the second form
// was written.
// fuse_first (inference only, zpre null): on grids whose sides are multiples
// of 16, layer 1 is computed inside layer 2's tiles and its activation is
// not kept in the handle (the network output is the same bit for bit)
int ldsv_launch_cnn(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                    float* out, float* const* zpre, hipStream_t st, uint16_t* coef16 = nullptr,
                    float* tc = nullptr, bool* bf16_out = nullptr, bool fuse_first = false);
int ldsv_launch_cnn_backward(ldsv_handle* h, const ldsv_net* net, const float* u, const float* v,
                             const float* gout, float* gu, float* gv, const ldsv_net_grad* dW,
                             hipStream_t st);
// launch the persistent LDS-tiled convolution (sides multiples of 16)
int ldsv_launch_conv_tile(ldsv_handle* h, int mt, int epi, const uint16_t* X, const uint16_t* W,
                          const float* bias, int cout, uint16_t* Y, float* zio, float* out,
                          hipStream_t st);
