// Host-side declarations of the surrogate's device kernels (BF16 MFMA convolutions and the
// elementwise / reduction pieces of its training step).
#pragma once

#include "common.hpp"

namespace vs {

// One convolution launch.  Activations are [B][H][W][C] BF16 (bit patterns), channels last.
// The input is the concatenation of two sources along channels: the first `cu` channels come
// from `xu`, a [B][H/2][W/2][cu] tensor read through nearest 2x upsampling (or cu = 0), the
// remaining `cx` channels from `x` ([B][H][W][cx]).  Weights: [cout][ks*ks][cu + cx] BF16.
struct NnConv {
  const uint16_t* x;
  const uint16_t* xu;
  int cu, cx;
  const uint16_t* w;  // [cout][k*k][cin] rows, or the blocked layout when wblk (see w_index)
  int wblk;           // 1: w is blocked (cout and cin multiples of 16 and 8)
  const float* bias;  // [cout] or null
  void* y;            // output, see NnEpi
  int B, H, W, cout;
  float out_scale;    // NN_EPI_SHUFFLE / NN_EPI_HEAD
  // NN_EPI_HEAD: a 1x1 layer of 16 outputs applied to this layer's ReLU output in registers
  const uint16_t* w2;  // [16][cout] BF16
  const float* bias2;  // [16]
};

enum NnEpi : int {
  NN_EPI_BF16 = 0,       // y: [B][H][W][cout] BF16 of (acc + bias), ReLU if requested
  NN_EPI_F32 = 1,        // y: [B][H][W][cout] FP32 of (acc + bias)
  NN_EPI_SHUFFLE = 2,    // cout = 16: y[b][4Y + j/4][4X + j%4] = out_scale (acc_j + bias_j), [B][4H][4W] FP32
  NN_EPI_HEAD = 3,       // cout = 32, ReLU: then y as NN_EPI_SHUFFLE of the 16-output layer (w2, bias2)
};


hipError_t nn_conv(int ks, int epi, bool relu, const NnConv& a, hipStream_t s);

// Weight gradient: part[s][cout][ks*ks][cin] = sum over pixel chunk s of dz (x) shifted input.
// n_split must be nn_wgrad_splits(ks, B, H, W, cu + cx, cout), the number of chunks of the
// kernel the shape selects (1 x 1 and 3 x 3 layers whose image width is a power of two up to 128
// and whose rows come in whole 128-pixel steps: every tap per workgroup; otherwise one tap each).
int nn_wgrad_splits(int ks, int B, int H, int W, int cin, int cout);
hipError_t nn_wgrad(int ks, const NnConv& a, const uint16_t* dz, float* part, int n_split, hipStream_t s);
// out[co][t][ci] (ci < cin_dst) = sum_s part[s][co][t][ci] (part has cin_src columns)
hipError_t nn_reduce_parts(const float* part, int n_split, int cout, int taps, int cin_src, int cin_dst, float* out,
                           hipStream_t s);

// dz = BF16 of g * [act > 0] (act may be null: no mask), where g at pixel p of the H x W grid is
// the sum of the sources that are given: da[p * lda + c] (same grid), the four values
// dfine[q * ldf + c] of the 2 x 2 block of p on the 2H x 2W grid (gradient of a nearest-neighbour
// upsampling) and 0.25 dpool[coarse(p) * C + c] (gradient of a 2 x 2 average pool); per-channel
// sums of g into part[block][C].  Strides in floats, multiples of 4.
constexpr int kNnReluBlocks = 2048;
hipError_t nn_relu_bwd(const float* da, int lda, const float* dfine, int ldf, const float* dpool, const uint16_t* act,
                       uint16_t* dz, int B, int H, int W, int C, float* part, hipStream_t s);
// out[c] = scale * sum_b part[b * stride + c], b < nb, c < C
hipError_t nn_colsum(const float* part, int nb, int stride, int C, float scale, float* out, hipStream_t s);

hipError_t nn_avgpool(const uint16_t* x, uint16_t* y, int B, int Hc, int Wc, int C, hipStream_t s);

struct NnFeat {
  float shift[3], scale[3];
  float k0;
};
// Features + 1x1 stem (48 -> cout = 32 or 64, ReLU) in one kernel.  Inputs: [B][n][n] FP32
// maps (sample b at idx[b] when idx is given; v, m may be null = 1).  Feature (py*4 + px)*3 + c
// of a coarse pixel's 4x4 patch is formed in the lane that feeds it to the matrix cores;
// feat_out ([B][n/4][n/4][64] BF16, features 48..63 zero) is written too when given (the
// training pass needs it).
hipError_t nn_stem(const float* q, const float* v, const float* m, const int* idx, int n, int B, const NnFeat& f,
                   const uint16_t* w, const float* bias, int cout, uint16_t* y, uint16_t* feat_out, hipStream_t s);
// dh[b][Y][X][j] = BF16 of out_scale * 2 (y - t) / (B n^2) at fine pixel (4Y + j/4, 4X + j%4);
// part[block][17] = per-block sums of the 16 FP32 dh values and of (y - t)^2
constexpr int kNnMseBlocks = 1024;
hipError_t nn_mse_grad(const float* y, const float* t, const int* idx, int n, int B, float out_scale, uint16_t* dh,
                       float* part, hipStream_t s);

hipError_t nn_adam(float* p, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                   float bc1, float bc2, hipStream_t s);
// Blocked weight layout: element (co, tap, ci) of a [C_out][taps][C_in] weight sits at
// ((co / 16 * taps + tap) * C_in / 8 + ci / 8) * 128 + (co % 16) * 8 + ci % 8, so the 16-byte A
// operands of one matrix-core step (16 output channels x 32 input channels of one tap) are one
// contiguous kilobyte.
__host__ __device__ inline long w_index(int blocked, int co, int tap, int ci, int taps, int c_in) {
  if (!blocked) return ((long)co * taps + tap) * c_in + ci;
  return (((long)(co >> 4) * taps + tap) * (c_in >> 3) + (ci >> 3)) * 128 + (co & 15) * 8 + (ci & 7);
}
// BF16 copies of one layer's weights src[cout][taps][cin_src] (FP32, or BF16 bit patterns):
// dst = [cout][taps][cin_pad] (zero padded) and dstT = [cin_pad][taps][cout] with the taps
// reversed (the input-gradient weights), both in rows or, with blocked, in the blocked layout;
// either output may be null
hipError_t nn_weight_cast(const float* src, int cout, int taps, int cin_src, int cin_pad, uint16_t* dst,
                          uint16_t* dstT, hipStream_t s, int blocked = 0);
hipError_t nn_weight_cast_bf16(const uint16_t* src, int cout, int taps, int cin_src, int cin_pad, uint16_t* dst,
                               uint16_t* dstT, hipStream_t s);

}  // namespace vs
