// Device kernels of the convolutional warm-start surrogate (gfx950, BF16 MFMA, FP32 accumulate).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: M = output channels, N = pixels,
// K = taps x input channels.  A lane supplies row (lane % 16) of A and column (lane % 16) of B,
// each with the same 8 consecutive K values (group lane / 16); with channels last and the input
// channel count a multiple of 16, those 8 values are one 16-byte load from one pixel and one tap.
// The output tile comes back as D[4 (lane / 16) + r][lane % 16], r = 0..3: four consecutive
// output channels of one pixel, one vector store.  The same kernel computes the input gradient
// with tap-reversed, channel-transposed weights.  The weight gradient contracts over pixels: its
// operand tiles are staged through LDS transposed so that K (pixels) is contiguous, and chunks
// of pixels write partial sums that a second kernel adds in a fixed order.
#include <cmath>

#include "fft.hpp"
#include "nn.hpp"

namespace vs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ bf16x8 as_bf(uint4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ unsigned pack2(float a, float b) { return (unsigned)f2bf(a) | ((unsigned)f2bf(b) << 16); }

// ------------------------------------------------------------------------------ convolution
// Bias, ReLU and the store of a wavefront's MW x NW accumulator tiles: tile (i, j) holds output
// channels co0 + 16 i + 4 lg + r (r = 0..3) of pixel (pb[j], py[j], px[j]) in lane (lr, lg).
template <int MW, int NW, int EPI, bool RELU>
__device__ __forceinline__ void conv_epilogue(const NnConv& a, const f32x4 (&acc)[MW][NW], const int (&pb)[NW],
                                              const int (&py)[NW], const int (&px)[NW], const bool (&pv)[NW], int lr,
                                              int lg, int co0) {
  if constexpr (EPI == NN_EPI_HEAD) {
    // this layer's 32 channels -> BF16 -> B operand of the 16-output layer.  Lane (lr, lg) holds
    // channels 4 lg + r (tile 0) and 16 + 4 lg + r (tile 1) of pixel lr: that is its K group, and
    // the head's A operand is loaded in the same channel order.
    static_assert(MW == 2, "head epilogue needs the 32 channels in two tiles");
    float b1[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b1[r] = a.bias[4 * lg + r];
      b1[4 + r] = a.bias[16 + 4 * lg + r];
    }
    const uint2 wl = *reinterpret_cast<const uint2*>(a.w2 + lr * 32 + 4 * lg);
    const uint2 wh = *reinterpret_cast<const uint2*>(a.w2 + lr * 32 + 16 + 4 * lg);
    const bf16x8 hw = as_bf(make_uint4(wl.x, wl.y, wh.x, wh.y));
    float hb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) hb[r] = a.bias2[4 * lg + r];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      float v[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = fmaxf(acc[0][j][r] + b1[r], 0.f);
        v[4 + r] = fmaxf(acc[1][j][r] + b1[4 + r], 0.f);
      }
      const uint4 d = make_uint4(pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7]));
      f32x4 h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hw, as_bf(d), f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if (!pv[j]) continue;
      float* out = (float*)a.y + ((long)pb[j] * (4 * a.H) + 4 * py[j] + lg) * (4L * a.W) + 4 * px[j];
      const float sc = a.out_scale;
      *reinterpret_cast<float4*>(out) =
          make_float4(sc * (h[0] + hb[0]), sc * (h[1] + hb[1]), sc * (h[2] + hb[2]), sc * (h[3] + hb[3]));
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    const int co = co0 + i * 16 + 4 * lg;
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (a.bias)
#pragma unroll
      for (int r = 0; r < 4; ++r) bias[r] = a.bias[co + r];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      if (!pv[j]) continue;
      const long p = ((long)pb[j] * a.H + py[j]) * a.W + px[j];
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = acc[i][j][r] + bias[r];
        if (RELU) v[r] = fmaxf(v[r], 0.f);
      }
      if constexpr (EPI == NN_EPI_BF16) {
        *reinterpret_cast<uint2*>((uint16_t*)a.y + p * a.cout + co) = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
      } else if constexpr (EPI == NN_EPI_F32) {
        *reinterpret_cast<float4*>((float*)a.y + p * a.cout + co) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        // cout = 16: output channel co + r = 4 lg + r is sub-pixel (lg, r) of the 4x4 patch
        float* out = (float*)a.y + ((long)pb[j] * (4 * a.H) + 4 * py[j] + lg) * (4L * a.W) + 4 * px[j];
        const float s = a.out_scale;
        *reinterpret_cast<float4*>(out) = make_float4(s * v[0], s * v[1], s * v[2], s * v[3]);
      }
    }
  }
}

template <int KS, int MW, int NW, int EPI, bool RELU>
__global__ void __launch_bounds__(256) conv_kernel(NnConv a) {
  constexpr int TAPS = KS * KS, R = KS / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int H = a.H, W = a.W, cu = a.cu, cx = a.cx, cin = cu + cx;
  const long HW = (long)H * W;
  const long P = (long)a.B * HW;
  const long p0 = ((long)blockIdx.x * 4 + wave) * (16 * NW);
  const int co0 = blockIdx.y * (16 * MW);
  int pb[NW], py[NW], px[NW];
  bool pv[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const long p = p0 + j * 16 + lr;
    pv[j] = p < P;
    const long q = pv[j] ? p : 0;
    pb[j] = (int)(q / HW);
    const int rem = (int)(q - (long)pb[j] * HW);
    py[j] = rem / W;
    px[j] = rem - py[j] * W;
  }
  f32x4 acc[MW][NW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);

  for (int tap = 0; tap < TAPS; ++tap) {
    const int dy = tap / KS - R, dx = tap % KS - R;
    for (int c0 = 0; c0 < cin; c0 += 32) {
      const int ci = c0 + 8 * lg;
      const bool kv = ci < cin;
      const bool up = ci < cu;
      uint4 av[MW], bv[NW];
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        const int co = co0 + i * 16 + lr;
        av[i] = kv ? ld16(a.w + w_index(a.wblk, co, tap, ci, TAPS, cin)) : z4;
      }
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int yy = py[j] + dy, xx = px[j] + dx;
        const bool in = kv && pv[j] && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const uint16_t* src = up ? a.xu + (((long)pb[j] * (H >> 1) + (yy >> 1)) * (W >> 1) + (xx >> 1)) * cu + ci
                                 : a.x + (((long)pb[j] * H + yy) * W + xx) * cx + (ci - cu);
        bv[j] = in ? ld16(src) : z4;
      }
#pragma unroll
      for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av[i]), as_bf(bv[j]), acc[i][j], 0, 0, 0);
    }
  }

  conv_epilogue<MW, NW, EPI, RELU>(a, acc, pb, py, px, pv, lr, lg, co0);
}

// 3x3 convolution of wide maps with the input staged in LDS.  A workgroup computes 4 rows x 64
// columns of one image (wavefront w: row w, 4 x 16 consecutive pixels).  The input channels are
// taken in phases of at most 64 channels of one source (the upsampled coarser level or the skip
// input, as in conv_kernel); per phase the workgroup copies the 6 x 66 input pixels around its
// tile -- zero outside the image and beyond the phase's channels up to the next multiple of 32 --
// into LDS with a pixel pitch of that multiple + 8 elements (an odd multiple of 16 bytes, so 8
// lanes reading 16 bytes at consecutive pixels use distinct banks), then runs the phase's part
// of the K loop reading B from LDS.  Each input pixel leaves L2 once per tile instead of once per
// tap and output pixel.  Requires H % 4 == 0 and W % 64 == 0.
constexpr int kLdsRows = 4, kLdsCols = 64, kLdsPhase = 64;
__host__ __device__ constexpr int conv_lds_pitch(int channels) { return ((channels + 31) & ~31) + 8; }
inline long conv_lds_bytes(int cu, int cx) {
  const int widest = cu > cx ? cu : cx;
  return (long)(kLdsRows + 2) * (kLdsCols + 2) * conv_lds_pitch(widest < kLdsPhase ? widest : kLdsPhase) * 2;
}

template <int MW, int EPI, bool RELU, bool BLK>
__global__ void __launch_bounds__(256) conv3_lds_kernel(NnConv a) {
  constexpr int TR = kLdsRows, NW = kLdsRows, TW = kLdsCols + 2;
  extern __shared__ __attribute__((aligned(16))) uint16_t tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int H = a.H, W = a.W, cu = a.cu, cx = a.cx, cin = cu + cx;
  const int tiles_x = W / kLdsCols, tiles_y = H / TR;
  const int tb = blockIdx.x / (tiles_x * tiles_y);
  const int trem = blockIdx.x - tb * tiles_x * tiles_y;
  const int y0 = (trem / tiles_x) * TR, x0 = (trem % tiles_x) * kLdsCols;
  const int co0 = blockIdx.y * (16 * MW);

  int pb[NW], py[NW], px[NW];
  bool pv[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    pb[j] = tb;
    py[j] = y0 + wave;
    px[j] = x0 + 16 * j + lr;
    pv[j] = true;
  }
  f32x4 acc[MW][NW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);

  for (int cs = 0; cs < cin;) {
    const int send = cs < cu ? cu : cin;
    const int len = send - cs < kLdsPhase ? send - cs : kLdsPhase;
    const int pitch = conv_lds_pitch(len);
    // stage the phase's halo, (pitch - 8) / 8 chunks of 8 channels per pixel; each thread issues
    // a batch of SB loads before storing them, so their latencies overlap
    constexpr int SB = 4;
    const int chunks = (pitch - 8) >> 3;
    const int total = (TR + 2) * TW * chunks;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * SB) {
      uint4 v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int e = e0 + 256 * u;
        const int k = e % chunks, pix = e / chunks;
        const int r = pix / TW, c = pix - r * TW;
        const int yy = y0 - 1 + r, xx = x0 - 1 + c, ch = cs + 8 * k;
        v[u] = z4;
        if (e < total && 8 * k < len && yy >= 0 && yy < H && xx >= 0 && xx < W)
          v[u] = ch < cu ? ld16(a.xu + (((long)tb * (H >> 1) + (yy >> 1)) * (W >> 1) + (xx >> 1)) * cu + ch)
                         : ld16(a.x + (((long)tb * H + yy) * W + xx) * cx + (ch - cu));
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int e = e0 + 256 * u;
        if (e < total) *reinterpret_cast<uint4*>(tile + (e / chunks) * pitch + 8 * (e % chunks)) = v[u];
      }
    }
    __syncthreads();

    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      const uint16_t* brow = tile + ((wave + 1 + dy) * TW + 1 + dx) * pitch;
      for (int c0 = 0; c0 < len; c0 += 32) {
        const int cl = c0 + 8 * lg;  // channel within the phase
        const bool kv = cl < len;
        uint4 av[MW], bv[NW];
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          const int co = co0 + i * 16 + lr;
          const long wi = BLK ? (((long)((co0 >> 4) + i) * 9 + tap) * (cin >> 3) + ((cs + cl) >> 3)) * 128 + lr * 8
                              : ((long)co * 9 + tap) * cin + cs + cl;
          av[i] = kv ? ld16(a.w + wi) : z4;
        }
#pragma unroll
        for (int j = 0; j < NW; ++j)  // zero past the phase's channels
          bv[j] = *reinterpret_cast<const uint4*>(brow + (16 * j + lr) * pitch + cl);
#pragma unroll
        for (int i = 0; i < MW; ++i)
#pragma unroll
          for (int j = 0; j < NW; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av[i]), as_bf(bv[j]), acc[i][j], 0, 0, 0);
      }
    }
    cs += len;
    if (cs < cin) __syncthreads();  // the next phase overwrites the tile
  }
  conv_epilogue<MW, NW, EPI, RELU>(a, acc, pb, py, px, pv, lr, lg, co0);
}

inline bool conv_lds_ok(const NnConv& a) {
  return a.W % kLdsCols == 0 && a.H % kLdsRows == 0 && conv_lds_bytes(a.cu, a.cx) <= 65536;
}

template <int MW, int EPI, bool RELU>
hipError_t conv_lds(const NnConv& a, hipStream_t s) {
  const dim3 grid((unsigned)((long)a.B * (a.H / kLdsRows) * (a.W / kLdsCols)), a.cout / (16 * MW));
  if (a.wblk)
    hipLaunchKernelGGL((conv3_lds_kernel<MW, EPI, RELU, true>), grid, dim3(256), (size_t)conv_lds_bytes(a.cu, a.cx), s,
                       a);
  else
    hipLaunchKernelGGL((conv3_lds_kernel<MW, EPI, RELU, false>), grid, dim3(256), (size_t)conv_lds_bytes(a.cu, a.cx),
                       s, a);
  return hipGetLastError();
}

template <int KS, int MW, int NW, int EPI, bool RELU>
hipError_t conv_launch(const NnConv& a, hipStream_t s) {
  const long P = (long)a.B * a.H * a.W;
  const dim3 grid((unsigned)((P + 64 * NW - 1) / (64 * NW)), a.cout / (16 * MW));
  hipLaunchKernelGGL((conv_kernel<KS, MW, NW, EPI, RELU>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int KS, int EPI, bool RELU>
hipError_t conv_tile(const NnConv& a, hipStream_t s) {
  if constexpr (KS == 3) {
    if (conv_lds_ok(a)) {
      // decoder input gradients (80 and 112 channels at the default widths) in one tile, so the
      // staged halo serves every output channel
      if (a.cout == 80) return conv_lds<5, EPI, RELU>(a, s);
      if (a.cout == 112) return conv_lds<7, EPI, RELU>(a, s);
      if (a.cout % 64 == 0) return conv_lds<4, EPI, RELU>(a, s);
      if (a.cout % 48 == 0) return conv_lds<3, EPI, RELU>(a, s);
      if (a.cout % 32 == 0) return conv_lds<2, EPI, RELU>(a, s);
      return conv_lds<1, EPI, RELU>(a, s);
    }
  }
  if (a.cout % 64 == 0) return conv_launch<KS, 4, 2, EPI, RELU>(a, s);
  if (a.cout % 48 == 0) return conv_launch<KS, 3, 2, EPI, RELU>(a, s);
  if (a.cout % 32 == 0) return conv_launch<KS, 2, 4, EPI, RELU>(a, s);
  return conv_launch<KS, 1, 8, EPI, RELU>(a, s);
}

template <int KS>
hipError_t conv_ks(int epi, bool relu, const NnConv& a, hipStream_t s) {
  switch (epi) {
    case NN_EPI_BF16: return relu ? conv_tile<KS, NN_EPI_BF16, true>(a, s) : conv_tile<KS, NN_EPI_BF16, false>(a, s);
    case NN_EPI_F32: return conv_tile<KS, NN_EPI_F32, false>(a, s);
    case NN_EPI_SHUFFLE:
      if (a.cout != 16) return hipErrorInvalidValue;
      if (KS == 3 && conv_lds_ok(a)) return conv_lds<1, NN_EPI_SHUFFLE, false>(a, s);
      return conv_launch<KS, 1, 8, NN_EPI_SHUFFLE, false>(a, s);
    case NN_EPI_HEAD:
      if (a.cout != 32 || !a.w2 || !a.bias2) return hipErrorInvalidValue;
      if (KS == 3 && conv_lds_ok(a)) return conv_lds<2, NN_EPI_HEAD, true>(a, s);
      return conv_launch<KS, 2, 4, NN_EPI_HEAD, true>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------ weight gradient
// Pixels per staging step and LDS row pitch (elements): rows 272 bytes apart, so the 16-byte
// operand reads of 8 consecutive rows fall on distinct banks.
constexpr int kWgK = 128;
constexpr int kWgPitch = kWgK + 8;

// Row c of the transpose of an 8 x 8 block of 16-bit values: element e of the result is element c
// of v[e].
__device__ __forceinline__ uint4 transpose8_row(const uint4 (&v)[8], int c) {
  unsigned w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned lo = reinterpret_cast<const unsigned*>(&v[2 * k])[c >> 1];
    const unsigned hi = reinterpret_cast<const unsigned*>(&v[2 * k + 1])[c >> 1];
    w[k] = (c & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Weight gradient of one tap (blockIdx.y) for a 64 x 64 block of (output, input) channels over
// one chunk of pixels (blockIdx.x).  Each step stages 128 pixels of dz and of the shifted input,
// transposed so that pixels (the contraction) are contiguous: thread t takes an 8-pixel x
// 8-channel block of one operand (eight 16-byte loads, one per pixel), transposes it in registers
// and writes eight 16-byte rows.  Four K steps of 32 pixels follow per staging, while the next
// step's operands load.
template <int KS>
__global__ void __launch_bounds__(256) wgrad_kernel(NnConv a, const uint16_t* __restrict__ dz, float* __restrict__ part,
                                                    long chunk) {
  constexpr int TAPS = KS * KS, R = KS / 2;
  __shared__ __attribute__((aligned(16))) uint16_t sz[64 * kWgPitch];
  __shared__ __attribute__((aligned(16))) uint16_t sx[64 * kWgPitch];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lg = lane >> 4;
  const int H = a.H, W = a.W, cu = a.cu, cx = a.cx, cin = cu + cx, cout = a.cout;
  const long HW = (long)H * W, P = (long)a.B * HW;
  const int tap = blockIdx.y, dy = tap / KS - R, dx = tap % KS - R;
  const int nco = (cout + 63) / 64;
  const int cob = (int)(blockIdx.z % nco) * 64, cib = (int)(blockIdx.z / nco) * 64;
  const int wco = (wave >> 1) * 32, wci = (wave & 1) * 32;
  const long pbeg = (long)blockIdx.x * chunk;
  const long pend = P < pbeg + chunk ? P : pbeg + chunk;
  // staging role: threads 0..127 take dz, 128..255 the input; pixel group pg (8 pixels), channel
  // group cg (8 channels) of the 64-channel block
  const bool stage_x = t >= 128;
  const int pg = t & 15, cg = (t >> 4) & 7;
  const int co = cob + cg * 8, ci = cib + cg * 8;
  uint16_t* const dst = (stage_x ? sx : sz) + (cg * 8) * kWgPitch + pg * 8;
  // W % 8 == 0: the 8 pixels of a group lie in one image row (chunks start at multiples of 128)
  const bool row8 = (W & 7) == 0;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  uint4 v[8];
  auto load = [&](long p) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = z4;
    const long q0 = p + pg * 8;
    if (!stage_x) {
      if (co < cout)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (q0 + e < pend) v[e] = ld16(dz + (q0 + e) * cout + co);
    } else if (ci < cin) {
      const uint16_t* src = ci < cu ? a.xu + ci : a.x + (ci - cu);
      const int cs = ci < cu ? cu : cx;
      if (row8) {
        if (q0 < pend) {
          const unsigned b = (unsigned)q0 / (unsigned)HW;
          const unsigned rem = (unsigned)q0 - b * (unsigned)HW;
          const int y = (int)(rem / (unsigned)W), x0 = (int)(rem - (unsigned)y * W);
          const int yy = y + dy;
          if (yy >= 0 && yy < H) {
            const long rowbase = ci < cu ? ((long)b * (H >> 1) + (yy >> 1)) * (W >> 1) : ((long)b * H + yy) * W;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int xx = x0 + e + dx;
              if (xx >= 0 && xx < W) v[e] = ld16(src + (rowbase + (ci < cu ? xx >> 1 : xx)) * cs);
            }
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const long q = q0 + e;
          if (q < pend) {
            const unsigned b = (unsigned)q / (unsigned)HW;
            const unsigned rem = (unsigned)q - b * (unsigned)HW;
            const int yy = (int)(rem / (unsigned)W) + dy, xx = (int)(rem % (unsigned)W) + dx;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
              v[e] = ld16(src + (ci < cu ? ((long)b * (H >> 1) + (yy >> 1)) * (W >> 1) + (xx >> 1)
                                         : ((long)b * H + yy) * W + xx) * cs);
          }
        }
      }
    }
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (pbeg < pend) load(pbeg);
  for (long p = pbeg; p < pend; p += kWgK) {
    __syncthreads();  // the previous step's operand reads are done
#pragma unroll
    for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4*>(dst + c * kWgPitch) = transpose8_row(v, c);
    __syncthreads();
    if (p + kWgK < pend) load(p + kWgK);  // next step's operands, in flight during the products
#pragma unroll
    for (int ks = 0; ks < kWgK / 32; ++ks) {
      uint4 av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        av[i] = *reinterpret_cast<const uint4*>(sz + (wco + i * 16 + lr) * kWgPitch + ks * 32 + 8 * lg);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bv[j] = *reinterpret_cast<const uint4*>(sx + (wci + j * 16 + lr) * kWgPitch + ks * 32 + 8 * lg);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av[i]), as_bf(bv[j]), acc[i][j], 0, 0, 0);
    }
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = cob + wco + i * 16 + 4 * lg + r, ci = cib + wci + j * 16 + lr;
        if (co < cout && ci < cin) part[(((long)blockIdx.x * cout + co) * TAPS + tap) * cin + ci] = acc[i][j][r];
      }
}

// Weight gradient of a 3 x 3 layer with the nine taps in one workgroup (a 1 x 1 layer: the same
// steps without the halo and with one tap).  A step covers R = 128 / W
// whole image rows (128 pixels).  dz of the step is staged once (16 MT channels x 128 pixels,
// pixels contiguous), and the input once as a halo of R + 2 rows by W + 2 columns (zero outside
// the image; 16 NT channels, columns contiguous, halo column h holding image column h - 1).  For
// the 8 pixels of a lane's K slice and a tap (dy, dx), the input operand is the halo run starting at
// column c + dx + 1: two aligned 16-byte reads per row serve all three dx (byte shifts of 0, 2
// and 4).  Wave w owns the (output block, input block) pairs w, w + 4, ... of the tile, each with
// nine accumulators; there is no cross-wave sum.  The input is staged once per step instead of
// once per tap.
template <int MT, int NT>
struct WgFused {
  static constexpr int PAIRS = MT * NT;
  static constexpr int PW = (PAIRS + 3) / 4;  // pairs per wave, at most
  static constexpr int ZP = 136;              // dz row pitch (elements): 272 bytes
  static constexpr int XPMAX = 456;           // largest halo pitch per channel
  static constexpr int LDS = 16 * MT * ZP + 16 * NT * XPMAX;
};

// halo geometry per image width: row pitch W + 16, channel pitch >= (R + 2) (W + 16) with
// pitch = 8 (mod 64) elements, so 8 consecutive channel rows start 16 bytes apart modulo 128
__host__ __device__ inline int wg3_hp(int W) { return W + 16; }
__host__ __device__ inline int wg3_xp(int W) {
  const int need = (128 / W + 2) * (W + 16);
  return (need + 55) / 64 * 64 + 8;
}

__device__ __forceinline__ uint4 shift_elems1(const uint4& a, const uint4& b) {
  return make_uint4(__builtin_amdgcn_alignbyte(a.y, a.x, 2), __builtin_amdgcn_alignbyte(a.z, a.y, 2),
                    __builtin_amdgcn_alignbyte(a.w, a.z, 2), __builtin_amdgcn_alignbyte(b.x, a.w, 2));
}

template <int KS, int MT, int NT>
__global__ void __launch_bounds__(256) wgrad3_kernel(NnConv a, const uint16_t* __restrict__ dz, float* __restrict__ part,
                                                     int steps_per_wg) {
  using F = WgFused<MT, NT>;
  constexpr int TAPS = KS * KS, PAD = KS / 2;  // a 1x1 layer stages no halo: one tap
  __shared__ __attribute__((aligned(16))) uint16_t lds[F::LDS];
  uint16_t* const sz = lds;
  uint16_t* const sx = lds + 16 * MT * F::ZP;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lg = lane >> 4;
  const int H = a.H, W = a.W, cu = a.cu, cx = a.cx, cin = cu + cx, cout = a.cout;
  const int R = 128 / W, HP = wg3_hp(W), XP = wg3_xp(W), HB = W / 8 + PAD, HR = R + 2 * PAD;
  const int spi = H / R;  // steps per image
  const int nsteps = a.B * spi;
  const int nco = (cout + 16 * MT - 1) / (16 * MT);
  const int cob = (int)(blockIdx.y % nco) * 16 * MT, cib = (int)(blockIdx.y / nco) * 16 * NT;
  const int s0 = blockIdx.x * steps_per_wg;
  const int s1 = nsteps < s0 + steps_per_wg ? nsteps : s0 + steps_per_wg;
  const int nzb = 2 * MT * 16, nblk = nzb + 2 * NT * HR * HB;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  f32x4 acc[F::PW][TAPS];
#pragma unroll
  for (int q = 0; q < F::PW; ++q)
#pragma unroll
    for (int k = 0; k < TAPS; ++k) acc[q][k] = f32x4{0.f, 0.f, 0.f, 0.f};

  // one 8-pixel x 8-channel staging block: its loads, and where its transpose goes
  auto fetch = [&](int blk, int b, int y0, long p0, uint4 (&v)[8], uint16_t*& dst, int& pitch) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = z4;
    dst = nullptr;
    if (blk >= nblk) return;
    if (blk < nzb) {
      const int cg = blk >> 4, pg = blk & 15;
      const int co = cob + cg * 8;
      if (co < cout)
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = ld16(dz + (p0 + pg * 8 + e) * cout + co);
      dst = sz + (cg * 8) * F::ZP + pg * 8;
      pitch = F::ZP;
    } else {
      const int xb = blk - nzb;
      const int hcb = xb % HB, rest = xb / HB;
      const int hr = rest % HR, cg = rest / HR;
      const int ci = cib + cg * 8, y = y0 - PAD + hr;
      if (ci < cin && y >= 0 && y < H) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int xc = hcb * 8 + e - PAD;
          if (xc >= 0 && xc < W)
            v[e] = ci < cu ? ld16(a.xu + (((long)b * (H >> 1) + (y >> 1)) * (W >> 1) + (xc >> 1)) * cu + ci)
                           : ld16(a.x + (((long)b * H + y) * W + xc) * cx + (ci - cu));
        }
      }
      dst = sx + (cg * 8) * XP + hr * HP + hcb * 8;
      pitch = XP;
    }
  };

  for (int st = s0; st < s1; ++st) {
    const int b = st / spi, y0 = (st - b * spi) * R;
    const long p0 = (long)st * 128;
    // at most two staging blocks per thread: both loads in flight before the writes
    uint4 v0[8], v1[8];
    uint16_t *d0, *d1;
    int pt0 = 0, pt1 = 0;
    fetch(t, b, y0, p0, v0, d0, pt0);
    fetch(t + 256, b, y0, p0, v1, d1, pt1);
    __syncthreads();  // the previous step's operand reads are done
    if (d0)
#pragma unroll
      for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4*>(d0 + c * pt0) = transpose8_row(v0, c);
    if (d1)
#pragma unroll
      for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4*>(d1 + c * pt1) = transpose8_row(v1, c);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k0 = ks * 32 + 8 * lg;
      const int r = k0 / W, c = k0 - r * W;
#pragma unroll
      for (int q = 0; q < F::PW; ++q) {
        const int pair = wave + 4 * q;
        if (pair < F::PAIRS) {
          const int i = pair / NT, j = pair % NT;
          const uint4 av = *reinterpret_cast<const uint4*>(sz + (i * 16 + lr) * F::ZP + k0);
          if constexpr (KS == 1) {
            const uint4 c0 = *reinterpret_cast<const uint4*>(sx + (j * 16 + lr) * XP + r * HP + c);
            acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(c0), acc[q][0], 0, 0, 0);
          } else {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
              const uint16_t* bx = sx + (j * 16 + lr) * XP + (r + dy) * HP + c;
              const uint4 c0 = *reinterpret_cast<const uint4*>(bx);
              const uint4 c1 = *reinterpret_cast<const uint4*>(bx + 8);
              const uint4 b1 = shift_elems1(c0, c1);
              const uint4 b2 = make_uint4(c0.y, c0.z, c0.w, c1.x);
              acc[q][dy * 3 + 0] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(c0), acc[q][dy * 3 + 0], 0, 0, 0);
              acc[q][dy * 3 + 1] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(b1), acc[q][dy * 3 + 1], 0, 0, 0);
              acc[q][dy * 3 + 2] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(b2), acc[q][dy * 3 + 2], 0, 0, 0);
            }
          }
        }
      }
    }
  }

#pragma unroll
  for (int q = 0; q < F::PW; ++q) {
    const int pair = wave + 4 * q;
    if (pair < F::PAIRS) {
      const int i = pair / NT, j = pair % NT;
#pragma unroll
      for (int tap = 0; tap < TAPS; ++tap)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int co = cob + i * 16 + 4 * lg + r4, ci = cib + j * 16 + lr;
          if (co < cout && ci < cin) part[(((long)blockIdx.x * cout + co) * TAPS + tap) * cin + ci] = acc[q][tap][r4];
        }
    }
  }
}

// 64 outputs per workgroup, four threads per output (chunks g, g + 4, ...), added in a fixed order
__global__ void __launch_bounds__(256) reduce_parts_kernel(const float* __restrict__ part, int ns, int cout, int taps,
                                                           int cin_src, int cin_dst, float* __restrict__ out) {
  __shared__ float s[4][64];
  const long n = (long)cout * taps * cin_dst, len = (long)cout * taps * cin_src;
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const long j = (long)blockIdx.x * 64 + o;
  float acc = 0.f;
  if (j < n) {
    const long rt = j / cin_dst;
    const long src = rt * cin_src + (j - rt * cin_dst);
    float a4[4] = {0.f, 0.f, 0.f, 0.f};
    int k = g;
    for (; k + 12 < ns; k += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] += part[(long)(k + 4 * u) * len + src];
    }
    for (; k < ns; k += 4) a4[0] += part[(long)k * len + src];
    acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
  s[g][o] = acc;
  __syncthreads();
  if (g == 0 && j < n) out[j] = (s[0][o] + s[1][o]) + (s[2][o] + s[3][o]);
}

// ------------------------------------------------------------------------------ elementwise
// Thread t owns channel group cg = t % G (8 channels, G = C / 8) of pixels slot, slot + T, ...
// (T = 256 / G threads per group); its channel sums stay in registers and the workgroup adds the
// T partials of each channel in a fixed order: no atomics, the same bits on every run.
__device__ __forceinline__ void add8(float (&g)[8], const float* __restrict__ p, float w) {
  const float4 lo = *reinterpret_cast<const float4*>(p), hi = *reinterpret_cast<const float4*>(p + 4);
  g[0] += w * lo.x, g[1] += w * lo.y, g[2] += w * lo.z, g[3] += w * lo.w;
  g[4] += w * hi.x, g[5] += w * hi.y, g[6] += w * hi.z, g[7] += w * hi.w;
}

__global__ void __launch_bounds__(256) relu_bwd_kernel(const float* __restrict__ da, int lda,
                                                       const float* __restrict__ dfine, int ldf,
                                                       const float* __restrict__ dpool, const uint16_t* __restrict__ act,
                                                       uint16_t* __restrict__ dz, int B, int H, int W, int C,
                                                       float* __restrict__ part) {
  __shared__ float s[256 * 8];
  const int G = C >> 3, T = 256 / G;
  const int cg = threadIdx.x % G, slot = threadIdx.x / G;
  const int c = 8 * cg;
  const long P = (long)B * H * W;
  const unsigned HW = (unsigned)H * W;
  float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (slot < T) {
    for (long p = (long)blockIdx.x * T + slot; p < P; p += (long)gridDim.x * T) {
      float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (da) {
        const float4 lo = *reinterpret_cast<const float4*>(da + p * lda + c);
        const float4 hi = *reinterpret_cast<const float4*>(da + p * lda + c + 4);
        g[0] = lo.x, g[1] = lo.y, g[2] = lo.z, g[3] = lo.w, g[4] = hi.x, g[5] = hi.y, g[6] = hi.z, g[7] = hi.w;
      }
      if (dfine || dpool) {
        const unsigned b = (unsigned)p / HW;
        const unsigned rem = (unsigned)p - b * HW;
        const int yq = (int)(rem / (unsigned)W), xq = (int)(rem - (unsigned)yq * W);
        if (dfine)  // nearest-neighbour upsampling: the sum over the 2 x 2 fine block
#pragma unroll
          for (int d = 0; d < 4; ++d)
            add8(g, dfine + (((long)b * 2 * H + 2 * yq + (d >> 1)) * (2L * W) + 2 * xq + (d & 1)) * ldf + c, 1.f);
        if (dpool)  // 2 x 2 average pool: a quarter of the coarse value
          add8(g, dpool + (((long)b * (H >> 1) + (yq >> 1)) * (W >> 1) + (xq >> 1)) * C + c, 0.25f);
      }
      if (act) {
        const uint4 u = ld16(act + p * C + c);
        const uint16_t* h = reinterpret_cast<const uint16_t*>(&u);
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = bf2f(h[k]) > 0.f ? g[k] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) sum[k] += g[k];
      if (dz)
        *reinterpret_cast<uint4*>(dz + p * C + c) = make_uint4(pack2(g[0], g[1]), pack2(g[2], g[3]),
                                                               pack2(g[4], g[5]), pack2(g[6], g[7]));
    }
  }
  // s[slot][c + k]: the T partials of every channel
  if (slot < T) {
#pragma unroll
    for (int k = 0; k < 8; ++k) s[slot * C + c + k] = sum[k];
  }
  __syncthreads();
  for (int ch = threadIdx.x; ch < C; ch += 256) {
    float acc = 0.f;
    for (int q = 0; q < T; ++q) acc += s[q * C + ch];
    part[(long)blockIdx.x * C + ch] = acc;
  }
}

// one workgroup per column c: thread t adds rows t, t + 256, ...; then a fixed-order tree
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ part, int nb, int stride, int C,
                                                     float scale, float* __restrict__ out) {
  __shared__ float s[256];
  const int c = blockIdx.x;
  float acc = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[(long)b * stride + c];
  s[threadIdx.x] = acc;
  __syncthreads();
#pragma unroll
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = scale * s[0];
}

// y = 2x2 mean of x; one thread per (coarse pixel, 8 channels)
__global__ void __launch_bounds__(256) avgpool_kernel(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, int B,
                                                      int Hc, int Wc, int C) {
  const int g8 = C / 8;
  const long n = (long)B * Hc * Wc * g8;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long pc = i / g8;
    const int c = (int)(i - pc * g8) * 8;
    const int b = (int)(pc / ((long)Hc * Wc));
    const int rem = (int)(pc - (long)b * Hc * Wc);
    const int Y = rem / Wc, X = rem % Wc;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const long pf = ((long)b * 2 * Hc + 2 * Y + (d >> 1)) * (2L * Wc) + 2 * X + (d & 1);
      const uint4 u = ld16(x + pf * C + c);
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&u);
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += bf2f(h[k]);
    }
    *reinterpret_cast<uint4*>(y + pc * C + c) =
        make_uint4(pack2(0.25f * acc[0], 0.25f * acc[1]), pack2(0.25f * acc[2], 0.25f * acc[3]),
                   pack2(0.25f * acc[4], 0.25f * acc[5]), pack2(0.25f * acc[6], 0.25f * acc[7]));
  }
}

// Features + 1x1 stem.  Wave = 16 coarse pixels.  Lane (lr, lg) reads row lg of pixel lr's 4x4
// patch (one 16-byte load per map) and forms its 12 features; they meet in LDS as [pixel][64]
// BF16 (slots 48..63 zero), from which each lane takes its B operand: slots 32 c + 8 lg .. + 7
// of pixel lr for the two K chunks c.
template <int MT>
__global__ void __launch_bounds__(256) stem_kernel(const float* __restrict__ q, const float* __restrict__ v,
                                                   const float* __restrict__ m, const int* __restrict__ idx, int n,
                                                   int B, NnFeat f, const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias, uint16_t* __restrict__ y,
                                                   uint16_t* __restrict__ feat_out) {
  constexpr int COUT = 16 * MT;
  constexpr int FP = 72;  // LDS pitch of a pixel's feature row (BF16 elements; rows stay 16-byte aligned)
  __shared__ __attribute__((aligned(16))) uint16_t sf[4][16 * FP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int mc = n / 4;
  const long P = (long)B * mc * mc;
  const long p = ((long)blockIdx.x * 4 + wave) * 16 + lr;
  const bool pv = p < P;
  uint16_t* row = sf[wave] + lr * FP;
  {
    float fv[12];
    if (pv) {
      const int b = (int)(p / ((long)mc * mc));
      const int rem = (int)(p - (long)b * mc * mc);
      const int Y = rem / mc, X = rem % mc;
      const long sidx = idx ? idx[b] : b;
      const long o = sidx * n * n + (long)(4 * Y + lg) * n + 4 * X;
      const float4 qq = *reinterpret_cast<const float4*>(q + o);
      const float4 vv = v ? *reinterpret_cast<const float4*>(v + o) : make_float4(1.f, 1.f, 1.f, 1.f);
      const float4 mm = m ? *reinterpret_cast<const float4*>(m + o) : make_float4(1.f, 1.f, 1.f, 1.f);
      const float qa[4] = {qq.x, qq.y, qq.z, qq.w}, va[4] = {vv.x, vv.y, vv.z, vv.w}, ma[4] = {mm.x, mm.y, mm.z, mm.w};
#pragma unroll
      for (int px = 0; px < 4; ++px) {
        fv[3 * px] = (qa[px] * 1e-6f - f.shift[0]) * f.scale[0];
        fv[3 * px + 1] = (__logf(va[px]) - f.shift[1]) * f.scale[1];
        fv[3 * px + 2] = (f.k0 * ma[px] * (1.f / 150.f) - f.shift[2]) * f.scale[2];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 12; ++i) fv[i] = 0.f;
    }
    // patch row lg holds slots 12 lg .. 12 lg + 11 (6 BF16 pairs)
    unsigned* dst = reinterpret_cast<unsigned*>(row + 12 * lg);
#pragma unroll
    for (int i = 0; i < 6; ++i) dst[i] = pack2(fv[2 * i], fv[2 * i + 1]);
    if (lg == 0) {
      uint4* z = reinterpret_cast<uint4*>(row + 48);
      z[0] = make_uint4(0u, 0u, 0u, 0u);
      z[1] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  wave_sync();
  f32x4 acc[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const uint4 bv = *reinterpret_cast<const uint4*>(row + 32 * c + 8 * lg);
    if (feat_out && pv) *reinterpret_cast<uint4*>(feat_out + p * 64 + 32 * c + 8 * lg) = bv;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const uint4 av = ld16(w + (long)(i * 16 + lr) * 64 + 32 * c + 8 * lg);
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(bv), acc[i], 0, 0, 0);
    }
  }
  if (!pv) return;
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int co = i * 16 + 4 * lg;
    float r4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) r4[r] = fmaxf(acc[i][r] + bias[co + r], 0.f);
    *reinterpret_cast<uint2*>(y + p * COUT + co) = make_uint2(pack2(r4[0], r4[1]), pack2(r4[2], r4[3]));
  }
}

__global__ void __launch_bounds__(256) mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                       const int* __restrict__ idx, int n, int B, float out_scale,
                                                       uint16_t* __restrict__ dh, float* __restrict__ part) {
  __shared__ float s[4][17];
  const int mc = n / 4;
  const long total = (long)B * mc * mc;
  const float k = 2.f / ((float)B * (float)n * (float)n);
  // per-thread sums in registers, then a butterfly over the wave and the four waves in a fixed
  // order: no atomics, the same bits on every run
  float acc[17];
#pragma unroll
  for (int j = 0; j < 17; ++j) acc[j] = 0.f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const unsigned per = (unsigned)mc * mc;
    const int b = (int)((unsigned long)i / per);
    const int rem = (int)(i - (long)b * per);
    const int Y = rem / mc, X = rem % mc;
    const long st = idx ? idx[b] : b;
    float g[16];
#pragma unroll
    for (int py = 0; py < 4; ++py) {
      const float4 yy = *reinterpret_cast<const float4*>(y + ((long)b * n + 4 * Y + py) * n + 4 * X);
      const float4 tt = *reinterpret_cast<const float4*>(t + (st * n + 4 * Y + py) * n + 4 * X);
      const float d[4] = {yy.x - tt.x, yy.y - tt.y, yy.z - tt.z, yy.w - tt.w};
#pragma unroll
      for (int px = 0; px < 4; ++px) {
        acc[16] += d[px] * d[px];
        g[py * 4 + px] = out_scale * k * d[px];
        acc[py * 4 + px] += g[py * 4 + px];
      }
    }
    uint4* o = reinterpret_cast<uint4*>(dh + i * 16);
    o[0] = make_uint4(pack2(g[0], g[1]), pack2(g[2], g[3]), pack2(g[4], g[5]), pack2(g[6], g[7]));
    o[1] = make_uint4(pack2(g[8], g[9]), pack2(g[10], g[11]), pack2(g[12], g[13]), pack2(g[14], g[15]));
  }
#pragma unroll
  for (int j = 0; j < 17; ++j)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 17; ++j) s[wave][j] = acc[j];
  __syncthreads();
  if (threadIdx.x < 17) {
    const int j = threadIdx.x;
    part[(long)blockIdx.x * 17 + j] = (s[0][j] + s[1][j]) + (s[2][j] + s[3][j]);
  }
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, long n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

__device__ __forceinline__ uint16_t to_bf(float x) { return f2bf(x); }
__device__ __forceinline__ uint16_t to_bf(uint16_t x) { return x; }

template <typename S>
__global__ void __launch_bounds__(256) weight_cast_kernel(const S* __restrict__ src, int cout, int taps, int cin_src,
                                                          int cin_pad, uint16_t* __restrict__ dst,
                                                          uint16_t* __restrict__ dstT, int blocked) {
  const long n = (long)cout * taps * cin_pad;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ci = (int)(i % cin_pad);
    const long rt = i / cin_pad;
    const int tap = (int)(rt % taps), co = (int)(rt / taps);
    const uint16_t h = ci < cin_src ? to_bf(src[rt * cin_src + ci]) : (uint16_t)0;
    if (dst) dst[w_index(blocked, co, tap, ci, taps, cin_pad)] = h;
    if (dstT) dstT[w_index(blocked, ci, taps - 1 - tap, co, taps, cout)] = h;
  }
}

unsigned blocks_for(long n, int per_thread = 1, unsigned cap = 4096) {
  const long b = (n / per_thread + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t nn_conv(int ks, int epi, bool relu, const NnConv& a, hipStream_t s) {
  if ((a.cu % 16) || (a.cx % 16) || a.cu + a.cx <= 0 || (a.cout % 16) || a.cout <= 0 || a.B <= 0 || a.H <= 0 ||
      a.W <= 0 || (a.cu && ((a.H | a.W) & 1)))
    return hipErrorInvalidValue;
  if (ks == 1) return conv_ks<1>(epi, relu, a, s);
  if (ks == 3) return conv_ks<3>(epi, relu, a, s);
  return hipErrorInvalidValue;
}

namespace {

// Tile of the nine-tap kernel for a layer: output blocks MT (<= 4, a divisor of cout / 16 when one
// exists), input blocks NT chosen for the least padded input channels plus a per-tile cost, within
// 12 pairs and 72 KB of LDS.  Returns false when the layer does not suit the kernel.
bool wgrad3_tile(int W, int H, int cout, int cin, int& mt, int& nt) {
  if (W < 8 || W > 128 || (W & (W - 1)) || H % (128 / W)) return false;
  const int cm = cout / 16;
  mt = cm % 4 == 0 ? 4 : (cm % 3 == 0 ? 3 : (cm % 2 == 0 ? 2 : 1));
  if (mt == 1 && cm > 1) mt = cm >= 4 ? 4 : cm;
  long best = -1;
  for (int n = 1; n <= 5; ++n) {
    if (mt * n > 12 || mt * n < 4) continue;
    const long lds = 2L * (16 * mt * 136 + 16 * n * 456);
    if (lds > 72 * 1024) continue;
    const long cost = (long)((cin + 16 * n - 1) / (16 * n)) * (n + 2);
    if (best < 0 || cost < best) best = cost, nt = n;
  }
  return best >= 0;
}

int wgrad3_steps_per_wg(int B, int H, int W, int tiles) {
  const long nsteps = (long)B * H * W / 128;
  long per = (nsteps * tiles + 767) / 768;
  if (per < 8) per = 8;
  return (int)per;
}

template <int KS, int MT, int NT>
hipError_t wgrad3_launch(const NnConv& a, const uint16_t* dz, float* part, int n_split, int per, hipStream_t s) {
  const int cin = a.cu + a.cx;
  const dim3 grid(n_split, ((a.cout + 16 * MT - 1) / (16 * MT)) * ((cin + 16 * NT - 1) / (16 * NT)));
  hipLaunchKernelGGL((wgrad3_kernel<KS, MT, NT>), grid, dim3(256), 0, s, a, dz, part, per);
  return hipGetLastError();
}

template <int KS>
hipError_t wgrad3_dispatch(int mt, int nt, const NnConv& a, const uint16_t* dz, float* part, int n_split, int per,
                           hipStream_t s) {
  switch (mt * 8 + nt) {
#define VS_WG3(M, N) \
  case M * 8 + N: return wgrad3_launch<KS, M, N>(a, dz, part, n_split, per, s);
    VS_WG3(1, 4) VS_WG3(1, 5) VS_WG3(2, 2) VS_WG3(2, 3) VS_WG3(2, 4) VS_WG3(2, 5) VS_WG3(3, 2) VS_WG3(3, 3)
    VS_WG3(3, 4) VS_WG3(4, 1) VS_WG3(4, 2) VS_WG3(4, 3)
#undef VS_WG3
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int nn_wgrad_splits(int ks, int B, int H, int W, int cin, int cout) {
  int mt, nt;
  if ((ks == 1 || ks == 3) && wgrad3_tile(W, H, cout, cin, mt, nt)) {
    const int tiles = ((cout + 16 * mt - 1) / (16 * mt)) * ((cin + 16 * nt - 1) / (16 * nt));
    const long nsteps = (long)B * H * W / 128;
    const int per = wgrad3_steps_per_wg(B, H, W, tiles);
    return (int)((nsteps + per - 1) / per);
  }
  const long s = ((long)B * H * W + 2047) / 2048;
  return (int)(s < 1 ? 1 : (s > 256 ? 256 : s));
}

hipError_t nn_wgrad(int ks, const NnConv& a, const uint16_t* dz, float* part, int n_split, hipStream_t s) {
  if ((a.cu % 16) || (a.cx % 16) || (a.cout % 16) || (a.cu && ((a.H | a.W) & 1))) return hipErrorInvalidValue;
  if (n_split != nn_wgrad_splits(ks, a.B, a.H, a.W, a.cu + a.cx, a.cout)) return hipErrorInvalidValue;
  const long P = (long)a.B * a.H * a.W;
  if (P > 0x7fffffffL) return hipErrorInvalidValue;  // pixel indices are divided in 32 bits
  int mt, nt;
  if ((ks == 1 || ks == 3) && wgrad3_tile(a.W, a.H, a.cout, a.cu + a.cx, mt, nt)) {
    const int cin = a.cu + a.cx;
    const int tiles = ((a.cout + 16 * mt - 1) / (16 * mt)) * ((cin + 16 * nt - 1) / (16 * nt));
    const int per = wgrad3_steps_per_wg(a.B, a.H, a.W, tiles);
    return ks == 1 ? wgrad3_dispatch<1>(mt, nt, a, dz, part, n_split, per, s)
                   : wgrad3_dispatch<3>(mt, nt, a, dz, part, n_split, per, s);
  }
  long chunk = (P + n_split - 1) / n_split;
  chunk = (chunk + kWgK - 1) / kWgK * kWgK;
  const int cin = a.cu + a.cx;
  const dim3 grid(n_split, ks * ks, ((a.cout + 63) / 64) * ((cin + 63) / 64));
  if (ks == 1)
    hipLaunchKernelGGL(wgrad_kernel<1>, grid, dim3(256), 0, s, a, dz, part, chunk);
  else if (ks == 3)
    hipLaunchKernelGGL(wgrad_kernel<3>, grid, dim3(256), 0, s, a, dz, part, chunk);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t nn_reduce_parts(const float* part, int n_split, int cout, int taps, int cin_src, int cin_dst, float* out,
                           hipStream_t s) {
  const long n = (long)cout * taps * cin_dst;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, part, n_split, cout, taps,
                     cin_src, cin_dst, out);
  return hipGetLastError();
}

hipError_t nn_relu_bwd(const float* da, int lda, const float* dfine, int ldf, const float* dpool, const uint16_t* act,
                       uint16_t* dz, int B, int H, int W, int C, float* part, hipStream_t s) {
  if (C % 8 || C > 256 || (da && (lda < C || lda % 4)) || (dfine && (ldf < C || ldf % 4)) ||
      (dpool && ((H | W) & 1)) || (long)B * H * W > 0x7fffffffL)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(kNnReluBlocks), dim3(256), 0, s, da, lda, dfine, ldf, dpool, act, dz, B, H,
                     W, C, part);
  return hipGetLastError();
}

hipError_t nn_colsum(const float* part, int nb, int stride, int C, float scale, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(C), dim3(256), 0, s, part, nb, stride, C, scale, out);
  return hipGetLastError();
}

hipError_t nn_avgpool(const uint16_t* x, uint16_t* y, int B, int Hc, int Wc, int C, hipStream_t s) {
  if (C % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(avgpool_kernel, dim3(blocks_for((long)B * Hc * Wc * (C / 8))), dim3(256), 0, s, x, y, B, Hc, Wc,
                     C);
  return hipGetLastError();
}

hipError_t nn_stem(const float* q, const float* v, const float* m, const int* idx, int n, int B, const NnFeat& f,
                   const uint16_t* w, const float* bias, int cout, uint16_t* y, uint16_t* feat_out, hipStream_t s) {
  if (n % 4) return hipErrorInvalidValue;
  const long P = (long)B * (n / 4) * (n / 4);
  const dim3 grid((unsigned)((P + 63) / 64));
  if (cout == 32)
    hipLaunchKernelGGL(stem_kernel<2>, grid, dim3(256), 0, s, q, v, m, idx, n, B, f, w, bias, y, feat_out);
  else if (cout == 64)
    hipLaunchKernelGGL(stem_kernel<4>, grid, dim3(256), 0, s, q, v, m, idx, n, B, f, w, bias, y, feat_out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t nn_mse_grad(const float* y, const float* t, const int* idx, int n, int B, float out_scale, uint16_t* dh,
                       float* part, hipStream_t s) {
  if (n % 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(kNnMseBlocks), dim3(256), 0, s, y, t, idx, n, B, out_scale, dh, part);
  return hipGetLastError();
}

hipError_t nn_adam(float* p, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                   float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t nn_weight_cast(const float* src, int cout, int taps, int cin_src, int cin_pad, uint16_t* dst,
                          uint16_t* dstT, hipStream_t s, int blocked) {
  if (blocked && ((cout % 16) || (cin_pad % 16))) return hipErrorInvalidValue;
  const long n = (long)cout * taps * cin_pad;
  hipLaunchKernelGGL(weight_cast_kernel<float>, dim3(blocks_for(n)), dim3(256), 0, s, src, cout, taps, cin_src, cin_pad,
                     dst, dstT, blocked);
  return hipGetLastError();
}

hipError_t nn_weight_cast_bf16(const uint16_t* src, int cout, int taps, int cin_src, int cin_pad, uint16_t* dst,
                               uint16_t* dstT, hipStream_t s) {
  const long n = (long)cout * taps * cin_pad;
  hipLaunchKernelGGL(weight_cast_kernel<uint16_t>, dim3(blocks_for(n)), dim3(256), 0, s, src, cout, taps, cin_src,
                     cin_pad, dst, dstT, 0);
  return hipGetLastError();
}

}  // namespace vs
