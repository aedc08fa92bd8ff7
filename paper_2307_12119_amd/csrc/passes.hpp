// Device helpers shared by the steady and transient passes: launch shapes, slot I/O of the
// register-resident row transforms, the pointwise physics (leakage law, Kirchhoff inverse of
// k(T)) and wavefront reductions.
#pragma once

#include <cmath>

#include "common.hpp"
#include "fft.hpp"

namespace vs {

template <int N>
struct RowCfg {
  static constexpr int TPF = Shape<N>::TPF;
  static constexpr int FFTS = (256 / TPF) < (N / 2) ? (256 / TPF) : (N / 2);
  static constexpr int THREADS = FFTS * TPF;
  static constexpr int WAVE = THREADS < 64 ? THREADS : 64;
  static constexpr int WAVES = THREADS / WAVE;
};

// columns per column-pass workgroup: at most 16, LDS <= 40 KB (two workgroups per CU),
// <= 512 threads
constexpr int col_count(int n, int esz, int tpf) {
  int c = 16;
  while (c > 2 && ((long)c * (n + n / 8 + 4) * esz > 40000 || (c / 2) * tpf > 512)) c /= 2;
  return c < n ? c : n;
}

// Workgroups are handed to the 8 XCDs round-robin in launch order; renumber them so that
// consecutive tiles (neighbouring column strips of one map, which share L2 lines) run on the
// same XCD.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ void xcd_tile(int& strip, int& map) {
  const int gx = gridDim.x, g = gx * gridDim.y;
  const int w = blockIdx.x + gx * blockIdx.y;
  const int l = (g & 7) ? w : (w & 7) * (g >> 3) + (w >> 3);
  strip = l % gx;
  map = l / gx;
}

// COLS_ = 0: the default strip width (col_count); otherwise an explicit even width.  Each
// transform group (one wavefront at N >= 512) handles PAIRS column pairs one after the other,
// so a strip can be wider (longer contiguous row segments) without more threads.
// INPL_: each pair's transform scratch is its own two tile columns (element i of the padded
// scratch at tile row lds_at(i)), so the tile needs no separate scratch and a wider strip fits
// two workgroups per CU.
template <typename Tc, int N, int COLS_ = 0, int PAIRS_ = 1, bool INPL_ = false>
struct ColCfg {
  static constexpr int TPF = Shape<N>::TPF;
  static constexpr int COLS = COLS_ ? (COLS_ < N ? COLS_ : N) : col_count(N, (int)sizeof(Tc), TPF);
  static constexpr int PAIRS = COLS / 2 >= PAIRS_ ? PAIRS_ : 1;
  static constexpr int FFTS = COLS / (2 * PAIRS);
  static constexpr int THREADS = FFTS * TPF;
  static constexpr int VEC = (int)(16 / sizeof(Tc)) < COLS ? (int)(16 / sizeof(Tc)) : COLS;
  // Staging tile [N][PITCH].  For N >= 256 its rows are stored in transform-slot order (row y
  // at slot perm(y)), so the column reads of a half-wavefront walk consecutive tile rows; with
  // pitch COLS + 1 that costs 1.5x the conflict-free LDS time against 2x in natural order.
  static constexpr bool SLOT = N >= 256;
  static constexpr bool INPL = INPL_;
  static constexpr int PITCH = (SLOT || INPL) ? COLS + 1 : (sizeof(Tc) == 4 ? COLS + 3 : COLS + 1);
  // tile rows: N, or the padded transform length when the scratch lives in the tile
  static constexpr int ROWS = INPL ? Shape<N>::STRIDE : N;
  static constexpr int TILE = ROWS * PITCH;
  static constexpr int SCRATCH = INPL ? 0 : FFTS * 2 * Shape<N>::STRIDE;
  // several column pairs per transform group: the transform scratch follows the tile, so each
  // pair is read from the tile only when its turn comes (one pair's values in registers)
  static constexpr bool LAZY = !INPL && PAIRS > 1;
  static constexpr int LDS = INPL ? TILE : (LAZY ? TILE + SCRATCH : (TILE > SCRATCH ? TILE : SCRATCH));
  // row-segment vectors each thread moves per tile
  static constexpr int LOADS = N * (COLS / VEC) / THREADS;
};

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
  T v[V];
};

// tile row of natural row y, and of transform slot k
template <typename Cfg, int N>
__device__ __forceinline__ int tile_row(int y) {
  return Cfg::SLOT ? perm<N>(y) : y;
}
template <typename Cfg, int N>
__device__ __forceinline__ int tile_slot(int k) {
  return Cfg::SLOT ? k : unperm<N>(k);
}

// Row values at the sample positions of this lane's slots (slot m <-> reordered index
// t + TPF m).  Each lane loads the adjacent pair (2k, 2k+1) of its even slot k = t + TPF m;
// the odd sample 2k+1 belongs to slot E-1-m of the mirror lane TPF-1-t and is swapped over.
// NT: non-temporal loads, for maps streamed once per pass (a batch's inputs outgrow the caches
// between passes); callers that re-read a map while it is still cached keep the default.
template <typename Tio, typename Tc, int N, bool NT = false>
__device__ __forceinline__ void load_slots(const Tio* __restrict__ row, Tc* out, int t, int mirror) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  typedef Tio pair_t __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
    const pair_t* p = reinterpret_cast<const pair_t*>(row + 2 * (t + TPF * m));
    const pair_t v = NT ? __builtin_nontemporal_load(p) : *p;
    out[m] = (Tc)v.x;
    out[E - 1 - m] = (Tc)lane_get(v.y, mirror);
  }
}

template <typename Tio, typename Tc, int N, bool NT = false>
__device__ __forceinline__ void store_slots(Tio* __restrict__ row, const Tc* val, int t, int mirror) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  typedef Tio pair_t __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
    pair_t v;
    v.x = (Tio)val[m];
    v.y = lane_get((Tio)val[E - 1 - m], mirror);
    pair_t* p = reinterpret_cast<pair_t*>(row + 2 * (t + TPF * m));
    if (NT)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
}

// Column-pass step between the forward and inverse column DFTs of a packed column pair: split
// into the two columns' cosine coefficients at (p, N - p), multiply by lambda, merge back.  ka, kb:
// the columns' (alpha, beta, gamma) at min(p, N - p); hi: p >= N / 2 (beta negated).  (zr, zi):
// Z[p] of the forward DFT, (pr, pim): Z[N - p]; (zr, zi) is overwritten with the merged Z[p] of
// the inverse.
template <typename Tc>
__device__ __forceinline__ void lambda_pair(const Vec<Tc, 4>& ka, const Vec<Tc, 4>& kb, bool hi, Tc& zr, Tc& zi,
                                            Tc pr, Tc pim) {
  const Tc ba = hi ? -ka.v[1] : ka.v[1], bb = hi ? -kb.v[1] : kb.v[1];
  const Tc u = zr + pr, v = zi - pim, w = zi + pim, x = pr - zr;
  zr = dot2(ka.v[0], u, ba, v) - dot2(bb, w, kb.v[2], x);
  zi = dot2(ba, u, ka.v[2], v) + dot2(kb.v[0], w, bb, x);
}

template <typename T>
__device__ __forceinline__ T ldm(const void* p, long i) {
  return ((const T*)p)[i];
}

// order-preserving key of a float for packed max / argmax
__device__ __forceinline__ unsigned order_key(float v) {
  const unsigned u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ unsigned long long pack_max(float v, long idx) {
  return ((unsigned long long)order_key(v) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)idx);
}

__device__ __forceinline__ float exp_leak(float x) { return __expf(x); }
__device__ __forceinline__ double exp_leak(double x) { return exp(x); }

template <typename Tc>
__device__ __forceinline__ Tc leak_factor(Tc dT, const PointParams& pp) {
  if (pp.leak == VARSIM_LEAK_EXP) return exp_leak((Tc)pp.beta * dT);
  if (pp.leak == VARSIM_LEAK_LINEAR) return (Tc)1 + (Tc)pp.beta * dT;
  return (Tc)0;
}

// dT = Phi^-1(theta) for k = k_ref (T / T_amb)^-eta (Kirchhoff inverse).  NaN outside the
// law's domain (1 + (1 - eta) theta / T_amb <= 0), which the caller reports as runaway.
template <typename Tc>
__device__ __forceinline__ Tc kirchhoff_inv(Tc theta, const PointParams& pp) {
  if (pp.eta_mode == 0) return theta;
  const Tc u = (Tc)pp.u_scale * theta;
  if constexpr (sizeof(Tc) == 4) {
    // FP32: Horner form of the Taylor series of (1 + u)^a - 1 (exp(u) - 1 for eta = 1) where
    // the first dropped term is negligible (|u| <= poly_umax <= 0.1); beyond it there is no
    // cancellation and the hardware exp2 / log2 (relative error ~1e-6) keep the code short.
    if (fabsf(u) <= (float)pp.poly_umax) {
      float acc = pp.polyf[kPoly - 1];
#pragma unroll
      for (int k = kPoly - 2; k >= 0; --k) acc = fmaf(acc, u, pp.polyf[k]);
      return (float)pp.t_amb * u * acc;
    }
    if (pp.eta_mode == 1) return (float)pp.t_amb * (__expf(u) - 1.f);
    if (!(u > -1.f)) return NAN;
    return (float)pp.t_amb * (__expf((float)pp.inv_1m_eta * __logf(1.f + u)) - 1.f);
  } else {
    // FP64: the same series to degree kPoly64 inside its range (about a tenth of the cost of
    // log1p + expm1, which the compiler inlines per element), the library forms beyond it
    if (fabs(u) <= pp.poly_umax64) {
      double acc = pp.polyd[kPoly64 - 1];
#pragma unroll
      for (int k = kPoly64 - 2; k >= 0; --k) acc = fma(acc, u, pp.polyd[k]);
      return pp.t_amb * u * acc;
    }
    if (pp.eta_mode == 1) return (Tc)pp.t_amb * expm1(u);
    if (!(u > (Tc)-1)) return (Tc)NAN;
    return (Tc)pp.t_amb * expm1((Tc)pp.inv_1m_eta * log1p(u));
  }
}

template <int W>
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
  return v;
}
template <int W>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W>
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, W);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ bool finished_before(const IterState& st, int map, int iter, double tol) {
  if (iter < 2) return false;
  const double prev = __longlong_as_double((long long)st.resid[(long)map * st.stride + iter - 1]);
  return prev <= tol;
}

}  // namespace vs
