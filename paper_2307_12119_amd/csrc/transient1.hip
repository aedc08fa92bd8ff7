// Transient-solve passes with one row (or one column) per transform group (Eqs. Ttran,
// tranGreen, tranapprox; Sec. IV-E).
//
// The same step as transient.hip computes (column pass: DCT-II down the columns, per-mode
// update theta_hat = a theta_hat + b P_hat, DCT-III; row pass: DCT-III, conductivity factor,
// Kirchhoff inverse, power of the next step, DCT-II), but each real sequence goes through a
// complex DFT of half its length (single.hpp) instead of sharing a full-length DFT with a second
// sequence.  A group then holds half as many elements per lane and one map yields twice as many
// wavefronts, which is what a single transient map needs: its passes are too small to fill the
// chip, so the time of one wavefront's serial chain sets the time of the pass.
//
// The row pass reads the static per-cell inputs (block ids, leakage density, 1 / conductivity
// multiplier) from copies in z order, made once per solve by zorder_kernel, so that every lane
// loads its own samples with contiguous vector loads.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "trpoint.hpp"
#include "single.hpp"

namespace vs {

namespace {

// dst[row][2j + k] = src[row][sample of part k of z[j]]
template <typename T>
__global__ void __launch_bounds__(256) zorder_kernel(const T* __restrict__ src, T* __restrict__ dst, int n) {
  const int row = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = i >> 1, k = i & 1;
  const int y = j < n / 4 ? 4 * j + 2 * k : 2 * n - 4 * j - 1 - 2 * k;
  dst[(long)row * n + i] = src[(long)row * n + y];
}

template <int N, int W>
struct TrRow1Cfg {
  static constexpr int M = N / 2;
  static constexpr int E = Shape<M>::E, TPF = Shape<M>::TPF;
  static constexpr int THREADS = 64 * W;   // W wavefronts
  static constexpr int ROWS = THREADS / TPF;  // one row per group of TPF lanes
};

template <typename Tio, typename Tc, int N, int MODE, int W>
__global__ void __launch_bounds__((TrRow1Cfg<N, W>::THREADS))
    transient_row1_kernel(TransArgs a, int step, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = TrRow1Cfg<N, W>;
  constexpr int M = Cfg::M, E = Cfg::E, TPF = Cfg::TPF;
  constexpr int ST = Shape<M>::STRIDE;
  constexpr bool INV = MODE != TR_HEAD;
  constexpr bool FWD = MODE != TR_LAST;
  __shared__ Tc s_re[Cfg::ROWS * ST];
  __shared__ Tc s_im[Cfg::ROWS * ST];

  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  const int row = blockIdx.x * Cfg::ROWS + f;
  Tc* re = s_re + f * ST;
  Tc* im = s_im + f * ST;
  const long off = (long)row * N;
  Tc* const Srow = (Tc*)a.S + off;
  const PointParams& pp = a.pp;

  // row spectrum of the previous column pass: (X[p], X[hi(p)]) per slot
  Tc zr[E], zi[E];
  if constexpr (INV) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m;
      zr[m] = Srow[p];
      zi[m] = Srow[spec_hi<N>(p)];
    }
  }
  // static inputs of this lane's samples, issued before the transform so that their latency
  // overlaps it: dynamic power of the next step from block ids + trace, leakage density, 1/m
  Tc qd[2 * E], ql[2 * E], mv[2 * E];
  const bool has_ql = a.qlz != nullptr, has_mv = a.minvz != nullptr;
  if constexpr (FWD) {
    const Vec<int, 2>* ids = reinterpret_cast<const Vec<int, 2>*>(a.idz + off);
    const Tio* tr = (const Tio*)a.trace + (long)step * a.n_blocks;  // trace row `step` holds step step+1
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const Vec<int, 2> id = ids[t + TPF * m];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int b = id.v[k];
        const Tc v = (Tc)tr[b < 0 ? 0 : b];
        qd[k * E + m] = b < 0 ? (Tc)0 : v;
      }
    }
    if (has_ql) {
      const Vec<Tio, 2>* src = reinterpret_cast<const Vec<Tio, 2>*>((const Tio*)a.qlz + off);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const Vec<Tio, 2> v = src[t + TPF * m];
        ql[m] = (Tc)v.v[0];
        ql[E + m] = (Tc)v.v[1];
      }
    }
  }
  // 1/m acts on the rise (target side, inverse half) or on the next power map (source side)
  const bool mv_inv = INV && has_mv && !pp.cond_src, mv_fwd = FWD && has_mv && pp.cond_src;
  if (mv_inv || mv_fwd) {
    const Vec<Tio, 2>* src = reinterpret_cast<const Vec<Tio, 2>*>((const Tio*)a.minvz + off);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const Vec<Tio, 2> v = src[t + TPF * m];
      mv[m] = (Tc)v.v[0];
      mv[E + m] = (Tc)v.v[1];
    }
  }

  // x[k E + m]: sample z_sample(t + TPF m, k) of this row
  Tc x[2 * E];
  bool bad = false;
  if constexpr (INV) {
    dct3_single<Tc, N>(zr, zi, re, im, tw, qw, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      x[m] = zr[m];
      x[E + m] = zi[m];
    }
    if (mv_inv) {
#pragma unroll
      for (int k = 0; k < 2 * E; ++k) x[k] *= mv[k];
    }
    kirchhoff_inv_n<Tc, 2 * E>(x, pp);
#pragma unroll
    for (int k = 0; k < 2 * E; ++k) {
      x[k] = (Tc)(Tio)x[k];  // the rise as stored
      bad = bad || !(x[k] <= (Tc)pp.cap) || !(x[k] == x[k]);
    }
    const bool snap = a.snaps && (step % a.out_every == 0);
    if (snap || MODE == TR_LAST) {
      Tio* dst = MODE == TR_LAST ? (Tio*)a.dT + off : (Tio*)a.snaps + (long)(step / a.out_every - 1) * N * N + off;
      if (MODE == TR_LAST && snap) {
        Tio* d2 = (Tio*)a.snaps + (long)(step / a.out_every - 1) * N * N + off;
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int j = t + TPF * m;
          d2[z_sample<N>(j, 0)] = (Tio)x[m];
          d2[z_sample<N>(j, 1)] = (Tio)x[E + m];
        }
      }
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int j = t + TPF * m;
        dst[z_sample<N>(j, 0)] = (Tio)x[m];
        dst[z_sample<N>(j, 1)] = (Tio)x[E + m];
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 2 * E; ++k) x[k] = (Tc)0;
  }
  if (INV && __any(bad) && (__lane_id() & 63) == 0) atomicOr(a.flags, kFlagRunaway);

  if constexpr (FWD) {
    // P_{n+1} = hx hy (q_dyn + QL L(dT_n)), then its row spectrum
    if (has_ql) add_leakage_n<Tc, 2 * E>(qd, ql, x, pp);
    const Tc hh = (Tc)pp.hxhy;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      zr[m] = hh * qd[m];
      zi[m] = hh * qd[E + m];
    }
    if (mv_fwd) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        zr[m] *= mv[m];
        zi[m] *= mv[E + m];
      }
    }
    dct2_single<Tc, N>(zr, zi, re, im, tw, qw, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m;
      Srow[p] = zr[m];
      Srow[spec_hi<N>(p)] = zi[m];
    }
  }
}

// Column pass: COLS columns per workgroup, one per group of TPF lanes.  The strip is staged in
// LDS with its rows in z order (tile row z_row(y)), so that lane t of a group reads consecutive
// tile rows t + TPF m (real parts) and M + t + TPF m (imaginary parts); the pitch COLS + 1 is odd,
// so those reads fall in distinct banks.
template <typename Tc, int N, int COLS_>
struct TrCol1Cfg {
  static constexpr int M = N / 2;
  static constexpr int E = Shape<M>::E, TPF = Shape<M>::TPF;
  static constexpr int COLS = COLS_;
  static constexpr int THREADS = COLS * TPF;
  static constexpr int VEC = (int)(16 / sizeof(Tc)) < COLS ? (int)(16 / sizeof(Tc)) : COLS;
  static constexpr int VPR = COLS / VEC;
  static constexpr int PITCH = COLS + 1;
  static constexpr int TILE = N * PITCH;
  static constexpr int SCRATCH = COLS * 2 * Shape<M>::STRIDE;
  static constexpr int LDS = TILE > SCRATCH ? TILE : SCRATCH;
};

// FIR: the truncated history of a.hist steps (the ring of past spectra and the fir planes)
template <typename Tc, int N, int COLS, bool FIR>
__global__ void __launch_bounds__((TrCol1Cfg<Tc, N, COLS>::THREADS))
    transient_col1_kernel(TransArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = TrCol1Cfg<Tc, N, COLS>;
  constexpr int M = Cfg::M, E = Cfg::E, TPF = Cfg::TPF;
  constexpr int ST = Shape<M>::STRIDE;
  constexpr int VEC = Cfg::VEC, VPR = Cfg::VPR, P = Cfg::PITCH;
  __shared__ Tc lds[Cfg::LDS];

  int strip, map;
  xcd_tile(strip, map);
  Tc* S = (Tc*)a.S;
  const int c0 = strip * COLS;
  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;

  // per-mode (a, b) and spectral state of column q = c0 + f at modes p and hi(p); in FP32 they
  // are loaded before the strip so that their latency overlaps the strip load and the transform
  const int q = c0 + f;
  Tc* st = (Tc*)a.state + (long)q * N;
  const Vec<Tc, 2>* ab = reinterpret_cast<const Vec<Tc, 2>*>(a.ab) + (long)q * N;
  constexpr bool EARLY = sizeof(Tc) == 4;
  Vec<Tc, 2> k0[E], k1[E];
  Tc s0[E], s1[E];
  if constexpr (EARLY) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m, h = spec_hi<N>(p);
      k0[m] = ab[p];
      k1[m] = ab[h];
      s0[m] = st[p];
      s1[m] = st[h];
    }
  }

  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Vec<Tc, VEC> v = *reinterpret_cast<const Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC);
    Tc* d = lds + z_row<N>(y) * P + j * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = v.v[e];
  }
  __syncthreads();

  Tc zr[E], zi[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    zr[m] = lds[(t + TPF * m) * P + f];
    zi[m] = lds[(M + t + TPF * m) * P + f];
  }
  __syncthreads();

  Tc* re = lds + f * ST;  // all real parts first, then all imaginary parts
  Tc* im = lds + COLS * ST + f * ST;
  dct2_single<Tc, N>(zr, zi, re, im, tw, qw, t);
  if constexpr (!EARLY) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m, h = spec_hi<N>(p);
      k0[m] = ab[p];
      k1[m] = ab[h];
      s0[m] = st[p];
      s1[m] = st[h];
    }
  }
  // per-mode update at modes p and hi(p) (mode_step: further poles, truncated history)
  Tc* rg = FIR ? (Tc*)a.ring + (long)a.slot * N * N + (long)q * N : nullptr;
  const Tc* fc = FIR ? (const Tc*)a.fir + (long)q * N : nullptr;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int p = t + TPF * m, h = spec_hi<N>(p);
    zr[m] = mode_step<Tc, FIR>(zr[m], k0[m], s0[m], st, ab, rg, fc, (long)N * N, a.poles, p);
    zi[m] = mode_step<Tc, FIR>(zi[m], k1[m], s1[m], st, ab, rg, fc, (long)N * N, a.poles, h);
  }
  dct3_single<Tc, N>(zr, zi, re, im, tw, qw, t);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    lds[(t + TPF * m) * P + f] = zr[m];
    lds[(M + t + TPF * m) * P + f] = zi[m];
  }
  __syncthreads();
  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Tc* s = lds + z_row<N>(y) * P + j * VEC;
    Vec<Tc, VEC> v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = s[e];
    *reinterpret_cast<Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC) = v;
  }
}

template <typename Tio, typename Tc, int N, int W>
hipError_t row1_shape(int mode, const TransArgs& a, int step, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = TrRow1Cfg<N, W>;
  static_assert(N % Cfg::ROWS == 0, "rows per workgroup must divide the grid");
  const dim3 grid(N / Cfg::ROWS), block(Cfg::THREADS);
  switch (mode) {
    case TR_HEAD:
      hipLaunchKernelGGL((transient_row1_kernel<Tio, Tc, N, TR_HEAD, W>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_MERGED:
      hipLaunchKernelGGL((transient_row1_kernel<Tio, Tc, N, TR_MERGED, W>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_LAST:
      hipLaunchKernelGGL((transient_row1_kernel<Tio, Tc, N, TR_LAST, W>), grid, block, 0, s, a, step, tw, qw);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// strip widths: the widest that keeps the tile within 64 KB and the workgroup within 1024 lanes
// (at most 16 columns), then half and a quarter of it
template <typename Tc, int N>
constexpr int col1_max() {
  constexpr int tpf = Shape<N / 2>::TPF;
  int c = 16;
  while (c > 1 && ((long)N * (c + 1) * (long)sizeof(Tc) > 65536 || c * tpf > 1024)) c /= 2;
  return c < N ? c : N;
}
template <typename Tc, int N, int V>
constexpr int col1_cols() {
  constexpr int c = col1_max<Tc, N>() >> V;
  return c < 1 ? 1 : c;
}

template <typename Tc, int N, int COLS>
hipError_t col1_shape(const TransArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = TrCol1Cfg<Tc, N, COLS>;
  if (a.ring)
    hipLaunchKernelGGL((transient_col1_kernel<Tc, N, COLS, true>), dim3(N / COLS, 1), dim3(Cfg::THREADS), 0, s, a, tw,
                       qw);
  else
    hipLaunchKernelGGL((transient_col1_kernel<Tc, N, COLS, false>), dim3(N / COLS, 1), dim3(Cfg::THREADS), 0, s, a, tw,
                       qw);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t tr1_launch(int which, int mode, int v, const TransArgs& a, int step, hipStream_t s) {
  const Cx<T>* tw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.tw32 : (const Cx<T>*)a.tw.tw64;
  const Cx<T>* qw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.qw32 : (const Cx<T>*)a.tw.qw64;
  if (which == 0) {
    switch (v) {
      case 0: return row1_shape<T, T, N, 1>(mode, a, step, tw, qw, s);
      case 1: return row1_shape<T, T, N, 2>(mode, a, step, tw, qw, s);
      case 2: return row1_shape<T, T, N, 4>(mode, a, step, tw, qw, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (v) {
    case 0: return col1_shape<T, N, col1_cols<T, N, 0>()>(a, tw, qw, s);
    case 1: return col1_shape<T, N, col1_cols<T, N, 1>()>(a, tw, qw, s);
    case 2: return col1_shape<T, N, col1_cols<T, N, 2>()>(a, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t tr1_dispatch(int which, int mode, int v, int n, const TransArgs& a, int step, hipStream_t s) {
  switch (n) {
    case 64: return tr1_launch<T, 64>(which, mode, v, a, step, s);
    case 128: return tr1_launch<T, 128>(which, mode, v, a, step, s);
    case 256: return tr1_launch<T, 256>(which, mode, v, a, step, s);
    case 512: return tr1_launch<T, 512>(which, mode, v, a, step, s);
    case 1024: return tr1_launch<T, 1024>(which, mode, v, a, step, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool transient_single_ok(int n) { return n >= 64 && n <= 1024; }

hipError_t launch_zorder(int esz, const void* src, void* dst, int n, hipStream_t stream) {
  const dim3 grid((n + 255) / 256, n);
  if (esz == 4)
    hipLaunchKernelGGL(zorder_kernel<int>, grid, dim3(256), 0, stream, (const int*)src, (int*)dst, n);
  else
    hipLaunchKernelGGL(zorder_kernel<long long>, grid, dim3(256), 0, stream, (const long long*)src, (long long*)dst, n);
  return hipGetLastError();
}

hipError_t launch_transient_row1(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant) {
  return io == VARSIM_F32 ? tr1_dispatch<float>(0, mode, variant, a.n, a, step, stream)
                          : tr1_dispatch<double>(0, mode, variant, a.n, a, step, stream);
}

hipError_t launch_transient_col1(int io, const TransArgs& a, hipStream_t stream, int variant) {
  return io == VARSIM_F32 ? tr1_dispatch<float>(1, 0, variant, a.n, a, 0, stream)
                          : tr1_dispatch<double>(1, 0, variant, a.n, a, 0, stream);
}

}  // namespace vs
