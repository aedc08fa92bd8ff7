// Transient-solve passes with each row (or column) spread over two wavefronts (Eqs. Ttran,
// tranGreen, tranapprox; Sec. IV-E).
//
// The step is the one of transient1.hip (column pass: DCT-II down the columns, per-mode update,
// DCT-III; row pass: DCT-III, conductivity factor, Kirchhoff inverse, power of the next step,
// DCT-II), each real sequence of length N again going through a complex DFT of M = N / 2 points,
// but that DFT is split in frequency into two DFTs of N / 4 points (single.hpp, dct2_split /
// dct3_split), one per wavefront: wavefront 0 owns the even cosine coefficients, wavefront 1 the
// odd ones.  The two wavefronts of a sequence meet twice through LDS: in the row pass after the
// synthesis (z[j] = A[j] +- B[j]) and before the analysis (a[j], b[j] from z[j] and z[j + N/4]);
// in the column pass the analysis inputs come straight from the staged strip and the synthesis
// halves meet once before the strip is written back.  A single 1024 x 1024 map thus gives two
// wavefronts per SIMD instead of one, and each wavefront's serial chain (loads, transforms,
// physics, stores) is half as long.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "single.hpp"
#include "trpoint.hpp"

namespace vs {

namespace {

// RPW rows per workgroup, two wavefronts per row
template <typename Tc, int N, int RPW>
struct TrRow2Cfg {
  using Sh = SplitShape<N>;
  static constexpr int H = Sh::H, EL = Sh::EL;
  static constexpr int THREADS = 128 * RPW;
  static constexpr int ST = Shape<H>::STRIDE;
};

template <typename Tio, typename Tc, int N, int MODE, int RPW>
__global__ void __launch_bounds__((TrRow2Cfg<Tc, N, RPW>::THREADS))
    transient_row2_kernel(TransArgs a, int step, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = TrRow2Cfg<Tc, N, RPW>;
  constexpr int H = Cfg::H, EL = Cfg::EL, ST = Cfg::ST;
  constexpr bool INV = MODE != TR_HEAD;
  constexpr bool FWD = MODE != TR_LAST;
  __shared__ Tc s_re[2 * RPW * ST];
  __shared__ Tc s_im[2 * RPW * ST];
  // per row and wavefront: the synthesis half (A or B) and the new power values, re / im
  __shared__ Tc x_inv[INV ? RPW * 2 * 2 * H : 1];
  __shared__ Tc x_fwd[FWD ? RPW * 2 * 2 * H : 1];

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int h = wave & 1, r = wave >> 1;
  const int t = threadIdx.x % 64;
  const int row = blockIdx.x * RPW + r;
  Tc* re = s_re + wave * ST;
  Tc* im = s_im + wave * ST;
  const long off = (long)row * N;
  Tc* const Srow = (Tc*)a.S + off;
  const PointParams& pp = a.pp;
  // z-order index of slot m: j = h H + t + 64 m (wavefront 0: z[j], wavefront 1: z[j + H])
  const int jz0 = h * H + t;

  Tc zr[EL], zi[EL];
  if constexpr (INV) {
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const int p = 2 * (t + 64 * m) + h;
      zr[m] = Srow[p];
      zi[m] = Srow[spec_hi<N>(p)];
    }
  }
  Tc qd[2 * EL], ql[2 * EL], mv[2 * EL];
  const bool has_ql = a.qlz != nullptr, has_mv = a.minvz != nullptr;
  if constexpr (FWD) {
    const Vec<int, 2>* ids = reinterpret_cast<const Vec<int, 2>*>(a.idz + off);
    const Tio* tr = (const Tio*)a.trace + (long)step * a.n_blocks;  // trace row `step` holds step step+1
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const Vec<int, 2> id = ids[jz0 + 64 * m];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int b = id.v[k];
        const Tc v = (Tc)tr[b < 0 ? 0 : b];
        qd[k * EL + m] = b < 0 ? (Tc)0 : v;
      }
    }
    if (has_ql) {
      const Vec<Tio, 2>* src = reinterpret_cast<const Vec<Tio, 2>*>((const Tio*)a.qlz + off);
#pragma unroll
      for (int m = 0; m < EL; ++m) {
        const Vec<Tio, 2> v = src[jz0 + 64 * m];
        ql[m] = (Tc)v.v[0];
        ql[EL + m] = (Tc)v.v[1];
      }
    }
  }
  const bool mv_inv = INV && has_mv && !pp.cond_src, mv_fwd = FWD && has_mv && pp.cond_src;
  if (mv_inv || mv_fwd) {
    const Vec<Tio, 2>* src = reinterpret_cast<const Vec<Tio, 2>*>((const Tio*)a.minvz + off);
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const Vec<Tio, 2> v = src[jz0 + 64 * m];
      mv[m] = (Tc)v.v[0];
      mv[EL + m] = (Tc)v.v[1];
    }
  }

  // x[k EL + m]: sample z_sample(jz0 + 64 m, k) of this row
  Tc x[2 * EL];
  bool bad = false;
  if constexpr (INV) {
    dct3_split<Tc, N>(zr, zi, re, im, tw, qw, t, h);
    Tc* mine = x_inv + (r * 2 + h) * 2 * H;
    const Tc* other = x_inv + (r * 2 + (h ^ 1)) * 2 * H;
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      mine[t + 64 * m] = zr[m];
      mine[H + t + 64 * m] = zi[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const Tc orr = other[t + 64 * m], oi = other[H + t + 64 * m];
      // z[j] = A[j] + B[j] (wavefront 0), z[j + H] = A[j] - B[j] (wavefront 1)
      x[m] = h == 0 ? zr[m] + orr : orr - zr[m];
      x[EL + m] = h == 0 ? zi[m] + oi : oi - zi[m];
    }
    if (mv_inv) {
#pragma unroll
      for (int k = 0; k < 2 * EL; ++k) x[k] *= mv[k];
    }
    kirchhoff_inv_n<Tc, 2 * EL>(x, pp);
#pragma unroll
    for (int k = 0; k < 2 * EL; ++k) {
      x[k] = (Tc)(Tio)x[k];  // the rise as stored
      bad = bad || !(x[k] <= (Tc)pp.cap) || !(x[k] == x[k]);
    }
    const bool snap = a.snaps && (step % a.out_every == 0);
    if (snap || MODE == TR_LAST) {
      Tio* dst = MODE == TR_LAST ? (Tio*)a.dT + off : (Tio*)a.snaps + (long)(step / a.out_every - 1) * N * N + off;
      if (MODE == TR_LAST && snap) {
        Tio* d2 = (Tio*)a.snaps + (long)(step / a.out_every - 1) * N * N + off;
#pragma unroll
        for (int m = 0; m < EL; ++m) {
          const int j = jz0 + 64 * m;
          d2[z_sample<N>(j, 0)] = (Tio)x[m];
          d2[z_sample<N>(j, 1)] = (Tio)x[EL + m];
        }
      }
#pragma unroll
      for (int m = 0; m < EL; ++m) {
        const int j = jz0 + 64 * m;
        dst[z_sample<N>(j, 0)] = (Tio)x[m];
        dst[z_sample<N>(j, 1)] = (Tio)x[EL + m];
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 2 * EL; ++k) x[k] = (Tc)0;
  }
  if (INV && __any(bad) && t == 0) atomicOr(a.flags, kFlagRunaway);

  if constexpr (FWD) {
    // P_{n+1} = hx hy (q_dyn + QL L(dT_n)) at this wavefront's z values, then the split inputs
    if (has_ql) add_leakage_n<Tc, 2 * EL>(qd, ql, x, pp);
    const Tc hh = (Tc)pp.hxhy;
    Tc pr[EL], pi[EL];
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      pr[m] = hh * qd[m];
      pi[m] = hh * qd[EL + m];
    }
    if (mv_fwd) {
#pragma unroll
      for (int m = 0; m < EL; ++m) {
        pr[m] *= mv[m];
        pi[m] *= mv[EL + m];
      }
    }
    Tc* mine = x_fwd + (r * 2 + h) * 2 * H;
    const Tc* other = x_fwd + (r * 2 + (h ^ 1)) * 2 * H;
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      mine[t + 64 * m] = pr[m];
      mine[H + t + 64 * m] = pi[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const int j = t + 64 * m;
      const Tc orr = other[j], oi = other[H + j];
      // wavefront 0 holds z[j] and reads z[j + H]; wavefront 1 the other way round
      if (h == 0)
        split_inputs<Tc, N>(zr[m], zi[m], pr[m], pi[m], orr, oi, j, 0, tw);
      else
        split_inputs<Tc, N>(zr[m], zi[m], orr, oi, pr[m], pi[m], j, 1, tw);
    }
    dct2_split<Tc, N>(zr, zi, re, im, tw, qw, t, h);
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const int p = 2 * (t + 64 * m) + h;
      Srow[p] = zr[m];
      Srow[spec_hi<N>(p)] = zi[m];
    }
  }
}

// Column pass: COLS columns per workgroup, two wavefronts per column.  The strip is staged in
// LDS with its rows in z order (as transient1.hip); the transform scratch of the wavefronts
// follows the tile and carries the synthesis halves from one wavefront of a column to the other.
template <typename Tc, int N, int COLS_>
struct TrCol2Cfg {
  using Sh = SplitShape<N>;
  static constexpr int M = Sh::M, H = Sh::H, EL = Sh::EL;
  static constexpr int COLS = COLS_;
  static constexpr int THREADS = COLS * 128;
  static constexpr int VEC = (int)(16 / sizeof(Tc)) < COLS ? (int)(16 / sizeof(Tc)) : COLS;
  static constexpr int VPR = COLS / VEC;
  static constexpr int PITCH = COLS + 1;
  static constexpr int TILE = N * PITCH;
  static constexpr int ST = Shape<H>::STRIDE;
  static constexpr int SCRATCH = 2 * COLS * 2 * ST;
  static constexpr int LDS = TILE + SCRATCH;
};

template <typename Tc, int N, int COLS, bool FIR>
__global__ void __launch_bounds__((TrCol2Cfg<Tc, N, COLS>::THREADS))
    transient_col2_kernel(TransArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = TrCol2Cfg<Tc, N, COLS>;
  constexpr int M = Cfg::M, H = Cfg::H, EL = Cfg::EL, ST = Cfg::ST;
  constexpr int VEC = Cfg::VEC, VPR = Cfg::VPR, P = Cfg::PITCH;
  __shared__ Tc lds[Cfg::LDS];

  int strip, map;
  xcd_tile(strip, map);
  Tc* S = (Tc*)a.S;
  const int c0 = strip * COLS;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int h = wave & 1, f = wave >> 1;
  const int t = threadIdx.x % 64;

  // (a, b) and state of column q at this wavefront's modes p = 2 (t + 64 m) + h and hi(p)
  const int q = c0 + f;
  Tc* st = (Tc*)a.state + (long)q * N;
  const Vec<Tc, 2>* ab = reinterpret_cast<const Vec<Tc, 2>*>(a.ab) + (long)q * N;
  Vec<Tc, 2> k0[EL], k1[EL];
  Tc s0[EL], s1[EL];
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int p = 2 * (t + 64 * m) + h, hp = spec_hi<N>(p);
    k0[m] = ab[p];
    k1[m] = ab[hp];
    s0[m] = st[p];
    s1[m] = st[hp];
  }

  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Vec<Tc, VEC> v = *reinterpret_cast<const Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC);
    Tc* d = lds + z_row<N>(y) * P + j * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = v.v[e];
  }
  __syncthreads();

  // z[j] at tile rows j (real) and M + j (imaginary); z[j + H] at rows H + j and M + H + j
  Tc zr[EL], zi[EL];
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int j = t + 64 * m;
    split_inputs<Tc, N>(zr[m], zi[m], lds[j * P + f], lds[(M + j) * P + f], lds[(H + j) * P + f],
                        lds[(M + H + j) * P + f], j, h, tw);
  }
  Tc* re = lds + Cfg::TILE + wave * 2 * ST;
  Tc* im = re + ST;
  dct2_split<Tc, N>(zr, zi, re, im, tw, qw, t, h);
  Tc* rg = FIR ? (Tc*)a.ring + (long)a.slot * N * N + (long)q * N : nullptr;
  const Tc* fc = FIR ? (const Tc*)a.fir + (long)q * N : nullptr;
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int p = 2 * (t + 64 * m) + h, hp = spec_hi<N>(p);
    zr[m] = mode_step<Tc, FIR>(zr[m], k0[m], s0[m], st, ab, rg, fc, (long)N * N, a.poles, p);
    zi[m] = mode_step<Tc, FIR>(zi[m], k1[m], s1[m], st, ab, rg, fc, (long)N * N, a.poles, hp);
  }
  dct3_split<Tc, N>(zr, zi, re, im, tw, qw, t, h);
  // this wavefront's half (A or B) into its own scratch, then the column's z values into the tile
  wave_sync();
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    re[t + 64 * m] = zr[m];
    im[t + 64 * m] = zi[m];
  }
  __syncthreads();
  const Tc* ore = lds + Cfg::TILE + (wave ^ 1) * 2 * ST;
  const Tc* oim = ore + ST;
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int j = t + 64 * m;
    const Tc orr = ore[j], oi = oim[j];
    if (h == 0) {  // z[j] = A[j] + B[j]
      lds[j * P + f] = zr[m] + orr;
      lds[(M + j) * P + f] = zi[m] + oi;
    } else {  // z[j + H] = A[j] - B[j]
      lds[(H + j) * P + f] = orr - zr[m];
      lds[(M + H + j) * P + f] = oi - zi[m];
    }
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

template <typename Tio, typename Tc, int N, int RPW>
hipError_t row2_shape(int mode, const TransArgs& a, int step, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = TrRow2Cfg<Tc, N, RPW>;
  static_assert(N % RPW == 0, "rows per workgroup must divide the grid");
  const dim3 grid(N / RPW), block(Cfg::THREADS);
  switch (mode) {
    case TR_HEAD:
      hipLaunchKernelGGL((transient_row2_kernel<Tio, Tc, N, TR_HEAD, RPW>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_MERGED:
      hipLaunchKernelGGL((transient_row2_kernel<Tio, Tc, N, TR_MERGED, RPW>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_LAST:
      hipLaunchKernelGGL((transient_row2_kernel<Tio, Tc, N, TR_LAST, RPW>), grid, block, 0, s, a, step, tw, qw);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Tc, int N, int COLS>
hipError_t col2_shape(const TransArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = TrCol2Cfg<Tc, N, COLS>;
  static_assert(N % COLS == 0, "strips must tile the columns");
  if (a.ring)
    hipLaunchKernelGGL((transient_col2_kernel<Tc, N, COLS, true>), dim3(N / COLS, 1), dim3(Cfg::THREADS), 0, s, a,
                       tw, qw);
  else
    hipLaunchKernelGGL((transient_col2_kernel<Tc, N, COLS, false>), dim3(N / COLS, 1), dim3(Cfg::THREADS), 0, s, a,
                       tw, qw);
  return hipGetLastError();
}

// candidates: 0 = one row per workgroup / four columns per strip, 1 = two rows / two columns
template <typename T, int N>
hipError_t tr2_launch(int which, int mode, int v, const TransArgs& a, int step, hipStream_t s) {
  const Cx<T>* tw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.tw32 : (const Cx<T>*)a.tw.tw64;
  const Cx<T>* qw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.qw32 : (const Cx<T>*)a.tw.qw64;
  if (which == 0) {
    switch (v) {
      case 0: return row2_shape<T, T, N, 1>(mode, a, step, tw, qw, s);
      case 1: return row2_shape<T, T, N, 2>(mode, a, step, tw, qw, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (v) {
    case 0: return col2_shape<T, N, 4>(a, tw, qw, s);
    case 1: return col2_shape<T, N, 2>(a, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool transient_split_ok(int n) { return n == 1024; }

hipError_t launch_transient_row2(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant) {
  if (a.n != 1024) return hipErrorInvalidValue;
  return io == VARSIM_F32 ? tr2_launch<float, 1024>(0, mode, variant, a, step, stream)
                          : tr2_launch<double, 1024>(0, mode, variant, a, step, stream);
}

hipError_t launch_transient_col2(int io, const TransArgs& a, hipStream_t stream, int variant) {
  if (a.n != 1024) return hipErrorInvalidValue;
  return io == VARSIM_F32 ? tr2_launch<float, 1024>(1, 0, variant, a, 0, stream)
                          : tr2_launch<double, 1024>(1, 0, variant, a, 0, stream);
}

}  // namespace vs
