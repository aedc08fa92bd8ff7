// The steady solve's row pass (one template for every mode; steady.hip launches the plain
// instantiations, steady_ct.hip the FP32 ones with compensated twiddles): per workgroup 2 FFTS
// rows of one map, each pair of rows packed into one complex transform of length N.
#pragma once

#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "rowops.hpp"

namespace vs {
namespace {  // each translation unit keeps its own instantiations

// Waves per SIMD the register allocation must leave room for: the FP32 merged pass of the
// two-pass sizes is HBM-bound and needs four to hide its load latency (it fits 128 VGPRs without
// spilling at N <= 512; at N = 1024 two, for 72 bytes of spills, against one wave per SIMD
// uncapped); other instantiations are left to the compiler.
template <typename Tio, typename Tc, int N, int MODE>
constexpr int row_min_waves() {
  if (sizeof(Tio) != 4 || sizeof(Tc) != 4 || MODE != ROW_MERGED) return 1;
  return N >= 128 && N <= 512 ? 4 : (N == 1024 ? 2 : 1);
}

// CT: compensated twiddles (twl, qwl: low parts of tw, qw; FP32 only)
template <typename Tio, typename Tc, int N, int MODE, bool CT = false>
__global__ void __launch_bounds__(RowCfg<N>::THREADS)
    __attribute__((amdgpu_waves_per_eu(row_min_waves<Tio, Tc, N, MODE>())))
    row_pass_kernel(PassArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw,
                    const Cx<Tc>* __restrict__ twl = nullptr, const Cx<Tc>* __restrict__ qwl = nullptr) {
  using Cfg = RowCfg<N>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int ST = Shape<N>::STRIDE;
  constexpr bool OS = MODE == ROW_OS_MID || MODE == ROW_OS_TAIL;
  constexpr bool AA = MODE == ROW_AA_EVAL || MODE == ROW_AA_MIX;
  constexpr bool INV = MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID || MODE == ROW_CONV_TAIL || OS ||
                       MODE == ROW_AA_EVAL;
  constexpr bool FWD = MODE == ROW_HEAD || MODE == ROW_MERGED || MODE == ROW_CONV_HEAD || MODE == ROW_OS_MID ||
                       MODE == ROW_AA_MIX;
  constexpr bool STATS = MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID || MODE == ROW_OS_TAIL ||
                         MODE == ROW_AA_EVAL;
  __shared__ Tc s_re[Cfg::FFTS * ST];
  __shared__ Tc s_im[Cfg::FFTS * ST];
  __shared__ double s_red[AA ? 5 : 3][Cfg::WAVES];
  __shared__ double s_gamma;

  // Maps in reverse launch order: the column pass walks them forward, so each pass starts on the
  // maps the previous one wrote last, which a batch larger than the 256 MB MALL still has there
  // (an LRU-like cache evicts first what a same-direction pass reads first).
  const int map = gridDim.y - 1 - blockIdx.y;
  unsigned flags = 0u;
  if (MODE != ROW_CONV_HEAD && MODE != ROW_CONV_TAIL) {
    flags = a.st.flags[map];
    if (flags & kFlagSkip) return;
    if ((MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_AA_EVAL) &&
        finished_before(a.st, map, a.iter, a.pp.tol))
      return;
    // the mixing pass follows this iteration's evaluation: a map that has just converged (or
    // converged before, its later increments staying 0) keeps G(x) in dT
    if (MODE == ROW_AA_MIX && __longlong_as_double((long long)a.st.resid[(long)map * a.st.stride + a.iter]) <= a.pp.tol)
      return;
  }
  const MapPtrs mp = a.maps[map];
  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  const int mirror = (__lane_id() & ~(TPF - 1)) + (TPF - 1 - t);
  const int row = (blockIdx.x * Cfg::FFTS + f) * 2;
  Tc* re = s_re + f * ST;
  Tc* im = s_im + f * ST;
  Tc* const Sa = (Tc*)(a.use_s64 ? mp.S64 : mp.S) + (long)row * N;
  Tc* const Sb = Sa + N;
  const long oa = (long)row * N, ob = oa + N;
  const PointParams& pp = a.pp;

  // slot m of this lane holds spectrum index / reordered sample t + TPF m
  Tc zr[E], zi[E];

  // ---- inverse half: spectrum rows -> theta (row DCT-III of the packed pair)
  if constexpr (INV) {
    Tc xa[E], xb[E], xa2[E], xb2[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      xa[m] = Sa[t + TPF * m];
      xb[m] = Sb[t + TPF * m];
    }
    partner<Tc, N, false>(xa, xa2, t);
    partner<Tc, N, false>(xb, xb2, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const Cx<Tc> q = qw[t + TPF * m];
      if constexpr (CT) {
        const Cx<Tc> ql = qwl[t + TPF * m];
        merge_pair_ct<Tc>(xa[m], xb[m], xa2[m], xb2[m], q.r, q.i, ql.r, ql.i, zr[m], zi[m]);
      } else {
        merge_pair<Tc>(xa[m], xb[m], xa2[m], xb2[m], q.r, q.i, zr[m], zi[m]);
      }
    }
    fft_reg<Tc, N, +1, 1, CT>(zr, zi, re, im, tw, t, twl);
  }

  // ---- pointwise: conductivity factor, Kirchhoff inverse, increment, stats, new power
  LaneStats<Tc> ls;
  const bool zero_old = (a.iter == 1) && (a.zero_start || (flags & kFlagWarmRejected));
  double d1 = 0.0, d2 = 0.0;  // Anderson dot products of this lane
  if constexpr (MODE == ROW_AA_MIX) {
    // gamma = <df, f> / <df, df> from the evaluation's per-workgroup sums, added in index order
    // (every workgroup of the map gets the same bits)
    if (threadIdx.x == 0) {
      double s1 = 0.0, s2 = 0.0;
      if (a.iter >= 2) {
        const double* pa = a.st.aa + (long)map * kRowGroupsMax * 2;
        for (int g = 0; g < (int)gridDim.x; ++g) {
          s1 += pa[2 * g];
          s2 += pa[2 * g + 1];
        }
      }
      s_gamma = s2 > 0.0 ? s1 / s2 : 0.0;
    }
    __syncthreads();
  }
  if constexpr (MODE == ROW_CONV_TAIL) {
    store_slots<Tio, Tc, N>((Tio*)mp.dT + oa, zr, t, mirror);
    store_slots<Tio, Tc, N>((Tio*)mp.dT + ob, zi, t, mirror);
  } else if constexpr (MODE == ROW_CONV_HEAD) {
    load_slots<Tio, Tc, N, true>((const Tio*)mp.qd + oa, zr, t, mirror);
    load_slots<Tio, Tc, N, true>((const Tio*)mp.qd + ob, zi, t, mirror);
  } else if constexpr (OS) {
    row_oneshot<Tio, Tc, N, MODE>(zr, mp, oa, t, mirror, pp, ls);
    row_oneshot<Tio, Tc, N, MODE>(zi, mp, ob, t, mirror, pp, ls);
  } else if constexpr (AA) {
    const double gamma = MODE == ROW_AA_MIX ? s_gamma : 0.0;
    row_anderson<Tio, Tc, N, MODE, true>(zr, mp, oa, t, mirror, zero_old, a.iter, gamma, pp, ls, d1, d2);
    row_anderson<Tio, Tc, N, MODE, true>(zi, mp, ob, t, mirror, zero_old, a.iter, gamma, pp, ls, d1, d2);
  } else {
    row_pointwise<Tio, Tc, N, MODE, true>(zr, mp, oa, t, mirror, zero_old, pp, ls);
    row_pointwise<Tio, Tc, N, MODE, true>(zi, mp, ob, t, mirror, zero_old, pp, ls);
  }

  if constexpr (STATS) {
    constexpr int W = Cfg::WAVE;
    const int wave = threadIdx.x / W;
    const bool bad = !(ls.xmax <= (Tc)pp.cap) || !isfinite(ls.sum);
    double inc = wave_max<W>((double)ls.inc);
    const unsigned bad_any = __any(bad);
    double sum = 0.0;
    unsigned long long best = 0ull;
    if (MODE != ROW_RESID) {
      sum = wave_sum<W>((double)ls.sum);
      best = ls.imax == 0x7fffffff ? 0ull : pack_max((float)ls.xmax, ls.imax);
      best = wave_max_u64<W>(best);
    }
    if constexpr (AA) {
      d1 = wave_sum<W>(d1);
      d2 = wave_sum<W>(d2);
    }
    if ((threadIdx.x % W) == 0) {
      s_red[0][wave] = bad_any ? (double)NAN : inc;
      s_red[1][wave] = sum;
      s_red[2][wave] = __longlong_as_double((long long)best);
      if constexpr (AA) {
        s_red[3][wave] = d1;
        s_red[4][wave] = d2;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double i0 = s_red[0][0], s0 = s_red[1][0];
      unsigned long long b0 = (unsigned long long)__double_as_longlong(s_red[2][0]);
      bool any_bad = isnan(i0);
      for (int w = 1; w < Cfg::WAVES; ++w) {
        any_bad = any_bad || isnan(s_red[0][w]);
        i0 = fmax(i0, s_red[0][w]);
        s0 += s_red[1][w];
        const unsigned long long bw = (unsigned long long)__double_as_longlong(s_red[2][w]);
        b0 = bw > b0 ? bw : b0;
      }
      if (MODE == ROW_RESID) {
        atomicMax(&a.st.resid64[map], (unsigned long long)__double_as_longlong(any_bad ? (double)INFINITY : i0));
      } else {
        const long slot = (long)map * a.st.stride + a.iter;
        atomicMax(&a.st.resid[slot], (unsigned long long)__double_as_longlong(any_bad ? (double)INFINITY : i0));
        a.st.part[(long)map * kRowGroupsMax + blockIdx.x] = s0;
        atomicMax(&a.st.maxpack[slot], b0);
        if (any_bad) atomicOr(&a.st.flags[map], kFlagRunaway);
        if constexpr (AA) {
          double e1 = s_red[3][0], e2 = s_red[4][0];
          for (int w = 1; w < Cfg::WAVES; ++w) {
            e1 += s_red[3][w];
            e2 += s_red[4][w];
          }
          double* pa = a.st.aa + ((long)map * kRowGroupsMax + blockIdx.x) * 2;
          pa[0] = e1;
          pa[1] = e2;
        }
      }
    }
  }

  // ---- forward half: P rows -> row DCT-II spectrum
  if constexpr (FWD) {
    wave_sync();
    fft_reg<Tc, N, -1, 1, CT>(zr, zi, re, im, tw, t, twl);
    Tc pr[E], pim[E];
    partner<Tc, N, true>(zr, pr, t);
    partner<Tc, N, true>(zi, pim, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m;
      const Cx<Tc> q = qw[p];
      Tc xa, xb, xa2, xb2;
      if constexpr (CT) {
        const Cx<Tc> ql = qwl[p];
        split_pair_ct<Tc>(zr[m], zi[m], pr[m], pim[m], q.r, q.i, ql.r, ql.i, xa, xb, xa2, xb2);
      } else {
        split_pair<Tc>(zr[m], zi[m], pr[m], pim[m], q.r, q.i, xa, xb, xa2, xb2);
      }
      Sa[p] = xa;
      Sb[p] = xb;
    }
  }
}


}  // namespace
}  // namespace vs
