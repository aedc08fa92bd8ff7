// Row-pass building blocks shared by the two-pass steady solve and the LDS-resident small-grid
// solve: per-lane statistics of a new iterate and the pointwise update of one row (theta ->
// [conductivity factor, target side] -> Kirchhoff inverse -> increment / statistics -> new total
// power -> [conductivity factor, source side]).
#pragma once

#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"

namespace vs {

// Per-lane running statistics of the new iterate.
template <typename Tc>
struct LaneStats {
  Tc inc = (Tc)0;       // max |dT_new - dT_old|
  Tc sum = (Tc)0;       // sum of dT_new (NaN / inf propagate: runaway detection)
  Tc xmax = (Tc)-INFINITY;
  int imax = 0x7fffffff;
  __device__ __forceinline__ void add(Tc x, Tc old, int idx) {
    inc = fmax(inc, fabs(x - old));
    sum += x;
    if (x > xmax || (x == xmax && idx < imax)) {
      xmax = x;
      imax = idx;
    }
  }
};

// one map's pointwise update of one row: theta slots -> dT (stored) -> total power slots
template <typename Tio, typename Tc, int N, int MODE, bool NT = false>
__device__ __forceinline__ void row_pointwise(Tc* z, const MapPtrs& mp, long off, int t, int mirror, bool zero_old,
                                              const PointParams& pp, LaneStats<Tc>& ls) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  Tc x[E];
  if constexpr (MODE == ROW_HEAD) {
    if (zero_old) {
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (Tc)0;
    } else {
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.dT + off, x, t, mirror);
    }
  } else {
    Tc old[E];
    if (mp.minv && !pp.cond_src) {  // target side: the rise is scaled
      Tc mv[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] *= mv[m];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = kirchhoff_inv<Tc>(z[m], pp);
    if (zero_old) {
#pragma unroll
      for (int m = 0; m < E; ++m) old[m] = (Tc)0;
    } else {
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.dT + off, old, t, mirror);
    }
    if constexpr (MODE == ROW_RESID) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        ls.inc = fmax(ls.inc, fabs(x[m] - old[m]));
        ls.sum += x[m];
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        x[m] = (Tc)(Tio)x[m];  // the iterate as stored
        ls.add(x[m], old[m], (int)off + unperm<N>(t + TPF * m));
      }
      store_slots<Tio, Tc, N, NT>((Tio*)mp.dT + off, x, t, mirror);
    }
  }
  if constexpr (MODE == ROW_HEAD || MODE == ROW_MERGED) {
    // FP32 transforms with the factor on the source side: the inputs come divided by m already
    constexpr bool kPre = sizeof(Tc) == 4;
    const bool pre = kPre && pp.cond_src;
    Tc q[E];
    load_slots<Tio, Tc, N, NT>((const Tio*)(pre ? mp.qs : mp.qd) + off, q, t, mirror);
    if (mp.ql) {
      Tc ql[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)(pre ? mp.qls : mp.ql) + off, ql, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) q[m] += ql[m] * leak_factor<Tc>(x[m], pp);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = (Tc)pp.hxhy * q[m];
    if constexpr (!kPre) {
      if (mp.minv && pp.cond_src) {  // source side: the power is scaled
        Tc mv[E];
        load_slots<Tio, Tc, N, NT>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] *= mv[m];
      }
    }
  }
}

// Anderson(1) mixing of the fixed point (a classical acceleration), pointwise part of one row.
//   ROW_AA_EVAL: theta slots -> g = G(x_k) -> dT; f = g - x_k -> af; increment / statistics of g;
//                d1 += (f - f_prev) f, d2 += (f - f_prev)^2 from iteration 2 on;
//   ROW_AA_MIX : g from dT -> x_{k+1} = g - gamma (g - g_prev) (gamma = 0 at iteration 1) -> ax,
//                g -> ag -> the total power of x_{k+1} (as ROW_HEAD) in the slots.
template <typename Tio, typename Tc, int N, int MODE, bool NT = false>
__device__ __forceinline__ void row_anderson(Tc* z, const MapPtrs& mp, long off, int t, int mirror, bool zero_old,
                                             int iter, double gamma, const PointParams& pp, LaneStats<Tc>& ls,
                                             double& d1, double& d2) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  if constexpr (MODE == ROW_AA_EVAL) {
    if (mp.minv && !pp.cond_src) {  // target side: the rise is scaled
      Tc mv[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] *= mv[m];
    }
    Tc g[E], x[E];
#pragma unroll
    for (int m = 0; m < E; ++m) g[m] = (Tc)(Tio)kirchhoff_inv<Tc>(z[m], pp);
    if (zero_old) {
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (Tc)0;
    } else {
      load_slots<Tio, Tc, N, NT>((const Tio*)(iter == 1 ? mp.dT : mp.ax) + off, x, t, mirror);
    }
    Tc f[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      ls.add(g[m], x[m], (int)off + unperm<N>(t + TPF * m));
      f[m] = (Tc)(Tio)(g[m] - x[m]);
    }
    if (iter >= 2) {
      Tc fp[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.af + off, fp, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const double df = (double)f[m] - (double)fp[m];
        d1 += df * (double)f[m];
        d2 += df * df;
      }
    }
    store_slots<Tio, Tc, N, NT>((Tio*)mp.dT + off, g, t, mirror);
    store_slots<Tio, Tc, N, NT>((Tio*)mp.af + off, f, t, mirror);
  } else {
    Tc g[E], x[E];
    load_slots<Tio, Tc, N, NT>((const Tio*)mp.dT + off, g, t, mirror);
    if (iter >= 2 && gamma != 0.0) {
      Tc gp[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.ag + off, gp, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (Tc)(Tio)fma(-(Tc)gamma, g[m] - gp[m], g[m]);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = g[m];
    }
    store_slots<Tio, Tc, N, NT>((Tio*)mp.ax + off, x, t, mirror);
    store_slots<Tio, Tc, N, NT>((Tio*)mp.ag + off, g, t, mirror);
    Tc q[E];
    load_slots<Tio, Tc, N, NT>((const Tio*)mp.qd + off, q, t, mirror);
    if (mp.ql) {
      Tc ql[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.ql + off, ql, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) q[m] += ql[m] * leak_factor<Tc>(x[m], pp);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = (Tc)pp.hxhy * q[m];
    if (mp.minv && pp.cond_src) {  // source side: the power is scaled
      Tc mv[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] *= mv[m];
    }
  }
}

// One-shot solve (Sec. IV-C, Eqs. detsol, randsol, detrandsol), pointwise part of one row.
//   ROW_OS_MID : theta_det slots -> stored in dT -> random-part source
//                beta hx hy (QL / m - mu) theta_det (W per cell) for the forward transform;
//   ROW_OS_TAIL: theta_rand slots (+ theta_det from dT when the random part is on) -> Phi^-1 ->
//                dT, statistics (max, sum, argmax; no increment).
template <typename Tio, typename Tc, int N, int MODE, bool NT = false>
__device__ __forceinline__ void row_oneshot(Tc* z, const MapPtrs& mp, long off, int t, int mirror, const PointParams& pp,
                                            LaneStats<Tc>& ls) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  if constexpr (MODE == ROW_OS_MID) {
    store_slots<Tio, Tc, N, NT>((Tio*)mp.dT + off, z, t, mirror);
    Tc r[E];
    if (mp.ql) {
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.ql + off, r, t, mirror);
      if (mp.minv) {
        Tc mv[E];
        load_slots<Tio, Tc, N, NT>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
        for (int m = 0; m < E; ++m) r[m] *= mv[m];
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) r[m] = (Tc)0;
    }
    const Tc bh = (Tc)(pp.beta * pp.hxhy), mu = (Tc)pp.os_mu;
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = bh * (r[m] - mu) * z[m];
  } else {
    if (pp.os_rand) {
      Tc d[E];
      load_slots<Tio, Tc, N, NT>((const Tio*)mp.dT + off, d, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] += d[m];
    }
    Tc x[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      x[m] = (Tc)(Tio)kirchhoff_inv<Tc>(z[m], pp);
      ls.add(x[m], x[m], (int)off + unperm<N>(t + TPF * m));
    }
    store_slots<Tio, Tc, N, NT>((Tio*)mp.dT + off, x, t, mirror);
  }
}

}  // namespace vs
