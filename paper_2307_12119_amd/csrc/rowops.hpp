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
