// Pointwise physics of the transient row passes over a lane's K values at once: the
// Kirchhoff inverse of k(T) and the leakage term of the next step's power, with the uniform
// mode tests taken once per call rather than once per value.
#pragma once

#include <cmath>

#include "common.hpp"
#include "passes.hpp"

namespace vs {

// theta -> dT (Kirchhoff inverse of k = k_ref (T / T_amb)^-eta) for K values in place; the same
// arithmetic as kirchhoff_inv, with the mode tests taken once for all K values and the FP32
// exp / log fallback entered only when some lane of the wavefront needs it.
template <typename Tc, int K>
__device__ __forceinline__ void kirchhoff_inv_n(Tc* v, const PointParams& pp) {
  if (pp.eta_mode == 0) return;
  if constexpr (sizeof(Tc) == 4) {
    const float us = (float)pp.u_scale, umax = (float)pp.poly_umax, ta = (float)pp.t_amb;
    float u[K];
    bool far = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      u[k] = us * v[k];
      far = far || !(fabsf(u[k]) <= umax);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float acc = pp.polyf[kPoly - 1];
#pragma unroll
      for (int c = kPoly - 2; c >= 0; --c) acc = fmaf(acc, u[k], pp.polyf[c]);
      v[k] = ta * u[k] * acc;
    }
    if (__any(far)) {
      if (pp.eta_mode == 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float fb = ta * (__expf(u[k]) - 1.f);
          v[k] = fabsf(u[k]) <= umax ? v[k] : fb;
        }
      } else {
        const float ie = (float)pp.inv_1m_eta;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float fb = u[k] > -1.f ? ta * (__expf(ie * __logf(1.f + u[k])) - 1.f) : NAN;
          v[k] = fabsf(u[k]) <= umax ? v[k] : fb;
        }
      }
    }
  } else {
    const Tc us = (Tc)pp.u_scale, ta = (Tc)pp.t_amb;
    if (pp.eta_mode == 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = ta * expm1(us * v[k]);
    } else {
      const Tc ie = (Tc)pp.inv_1m_eta;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const Tc u = us * v[k];
        const Tc r = ta * expm1(ie * log1p(u));
        v[k] = u > (Tc)-1 ? r : (Tc)NAN;
      }
    }
  }
}

// q[k] += ql[k] L(dT[k]) for K values, the leakage law chosen once for all of them
template <typename Tc, int K>
__device__ __forceinline__ void add_leakage_n(Tc* q, const Tc* ql, const Tc* dT, const PointParams& pp) {
  if (pp.leak == VARSIM_LEAK_EXP) {
#pragma unroll
    for (int k = 0; k < K; ++k) q[k] += ql[k] * exp_leak((Tc)pp.beta * dT[k]);
  } else if (pp.leak == VARSIM_LEAK_LINEAR) {
#pragma unroll
    for (int k = 0; k < K; ++k) q[k] += ql[k] * ((Tc)1 + (Tc)pp.beta * dT[k]);
  }
}

// One mode's state update in the column pass (Eqs. tranGreen, tranapprox): theta_hat = a theta_hat
// + b P_hat for the first pole ((a, b) in k and its state s already loaded); further poles of the
// multi-pole model keep their states and (a, b) in planes of `plane` values (pole j at st, ab
// + j plane) and add to the mode's rise; with a truncated history (FIR) the spectrum of h - 1
// steps ago leaves ring slot rg[p] as this step's P_hat enters, weighted by the per-pole FIR
// coefficients and finally the saturated part (fc planes 0..poles).  Returns the mode's rise.
template <typename Tc, bool FIR>
__device__ __forceinline__ Tc mode_step(Tc P, Vec<Tc, 2> k, Tc s, Tc* st, const Vec<Tc, 2>* ab, Tc* rg,
                                        const Tc* fc, long plane, int poles, int p) {
  Tc o = 0;
  if constexpr (FIR) {
    o = rg[p];
    rg[p] = P;
  }
  Tc n = dot2(k.v[0], s, k.v[1], P);
  if constexpr (FIR) n = fma(fc[p], o, n);
  st[p] = n;
  for (int j = 1; j < poles; ++j) {
    Tc* sj = st + (long)j * plane;
    const Vec<Tc, 2> kj = ab[(long)j * plane + p];
    Tc u = dot2(kj.v[0], sj[p], kj.v[1], P);
    if constexpr (FIR) u = fma(fc[(long)j * plane + p], o, u);
    sj[p] = u;
    n += u;
  }
  if constexpr (FIR) n = fma(fc[(long)poles * plane + p], o, n);  // the saturated step response
  return n;
}

}  // namespace vs
