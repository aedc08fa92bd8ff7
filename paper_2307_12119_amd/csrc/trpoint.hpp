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

}  // namespace vs
