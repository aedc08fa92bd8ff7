// Shared definitions of the varsim HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "varsim.h"

namespace vs {

template <typename T>
struct Cx {
  T r, i;
};

constexpr int kMinN = 16;
constexpr int kMaxN = 1024;
constexpr int kMaxIter = 1000;

// per-map flag bits (IterState::flags)
constexpr unsigned kFlagRunaway = 1u;       // non-finite / above cap / Kirchhoff domain left
constexpr unsigned kFlagWarmRejected = 2u;  // dT_init had a non-finite entry: start from 0
constexpr unsigned kFlagInvalid = 4u;       // conductivity map not strictly positive
constexpr unsigned kFlagSkip = kFlagRunaway | kFlagInvalid;
constexpr unsigned kFlagOwnLoop = 8u;  // solved start to finish by one LDS-resident workgroup

// Device pointers of one map (all [n][n] row-major).
struct MapPtrs {
  const void* qd;    // dynamic power density (io type)
  const void* ql;    // leakage density at ambient times variation (io type), or null
  const void* minv;  // 1 / conductivity multiplier (io type), or null
  void* dT;          // temperature rise, in/out (io type)
  void* S;           // transform work array (compute type of the main loop)
  void* S64;         // FP64 work array for the residual pass, or null
  const void* init;  // warm start (io type), or null
  void* aux;         // spare per-map pointer (transient state)
  // Anderson mixing (io type, or null): the current iterate x_k, the previous G(x), the
  // previous residual G(x) - x
  void* ax;
  void* ag;
  void* af;
  // FP32 passes with the conductivity factor on the source side read the power inputs already
  // divided by m (io type): q_dyn / m and QL / m, written once per solve by the prep kernel (qd
  // and ql themselves where no conductivity map is given), so that no 1/m map is read per iteration
  const void* qs;
  const void* qls;
};

// Pointwise physics constants of one geometry.
struct PointParams {
  double hxhy;        // cell area, m^2
  double beta;        // leakage temperature coefficient, 1/K
  double t_amb;       // K
  double inv_1m_eta;  // 1 / (1 - eta)
  double c_1m_eta;    // (1 - eta) / T_amb
  double cap;         // runaway cap, K
  double tol;         // convergence tolerance, K
  int leak;           // VARSIM_LEAK_*
  int eta_mode;       // 0: eta == 0, 1: eta == 1, 2: general
  int cond_src;       // 1: the factor 1/m scales the power (source side), 0: the rise (target side)
  // Taylor coefficients of (1 + u)^(1/(1-eta)) - 1 = sum_k poly[k-1] u^k (k = 1..kPoly), used
  // by the FP32 path for |u| <= poly_umax, u = (1 - eta) theta / T_amb; 0 disables it.  The FP64
  // steady path uses the first kPoly64 coefficients for |u| <= poly_umax64 (first dropped term
  // below 1e-17 of the leading one).
  double u_scale;     // u = u_scale * theta: (1 - eta) / T_amb, or 1 / T_amb when eta == 1
  double poly_umax;
  float polyf[10];
  double poly_umax64;
  double polyd[20];
  // one-shot solve (Sec. IV-C): leakage density mu (W/m^2, per unit conductivity multiplier) that
  // the deterministic operator treats as uniform, and whether the random part is added
  double os_mu;
  int os_rand;
};
constexpr int kPoly = 10;
constexpr int kPoly64 = 20;

// Per-map iteration state in the workspace.
struct IterState {
  unsigned long long* resid;    // [maps][stride] double bits of max |dT_k - dT_{k-1}|
  double* sum;                  // [maps][stride] sum of dT_k
  unsigned long long* maxpack;  // [maps][stride] (orderable bits of dT_k << 32) | ~index
  unsigned* flags;              // [maps]
  unsigned long long* resid64;  // [maps] double bits of the FP64 residual
  int stride;
  // two-pass row passes: [maps][kRowGroupsMax] sum of dT over each workgroup's rows in the last
  // iteration that ran (overwritten each iteration, no atomics); added in a fixed order at the end
  double* part;
  // Anderson mixing: [maps][kRowGroupsMax][2] each row-pass workgroup's sums of df f and df df
  // (df = f_k - f_{k-1}) in the last evaluation, added in a fixed order by the mixing pass
  double* aa;
};
constexpr int kRowGroupsMax = 128;  // row-pass workgroups of one map, at most

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

}  // namespace vs
