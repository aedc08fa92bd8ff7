// Transient-solve kernels (Eqs. Ttran, tranGreen, tranapprox; Sec. IV-E).
//
// Each cosine mode (p, q) of the mirrored die responds to a power step with a single pole:
// steady gain lambda[p][q], time constant tau[p][q].  With the power held constant over a step
// of length dt, the exact update of the mode's rise is
//     theta_hat_n = a theta_hat_{n-1} + b P_hat_n,   a = exp(-dt / tau),  b = (1 - a) lambda,
// which is the full-history superposition of step responses (Eq. tranapprox) in recursive form.
// One step is two passes:
//   column pass : column DCT-II of the row spectrum of P_n, the per-mode update of the
//                 spectral state theta_hat (kept in HBM, layout [q][p]), column DCT-III;
//   row pass    : row DCT-III -> theta_n, conductivity factor, Kirchhoff inverse -> dT_n (kept in
//                 registers; written only for snapshots and the last step), then the power of the
//                 next step P_{n+1} = hx hy (q_dyn(t_{n+1}) + QL L(dT_n)) and its row DCT-II.
// q_dyn(t_n) comes from the block trace through a per-cell block id map.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "trpoint.hpp"

namespace vs {

namespace {

__device__ __forceinline__ int lane_get_i(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

template <int N>
__device__ __forceinline__ void load_ids(const int* __restrict__ row, int* out, int t, int mirror) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
    const Vec<int, 2> v = *reinterpret_cast<const Vec<int, 2>*>(row + 2 * (t + TPF * m));
    out[m] = v.v[0];
    out[E - 1 - m] = lane_get_i(v.v[1], mirror);
  }
}

// exact first moment of the slab's step response at lateral wavenumber s
__device__ double tau_moment(double s, double t, double alpha) {
  const double x = 2.0 * s * t;
  if (x < 1e-3) return t * t / (3.0 * alpha) * (1.0 - 7.0 * x * x / 60.0 + 31.0 * x * x * x * x / 2520.0);
  return (1.0 - x / sinh(x)) / (2.0 * alpha * s * s);
}

// ab[j][q][p] = (exp(-dt/tau_j), -expm1(-dt/tau_j) w_j lambda'), lambda' = lamT[q][p] (scaled by
// 1/(nx ny)), for the poles j < poles of mode (p, q).  One pole: tau = the lumped (rho c t / 3)
// hx hy lambda or the moment tau(s), w = 1.  Modal (poles >= 1): the slab's depth modes
// m < poles - 1, tau_m = t^2 / (alpha ((s t)^2 + ((m + 1/2) pi)^2)), w_m = 2 (s t / tanh(s t)) /
// ((s t)^2 + ((m + 1/2) pi)^2), and one last pole with the remaining weight whose time constant
// keeps the first moment sum_j w_j tau_j = tau(s).
// Truncated history of h steps (fir non-null): with c_j = w_j lambda' and r_j = exp(-(h - 1) dt /
// tau_j), fir[j][q][p] = -b_j r_j for each pole and fir[poles][q][p] = sum_j c_j r_j.
template <typename T>
__global__ void __launch_bounds__(256) transient_coef_kernel(const double* __restrict__ lamT, T* __restrict__ ab,
                                                             T* __restrict__ fir, int nx, int ny, double lx, double ly,
                                                             double t, double alpha, double dt, int tau_model,
                                                             double lumped_c, int poles, int hist) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= ny) return;
  const double lam = lamT[(size_t)q * ny + p];
  const double s = M_PI * sqrt(((double)p / ly) * ((double)p / ly) + ((double)q / lx) * ((double)q / lx));
  const size_t plane = (size_t)nx * ny * 2, cell = (size_t)q * ny + p;
  double tail = 0.0;  // sum_j c_j r_j of the truncated history
  auto put = [&](int j, double tau, double w) {
    const size_t o = j * plane + cell * 2;
    const double b = -expm1(-dt / tau) * w * lam;
    ab[o] = (T)exp(-dt / tau);
    ab[o + 1] = (T)b;
    if (fir) {
      const double r = exp(-(double)(hist - 1) * dt / tau);
      fir[j * (plane / 2) + cell] = (T)(-b * r);
      tail += w * lam * r;
    }
  };
  auto finish = [&]() {
    if (fir) fir[poles * (plane / 2) + cell] = (T)tail;
  };
  if (tau_model == VARSIM_TAU_LUMPED) {
    put(0, lumped_c * lam, 1.0);  // (rho c t / 3) hx hy lambda = (rho c t / 3) (lx ly) lambda'
    finish();
    return;
  }
  const double tm = tau_moment(s, t, alpha);
  if (tau_model != VARSIM_TAU_MODAL || poles <= 1) {
    put(0, tm, 1.0);
    finish();
    return;
  }
  const double x = s * t, xt = x < 1e-8 ? 1.0 : x / tanh(x);
  double wsum = 0.0, first = 0.0;
  for (int m = 0; m < poles - 1; ++m) {
    const double bt = (m + 0.5) * M_PI, d = x * x + bt * bt;
    const double w = 2.0 * xt / d, tau = t * t / (alpha * d);
    put(m, tau, w);
    wsum += w;
    first += w * tau;
  }
  const double wr = 1.0 - wsum;
  put(poles - 1, (tm - first) / wr, wr);
  finish();
}

// block id of each cell: the last block (painter's order) whose rectangle covers it, else -1
__global__ void __launch_bounds__(256) block_id_kernel(const int* __restrict__ rects, int n_blocks, int* __restrict__ ids,
                                                       int nx, int ny) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nx * ny) return;
  const int x = (int)(c % nx), y = (int)(c / nx);
  int id = -1;
  for (int b = 0; b < n_blocks; ++b) {
    const int x0 = rects[4 * b], y0 = rects[4 * b + 1], w = rects[4 * b + 2], h = rects[4 * b + 3];
    if (x >= x0 && x < x0 + w && y >= y0 && y < y0 + h) id = b;
  }
  ids[c] = id;
}

// Row-pass launch shape of the transient: FFTS_ row pairs per workgroup (0: the steady pass's
// default).  A single map has only N/2 row pairs, so fewer per workgroup spreads them over more CUs.
template <int N, int FFTS_>
struct TrRowCfg {
  static constexpr int TPF = Shape<N>::TPF;
  static constexpr int FFTS = FFTS_ ? FFTS_ : RowCfg<N>::FFTS;
  static constexpr int THREADS = FFTS * TPF;
};

template <typename Tio, typename Tc, int N, int MODE, int FFTS_>
__global__ void __launch_bounds__((TrRowCfg<N, FFTS_>::THREADS))
    transient_row_kernel(TransArgs a, int step, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = TrRowCfg<N, FFTS_>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int ST = Shape<N>::STRIDE;
  constexpr bool INV = MODE != TR_HEAD;
  constexpr bool FWD = MODE != TR_LAST;
  __shared__ Tc s_re[Cfg::FFTS * ST];
  __shared__ Tc s_im[Cfg::FFTS * ST];

  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  const int mirror = (__lane_id() & ~(TPF - 1)) + (TPF - 1 - t);
  const int row = (blockIdx.x * Cfg::FFTS + f) * 2;
  Tc* re = s_re + f * ST;
  Tc* im = s_im + f * ST;
  Tc* const Sa = (Tc*)a.S + (long)row * N;
  Tc* const Sb = Sa + N;
  const long oa = (long)row * N, ob = oa + N;
  const PointParams& pp = a.pp;

  Tc zr[E], zi[E];
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
      merge_pair<Tc>(xa[m], xb[m], xa2[m], xb2[m], q.r, q.i, zr[m], zi[m]);
    }
    fft_reg<Tc, N, +1>(zr, zi, re, im, tw, t);
  }

  bool bad = false;
  const bool snap = INV && a.snaps && (step % a.out_every == 0);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    Tc* z = half ? zi : zr;
    const long off = half ? ob : oa;
    Tc x[E];
    if constexpr (INV) {
      if (a.minv && !pp.cond_src) {  // conductivity factor on the target side
        Tc mv[E];
        load_slots<Tio, Tc, N>((const Tio*)a.minv + off, mv, t, mirror);
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] *= mv[m];
      }
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = z[m];
      kirchhoff_inv_n<Tc, E>(x, pp);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        x[m] = (Tc)(Tio)x[m];
        bad = bad || !(x[m] <= (Tc)pp.cap) || !(x[m] == x[m]);
      }
      if (snap)
        store_slots<Tio, Tc, N>((Tio*)a.snaps + (long)(step / a.out_every - 1) * N * N + off, x, t, mirror);
      if (MODE == TR_LAST) store_slots<Tio, Tc, N>((Tio*)a.dT + off, x, t, mirror);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (Tc)0;
    }
    if constexpr (FWD) {
      // power of the next step: trace row `step` (0-based) holds step step+1
      int id[E];
      load_ids<N>(a.ids + off, id, t, mirror);
      const Tio* tr = (const Tio*)a.trace + (long)step * a.n_blocks;
      Tc q[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const Tc v = (Tc)tr[id[m] < 0 ? 0 : id[m]];
        q[m] = id[m] < 0 ? (Tc)0 : v;
      }
      if (a.ql) {
        Tc ql[E];
        load_slots<Tio, Tc, N>((const Tio*)a.ql + off, ql, t, mirror);
        add_leakage_n<Tc, E>(q, ql, x, pp);
      }
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] = (Tc)pp.hxhy * q[m];
      if (a.minv && pp.cond_src) {  // conductivity factor on the source side
        Tc mv[E];
        load_slots<Tio, Tc, N>((const Tio*)a.minv + off, mv, t, mirror);
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] *= mv[m];
      }
    }
  }
  if (INV && __any(bad) && (__lane_id() & 63) == 0) atomicOr(a.flags, kFlagRunaway);

  if constexpr (FWD) {
    wave_sync();
    fft_reg<Tc, N, -1>(zr, zi, re, im, tw, t);
    Tc pr[E], pim[E];
    partner<Tc, N, true>(zr, pr, t);
    partner<Tc, N, true>(zi, pim, t);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m;
      const Cx<Tc> q = qw[p];
      Tc xa, xb, xa2, xb2;
      split_pair<Tc>(zr[m], zi[m], pr[m], pim[m], q.r, q.i, xa, xb, xa2, xb2);
      Sa[p] = xa;
      Sb[p] = xb;
    }
  }
}

// FIR: the truncated history of a.hist steps (the ring of past spectra and the fir planes)
template <typename Tc, int N, int COLS, bool FIR>
__global__ void __launch_bounds__((ColCfg<Tc, N, COLS>::THREADS))
    transient_col_kernel(TransArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = ColCfg<Tc, N, COLS>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int ST = Shape<N>::STRIDE;
  constexpr int VEC = Cfg::VEC;
  constexpr int VPR = Cfg::COLS / VEC;
  constexpr int P = Cfg::PITCH;
  __shared__ Tc lds[Cfg::LDS];

  int strip, map;
  xcd_tile(strip, map);
  Tc* S = (Tc*)a.S;
  const int c0 = strip * Cfg::COLS;

  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Vec<Tc, VEC> v = *reinterpret_cast<const Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC);
#pragma unroll
    for (int e = 0; e < VEC; ++e) lds[tile_row<Cfg, N>(y) * P + j * VEC + e] = v.v[e];
  }
  __syncthreads();

  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  Tc zr[E], zi[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int y = tile_slot<Cfg, N>(t + TPF * m);
    zr[m] = lds[y * P + 2 * f];
    zi[m] = lds[y * P + 2 * f + 1];
  }
  __syncthreads();

  Tc* re = lds + f * ST;  // all real parts first, then all imaginary parts
  Tc* im = lds + Cfg::FFTS * ST + f * ST;
  fft_reg<Tc, N, -1>(zr, zi, re, im, tw, t);
  Tc pr[E], pim[E];
  partner<Tc, N, true>(zr, pr, t);
  partner<Tc, N, true>(zi, pim, t);
  // per-mode update of the spectral state of columns qa = c0 + 2f and qb = qa + 1
  const int qa = c0 + 2 * f;
  Tc* sta = (Tc*)a.state + (long)qa * N;
  Tc* stb = sta + N;
  const Vec<Tc, 2>* aba = reinterpret_cast<const Vec<Tc, 2>*>(a.ab) + (long)qa * N;
  const Vec<Tc, 2>* abb = aba + N;
  // truncated history: the spectrum of h - 1 steps ago leaves the ring slot this step's enters
  Tc* ra = FIR ? (Tc*)a.ring + (long)a.slot * N * N + (long)qa * N : nullptr;
  const Tc* fa = FIR ? (const Tc*)a.fir + (long)qa * N : nullptr;
  Tc na[E], nb[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int p = t + TPF * m;
    const Cx<Tc> q = qw[p];
    Tc xa, xb, xa2, xb2;
    split_pair<Tc>(zr[m], zi[m], pr[m], pim[m], q.r, q.i, xa, xb, xa2, xb2);
    Tc oa = 0, ob = 0;
    if constexpr (FIR) {
      oa = ra[p];
      ob = ra[N + p];
      ra[p] = xa;
      ra[N + p] = xb;
    }
    const Vec<Tc, 2> ka = aba[p], kb = abb[p];
    na[m] = dot2(ka.v[0], sta[p], ka.v[1], xa);
    nb[m] = dot2(kb.v[0], stb[p], kb.v[1], xb);
    if constexpr (FIR) {
      na[m] = fma(fa[p], oa, na[m]);
      nb[m] = fma(fa[N + p], ob, nb[m]);
    }
    sta[p] = na[m];
    stb[p] = nb[m];
    // further poles of the multi-pole model: their states follow in planes of N^2, and the
    // mode's rise is the sum over poles (pole 0 first)
    for (int j = 1; j < a.poles; ++j) {
      Tc* sja = sta + (long)j * N * N;
      Tc* sjb = sja + N;
      const Vec<Tc, 2> ja = aba[(long)j * N * N + p], jb = abb[(long)j * N * N + p];
      Tc ua = dot2(ja.v[0], sja[p], ja.v[1], xa);
      Tc ub = dot2(jb.v[0], sjb[p], jb.v[1], xb);
      if constexpr (FIR) {
        ua = fma(fa[(long)j * N * N + p], oa, ua);
        ub = fma(fa[(long)j * N * N + N + p], ob, ub);
      }
      sja[p] = ua;
      sjb[p] = ub;
      na[m] += ua;
      nb[m] += ub;
    }
    if constexpr (FIR) {  // the saturated step response on the leaving spectrum
      na[m] = fma(fa[(long)a.poles * N * N + p], oa, na[m]);
      nb[m] = fma(fa[(long)a.poles * N * N + N + p], ob, nb[m]);
    }
  }
  Tc na2[E], nb2[E];
  partner<Tc, N, false>(na, na2, t);
  partner<Tc, N, false>(nb, nb2, t);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const Cx<Tc> q = qw[t + TPF * m];
    merge_pair<Tc>(na[m], nb[m], na2[m], nb2[m], q.r, q.i, zr[m], zi[m]);
  }
  wave_sync();
  fft_reg<Tc, N, +1>(zr, zi, re, im, tw, t);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int y = tile_slot<Cfg, N>(t + TPF * m);
    lds[y * P + 2 * f] = zr[m];
    lds[y * P + 2 * f + 1] = zi[m];
  }
  __syncthreads();
  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    Vec<Tc, VEC> v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = lds[tile_row<Cfg, N>(y) * P + j * VEC + e];
    *reinterpret_cast<Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC) = v;
  }
}

// statistics of one final map (one workgroup)
template <typename Tio>
__global__ void __launch_bounds__(1024) map_stats_kernel(const Tio* __restrict__ dT, long cells,
                                                         const unsigned* __restrict__ flags, int steps,
                                                         varsim_stats* __restrict__ out) {
  __shared__ double s_sum[16];
  __shared__ unsigned long long s_best[16];
  double sum = 0.0;
  unsigned long long best = 0ull;
  for (long i = threadIdx.x; i < cells; i += blockDim.x) {
    const float v = (float)dT[i];
    sum += (double)dT[i];
    const unsigned long long k = pack_max(v, i);
    best = k > best ? k : best;
  }
  sum = wave_sum<64>(sum);
  best = wave_max_u64<64>(best);
  if ((threadIdx.x & 63) == 0) {
    s_sum[threadIdx.x >> 6] = sum;
    s_best[threadIdx.x >> 6] = best;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      s_sum[0] += s_sum[w];
      s_best[0] = s_best[w] > s_best[0] ? s_best[w] : s_best[0];
    }
    varsim_stats s;
    const long idx = (long)(0xFFFFFFFFu - (unsigned)(s_best[0] & 0xFFFFFFFFull));
    const bool run = (*flags & kFlagRunaway) != 0;
    s.status = run ? VARSIM_ERR_RUNAWAY : VARSIM_OK;
    s.iterations = steps;
    s.last_increment_K = NAN;
    s.residual_f64_K = NAN;
    s.dT_mean_K = run ? NAN : s_sum[0] / (double)cells;
    s.hotspot_index = (run || idx < 0 || idx >= cells) ? -1 : idx;
    s.dT_max_K = s.hotspot_index >= 0 ? (double)dT[idx] : NAN;
    s.warm_start_rejected = 0;
    s.reserved = 0;
    *out = s;
  }
}

template <typename Tio, typename Tc, int N, int FFTS>
hipError_t tr_row_shape(int mode, const TransArgs& a, int step, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = TrRowCfg<N, FFTS>;
  const dim3 grid((N / 2) / Cfg::FFTS), block(Cfg::THREADS);
  switch (mode) {
    case TR_HEAD:
      hipLaunchKernelGGL((transient_row_kernel<Tio, Tc, N, TR_HEAD, FFTS>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_MERGED:
      hipLaunchKernelGGL((transient_row_kernel<Tio, Tc, N, TR_MERGED, FFTS>), grid, block, 0, s, a, step, tw, qw);
      break;
    case TR_LAST:
      hipLaunchKernelGGL((transient_row_kernel<Tio, Tc, N, TR_LAST, FFTS>), grid, block, 0, s, a, step, tw, qw);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// row-pass candidates: 0 = default rows per workgroup, 1 = half of them, 2 = one row pair
template <int N, int V>
constexpr int tr_row_ffts() {
  constexpr int f0 = RowCfg<N>::FFTS;
  return V == 0 ? f0 : (V == 1 ? (f0 / 2 > 0 ? f0 / 2 : 1) : 1);
}

template <typename Tio, typename Tc, int N>
hipError_t tr_row_launch(int mode, int v, const TransArgs& a, int step, const Cx<Tc>* tw, const Cx<Tc>* qw,
                         hipStream_t s) {
  switch (v) {
    case 0: return tr_row_shape<Tio, Tc, N, tr_row_ffts<N, 0>()>(mode, a, step, tw, qw, s);
    case 1: return tr_row_shape<Tio, Tc, N, tr_row_ffts<N, 1>()>(mode, a, step, tw, qw, s);
    case 2: return tr_row_shape<Tio, Tc, N, tr_row_ffts<N, 2>()>(mode, a, step, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

// column-pass candidates: 0 = default strip width, 1 = half, 2 = quarter (at least 2 columns)
template <typename Tc, int N, int V>
constexpr int tr_col_cols() {
  constexpr int c0 = ColCfg<Tc, N>::COLS;
  constexpr int c = V == 0 ? c0 : (V == 1 ? c0 / 2 : c0 / 4);
  return c < 2 ? 2 : c;
}

template <typename Tc, int N, int COLS>
hipError_t tr_col_shape(const TransArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = ColCfg<Tc, N, COLS>;
  const dim3 grid(N / Cfg::COLS, 1), block(Cfg::THREADS);
  if (a.ring)
    hipLaunchKernelGGL((transient_col_kernel<Tc, N, COLS, true>), grid, block, 0, s, a, tw, qw);
  else
    hipLaunchKernelGGL((transient_col_kernel<Tc, N, COLS, false>), grid, block, 0, s, a, tw, qw);
  return hipGetLastError();
}

template <typename Tc, int N>
hipError_t tr_col_launch(int v, const TransArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  switch (v) {
    case 0: return tr_col_shape<Tc, N, tr_col_cols<Tc, N, 0>()>(a, tw, qw, s);
    case 1: return tr_col_shape<Tc, N, tr_col_cols<Tc, N, 1>()>(a, tw, qw, s);
    case 2: return tr_col_shape<Tc, N, tr_col_cols<Tc, N, 2>()>(a, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t tr_dispatch(int which, int mode, int v, int n, const TransArgs& a, int step, hipStream_t s) {
  const Cx<T>* tw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.tw32 : (const Cx<T>*)a.tw.tw64;
  const Cx<T>* qw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.qw32 : (const Cx<T>*)a.tw.qw64;
#define VS_TR_CASE(NN)                                                       \
  case NN:                                                                   \
    return which == 0 ? tr_row_launch<T, T, NN>(mode, v, a, step, tw, qw, s) : \
                        tr_col_launch<T, NN>(v, a, tw, qw, s);
  switch (n) {
    VS_TR_CASE(16)
    VS_TR_CASE(32)
    VS_TR_CASE(64)
    VS_TR_CASE(128)
    VS_TR_CASE(256)
    VS_TR_CASE(512)
    VS_TR_CASE(1024)
    default: return hipErrorInvalidValue;
  }
#undef VS_TR_CASE
}

}  // namespace

hipError_t launch_transient_coef(const TableSpec& sp, const double* lam64T, int io, void* ab, void* fir, int hist,
                                 double alpha, double dt, int tau_model, double rho_c, int poles, hipStream_t stream) {
  // lumped: tau = (rho c t / 3) hx hy lambda = (rho c t / 3) lx ly lambda'
  const double lumped_c = rho_c * sp.t / 3.0 * sp.lx * sp.ly;
  const dim3 grid((sp.ny + 255) / 256, sp.nx);
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(transient_coef_kernel<float>, grid, dim3(256), 0, stream, lam64T, (float*)ab, (float*)fir, sp.nx,
                       sp.ny, sp.lx, sp.ly, sp.t, alpha, dt, tau_model, lumped_c, poles, hist);
  else
    hipLaunchKernelGGL(transient_coef_kernel<double>, grid, dim3(256), 0, stream, lam64T, (double*)ab, (double*)fir,
                       sp.nx, sp.ny, sp.lx, sp.ly, sp.t, alpha, dt, tau_model, lumped_c, poles, hist);
  return hipGetLastError();
}

hipError_t launch_block_ids(const int* rects, int n_blocks, int* ids, int nx, int ny, hipStream_t stream) {
  const long cells = (long)nx * ny;
  hipLaunchKernelGGL(block_id_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, stream, rects, n_blocks, ids,
                     nx, ny);
  return hipGetLastError();
}

int transient_variants(int n) { return transient_split_ok(n) ? kTrVariants : transient_single_ok(n) ? 6 : 3; }

hipError_t launch_transient_row(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant) {
  if (variant >= 6) return launch_transient_row2(mode, io, a, step, stream, variant - 6);
  if (variant >= 3) return launch_transient_row1(mode, io, a, step, stream, variant - 3);
  return io == VARSIM_F32 ? tr_dispatch<float>(0, mode, variant, a.n, a, step, stream)
                          : tr_dispatch<double>(0, mode, variant, a.n, a, step, stream);
}

hipError_t launch_transient_col(int io, const TransArgs& a, hipStream_t stream, int variant) {
  if (variant >= 6) return launch_transient_col2(io, a, stream, variant - 6);
  if (variant >= 3) return launch_transient_col1(io, a, stream, variant - 3);
  return io == VARSIM_F32 ? tr_dispatch<float>(1, 0, variant, a.n, a, 0, stream)
                          : tr_dispatch<double>(1, 0, variant, a.n, a, 0, stream);
}

hipError_t launch_map_stats(int io, const void* dT, long cells, const unsigned* flags, int steps, varsim_stats* out,
                            hipStream_t stream) {
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(map_stats_kernel<float>, dim3(1), dim3(1024), 0, stream, (const float*)dT, cells, flags, steps,
                       out);
  else
    hipLaunchKernelGGL(map_stats_kernel<double>, dim3(1), dim3(1024), 0, stream, (const double*)dT, cells, flags, steps,
                       out);
  return hipGetLastError();
}

}  // namespace vs
