// Steady-solve kernels: the fixed point dT = G(dT) of the leakage- and conductivity-coupled
// Green's-function convolution (Eqs. Green, Pt, Pleak, condsi, fspvsk; Sec. IV-F images).
//
// One iteration is two passes over each map:
//   row pass    : cosine-synthesis of each row (row DCT-III) of the previous spectrum, the
//                 conductivity-variation factor, the Kirchhoff inverse of k(T), the increment
//                 and statistics, the new total power P = hx hy (q_dyn + QL L(dT)), and the
//                 row DCT-II of P into the spectrum array (in place, same rows);
//   column pass : column DCT-II, multiplication by the cosine eigenvalues lambda of the
//                 mirrored Green's operator, column DCT-III (in place, column tiles in LDS;
//                 colpass.hip).
// The first row pass of a solve starts from dT_init (or 0), the last one skips the forward part.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"

namespace vs {

namespace {

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
template <typename Tio, typename Tc, int N, int MODE>
__device__ __forceinline__ void row_pointwise(Tc* z, const MapPtrs& mp, long off, int t, int mirror, bool zero_old,
                                              const PointParams& pp, LaneStats<Tc>& ls) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  Tc x[E];
  if constexpr (MODE == ROW_HEAD) {
    if (zero_old) {
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (Tc)0;
    } else {
      load_slots<Tio, Tc, N>((const Tio*)mp.dT + off, x, t, mirror);
    }
  } else {
    Tc old[E];
    if (mp.minv) {
      Tc mv[E];
      load_slots<Tio, Tc, N>((const Tio*)mp.minv + off, mv, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) z[m] *= mv[m];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = kirchhoff_inv<Tc>(z[m], pp);
    if (zero_old) {
#pragma unroll
      for (int m = 0; m < E; ++m) old[m] = (Tc)0;
    } else {
      load_slots<Tio, Tc, N>((const Tio*)mp.dT + off, old, t, mirror);
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
      store_slots<Tio, Tc, N>((Tio*)mp.dT + off, x, t, mirror);
    }
  }
  if constexpr (MODE == ROW_HEAD || MODE == ROW_MERGED) {
    Tc q[E];
    load_slots<Tio, Tc, N>((const Tio*)mp.qd + off, q, t, mirror);
    if (mp.ql) {
      Tc ql[E];
      load_slots<Tio, Tc, N>((const Tio*)mp.ql + off, ql, t, mirror);
#pragma unroll
      for (int m = 0; m < E; ++m) q[m] += ql[m] * leak_factor<Tc>(x[m], pp);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = (Tc)pp.hxhy * q[m];
  }
}

template <typename Tio, typename Tc, int N, int MODE>
__global__ void __launch_bounds__(RowCfg<N>::THREADS)
    row_pass_kernel(PassArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = RowCfg<N>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int ST = Shape<N>::STRIDE;
  constexpr bool INV = MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID || MODE == ROW_CONV_TAIL;
  constexpr bool FWD = MODE == ROW_HEAD || MODE == ROW_MERGED || MODE == ROW_CONV_HEAD;
  constexpr bool STATS = MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID;
  __shared__ Tc s_re[Cfg::FFTS * ST];
  __shared__ Tc s_im[Cfg::FFTS * ST];
  __shared__ double s_red[3][Cfg::WAVES];

  const int map = blockIdx.y;
  unsigned flags = 0u;
  if (MODE != ROW_CONV_HEAD && MODE != ROW_CONV_TAIL) {
    flags = a.st.flags[map];
    if (flags & kFlagSkip) return;
    if ((MODE == ROW_MERGED || MODE == ROW_LAST) && finished_before(a.st, map, a.iter, a.pp.tol)) return;
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
      merge_pair<Tc>(xa[m], xb[m], xa2[m], xb2[m], q.r, q.i, zr[m], zi[m]);
    }
    fft_reg<Tc, N, +1>(zr, zi, re, im, tw, t);
  }

  // ---- pointwise: conductivity factor, Kirchhoff inverse, increment, stats, new power
  LaneStats<Tc> ls;
  const bool zero_old = (a.iter == 1) && (a.zero_start || (flags & kFlagWarmRejected));
  if constexpr (MODE == ROW_CONV_TAIL) {
    store_slots<Tio, Tc, N>((Tio*)mp.dT + oa, zr, t, mirror);
    store_slots<Tio, Tc, N>((Tio*)mp.dT + ob, zi, t, mirror);
  } else if constexpr (MODE == ROW_CONV_HEAD) {
    load_slots<Tio, Tc, N>((const Tio*)mp.qd + oa, zr, t, mirror);
    load_slots<Tio, Tc, N>((const Tio*)mp.qd + ob, zi, t, mirror);
  } else {
    row_pointwise<Tio, Tc, N, MODE>(zr, mp, oa, t, mirror, zero_old, pp, ls);
    row_pointwise<Tio, Tc, N, MODE>(zi, mp, ob, t, mirror, zero_old, pp, ls);
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
    if ((threadIdx.x % W) == 0) {
      s_red[0][wave] = bad_any ? (double)NAN : inc;
      s_red[1][wave] = sum;
      s_red[2][wave] = __longlong_as_double((long long)best);
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
        atomicAdd(&a.st.sum[slot], s0);
        atomicMax(&a.st.maxpack[slot], b0);
        if (any_bad) atomicOr(&a.st.flags[map], kFlagRunaway);
      }
    }
  }

  // ---- forward half: P rows -> row DCT-II spectrum
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

// ---------------------------------------------------------------------------------------
// Small grids (N <= 128 FP32, N <= 64 FP64): one workgroup holds a map's spectrum in LDS and runs
// the whole fixed point -- column phase, merged row phase, statistics, convergence test -- in
// one launch.  Group g owns rows (2g, 2g+1) in the row phase and columns (2g, 2g+1) in the
// column phase; the transforms, pointwise physics and statistics are those of the two-pass
// path, so the iterates are the same numbers.
template <typename Tc, int N>
struct SmallCfg {
  static constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
  static constexpr int GROUPS = N / 2;
  static constexpr int THREADS = GROUPS * TPF;
  static constexpr int WAVE = THREADS < 64 ? THREADS : 64;
  static constexpr int WAVES = THREADS / WAVE;
  static constexpr int SP = N + 1;  // spectrum row pitch
  static constexpr int ST = Shape<N>::STRIDE;
  static constexpr int LDS = N * SP + GROUPS * 2 * ST;
};

template <typename Tc, int N>
__device__ __forceinline__ void small_row_inverse(const Tc* Sa, const Tc* Sb, Tc* zr, Tc* zi, Tc* re, Tc* im,
                                                  const Cx<Tc>* tw, const Cx<Tc>* qw, int t) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
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
  wave_sync();
  fft_reg<Tc, N, +1>(zr, zi, re, im, tw, t);
}

template <typename Tc, int N>
__device__ __forceinline__ void small_row_forward(Tc* Sa, Tc* Sb, Tc* zr, Tc* zi, Tc* re, Tc* im, const Cx<Tc>* tw,
                                                  const Cx<Tc>* qw, int t) {
  constexpr int E = Shape<N>::E, TPF = Shape<N>::TPF;
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

template <typename Tio, typename Tc, int N>
__global__ void __launch_bounds__((SmallCfg<Tc, N>::THREADS))
    small_solve_kernel(PassArgs a, int max_iter, const Tc* __restrict__ coef, const Cx<Tc>* __restrict__ tw,
                       const Cx<Tc>* __restrict__ qw) {
  using Cfg = SmallCfg<Tc, N>;
  constexpr int TPF = Cfg::TPF, E = Cfg::E, SP = Cfg::SP, ST = Cfg::ST, W = Cfg::WAVE;
  __shared__ Tc lds[Cfg::LDS];
  __shared__ double s_red[3][Cfg::WAVES];
  __shared__ int s_stop;

  const int map = blockIdx.x;
  const unsigned flags0 = a.st.flags[map];
  if (flags0 & kFlagSkip) return;
  const MapPtrs mp = a.maps[map];
  int g = threadIdx.x / TPF;
  if constexpr (TPF == 64) g = __builtin_amdgcn_readfirstlane(g);
  const int t = threadIdx.x % TPF;
  const int mirror = (__lane_id() & ~(TPF - 1)) + (TPF - 1 - t);
  Tc* re = lds + N * SP + g * ST;
  Tc* im = lds + N * SP + Cfg::GROUPS * ST + g * ST;
  Tc* Sa = lds + 2 * g * SP;
  Tc* Sb = Sa + SP;
  const long oa = (long)(2 * g) * N, ob = oa + N;
  const PointParams& pp = a.pp;
  const long base = (long)map * a.st.stride;
  const bool zero0 = a.zero_start || (flags0 & kFlagWarmRejected);
  if (threadIdx.x == 0) a.st.flags[map] = flags0 | kFlagOwnLoop;

  Tc zr[E], zi[E];
  {  // iteration 1 head: P(dT_0) -> row DCT-II
    LaneStats<Tc> ls;
    row_pointwise<Tio, Tc, N, ROW_HEAD>(zr, mp, oa, t, mirror, zero0, pp, ls);
    row_pointwise<Tio, Tc, N, ROW_HEAD>(zi, mp, ob, t, mirror, zero0, pp, ls);
    small_row_forward<Tc, N>(Sa, Sb, zr, zi, re, im, tw, qw, t);
  }
  int done = max_iter;
  for (int k = 1; k <= max_iter; ++k) {
    __syncthreads();
    {  // column phase: columns (2g, 2g+1) of the spectrum
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = unperm<N>(t + TPF * m);
        zr[m] = lds[y * SP + 2 * g];
        zi[m] = lds[y * SP + 2 * g + 1];
      }
      wave_sync();
      fft_reg<Tc, N, -1>(zr, zi, re, im, tw, t);
      Tc pr[E], pim[E];
      partner<Tc, N, true>(zr, pr, t);
      partner<Tc, N, true>(zi, pim, t);
      const Vec<Tc, 4>* ca = reinterpret_cast<const Vec<Tc, 4>*>(coef) + (long)(2 * g) * (N / 2 + 1);
      const Vec<Tc, 4>* cb = ca + (N / 2 + 1);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int p = t + TPF * m;
        const bool hi = m >= E / 2;
        const int pi = hi ? N - p : p;
        const Vec<Tc, 4> ka = ca[pi], kb = cb[pi];
        const Tc ba = hi ? -ka.v[1] : ka.v[1], bb = hi ? -kb.v[1] : kb.v[1];
        const Tc u = zr[m] + pr[m], v = zi[m] - pim[m], w = zi[m] + pim[m], x = pr[m] - zr[m];
        zr[m] = ka.v[0] * u + ba * v - bb * w - kb.v[2] * x;
        zi[m] = ba * u + ka.v[2] * v + kb.v[0] * w + bb * x;
      }
      wave_sync();
      fft_reg<Tc, N, +1>(zr, zi, re, im, tw, t);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = unperm<N>(t + TPF * m);
        lds[y * SP + 2 * g] = zr[m];
        lds[y * SP + 2 * g + 1] = zi[m];
      }
    }
    __syncthreads();
    // merged row phase: synthesis, pointwise physics + statistics, new power, row DCT-II
    small_row_inverse<Tc, N>(Sa, Sb, zr, zi, re, im, tw, qw, t);
    LaneStats<Tc> ls;
    const bool zero_old = k == 1 && zero0;
    row_pointwise<Tio, Tc, N, ROW_MERGED>(zr, mp, oa, t, mirror, zero_old, pp, ls);
    row_pointwise<Tio, Tc, N, ROW_MERGED>(zi, mp, ob, t, mirror, zero_old, pp, ls);
    small_row_forward<Tc, N>(Sa, Sb, zr, zi, re, im, tw, qw, t);

    const int wave = threadIdx.x / W;
    const bool bad = !(ls.xmax <= (Tc)pp.cap) || !isfinite(ls.sum);
    const double inc = wave_max<W>((double)ls.inc);
    const unsigned bad_any = __any(bad);
    const double sum = wave_sum<W>((double)ls.sum);
    unsigned long long best = ls.imax == 0x7fffffff ? 0ull : pack_max((float)ls.xmax, ls.imax);
    best = wave_max_u64<W>(best);
    if ((threadIdx.x % W) == 0) {
      s_red[0][wave] = bad_any ? (double)NAN : inc;
      s_red[1][wave] = sum;
      s_red[2][wave] = __longlong_as_double((long long)best);
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
      a.st.resid[base + k] = (unsigned long long)__double_as_longlong(any_bad ? (double)INFINITY : i0);
      a.st.sum[base + k] = s0;
      a.st.maxpack[base + k] = b0;
      if (any_bad) a.st.flags[map] = flags0 | kFlagOwnLoop | kFlagRunaway;
      s_stop = any_bad || i0 <= pp.tol;
    }
    __syncthreads();
    if (s_stop) {
      done = k;
      break;
    }
  }
  if (threadIdx.x == 0) a.st.maxpack[base] = (unsigned long long)done;
}

// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) prep_kernel(const PrepArgs* __restrict__ args, long count) {
  const PrepArgs pa = args[blockIdx.y];
  bool invalid = false, warm_bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    if (pa.ql_out) {
      T v = ((const T*)pa.q_leak0)[i];
      if (pa.leak_var) v *= ((const T*)pa.leak_var)[i];
      ((T*)pa.ql_out)[i] = v;
    }
    if (pa.minv_out) {
      const T m = ((const T*)pa.cond_map)[i];
      if (!(m > (T)0) || !isfinite(m)) invalid = true;
      ((T*)pa.minv_out)[i] = (T)1 / m;
    }
    if (pa.init && !isfinite(((const T*)pa.init)[i])) warm_bad = true;
  }
  if (invalid) atomicOr(pa.flags, kFlagInvalid);
  if (warm_bad) atomicOr(pa.flags, kFlagWarmRejected);
}

template <typename T>
__global__ void __launch_bounds__(256) init_copy_kernel(const PrepArgs* __restrict__ args, long count) {
  const PrepArgs pa = args[blockIdx.y];
  // a rejected warm start is replaced by 0 through the iteration-1 flag, nothing to copy
  if (!pa.init || pa.init == pa.dT || (*pa.flags & kFlagWarmRejected)) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    ((T*)pa.dT)[i] = ((const T*)pa.init)[i];
}

__global__ void zero_words_kernel(unsigned* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void count_active_kernel(IterState st, int n_maps, int iter, double tol, int* out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_maps) return;
  if (st.flags[m] & (kFlagSkip | kFlagOwnLoop)) return;
  const double r = __longlong_as_double((long long)st.resid[(long)m * st.stride + iter]);
  if (!(r <= tol)) atomicAdd(out, 1);
}

template <typename Tio>
__global__ void finalize_kernel(IterState st, const MapPtrs* __restrict__ maps, int n_maps, long cells, int max_iter,
                                int iters_run, double tol, int residual_done, varsim_stats* out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_maps) return;
  varsim_stats s;
  const unsigned fl = st.flags[m];
  const long base = (long)m * st.stride;
  // a map solved by its own workgroup records its iteration count in slot 0
  if (fl & kFlagOwnLoop) iters_run = (int)st.maxpack[base];
  int kf = 0;
  for (int k = 1; k <= iters_run; ++k) {
    const double r = __longlong_as_double((long long)st.resid[base + k]);
    if (r <= tol) {
      kf = k;
      break;
    }
  }
  s.warm_start_rejected = (fl & kFlagWarmRejected) ? 1 : 0;
  s.reserved = 0;
  s.residual_f64_K = residual_done ? __longlong_as_double((long long)st.resid64[m]) : NAN;
  if (fl & kFlagInvalid) {
    s.status = VARSIM_ERR_INVALID;
    kf = 0;
  } else if (fl & kFlagRunaway) {
    s.status = VARSIM_ERR_RUNAWAY;
    kf = 0;
    for (int k = 1; k <= iters_run; ++k)
      if (st.resid[base + k] != 0ull) kf = k;
  } else if (kf > 0) {
    s.status = VARSIM_OK;
  } else {
    s.status = VARSIM_ERR_NOT_CONVERGED;
    kf = iters_run;
  }
  s.iterations = kf;
  if (kf > 0 && !(fl & kFlagSkip)) {
    s.last_increment_K = __longlong_as_double((long long)st.resid[base + kf]);
    s.dT_mean_K = st.sum[base + kf] / (double)cells;
    const unsigned long long mp = st.maxpack[base + kf];
    const long idx = (long)(0xFFFFFFFFu - (unsigned)(mp & 0xFFFFFFFFull));
    const bool valid = mp != 0ull && idx >= 0 && idx < cells;
    s.hotspot_index = valid ? idx : -1;
    s.dT_max_K = valid ? (double)((const Tio*)maps[m].dT)[idx] : NAN;
  } else {
    s.last_increment_K = kf > 0 ? __longlong_as_double((long long)st.resid[base + kf]) : NAN;
    s.dT_mean_K = NAN;
    s.dT_max_K = NAN;
    s.hotspot_index = -1;
  }
  out[m] = s;
}

// ---------------------------------------------------------------------------------------
template <typename Tio, typename Tc, int N>
hipError_t row_dispatch_mode(int mode, const PassArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = RowCfg<N>;
  const dim3 grid((N / 2) / Cfg::FFTS, a.n_maps), block(Cfg::THREADS);
  switch (mode) {
    case ROW_HEAD: hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_HEAD>), grid, block, 0, s, a, tw, qw); break;
    case ROW_MERGED: hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_MERGED>), grid, block, 0, s, a, tw, qw); break;
    case ROW_LAST: hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_LAST>), grid, block, 0, s, a, tw, qw); break;
    case ROW_RESID: hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_RESID>), grid, block, 0, s, a, tw, qw); break;
    case ROW_CONV_HEAD:
      hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_CONV_HEAD>), grid, block, 0, s, a, tw, qw);
      break;
    case ROW_CONV_TAIL:
      hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_CONV_TAIL>), grid, block, 0, s, a, tw, qw);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Tio, typename Tc>
hipError_t row_dispatch_n(int mode, const PassArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  switch (a.n) {
    case 16: return row_dispatch_mode<Tio, Tc, 16>(mode, a, tw, qw, s);
    case 32: return row_dispatch_mode<Tio, Tc, 32>(mode, a, tw, qw, s);
    case 64: return row_dispatch_mode<Tio, Tc, 64>(mode, a, tw, qw, s);
    case 128: return row_dispatch_mode<Tio, Tc, 128>(mode, a, tw, qw, s);
    case 256: return row_dispatch_mode<Tio, Tc, 256>(mode, a, tw, qw, s);
    case 512: return row_dispatch_mode<Tio, Tc, 512>(mode, a, tw, qw, s);
    case 1024: return row_dispatch_mode<Tio, Tc, 1024>(mode, a, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_row_pass(int mode, int io, int compute, const PassArgs& a, hipStream_t stream) {
  if (compute == VARSIM_F32) {
    if (io != VARSIM_F32) return hipErrorInvalidValue;
    return row_dispatch_n<float, float>(mode, a, a.tw.tw32, a.tw.qw32, stream);
  }
  if (io == VARSIM_F32) return row_dispatch_n<float, double>(mode, a, a.tw.tw64, a.tw.qw64, stream);
  return row_dispatch_n<double, double>(mode, a, a.tw.tw64, a.tw.qw64, stream);
}

hipError_t launch_prep(int io, const PrepArgs* args, int n_maps, long count, hipStream_t stream) {
  const int bx = (int)((count + 255) / 256 < 64 ? (count + 255) / 256 : 64);
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(prep_kernel<float>, dim3(bx, n_maps), dim3(256), 0, stream, args, count);
  else
    hipLaunchKernelGGL(prep_kernel<double>, dim3(bx, n_maps), dim3(256), 0, stream, args, count);
  return hipGetLastError();
}

hipError_t launch_init_copy(int io, const PrepArgs* args, int n_maps, long count, hipStream_t stream) {
  const int bx = (int)((count + 255) / 256 < 64 ? (count + 255) / 256 : 64);
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(init_copy_kernel<float>, dim3(bx, n_maps), dim3(256), 0, stream, args, count);
  else
    hipLaunchKernelGGL(init_copy_kernel<double>, dim3(bx, n_maps), dim3(256), 0, stream, args, count);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t small_launch(const PassArgs& a, int max_iter, const void* coef, hipStream_t s) {
  const Cx<T>* tw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.tw32 : (const Cx<T>*)a.tw.tw64;
  const Cx<T>* qw = sizeof(T) == 4 ? (const Cx<T>*)a.tw.qw32 : (const Cx<T>*)a.tw.qw64;
  hipLaunchKernelGGL((small_solve_kernel<T, T, N>), dim3(a.n_maps), dim3(SmallCfg<T, N>::THREADS), 0, s, a, max_iter,
                     (const T*)coef, tw, qw);
  return hipGetLastError();
}

int small_max_n(int io) { return io == VARSIM_F32 ? 128 : 64; }

hipError_t launch_small_solve(int io, const PassArgs& a, int max_iter, const void* coef, hipStream_t stream) {
  if (a.n > small_max_n(io)) return hipErrorInvalidValue;
  if (io == VARSIM_F32) {
    switch (a.n) {
      case 16: return small_launch<float, 16>(a, max_iter, coef, stream);
      case 32: return small_launch<float, 32>(a, max_iter, coef, stream);
      case 64: return small_launch<float, 64>(a, max_iter, coef, stream);
      case 128: return small_launch<float, 128>(a, max_iter, coef, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.n) {
    case 16: return small_launch<double, 16>(a, max_iter, coef, stream);
    case 32: return small_launch<double, 32>(a, max_iter, coef, stream);
    case 64: return small_launch<double, 64>(a, max_iter, coef, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t stream) {
  const size_t words = bytes / 4;
  if (!words) return hipSuccess;
  const size_t blocks = (words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (unsigned*)p, words);
  return hipGetLastError();
}

hipError_t launch_count_active(const IterState& st, int n_maps, int iter, double tol, int* out, hipStream_t stream) {
  hipLaunchKernelGGL(count_active_kernel, dim3((n_maps + 255) / 256), dim3(256), 0, stream, st, n_maps, iter, tol, out);
  return hipGetLastError();
}

hipError_t launch_finalize(const IterState& st, const MapPtrs* maps, int n_maps, int io, long cells, int max_iter,
                           int iters_run, double tol, int residual_done, varsim_stats* out, hipStream_t stream) {
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(finalize_kernel<float>, dim3((n_maps + 127) / 128), dim3(128), 0, stream, st, maps, n_maps,
                       cells, max_iter, iters_run, tol, residual_done, out);
  else
    hipLaunchKernelGGL(finalize_kernel<double>, dim3((n_maps + 127) / 128), dim3(128), 0, stream, st, maps, n_maps,
                       cells, max_iter, iters_run, tol, residual_done, out);
  return hipGetLastError();
}

}  // namespace vs
