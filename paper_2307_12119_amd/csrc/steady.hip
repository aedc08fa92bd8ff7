// Steady-solve kernels: the fixed point dT = G(dT) of the leakage- and conductivity-coupled
// Green's-function convolution (Eqs. Green, Pt, Pleak, condsi, fspvsk; Sec. IV-F images).
//
// One iteration is two passes over each map:
//   row pass    : cosine-synthesis of each row (row DCT-III) of the previous spectrum, the
//                 conductivity-variation factor, the Kirchhoff inverse of k(T), the increment
//                 and statistics, the new total power P = hx hy (q_dyn + QL L(dT)), and the
//                 row DCT-II of P into the spectrum array (in place, same rows);
//   column pass : column DCT-II, multiplication by the cosine eigenvalues lambda of the
//                 mirrored Green's operator, column DCT-III (in place, column tiles in LDS).
// The first row pass of a solve starts from dT_init (or 0), the last one skips the forward part.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"

namespace vs {

namespace {

template <int N>
struct RowCfg {
  static constexpr int TPF = N / 8;
  static constexpr int FFTS = (256 / TPF) < (N / 2) ? (256 / TPF) : (N / 2);
  static constexpr int THREADS = FFTS * TPF;
  static constexpr int WAVE = THREADS < 64 ? THREADS : 64;
};

constexpr int col_count(int n, int esz) {
  int c = 32;
  while (c > 2 && (long)c * 2 * (n + n / 8 + 1) * esz > 78000) c /= 2;
  return c < n ? c : n;
}

template <typename Tc, int N>
struct ColCfg {
  static constexpr int TPF = N / 8;
  static constexpr int COLS = col_count(N, (int)sizeof(Tc));
  static constexpr int FFTS = COLS / 2;
  static constexpr int GROUPS = (256 / TPF) < FFTS ? (256 / TPF) : FFTS;
  static constexpr int THREADS = GROUPS * TPF;
  static constexpr int ROUNDS = FFTS / GROUPS;
  static constexpr int VEC = (int)(16 / sizeof(Tc)) < COLS ? (int)(16 / sizeof(Tc)) : COLS;
};

template <typename T>
__device__ __forceinline__ T ldm(const void* p, long i) {
  return ((const T*)p)[i];
}

// order-preserving key of a float for packed max / argmax
__device__ __forceinline__ unsigned order_key(float v) {
  const unsigned u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ unsigned long long pack_max(float v, long idx) {
  return ((unsigned long long)order_key(v) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)idx);
}

template <typename Tc>
__device__ __forceinline__ Tc leak_factor(Tc dT, const PointParams& pp) {
  if (pp.leak == VARSIM_LEAK_EXP) return exp((Tc)pp.beta * dT);
  if (pp.leak == VARSIM_LEAK_LINEAR) return (Tc)1 + (Tc)pp.beta * dT;
  return (Tc)0;
}

// dT = Phi^-1(theta) for k = k_ref (T / T_amb)^-eta
template <typename Tc>
__device__ __forceinline__ Tc kirchhoff_inv(Tc theta, const PointParams& pp, bool& bad) {
  if (pp.eta_mode == 0) return theta;
  if (pp.eta_mode == 1) return (Tc)pp.t_amb * expm1(theta / (Tc)pp.t_amb);
  const Tc x = (Tc)pp.c_1m_eta * theta;
  if (!(x > (Tc)-1)) {
    bad = true;
    return (Tc)0;
  }
  return (Tc)pp.t_amb * expm1((Tc)pp.inv_1m_eta * log1p(x));
}

template <int W>
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
  return v;
}
template <int W>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W>
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, W);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ bool finished_before(const IterState& st, int map, int iter, double tol) {
  if (iter < 2) return false;
  const double prev = __longlong_as_double((long long)st.resid[(long)map * st.stride + iter - 1]);
  return prev <= tol;
}

template <typename Tio, typename Tc, int N, int MODE>
__global__ void __launch_bounds__(RowCfg<N>::THREADS)
    row_pass_kernel(PassArgs a, const Cx<Tc>* __restrict__ tw, const Cx<Tc>* __restrict__ qw) {
  using Cfg = RowCfg<N>;
  constexpr int TPF = Cfg::TPF;
  constexpr int ST = Lds<N>::STRIDE;
  __shared__ Tc s_re[Cfg::FFTS * ST];
  __shared__ Tc s_im[Cfg::FFTS * ST];

  const int map = blockIdx.y;
  unsigned flags = 0u;
  if (MODE != ROW_CONV_HEAD && MODE != ROW_CONV_TAIL) {
    flags = a.st.flags[map];
    if (flags & kFlagSkip) return;
    if ((MODE == ROW_MERGED || MODE == ROW_LAST) && finished_before(a.st, map, a.iter, a.pp.tol)) return;
  }
  const MapPtrs mp = a.maps[map];
  const int f = threadIdx.x / TPF, t = threadIdx.x % TPF;
  const int row = (blockIdx.x * Cfg::FFTS + f) * 2;
  Tc* re = s_re + f * ST;
  Tc* im = s_im + f * ST;
  Tc* S = (Tc*)(a.use_s64 ? mp.S64 : mp.S);
  const long oa = (long)row * N, ob = oa + N;
  const PointParams& pp = a.pp;
  const Tc sqrt2 = (Tc)1.4142135623730950488016887242097;
  const Tc half_sqrt2 = (Tc)0.70710678118654752440084436210485;

  // ---- inverse half: spectrum rows -> theta (row DCT-III of the packed pair)
  if constexpr (MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID || MODE == ROW_CONV_TAIL) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int p = t + s4 * TPF;
      if (p == 0) {
        re[Lds<N>::at(0)] = S[oa];
        im[Lds<N>::at(0)] = S[ob];
        re[Lds<N>::at(N / 2)] = sqrt2 * S[oa + N / 2];
        im[Lds<N>::at(N / 2)] = sqrt2 * S[ob + N / 2];
      } else {
        const Cx<Tc> q = qw[p];
        Tc zr, zi, z2r, z2i;
        merge_pair<Tc>(S[oa + p], S[ob + p], S[oa + N - p], S[ob + N - p], q.r, q.i, zr, zi, z2r, z2i);
        re[Lds<N>::at(p)] = zr;
        im[Lds<N>::at(p)] = zi;
        re[Lds<N>::at(N - p)] = z2r;
        im[Lds<N>::at(N - p)] = z2i;
      }
    }
    __syncthreads();
    fft_stages<Tc, N, 1, +1>(re, im, tw, t);
  }

  // ---- pointwise: conductivity factor, Kirchhoff inverse, increment, stats, new power
  double inc = 0.0, sum = 0.0;
  unsigned long long best = 0ull;
  bool bad = false;
  const bool zero_old = (a.iter == 1) && (a.zero_start || (flags & kFlagWarmRejected));
#pragma unroll
  for (int s8 = 0; s8 < 8; ++s8) {
    const int i = t + s8 * TPF;
    const int li = Lds<N>::at(perm<N>(i));
    if constexpr (MODE == ROW_CONV_TAIL) {
      ((Tio*)mp.dT)[oa + i] = (Tio)re[li];
      ((Tio*)mp.dT)[ob + i] = (Tio)im[li];
      continue;
    } else if constexpr (MODE == ROW_CONV_HEAD) {
      re[li] = (Tc)ldm<Tio>(mp.qd, oa + i);
      im[li] = (Tc)ldm<Tio>(mp.qd, ob + i);
      continue;
    } else {
      Tc xa, xb;
      if constexpr (MODE == ROW_HEAD) {
        if (zero_old) {
          xa = (Tc)0;
          xb = (Tc)0;
        } else {
          xa = (Tc)ldm<Tio>(mp.dT, oa + i);
          xb = (Tc)ldm<Tio>(mp.dT, ob + i);
        }
      } else {
        Tc ta = re[li], tb = im[li];
        if (mp.minv) {
          ta *= (Tc)ldm<Tio>(mp.minv, oa + i);
          tb *= (Tc)ldm<Tio>(mp.minv, ob + i);
        }
        xa = kirchhoff_inv<Tc>(ta, pp, bad);
        xb = kirchhoff_inv<Tc>(tb, pp, bad);
        const Tc olda = zero_old ? (Tc)0 : (Tc)ldm<Tio>(mp.dT, oa + i);
        const Tc oldb = zero_old ? (Tc)0 : (Tc)ldm<Tio>(mp.dT, ob + i);
        const Tc da = xa - olda, db = xb - oldb;
        inc = fmax(inc, (double)fmax(fabs(da), fabs(db)));
        if (!isfinite(xa) || !isfinite(xb) || xa > (Tc)pp.cap || xb > (Tc)pp.cap) bad = true;
        if constexpr (MODE != ROW_RESID) {
          const Tio sa = (Tio)xa, sb = (Tio)xb;
          ((Tio*)mp.dT)[oa + i] = sa;
          ((Tio*)mp.dT)[ob + i] = sb;
          sum += (double)sa + (double)sb;
          const unsigned long long ka = pack_max((float)sa, oa + i), kb = pack_max((float)sb, ob + i);
          best = ka > best ? ka : best;
          best = kb > best ? kb : best;
        }
      }
      if constexpr (MODE == ROW_HEAD || MODE == ROW_MERGED) {
        Tc qa = (Tc)ldm<Tio>(mp.qd, oa + i), qb = (Tc)ldm<Tio>(mp.qd, ob + i);
        if (mp.ql) {
          qa += (Tc)ldm<Tio>(mp.ql, oa + i) * leak_factor<Tc>(xa, pp);
          qb += (Tc)ldm<Tio>(mp.ql, ob + i) * leak_factor<Tc>(xb, pp);
        }
        re[li] = (Tc)pp.hxhy * qa;
        im[li] = (Tc)pp.hxhy * qb;
      }
    }
  }

  if constexpr (MODE == ROW_MERGED || MODE == ROW_LAST || MODE == ROW_RESID) {
    constexpr int W = Cfg::WAVE;
    inc = wave_max<W>(inc);
    const bool lane0 = (threadIdx.x % W) == 0;
    const unsigned bad_any = __any(bad);
    if (MODE == ROW_RESID) {
      if (lane0) atomicMax(&a.st.resid64[map], (unsigned long long)__double_as_longlong(inc));
    } else {
      sum = wave_sum<W>(sum);
      best = wave_max_u64<W>(best);
      if (lane0) {
        const long slot = (long)map * a.st.stride + a.iter;
        atomicMax(&a.st.resid[slot], (unsigned long long)__double_as_longlong(inc));
        atomicAdd(&a.st.sum[slot], sum);
        atomicMax(&a.st.maxpack[slot], best);
      }
    }
    if (lane0 && bad_any) atomicOr(&a.st.flags[map], kFlagRunaway);
  }

  // ---- forward half: P rows -> row DCT-II spectrum
  if constexpr (MODE == ROW_HEAD || MODE == ROW_MERGED || MODE == ROW_CONV_HEAD) {
    __syncthreads();
    fft_stages<Tc, N, 1, -1>(re, im, tw, t);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int p = t + s4 * TPF;
      if (p == 0) {
        S[oa] = re[Lds<N>::at(0)];
        S[ob] = im[Lds<N>::at(0)];
        S[oa + N / 2] = half_sqrt2 * re[Lds<N>::at(N / 2)];
        S[ob + N / 2] = half_sqrt2 * im[Lds<N>::at(N / 2)];
      } else {
        const Cx<Tc> q = qw[p];
        Tc xa, xb, xa2, xb2;
        split_pair<Tc>(re[Lds<N>::at(p)], im[Lds<N>::at(p)], re[Lds<N>::at(N - p)], im[Lds<N>::at(N - p)], q.r, q.i,
                       xa, xb, xa2, xb2);
        S[oa + p] = xa;
        S[ob + p] = xb;
        S[oa + N - p] = xa2;
        S[ob + N - p] = xb2;
      }
    }
  }
}

template <typename Tc, int N>
__global__ void __launch_bounds__((ColCfg<Tc, N>::THREADS))
    col_pass_kernel(PassArgs a, const Tc* __restrict__ lamT, const Cx<Tc>* __restrict__ tw,
                    const Cx<Tc>* __restrict__ qw) {
  using Cfg = ColCfg<Tc, N>;
  constexpr int TPF = Cfg::TPF;
  constexpr int ST = Lds<N>::STRIDE;
  constexpr int VEC = Cfg::VEC;
  constexpr int VPR = Cfg::COLS / VEC;
  __shared__ Tc s_re[Cfg::FFTS * ST];
  __shared__ Tc s_im[Cfg::FFTS * ST];

  const int map = blockIdx.y;
  if (a.iter >= 0) {  // iter < 0: plain convolution, no solver state
    if (a.st.flags[map] & kFlagSkip) return;
    if (!a.resid_pass && finished_before(a.st, map, a.iter, a.pp.tol)) return;
  }
  const MapPtrs mp = a.maps[map];
  Tc* S = (Tc*)(a.use_s64 ? mp.S64 : mp.S);
  const int c0 = blockIdx.x * Cfg::COLS;

  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Tc* src = S + (long)y * N + c0 + j * VEC;
    Tc v[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = src[e];
    const int li = Lds<N>::at(perm<N>(y));
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int col = j * VEC + e;
      ((col & 1) ? s_im : s_re)[(col >> 1) * ST + li] = v[e];
    }
  }
  __syncthreads();

  const int g = threadIdx.x / TPF, t = threadIdx.x % TPF;
  for (int rd = 0; rd < Cfg::ROUNDS; ++rd) {
    const int fi = rd * Cfg::GROUPS + g;
    Tc* re = s_re + fi * ST;
    Tc* im = s_im + fi * ST;
    fft_stages<Tc, N, 1, -1>(re, im, tw, t);
    const Tc* la = lamT + (long)(c0 + 2 * fi) * N;
    const Tc* lb = la + N;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int p = t + s4 * TPF;
      if (p == 0) {
        re[Lds<N>::at(0)] *= la[0];
        im[Lds<N>::at(0)] *= lb[0];
        re[Lds<N>::at(N / 2)] *= la[N / 2];
        im[Lds<N>::at(N / 2)] *= lb[N / 2];
      } else {
        const Cx<Tc> q = qw[p];
        const int lp = Lds<N>::at(p), lq = Lds<N>::at(N - p);
        Tc xa, xb, xa2, xb2;
        split_pair<Tc>(re[lp], im[lp], re[lq], im[lq], q.r, q.i, xa, xb, xa2, xb2);
        xa *= la[p];
        xb *= lb[p];
        xa2 *= la[N - p];
        xb2 *= lb[N - p];
        Tc zr, zi, z2r, z2i;
        merge_pair<Tc>(xa, xb, xa2, xb2, q.r, q.i, zr, zi, z2r, z2i);
        re[lp] = zr;
        im[lp] = zi;
        re[lq] = z2r;
        im[lq] = z2i;
      }
    }
    __syncthreads();
    fft_stages<Tc, N, 1, +1>(re, im, tw, t);
  }

  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    Tc* dst = S + (long)y * N + c0 + j * VEC;
    const int li = Lds<N>::at(perm<N>(y));
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int col = j * VEC + e;
      dst[e] = ((col & 1) ? s_im : s_re)[(col >> 1) * ST + li];
    }
  }
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
  if (st.flags[m] & kFlagSkip) return;
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

template <typename Tc, int N>
hipError_t col_launch(const PassArgs& a, const Tc* lamT, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = ColCfg<Tc, N>;
  hipLaunchKernelGGL((col_pass_kernel<Tc, N>), dim3(N / Cfg::COLS, a.n_maps), dim3(Cfg::THREADS), 0, s, a, lamT, tw,
                     qw);
  return hipGetLastError();
}

template <typename Tc>
hipError_t col_dispatch_n(const PassArgs& a, const Tc* lamT, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  switch (a.n) {
    case 16: return col_launch<Tc, 16>(a, lamT, tw, qw, s);
    case 32: return col_launch<Tc, 32>(a, lamT, tw, qw, s);
    case 64: return col_launch<Tc, 64>(a, lamT, tw, qw, s);
    case 128: return col_launch<Tc, 128>(a, lamT, tw, qw, s);
    case 256: return col_launch<Tc, 256>(a, lamT, tw, qw, s);
    case 512: return col_launch<Tc, 512>(a, lamT, tw, qw, s);
    case 1024: return col_launch<Tc, 1024>(a, lamT, tw, qw, s);
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

hipError_t launch_col_pass(int compute, const PassArgs& a, const void* lamT, hipStream_t stream) {
  if (compute == VARSIM_F32) return col_dispatch_n<float>(a, (const float*)lamT, a.tw.tw32, a.tw.qw32, stream);
  return col_dispatch_n<double>(a, (const double*)lamT, a.tw.tw64, a.tw.qw64, stream);
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
