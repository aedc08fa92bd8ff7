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
#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "rowops.hpp"
#include "rowpass.hpp"

namespace vs {

namespace {

// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) prep_kernel(const PrepArgs* __restrict__ args, long count) {
  // 16 bytes per lane and step; the inputs are read once (non-temporal), QL and 1/m are read
  // again by the first row pass
  constexpr int V = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  const PrepArgs pa = args[blockIdx.y];
  bool invalid = false, warm_bad = false;
  const long nv = count / V;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (long)gridDim.x * blockDim.x) {
    vec_t v = (T)0;
    if (pa.ql_out || pa.qls_out) {
      v = __builtin_nontemporal_load((const vec_t*)pa.q_leak0 + i);
      if (pa.leak_var) v *= __builtin_nontemporal_load((const vec_t*)pa.leak_var + i);
    }
    if (pa.ql_out) ((vec_t*)pa.ql_out)[i] = v;
    if (pa.minv_out) {
      const vec_t m = __builtin_nontemporal_load((const vec_t*)pa.cond_map + i);
      vec_t r;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if (!(m[e] > (T)0) || !isfinite(m[e])) invalid = true;
        r[e] = (T)1 / m[e];
      }
      ((vec_t*)pa.minv_out)[i] = r;
      if (pa.qs_out) ((vec_t*)pa.qs_out)[i] = __builtin_nontemporal_load((const vec_t*)pa.q_dyn + i) * r;
      if (pa.qls_out) ((vec_t*)pa.qls_out)[i] = v * r;
    }
    if (pa.init) {
      const vec_t w = ((const vec_t*)pa.init)[i];
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (!isfinite(w[e])) warm_bad = true;
    }
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

// Number of maps still iterating after iteration `iter`, stored to *out by one workgroup (out
// may be pinned host memory: the host reads it once an event behind this kernel has completed).
__global__ void __launch_bounds__(1024) count_active_kernel(IterState st, int n_maps, int iter, double tol, int* out) {
  __shared__ int s_cnt[16];
  int c = 0;
  for (int m = threadIdx.x; m < n_maps; m += blockDim.x) {
    if (st.flags[m] & (kFlagSkip | kFlagOwnLoop)) continue;
    const double r = __longlong_as_double((long long)st.resid[(long)m * st.stride + iter]);
    if (!(r <= tol)) ++c;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) total += s_cnt[w];
    *out = total;
    __threadfence_system();
  }
}

// Per-map statistics.  The mean of a map iterated by the two-pass loop adds the row-pass
// workgroups' sums of its last iteration (row_groups of them) in index order; a map solved by its
// own LDS-resident workgroup has its sum in the iteration's slot.
template <typename Tio>
__global__ void finalize_kernel(IterState st, const MapPtrs* __restrict__ maps, int n_maps, long cells, int max_iter,
                                int iters_run, double tol, int residual_done, int row_groups, int oneshot,
                                varsim_stats* out) {
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
    double total = 0.0;
    if (fl & kFlagOwnLoop) {
      total = st.sum[base + kf];
    } else {
      const double* p = st.part + (long)m * kRowGroupsMax;
      for (int g = 0; g < row_groups; ++g) total += p[g];
    }
    s.dT_mean_K = total / (double)cells;
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
  if (oneshot) {  // the one-shot solve iterates nothing: no count, no increment
    s.iterations = 0;
    s.last_increment_K = NAN;
  }
  out[m] = s;
}

// ---------------------------------------------------------------------------------------
template <typename Tio, typename Tc, int N>
hipError_t row_dispatch_mode(int mode, const PassArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = RowCfg<N>;
  // rows of the map: a.ny, 2 FFTS per workgroup (the host admits only grids where they divide)
  if (a.ny < 2 * Cfg::FFTS || a.ny % (2 * Cfg::FFTS)) return hipErrorInvalidValue;
  const dim3 grid((a.ny / 2) / Cfg::FFTS, a.n_maps), block(Cfg::THREADS);
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
    case ROW_OS_MID:
      if constexpr (std::is_same<Tio, Tc>::value)
        hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_OS_MID>), grid, block, 0, s, a, tw, qw);
      else
        return hipErrorInvalidValue;
      break;
    case ROW_OS_TAIL:
      if constexpr (std::is_same<Tio, Tc>::value)
        hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_OS_TAIL>), grid, block, 0, s, a, tw, qw);
      else
        return hipErrorInvalidValue;
      break;
    case ROW_AA_EVAL:
      if constexpr (std::is_same<Tio, Tc>::value)
        hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_AA_EVAL>), grid, block, 0, s, a, tw, qw);
      else
        return hipErrorInvalidValue;
      break;
    case ROW_AA_MIX:
      if constexpr (std::is_same<Tio, Tc>::value)
        hipLaunchKernelGGL((row_pass_kernel<Tio, Tc, N, ROW_AA_MIX>), grid, block, 0, s, a, tw, qw);
      else
        return hipErrorInvalidValue;
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
    if (a.ct && (mode == ROW_HEAD || mode == ROW_MERGED || mode == ROW_LAST)) return launch_row_pass_ct(mode, a, stream);
    return row_dispatch_n<float, float>(mode, a, a.tw.tw32, a.tw.qw32, stream);
  }
  if (io == VARSIM_F32) return row_dispatch_n<float, double>(mode, a, a.tw.tw64, a.tw.qw64, stream);
  return row_dispatch_n<double, double>(mode, a, a.tw.tw64, a.tw.qw64, stream);
}

hipError_t launch_prep(int io, const PrepArgs* args, int n_maps, long count, hipStream_t stream) {
  if (count % 4) return hipErrorInvalidValue;  // whole 16-byte vectors (grids are 16 x 16 or larger)
  const long nv = count / (io == VARSIM_F32 ? 4 : 2);
  const int bx = (int)((nv + 255) / 256 < 64 ? (nv + 255) / 256 : 64);
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
  hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(1024), 0, stream, st, n_maps, iter, tol, out);
  return hipGetLastError();
}

namespace {
__global__ void scatter_stats_kernel(const varsim_stats* __restrict__ src, const int* __restrict__ order, int n,
                                     varsim_stats* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[order[i]] = src[i];
}
}  // namespace

hipError_t launch_scatter_stats(const varsim_stats* src, const int* order, int n, varsim_stats* dst, hipStream_t s) {
  hipLaunchKernelGGL(scatter_stats_kernel, dim3((n + 127) / 128), dim3(128), 0, s, src, order, n, dst);
  return hipGetLastError();
}

hipError_t launch_finalize(const IterState& st, const MapPtrs* maps, int n_maps, int io, int nx, int ny, int max_iter,
                           int iters_run, double tol, int residual_done, varsim_stats* out, hipStream_t stream,
                           int oneshot) {
  const long cells = (long)nx * ny;
  const int groups = row_pass_groups(nx, ny);
  if (groups < 1 || groups > kRowGroupsMax) return hipErrorInvalidValue;
  if (io == VARSIM_F32)
    hipLaunchKernelGGL(finalize_kernel<float>, dim3((n_maps + 127) / 128), dim3(128), 0, stream, st, maps, n_maps,
                       cells, max_iter, iters_run, tol, residual_done, groups, oneshot, out);
  else
    hipLaunchKernelGGL(finalize_kernel<double>, dim3((n_maps + 127) / 128), dim3(128), 0, stream, st, maps, n_maps,
                       cells, max_iter, iters_run, tol, residual_done, groups, oneshot, out);
  return hipGetLastError();
}

int row_pass_rows(int nx) {
  switch (nx) {
    case 16: return 2 * RowCfg<16>::FFTS;
    case 32: return 2 * RowCfg<32>::FFTS;
    case 64: return 2 * RowCfg<64>::FFTS;
    case 128: return 2 * RowCfg<128>::FFTS;
    case 256: return 2 * RowCfg<256>::FFTS;
    case 512: return 2 * RowCfg<512>::FFTS;
    case 1024: return 2 * RowCfg<1024>::FFTS;
    default: return 0;
  }
}

int row_pass_groups(int nx, int ny) {
  const int r = row_pass_rows(nx);
  return r > 0 && ny % r == 0 ? ny / r : 0;
}

}  // namespace vs
