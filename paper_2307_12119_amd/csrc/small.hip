// Small grids: the whole steady fixed point of a map by one workgroup whose LDS holds the map's
// spectrum (see the kernel comment); the two-pass path drives larger maps.
#include <cmath>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "rowops.hpp"

namespace vs {

namespace {

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
        lambda_pair<Tc>(ca[pi], cb[pi], hi, zr[m], zi[m], pr[m], pim[m]);
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

}  // namespace

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

}  // namespace vs
