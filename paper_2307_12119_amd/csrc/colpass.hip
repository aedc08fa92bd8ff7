// Column pass of the steady solve and of the plain convolution: per strip of COLS columns of
// one map, the column DCT-II, the multiplication by the cosine eigenvalues lambda of the
// mirrored Green's operator (folded into one step with the split of the two packed columns and
// the merge for the inverse), and the column DCT-III, in place.  The strip width is a tuning
// parameter: the library times the candidates on the actual batch and keeps the fastest.
#include <atomic>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "passes.hpp"
#include "single.hpp"

namespace vs {

namespace {

// When the strips split evenly over the eight XCDs (workgroups are handed to them round-robin
// in launch order), XCD x takes strips [x gx/8, (x+1) gx/8) of every map, so its L2 holds one
// eighth of the column coefficient table (the whole FP64 table at N = 512 is 4.2 MB, as large as
// one XCD's L2) while each XCD still reads whole 128-byte lines of a map's rows; otherwise the
// map-major split of the row passes.
__device__ __forceinline__ void xcd_strip_tile(int& strip, int& map) {
  const int gx = gridDim.x;
  if (gx & 7) {
    xcd_tile(strip, map);
    return;
  }
  const int w = blockIdx.x + gx * blockIdx.y;
  const int per = gx >> 3, i = w >> 3;
  strip = (w & 7) * per + i % per;
  map = i / per;
}

// Waves per SIMD the register allocation must leave room for: the FP64 1024-point transforms
// with one pair per transform group need a few registers more than 256 and would otherwise run
// one wave per SIMD; other instantiations are left to the compiler.
template <typename Tc, int N, int PAIRS>
constexpr int col_min_waves() {
  return sizeof(Tc) == 8 && N == 1024 && PAIRS == 1 ? 2 : 1;
}

// SQ: square map, row stride N known at compile time (otherwise the run-time row length a.n;
// a run-time stride costs the square maps about 15 % of the pass).  CT: compensated twiddles
// (twl: low parts of tw; FP32 only).
template <typename Tc, int N, int COLS, int PAIRS, bool SQ, bool CT = false, bool INPL = false>
__global__ void __launch_bounds__((ColCfg<Tc, N, COLS, PAIRS, INPL>::THREADS))
    __attribute__((amdgpu_waves_per_eu(col_min_waves<Tc, N, ColCfg<Tc, N, COLS, PAIRS, INPL>::PAIRS>())))
    col_pass_kernel(PassArgs a, const Tc* __restrict__ coef, const Cx<Tc>* __restrict__ tw,
                    const Cx<Tc>* __restrict__ qw, const Cx<Tc>* __restrict__ twl) {
  using Cfg = ColCfg<Tc, N, COLS, PAIRS, INPL>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int ST = Shape<N>::STRIDE;
  constexpr int VEC = Cfg::VEC;
  constexpr int VPR = Cfg::COLS / VEC;
  constexpr int P = Cfg::PITCH;
  constexpr int NP = Cfg::PAIRS;
  // one LDS block: first the staging tile, then (after a barrier) the transform scratch
  __shared__ Tc lds[Cfg::LDS];

  int strip, map;
  xcd_strip_tile(strip, map);
  if (a.iter >= 0) {  // iter < 0: plain convolution, no solver state
    if (a.st.flags[map] & kFlagSkip) return;
    if (!a.resid_pass && finished_before(a.st, map, a.iter, a.pp.tol)) return;
  }
  const MapPtrs mp = a.maps[map];
  Tc* S = (Tc*)(a.use_s64 ? mp.S64 : mp.S);
  const int c0 = strip * Cfg::COLS;
  const long rs = SQ ? (long)N : (long)a.n;  // row stride: the row length nx (N = ny is the column length)

#pragma unroll
  for (int k = 0; k < Cfg::LOADS; ++k) {
    const int it = threadIdx.x + k * Cfg::THREADS;
    const int y = it / VPR, j = it % VPR;
    const Vec<Tc, VEC> v = *reinterpret_cast<const Vec<Tc, VEC>*>(S + y * rs + c0 + j * VEC);
#pragma unroll
    for (int e = 0; e < VEC; ++e) lds[tile_row<Cfg, N>(y) * P + j * VEC + e] = v.v[e];
  }
  __syncthreads();

  // pair q of group f: tile columns (2 (f + FFTS q), 2 (f + FFTS q) + 1) -> one complex sequence
  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  // split, multiply by lambda and merge in one step (coefficients alpha, beta, gamma per column)
  // LS: element stride of the transform scratch (P when it is the pair's own tile columns)
  constexpr int LS = Cfg::INPL ? P : 1;
  auto spectral = [&](Tc* zr, Tc* zi, int q, Tc* re, Tc* im) {
    fft_reg<Tc, N, -1, 1, CT, LS>(zr, zi, re, im, tw, t, twl);
    Tc pr[E], pim[E];
    partner<Tc, N, true>(zr, pr, t);
    partner<Tc, N, true>(zi, pim, t);
    const Vec<Tc, 4>* ca = reinterpret_cast<const Vec<Tc, 4>*>(coef) + (long)(c0 + 2 * (f + Cfg::FFTS * q)) * (N / 2 + 1);
    const Vec<Tc, 4>* cb = ca + (N / 2 + 1);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int p = t + TPF * m;
      const bool hi = m >= E / 2;  // p >= N/2: stored at N - p with beta negated
      const int pi = hi ? N - p : p;
      lambda_pair<Tc>(ca[pi], cb[pi], hi, zr[m], zi[m], pr[m], pim[m]);
    }
    wave_sync();
    fft_reg<Tc, N, +1, 1, CT, LS>(zr, zi, re, im, tw, t, twl);
  };
  if constexpr (Cfg::INPL) {
    // pair q's scratch is its own tile columns c (real) and c + 1 (imaginary): the values are
    // in registers before the transform first writes there, and other pairs never touch them
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      const int c = 2 * (f + Cfg::FFTS * q);
      Tc zr[E], zi[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        zr[m] = lds[y * P + c];
        zi[m] = lds[y * P + c + 1];
      }
      spectral(zr, zi, q, lds + c, lds + c + 1);
      wave_sync();  // the transform's last scratch reads are done before the results overwrite rows
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        lds[y * P + c] = zr[m];
        lds[y * P + c + 1] = zi[m];
      }
    }
    __syncthreads();
  } else if constexpr (Cfg::LAZY) {
    Tc* re = lds + Cfg::TILE + f * ST;  // scratch after the tile: real parts, then imaginary parts
    Tc* im = lds + Cfg::TILE + Cfg::FFTS * ST + f * ST;
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      const int c = 2 * (f + Cfg::FFTS * q);
      Tc zr[E], zi[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        zr[m] = lds[y * P + c];
        zi[m] = lds[y * P + c + 1];
      }
      if (q > 0) wave_sync();  // the previous pair's scratch reads are done
      spectral(zr, zi, q, re, im);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        lds[y * P + c] = zr[m];
        lds[y * P + c + 1] = zi[m];
      }
    }
    __syncthreads();
  } else {
    Tc zr[NP][E], zi[NP][E];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        const int c = 2 * (f + Cfg::FFTS * q);
        zr[q][m] = lds[y * P + c];
        zi[q][m] = lds[y * P + c + 1];
      }
    __syncthreads();

    Tc* re = lds + f * ST;  // all real parts first, then all imaginary parts
    Tc* im = lds + Cfg::FFTS * ST + f * ST;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (q > 0) wave_sync();
      spectral(zr[q], zi[q], q, re, im);
    }
    __syncthreads();

#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        const int c = 2 * (f + Cfg::FFTS * q);
        lds[y * P + c] = zr[q][m];
        lds[y * P + c + 1] = zi[q][m];
      }
    __syncthreads();
  }

#pragma unroll
  for (int k = 0; k < Cfg::LOADS; ++k) {
    const int it = threadIdx.x + k * Cfg::THREADS;
    const int y = it / VPR, j = it % VPR;
    Vec<Tc, VEC> v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = lds[tile_row<Cfg, N>(y) * P + j * VEC + e];
    *reinterpret_cast<Vec<Tc, VEC>*>(S + y * rs + c0 + j * VEC) = v;
  }
}

// Pipelined column pass: a grid of a few workgroups per CU, each walking a list of strips and
// loading the next strip's rows into registers while the current strip is transformed in place
// in LDS, so the HBM reads of one strip overlap the transforms of the previous one (a one-shot
// workgroup sits idle on its loads and its CU's memory pipe idles while all its workgroups
// transform).  Strips are COLS columns wide (128-byte row segments); the tile and its in-place
// transform scratch are those of the in-place strip.  Strips split over the XCDs as in
// xcd_strip_tile: XCD x walks strips [x S/8, (x+1) S/8) of every map.
template <typename Tc, int N>
constexpr int pipe_cols() {
  int c = 128 / (int)sizeof(Tc);
  if (c > N / 8) c = N / 8;
  while (c > 2 && (long)Shape<N>::STRIDE * (c + 1) * (long)sizeof(Tc) > 150 * 1024) c /= 2;
  return c;
}
// register budget: the waves per SIMD that the workgroups fitting one CU's 160 KB of LDS bring
template <typename Tc, int N, int COLS, int PAIRS>
constexpr int pipe_waves_per_eu() {
  using Cfg = ColCfg<Tc, N, COLS, PAIRS, true>;
  const long bytes = (long)Cfg::LDS * (long)sizeof(Tc);
  const int wgs = (int)(160 * 1024 / bytes);
  const int w = wgs * (Cfg::THREADS / 64) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}
template <typename Tc, int N, int COLS, int PAIRS, bool CT = false>
__global__ void __launch_bounds__((ColCfg<Tc, N, COLS, PAIRS, true>::THREADS))
    __attribute__((amdgpu_waves_per_eu(pipe_waves_per_eu<Tc, N, COLS, PAIRS>())))
    col_pipe_kernel(PassArgs a, const Tc* __restrict__ coef, const Cx<Tc>* __restrict__ tw,
                    const Cx<Tc>* __restrict__ twl) {
  using Cfg = ColCfg<Tc, N, COLS, PAIRS, true>;
  constexpr int TPF = Cfg::TPF;
  constexpr int E = Shape<N>::E;
  constexpr int VEC = Cfg::VEC;
  constexpr int VPR = Cfg::COLS / VEC;
  constexpr int P = Cfg::PITCH;
  constexpr int NP = Cfg::PAIRS;
  constexpr int SP = N / Cfg::COLS / 8;  // strips per XCD
  static_assert(SP >= 1 && (N / Cfg::COLS) % 8 == 0, "strips must split over the 8 XCDs");
  __shared__ Tc lds[Cfg::LDS];

  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
  const long count = (long)SP * a.n_maps;  // strips of this XCD
  auto map_of = [&](long j) { return (int)(j / SP); };
  auto strip_of = [&](long j) { return xcd * SP + (int)(j % SP); };
  auto active = [&](int map) {
    if (a.iter < 0) return true;  // plain convolution: no solver state
    if (a.st.flags[map] & kFlagSkip) return false;
    return a.resid_pass || !finished_before(a.st, map, a.iter, a.pp.tol);
  };
  auto next_active = [&](long j) {
    while (j < count && !active(map_of(j))) j += per;
    return j;
  };
  auto strip_base = [&](long j) {
    const MapPtrs mp = a.maps[map_of(j)];
    return (Tc*)(a.use_s64 ? mp.S64 : mp.S) + strip_of(j) * Cfg::COLS;
  };

  long j = next_active(blockIdx.x >> 3);
  if (j >= count) return;
  Vec<Tc, VEC> pre[Cfg::LOADS];
  {
    const Tc* S = strip_base(j);
#pragma unroll
    for (int k = 0; k < Cfg::LOADS; ++k) {
      const int it = threadIdx.x + k * Cfg::THREADS;
      pre[k] = *reinterpret_cast<const Vec<Tc, VEC>*>(S + (long)(it / VPR) * N + (it % VPR) * VEC);
    }
  }

  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
#pragma unroll 1
  while (true) {
#pragma unroll
    for (int k = 0; k < Cfg::LOADS; ++k) {
      const int it = threadIdx.x + k * Cfg::THREADS;
      const int y = it / VPR, jj = it % VPR;
#pragma unroll
      for (int e = 0; e < VEC; ++e) lds[tile_row<Cfg, N>(y) * P + jj * VEC + e] = pre[k].v[e];
    }
    __syncthreads();
    const long jn = next_active(j + per);
    if (jn < count) {
      const Tc* Sn = strip_base(jn);
#pragma unroll
      for (int k = 0; k < Cfg::LOADS; ++k) {
        const int it = threadIdx.x + k * Cfg::THREADS;
        pre[k] = *reinterpret_cast<const Vec<Tc, VEC>*>(Sn + (long)(it / VPR) * N + (it % VPR) * VEC);
      }
    }

    const int c0 = strip_of(j) * Cfg::COLS;
#pragma unroll 1
    for (int q = 0; q < NP; ++q) {
      const int c = 2 * (f + Cfg::FFTS * q);
      Tc zr[E], zi[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        zr[m] = lds[y * P + c];
        zi[m] = lds[y * P + c + 1];
      }
      fft_reg<Tc, N, -1, 1, CT, P>(zr, zi, lds + c, lds + c + 1, tw, t, twl);
      Tc pr[E], pim[E];
      partner<Tc, N, true>(zr, pr, t);
      partner<Tc, N, true>(zi, pim, t);
      const Vec<Tc, 4>* ca = reinterpret_cast<const Vec<Tc, 4>*>(coef) + (long)(c0 + c) * (N / 2 + 1);
      const Vec<Tc, 4>* cb = ca + (N / 2 + 1);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int p = t + TPF * m;
        const bool hi = m >= E / 2;
        const int pi = hi ? N - p : p;
        lambda_pair<Tc>(ca[pi], cb[pi], hi, zr[m], zi[m], pr[m], pim[m]);
      }
      wave_sync();
      fft_reg<Tc, N, +1, 1, CT, P>(zr, zi, lds + c, lds + c + 1, tw, t, twl);
      wave_sync();
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int y = tile_slot<Cfg, N>(t + TPF * m);
        lds[y * P + c] = zr[m];
        lds[y * P + c + 1] = zi[m];
      }
    }
    __syncthreads();

    Tc* S = strip_base(j);
#pragma unroll
    for (int k = 0; k < Cfg::LOADS; ++k) {
      const int it = threadIdx.x + k * Cfg::THREADS;
      const int y = it / VPR, jj = it % VPR;
      Vec<Tc, VEC> v;
#pragma unroll
      for (int e = 0; e < VEC; ++e) v.v[e] = lds[tile_row<Cfg, N>(y) * P + jj * VEC + e];
      *reinterpret_cast<Vec<Tc, VEC>*>(S + (long)y * N + jj * VEC) = v;
    }
    if (jn >= count) break;
    __syncthreads();  // the stores' LDS reads are done before the next strip is written there
    j = jn;
  }
}

// One-sequence column pass: each column through a complex DFT of N/2 points (single.hpp),
// COLS columns per workgroup, one per group of TPF lanes.  The DFT leaves the column's cosine
// coefficients X[p] and X[hi(p)] in one lane, so lambda multiplies them directly (no split and
// merge of two packed columns); a column needs half the registers of a packed pair, which is
// what the 1024-point columns (16 elements per lane in the packed form) are short of.  The
// strip is staged in LDS with its rows in z order; the transform scratch reuses the tile.
template <typename Tc, int N, int COLS_>
struct Col1Cfg {
  static constexpr int M = N / 2;
  static constexpr int E = Shape<M>::E, TPF = Shape<M>::TPF;
  static constexpr int COLS = COLS_;
  static constexpr int THREADS = COLS * TPF;
  static constexpr int VEC = (int)(16 / sizeof(Tc)) < COLS ? (int)(16 / sizeof(Tc)) : COLS;
  static constexpr int VPR = COLS / VEC;
  static constexpr int PITCH = COLS + 1;
  static constexpr int TILE = N * PITCH;
  static constexpr int ST = Shape<M>::STRIDE;
  static constexpr int SCRATCH = COLS * 2 * ST;
  static constexpr int LDS = TILE > SCRATCH ? TILE : SCRATCH;
};

template <typename Tc, int N, int COLS>
__global__ void __launch_bounds__((Col1Cfg<Tc, N, COLS>::THREADS))
    col1_pass_kernel(PassArgs a, const Tc* __restrict__ lam, const Cx<Tc>* __restrict__ tw,
                     const Cx<Tc>* __restrict__ qw) {
  using Cfg = Col1Cfg<Tc, N, COLS>;
  constexpr int M = Cfg::M, E = Cfg::E, TPF = Cfg::TPF, ST = Cfg::ST;
  constexpr int VEC = Cfg::VEC, VPR = Cfg::VPR, P = Cfg::PITCH;
  __shared__ Tc lds[Cfg::LDS];

  int strip, map;
  xcd_strip_tile(strip, map);
  if (a.iter >= 0) {
    if (a.st.flags[map] & kFlagSkip) return;
    if (!a.resid_pass && finished_before(a.st, map, a.iter, a.pp.tol)) return;
  }
  const MapPtrs mp = a.maps[map];
  Tc* S = (Tc*)(a.use_s64 ? mp.S64 : mp.S);
  const int c0 = strip * COLS;
  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Vec<Tc, VEC> v = *reinterpret_cast<const Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC);
    Tc* d = lds + z_row<N>(y) * P + j * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = v.v[e];
  }
  __syncthreads();

  int f = threadIdx.x / TPF;
  if constexpr (TPF == 64) f = __builtin_amdgcn_readfirstlane(f);
  const int t = threadIdx.x % TPF;
  Tc zr[E], zi[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    zr[m] = lds[(t + TPF * m) * P + f];
    zi[m] = lds[(M + t + TPF * m) * P + f];
  }
  __syncthreads();
  Tc* re = lds + f * ST;
  Tc* im = lds + COLS * ST + f * ST;
  dct2_single<Tc, N>(zr, zi, re, im, tw, qw, t);
  const Tc* lq = lam + (long)(c0 + f) * N;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int p = t + TPF * m;
    zr[m] *= lq[p];
    zi[m] *= lq[spec_hi<N>(p)];
  }
  dct3_single<Tc, N>(zr, zi, re, im, tw, qw, t);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    lds[(t + TPF * m) * P + f] = zr[m];
    lds[(M + t + TPF * m) * P + f] = zi[m];
  }
  __syncthreads();
  for (int it = threadIdx.x; it < N * VPR; it += Cfg::THREADS) {
    const int y = it / VPR, j = it % VPR;
    const Tc* src = lds + z_row<N>(y) * P + j * VEC;
    Vec<Tc, VEC> v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = src[e];
    *reinterpret_cast<Vec<Tc, VEC>*>(S + (long)y * N + c0 + j * VEC) = v;
  }
}

// strip width of the one-sequence pass: the widest (at most 16 columns) whose tile fits 64 KB,
// halved for candidate 8
template <typename Tc, int N, int V>
constexpr int col1_cols() {
  int c = 16;
  while (c > 1 && ((long)N * (c + 1) * (long)sizeof(Tc) > 65536 || c * Shape<N / 2>::TPF > 1024)) c /= 2;
  if (V == 8 && c > 1) c /= 2;
  return c;
}
template <typename Tc, int N>
constexpr bool col1_ok() {
  return N >= 256;
}

template <typename Tc, int N, int V>
hipError_t col1_launch(const PassArgs& a, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  constexpr int COLS = col1_cols<Tc, N, V>();
  using Cfg = Col1Cfg<Tc, N, COLS>;
  const Tc* lam;
  if constexpr (sizeof(Tc) == 4)
    lam = a.lam32;
  else
    lam = a.lam64;
  if (!lam || a.n != N || a.ny != N) return hipErrorInvalidValue;
  hipLaunchKernelGGL((col1_pass_kernel<Tc, N, COLS>), dim3(N / COLS, a.n_maps), dim3(Cfg::THREADS), 0, s, a, lam, tw,
                     qw);
  return hipGetLastError();
}

// Workgroups per CU of a pipelined instantiation (from its LDS and register use) times the CU
// count, a multiple of 8, taken once per instantiation and device (the grid size changes only
// the speed: any grid walks every strip).
template <typename K>
int pipe_grid(K kernel, int threads) {
  constexpr int kDevices = 64;
  static std::atomic<int> grid[kDevices];  // zero-initialised (static storage); host threads may race here
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < kDevices) {
    const int g = grid[dev].load(std::memory_order_relaxed);
    if (g) return g;
  }
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1)
    return 0;
  const int g = (cus * per + 7) / 8 * 8;
  if (dev < kDevices) grid[dev].store(g, std::memory_order_relaxed);
  return g;
}

template <typename Tc, int N, int COLS, int PAIRS, bool CT>
hipError_t col_pipe_launch(const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, hipStream_t s) {
  using Cfg = ColCfg<Tc, N, COLS, PAIRS, true>;
  if (a.n != N || a.ny != N) return hipErrorInvalidValue;  // square maps only
  const Cx<Tc>* twl = nullptr;
  if constexpr (CT) {
    twl = (const Cx<Tc>*)a.twc.tw32lo;
    if (!twl) return hipErrorInvalidValue;
  }
  auto k = col_pipe_kernel<Tc, N, COLS, PAIRS, CT>;
  int grid = pipe_grid(k, Cfg::THREADS);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  const long tiles = (long)(N / Cfg::COLS) * a.n_maps;
  if (tiles < grid) grid = (int)((tiles + 7) / 8 * 8);
  hipLaunchKernelGGL(k, dim3(grid), dim3(Cfg::THREADS), 0, s, a, coef, tw, twl);
  return hipGetLastError();
}

// Strip-width candidates: 0 = the default width, 1 = the default width with two column pairs
// per transform group (half the wavefronts, each taking its pairs from the tile in turn), 2 =
// half the default width, 3 / 4 = the wide in-place strip (128-byte row segments where two
// workgroups' tiles fit one CU's LDS) with one / two pairs per transform group, 5 / 6 = the
// pipelined pass on 128-byte strips with two / four pairs per transform group (where the strips
// split over the 8 XCDs; otherwise candidate 0).
template <typename Tc, int N>
constexpr int col_wide() {
  int c = 128 / (int)sizeof(Tc);
  while (c > 2 && (long)Shape<N>::STRIDE * (c + 1) * (long)sizeof(Tc) > 80000) c /= 2;
  return c < N ? c : N;
}
template <typename Tc, int N, int V>
constexpr int col_candidate() {
  constexpr int c0 = ColCfg<Tc, N>::COLS;
  constexpr int c = V >= 3 ? col_wide<Tc, N>() : (V == 2 ? c0 / 2 : c0);
  return c < 2 ? 2 : (c > N ? N : c);
}
template <int V>
constexpr int col_pairs() {
  return V == 1 || V == 4 ? 2 : 1;
}
template <int V>
constexpr bool col_inplace() {
  return V >= 3;
}

template <typename Tc, int N, int COLS, int PAIRS, bool SQ = true, bool CT = false, bool INPL = false>
hipError_t col_launch(const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  using Cfg = ColCfg<Tc, N, COLS, PAIRS, INPL>;
  // strips of COLS columns across the row length a.n (a power of two >= 16 >= COLS)
  if (a.n < Cfg::COLS || a.n % Cfg::COLS || (SQ && a.n != N)) return hipErrorInvalidValue;
  const Cx<Tc>* twl = nullptr;
  if constexpr (CT) {
    twl = (const Cx<Tc>*)a.twc.tw32lo;
    if (!twl) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((col_pass_kernel<Tc, N, COLS, PAIRS, SQ, CT, INPL>), dim3(a.n / Cfg::COLS, a.n_maps),
                     dim3(Cfg::THREADS), 0, s, a, coef, tw, qw, twl);
  return hipGetLastError();
}

// Rectangular maps take the default strip width only (the tuner times square maps); compensated
// twiddles are an FP32 option of square maps.
template <typename Tc, int N, int V, bool CT>
hipError_t col_launch_v(const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  return col_launch<Tc, N, col_candidate<Tc, N, V>(), col_pairs<V>(), true, CT, col_inplace<V>()>(a, coef, tw, qw, s);
}
template <int V>
constexpr int pipe_pairs() {
  return V == 5 ? 2 : 4;
}
template <typename Tc, int N, int V>
constexpr bool pipe_ok() {
  return V >= 5 && (N / pipe_cols<Tc, N>()) % 8 == 0 && N / pipe_cols<Tc, N>() >= 8;
}
template <typename Tc, int N, int V, bool CT>
hipError_t col_pipe_v(const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  if constexpr (pipe_ok<Tc, N, V>())
    return col_pipe_launch<Tc, N, pipe_cols<Tc, N>(), pipe_pairs<V>(), CT>(a, coef, tw, s);
  else
    return col_launch_v<Tc, N, 0, CT>(a, coef, tw, qw, s);
}
// one-sequence candidates where available (and lambda is given), else candidate 0
template <typename Tc, int N, int V, bool CT>
hipError_t col1_v(const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  const bool have = sizeof(Tc) == 4 ? a.lam32 != nullptr : a.lam64 != nullptr;
  if constexpr (col1_ok<Tc, N>() && !CT)
    if (have) return col1_launch<Tc, N, V>(a, tw, qw, s);
  return col_launch_v<Tc, N, 0, CT>(a, coef, tw, qw, s);
}
template <typename Tc, int N, bool CT>
hipError_t col_variant_ct(int v, const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  switch (v) {
    case 5: return col_pipe_v<Tc, N, 5, CT>(a, coef, tw, qw, s);
    case 6: return col_pipe_v<Tc, N, 6, CT>(a, coef, tw, qw, s);
    case 7: return col1_v<Tc, N, 7, CT>(a, coef, tw, qw, s);
    case 8: return col1_v<Tc, N, 8, CT>(a, coef, tw, qw, s);
    case 0: return col_launch_v<Tc, N, 0, CT>(a, coef, tw, qw, s);
    case 1: return col_launch_v<Tc, N, 1, CT>(a, coef, tw, qw, s);
    case 2: return col_launch_v<Tc, N, 2, CT>(a, coef, tw, qw, s);
    case 3: return col_launch_v<Tc, N, 3, CT>(a, coef, tw, qw, s);
    case 4: return col_launch_v<Tc, N, 4, CT>(a, coef, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}
template <typename Tc, int N>
hipError_t col_variant(int v, const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw, hipStream_t s) {
  if (a.n != N) return col_launch<Tc, N, col_candidate<Tc, N, 0>(), col_pairs<0>(), false>(a, coef, tw, qw, s);
  if constexpr (std::is_same<Tc, float>::value) {
    if (a.ct) return col_variant_ct<Tc, N, true>(v, a, coef, tw, qw, s);
  }
  return col_variant_ct<Tc, N, false>(v, a, coef, tw, qw, s);
}

template <typename Tc>
hipError_t col_dispatch_n(int v, const PassArgs& a, const Tc* coef, const Cx<Tc>* tw, const Cx<Tc>* qw,
                          hipStream_t s) {
  switch (a.ny) {
    case 16: return col_variant<Tc, 16>(v, a, coef, tw, qw, s);
    case 32: return col_variant<Tc, 32>(v, a, coef, tw, qw, s);
    case 64: return col_variant<Tc, 64>(v, a, coef, tw, qw, s);
    case 128: return col_variant<Tc, 128>(v, a, coef, tw, qw, s);
    case 256: return col_variant<Tc, 256>(v, a, coef, tw, qw, s);
    case 512: return col_variant<Tc, 512>(v, a, coef, tw, qw, s);
    case 1024: return col_variant<Tc, 1024>(v, a, coef, tw, qw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename Tc, int N>
int col_cols_of(int v) {
  switch (v) {
    case 7: return col1_ok<Tc, N>() ? col1_cols<Tc, N, 7>() : col_candidate<Tc, N, 0>();
    case 8: return col1_ok<Tc, N>() ? col1_cols<Tc, N, 8>() : col_candidate<Tc, N, 0>();
    case 5: return pipe_ok<Tc, N, 5>() ? pipe_cols<Tc, N>() : col_candidate<Tc, N, 0>();
    case 6: return pipe_ok<Tc, N, 6>() ? pipe_cols<Tc, N>() : col_candidate<Tc, N, 0>();
    case 0: return col_candidate<Tc, N, 0>();
    case 1: return col_candidate<Tc, N, 1>();
    case 2: return col_candidate<Tc, N, 2>();
    case 3: return col_candidate<Tc, N, 3>();
    case 4: return col_candidate<Tc, N, 4>();
    default: return 0;
  }
}
template <typename Tc, int N, int V>
constexpr int col_pairs_eff() {
  return ColCfg<Tc, N, col_candidate<Tc, N, V>(), col_pairs<V>(), col_inplace<V>()>::PAIRS;
}
template <typename Tc, int N, int V>
constexpr int pipe_pairs_eff() {
  if constexpr (pipe_ok<Tc, N, V>())
    return ColCfg<Tc, N, pipe_cols<Tc, N>(), pipe_pairs<V>(), true>::PAIRS;
  else
    return col_pairs_eff<Tc, N, 0>();
}
template <typename Tc, int N>
int col_pairs_of(int v) {
  switch (v) {
    case 7:
    case 8: return col1_ok<Tc, N>() ? 1 : col_pairs_eff<Tc, N, 0>();
    case 5: return pipe_pairs_eff<Tc, N, 5>();
    case 6: return pipe_pairs_eff<Tc, N, 6>();
    case 0: return col_pairs_eff<Tc, N, 0>();
    case 1: return col_pairs_eff<Tc, N, 1>();
    case 2: return col_pairs_eff<Tc, N, 2>();
    case 3: return col_pairs_eff<Tc, N, 3>();
    case 4: return col_pairs_eff<Tc, N, 4>();
    default: return 0;
  }
}

}  // namespace

hipError_t launch_col_pass(int compute, const PassArgs& a, const void* coef, hipStream_t stream, int variant) {
  if (compute == VARSIM_F32) return col_dispatch_n<float>(variant, a, (const float*)coef, a.twc.tw32, a.twc.qw32, stream);
  return col_dispatch_n<double>(variant, a, (const double*)coef, a.twc.tw64, a.twc.qw64, stream);
}

int col_pass_pairs(int compute, int n, int variant) {
  const bool f = compute == VARSIM_F32;
  switch (n) {
    case 16: return f ? col_pairs_of<float, 16>(variant) : col_pairs_of<double, 16>(variant);
    case 32: return f ? col_pairs_of<float, 32>(variant) : col_pairs_of<double, 32>(variant);
    case 64: return f ? col_pairs_of<float, 64>(variant) : col_pairs_of<double, 64>(variant);
    case 128: return f ? col_pairs_of<float, 128>(variant) : col_pairs_of<double, 128>(variant);
    case 256: return f ? col_pairs_of<float, 256>(variant) : col_pairs_of<double, 256>(variant);
    case 512: return f ? col_pairs_of<float, 512>(variant) : col_pairs_of<double, 512>(variant);
    case 1024: return f ? col_pairs_of<float, 1024>(variant) : col_pairs_of<double, 1024>(variant);
    default: return 0;
  }
}

int col_pass_pipelined(int compute, int n, int variant) {
  const bool f = compute == VARSIM_F32;
  if (variant != 5 && variant != 6) return 0;
  const bool six = variant == 6;
  switch (n) {
#define VS_PIPE_OK(NN) \
  case NN: return f ? (six ? pipe_ok<float, NN, 6>() : pipe_ok<float, NN, 5>()) : (six ? pipe_ok<double, NN, 6>() : pipe_ok<double, NN, 5>());
    VS_PIPE_OK(16) VS_PIPE_OK(32) VS_PIPE_OK(64) VS_PIPE_OK(128) VS_PIPE_OK(256) VS_PIPE_OK(512) VS_PIPE_OK(1024)
#undef VS_PIPE_OK
    default: return 0;
  }
}

int col_pass_family(int compute, int n, int variant) {
  (void)compute;
  return (variant == 7 || variant == 8) && n >= 256 ? 1 : 0;
}

int col_pass_columns(int compute, int n, int variant) {
  const bool f = compute == VARSIM_F32;
  switch (n) {
    case 16: return f ? col_cols_of<float, 16>(variant) : col_cols_of<double, 16>(variant);
    case 32: return f ? col_cols_of<float, 32>(variant) : col_cols_of<double, 32>(variant);
    case 64: return f ? col_cols_of<float, 64>(variant) : col_cols_of<double, 64>(variant);
    case 128: return f ? col_cols_of<float, 128>(variant) : col_cols_of<double, 128>(variant);
    case 256: return f ? col_cols_of<float, 256>(variant) : col_cols_of<double, 256>(variant);
    case 512: return f ? col_cols_of<float, 512>(variant) : col_cols_of<double, 512>(variant);
    case 1024: return f ? col_cols_of<float, 1024>(variant) : col_cols_of<double, 1024>(variant);
    default: return 0;
  }
}

}  // namespace vs
