// Cosine transforms of ONE real sequence of length N through a complex DFT of length M = N / 2
// held in registers (the transform pair behind the slab Green's function diagonalisation,
// Sec. IV-B, computed with the classical real-input DFT split).
//
// Real-space layout ("z order").  With the even/odd reordering v[k] = x[2k], v[N-1-k] = x[2k+1]
// (k < M), the packed sequence z[j] = v[2j] + i v[2j+1] holds
//     j <  M/2 : (x[4j],        x[4j+2])
//     j >= M/2 : (x[2N-4j-1],   x[2N-4j-3]),
// so slot m of lane t (j = t + TPF m) holds two samples of x, z_sample<N>(j, 0/1).
//
// Spectral layout.  The same slot holds the cosine coefficients X[p] and X[hi(p)] for
// p = t + TPF m, hi(p) = N - p (p > 0) and hi(0) = N / 2, so the M slots of a group hold all N
// coefficients once.
//
// Scaling matches the two-sequence transforms of fft.hpp: forward gives the unnormalised DCT-II
// X[p] = sum_n x[n] cos(pi p (2n + 1) / 2N); inverse gives N times the sequence whose DCT-II is
// X (with the p = 0 term at weight 1/2).
#pragma once

#include "fft.hpp"

namespace vs {

// sample index of the real (k = 0) or imaginary (k = 1) part of z[j]
template <int N>
__device__ __forceinline__ int z_sample(int j, int k) {
  return j < N / 4 ? 4 * j + 2 * k : 2 * N - 4 * j - 1 - 2 * k;
}

// row of a column tile in z order: sample y sits at row j (real part of z[j]) or M + j (imaginary)
template <int N>
__device__ __forceinline__ int z_row(int y) {
  constexpr int M = N / 2;
  switch (y & 3) {
    case 0: return y >> 2;
    case 2: return M + ((y - 2) >> 2);
    case 3: return (2 * N - 1 - y) >> 2;
    default: return M + ((2 * N - 3 - y) >> 2);
  }
}

template <int N>
__device__ __forceinline__ int spec_hi(int p) {
  return p ? N - p : N / 2;
}

// z (z order, in zr / zi) -> (X[p], X[hi(p)]) in (zr, zi).  tw, qw: tables of N.
template <typename T, int N>
__device__ __forceinline__ void dct2_single(T* zr, T* zi, T* re, T* im, const Cx<T>* __restrict__ tw,
                                            const Cx<T>* __restrict__ qw, int t) {
  constexpr int M = N / 2, E = Shape<M>::E, TPF = Shape<M>::TPF;
  wave_sync();
  fft_reg<T, M, -1, 2>(zr, zi, re, im, tw, t);
  T cr[E], ci[E];
  partner<T, M, true>(zr, cr, t);
  partner<T, M, true>(zi, ci, t);
  const bool head = t == 0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int p = t + TPF * m;
    // DFTs of the even (ev) and odd (od) elements of v at p, from Z[p] and Z[M - p]
    const T evr = (T)0.5 * (zr[m] + cr[m]), evi = (T)0.5 * (zi[m] - ci[m]);
    const T odr = (T)0.5 * (zi[m] + ci[m]), odi = (T)0.5 * (cr[m] - zr[m]);
    const Cx<T> w = tw[p];  // exp(-2 pi i p / N)
    const T vr = evr + dot2(w.r, odr, -w.i, odi);
    const T vi = evi + dot2(w.r, odi, w.i, odr);
    const Cx<T> q = qw[p];  // (cos, sin)(pi p / 2N)
    zr[m] = dot2(q.r, vr, q.i, vi);
    T hi = dot2(q.i, vr, -q.r, vi);
    if (m == 0) hi = head ? (evr - odr) * (T)0.70710678118654752440 : hi;  // X[N/2] = V[M] / sqrt 2
    zi[m] = hi;
  }
}

// (X[p], X[hi(p)]) in (zr, zi) -> N x in z order.  tw, qw: tables of N.
template <typename T, int N>
__device__ __forceinline__ void dct3_single(T* zr, T* zi, T* re, T* im, const Cx<T>* __restrict__ tw,
                                            const Cx<T>* __restrict__ qw, int t) {
  constexpr int M = N / 2, E = Shape<M>::E, TPF = Shape<M>::TPF;
  const bool head = t == 0;
  // V[p] = exp(i pi p / 2N) (X[p] - i X[N - p]); slot 0 of the head lane: V[0] = X[0] and
  // V[M] = sqrt 2 X[N/2]
  T vr[E], vi[E];
  const T vm = (T)1.41421356237309504880 * zi[0];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const Cx<T> q = qw[t + TPF * m];
    vr[m] = dot2(q.r, zr[m], q.i, zi[m]);
    vi[m] = dot2(q.i, zr[m], -q.r, zi[m]);
  }
  vi[0] = head ? (T)0 : vi[0];
  T cr[E], ci[E];
  partner<T, M, true>(vr, cr, t);
  partner<T, M, true>(vi, ci, t);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int p = t + TPF * m;
    // c = conj V[M - p] = V[p + M]
    T gr = cr[m], gi = -ci[m];
    if (m == 0) {
      gr = head ? vm : gr;
      gi = head ? (T)0 : gi;
    }
    const T sr = vr[m] + gr, si = vi[m] + gi;
    const T dr = vr[m] - gr, di = vi[m] - gi;
    const Cx<T> w = tw[p];  // conj(w) (V[p] - V[p + M]) = 2 x DFT of the odd elements
    zr[m] = sr - dot2(w.r, di, -w.i, dr);
    zi[m] = si + dot2(w.r, dr, w.i, di);
  }
  wave_sync();
  fft_reg<T, M, +1, 2>(zr, zi, re, im, tw, t);
}

// ---------------------------------------------------------------------------------------
// The same transforms with the DFT of length M split over two wavefronts (radix 2 in
// frequency): with H = M / 2,
//     Z[2k]     = DFT_H(z[j] + z[j + H])[k]
//     Z[2k + 1] = DFT_H((z[j] - z[j + H]) W_M^j)[k],
// so wavefront h = 0 transforms a[j] = z[j] + z[j + H] into the even-indexed spectrum and h = 1
// transforms b[j] = (z[j] - z[j + H]) W_M^j into the odd one, each lane holding EL = H / 64
// elements (j = t + 64 m).  The split into cosine coefficients pairs Z[p] with Z[M - p], which
// lies in the same half (even p: element (H - k) mod H of wavefront 0; odd p: element H - 1 - k
// of wavefront 1), so each wavefront finishes its half of the coefficients on its own:
// wavefront h ends with (X[p], X[hi(p)]) for p = 2 (t + 64 m) + h.  The inverse runs the same
// steps backwards: wavefront 0 returns A[j] = IDFT_H of the even half, wavefront 1
// B[j] = W_M^-j IDFT_H of the odd half, and z[j] = A[j] + B[j], z[j + H] = A[j] - B[j]
// (combined by the caller through LDS).  One sequence then occupies two wavefronts, which
// halves each wavefront's serial chain where a single map cannot fill the chip.
template <int N>
struct SplitShape {
  static constexpr int M = N / 2, H = N / 4, EL = H / 64, TS = N / H;
  static_assert(EL >= 2 && EL * 64 == H, "one sequence half per wavefront of 64 lanes");
};

// element E-1-m of lane 63-t: H - 1 - (t + 64 m) of the wavefront's sequence
template <typename T, int EL>
__device__ __forceinline__ void reversed(const T* own, T* out, int t) {
#pragma unroll
  for (int m = 0; m < EL; ++m) out[m] = lane_get(own[EL - 1 - m], 63 - t);
}

// (zr, zi): a[j] (h = 0) or b[j] (h = 1) at j = t + 64 m -> (X[p], X[hi(p)]), p = 2 (t + 64 m) + h
template <typename T, int N>
__device__ __forceinline__ void dct2_split(T* zr, T* zi, T* re, T* im, const Cx<T>* __restrict__ tw,
                                           const Cx<T>* __restrict__ qw, int t, int h) {
  using Sh = SplitShape<N>;
  constexpr int H = Sh::H, EL = Sh::EL;
  wave_sync();
  fft_reg<T, H, -1, Sh::TS, false, 1, EL>(zr, zi, re, im, tw, t);
  T cr[EL], ci[EL];
  if (h == 0) {
    partner<T, H, true, EL>(zr, cr, t);
    partner<T, H, true, EL>(zi, ci, t);
  } else {
    reversed<T, EL>(zr, cr, t);
    reversed<T, EL>(zi, ci, t);
  }
  const bool head = h == 0 && t == 0;
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int p = 2 * (t + 64 * m) + h;
    const T evr = (T)0.5 * (zr[m] + cr[m]), evi = (T)0.5 * (zi[m] - ci[m]);
    const T odr = (T)0.5 * (zi[m] + ci[m]), odi = (T)0.5 * (cr[m] - zr[m]);
    const Cx<T> w = tw[p];
    const T vr = evr + dot2(w.r, odr, -w.i, odi);
    const T vi = evi + dot2(w.r, odi, w.i, odr);
    const Cx<T> q = qw[p];
    zr[m] = dot2(q.r, vr, q.i, vi);
    T hi = dot2(q.i, vr, -q.r, vi);
    if (m == 0) hi = head ? (evr - odr) * (T)0.70710678118654752440 : hi;
    zi[m] = hi;
  }
}

// (X[p], X[hi(p)]), p = 2 (t + 64 m) + h -> A[j] (h = 0) or B[j] (h = 1) at j = t + 64 m
template <typename T, int N>
__device__ __forceinline__ void dct3_split(T* zr, T* zi, T* re, T* im, const Cx<T>* __restrict__ tw,
                                           const Cx<T>* __restrict__ qw, int t, int h) {
  using Sh = SplitShape<N>;
  constexpr int H = Sh::H, EL = Sh::EL;
  const bool head = h == 0 && t == 0;
  T vr[EL], vi[EL];
  const T vm = (T)1.41421356237309504880 * zi[0];
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const Cx<T> q = qw[2 * (t + 64 * m) + h];
    vr[m] = dot2(q.r, zr[m], q.i, zi[m]);
    vi[m] = dot2(q.i, zr[m], -q.r, zi[m]);
  }
  vi[0] = head ? (T)0 : vi[0];
  T cr[EL], ci[EL];
  if (h == 0) {
    partner<T, H, true, EL>(vr, cr, t);
    partner<T, H, true, EL>(vi, ci, t);
  } else {
    reversed<T, EL>(vr, cr, t);
    reversed<T, EL>(vi, ci, t);
  }
#pragma unroll
  for (int m = 0; m < EL; ++m) {
    const int p = 2 * (t + 64 * m) + h;
    T gr = cr[m], gi = -ci[m];
    if (m == 0) {
      gr = head ? vm : gr;
      gi = head ? (T)0 : gi;
    }
    const T sr = vr[m] + gr, si = vi[m] + gi;
    const T dr = vr[m] - gr, di = vi[m] - gi;
    const Cx<T> w = tw[p];
    zr[m] = sr - dot2(w.r, di, -w.i, dr);
    zi[m] = si + dot2(w.r, dr, w.i, di);
  }
  wave_sync();
  fft_reg<T, H, +1, Sh::TS, false, 1, EL>(zr, zi, re, im, tw, t);
  if (h == 1) {
#pragma unroll
    for (int m = 0; m < EL; ++m) {
      const Cx<T> w = tw[2 * (t + 64 * m)];  // W_M^j; multiplied by its conjugate
      const T r = zr[m], i = zi[m];
      zr[m] = dot2(w.r, r, w.i, i);
      zi[m] = dot2(w.r, i, -w.i, r);
    }
  }
}

// a[j] (h = 0) or b[j] (h = 1) from z[j] = (ar, ai) and z[j + H] = (br, bi) at j = t + 64 m
template <typename T, int N>
__device__ __forceinline__ void split_inputs(T& zr, T& zi, T ar, T ai, T br, T bi, int j, int h,
                                             const Cx<T>* __restrict__ tw) {
  if (h == 0) {
    zr = ar + br;
    zi = ai + bi;
  } else {
    const Cx<T> w = tw[2 * j];  // W_M^j
    const T dr = ar - br, di = ai - bi;
    zr = dot2(dr, w.r, -di, w.i);
    zi = dot2(dr, w.i, di, w.r);
  }
}

}  // namespace vs
