// Device building blocks for the real 2-D cosine transforms of the convolution.
//
// A length-N complex DFT runs on N/8 threads, each owning 8 elements, as a sequence of
// Stockham autosort stages of radix 8 (a final radix 4 or 2 when log2 N is not a multiple of
// 3) through LDS.  LDS holds real and imaginary parts in separate arrays with one pad word
// every 8 entries so that the strided butterfly stores do not collide in the LDS banks.
//
// Two real sequences share one complex DFT (one as the real part, one as the imaginary
// part).  The cosine transforms use the N-point reordering of the sequence (even samples
// ascending, odd samples descending), after which
//     DCT-II:  X[p] = Re( e^{-i pi p / 2N} V[p] ),  V = DFT(v)
//     inverse: V[p] = e^{+i pi p / 2N} (X[p] - i X[N-p]),  v = unnormalised inverse DFT(V)
// The pair split / merge formulas below combine both identities for the two packed rows.
#pragma once

#include "common.hpp"

namespace vs {

template <int N>
struct Lds {
  static constexpr int STRIDE = N + N / 8 + 1;  // odd: consecutive buffers start in other banks
  __device__ __forceinline__ static int at(int i) { return i + (i >> 3); }
};

// position of sample i in the reordered sequence
template <int N>
__device__ __forceinline__ int perm(int i) {
  return (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
}

// multiply by DIR * i
template <typename T, int DIR>
__device__ __forceinline__ void mul_i(T& r, T& i) {
  const T tr = r;
  if (DIR < 0) {
    r = i;
    i = -tr;
  } else {
    r = -i;
    i = tr;
  }
}

template <typename T, int DIR>
__device__ __forceinline__ void dft2(T* r, T* i) {
  const T ar = r[0], ai = i[0];
  r[0] = ar + r[1];
  i[0] = ai + i[1];
  r[1] = ar - r[1];
  i[1] = ai - i[1];
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(T* r, T* i) {
  const T s0r = r[0] + r[2], s0i = i[0] + i[2];
  const T d0r = r[0] - r[2], d0i = i[0] - i[2];
  const T s1r = r[1] + r[3], s1i = i[1] + i[3];
  T d1r = r[1] - r[3], d1i = i[1] - i[3];
  mul_i<T, DIR>(d1r, d1i);
  r[0] = s0r + s1r;
  i[0] = s0i + s1i;
  r[2] = s0r - s1r;
  i[2] = s0i - s1i;
  r[1] = d0r + d1r;
  i[1] = d0i + d1i;
  r[3] = d0r - d1r;
  i[3] = d0i - d1i;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft8(T* r, T* i) {
  T er[4] = {r[0], r[2], r[4], r[6]}, ei[4] = {i[0], i[2], i[4], i[6]};
  T orr[4] = {r[1], r[3], r[5], r[7]}, oi[4] = {i[1], i[3], i[5], i[7]};
  dft4<T, DIR>(er, ei);
  dft4<T, DIR>(orr, oi);
  const T c = (T)0.70710678118654752440084436210485;
  {
    const T a = orr[1], b = oi[1];
    orr[1] = c * (a - (T)DIR * b);
    oi[1] = c * (b + (T)DIR * a);
  }
  mul_i<T, DIR>(orr[2], oi[2]);
  {
    const T a = orr[3], b = oi[3];
    orr[3] = c * (-a - (T)DIR * b);
    oi[3] = c * (-b + (T)DIR * a);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[k] = er[k] + orr[k];
    i[k] = ei[k] + oi[k];
    r[k + 4] = er[k] - orr[k];
    i[k + 4] = ei[k] - oi[k];
  }
}

// One Stockham stage of radix R and span NS on the buffer (re, im); thread t of N/8.
// tw[k] = exp(-2 pi i k / N); the inverse direction uses the conjugates.
template <typename T, int N, int R, int NS, int DIR>
__device__ __forceinline__ void stockham_stage(T* re, T* im, const Cx<T>* __restrict__ tw, int t) {
  constexpr int NB = N / R;
  constexpr int PER = 8 / R;
  constexpr int TPF = N / 8;
  T xr[8], xi[8];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = t + u * TPF;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = Lds<N>::at(b + r * NB);
      xr[u * R + r] = re[s];
      xi[u * R + r] = im[s];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = t + u * TPF;
    const int j = b & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const Cx<T> w = tw[j * r * (N / (NS * R))];
        const T wi = DIR < 0 ? w.i : -w.i;
        const T a = xr[u * R + r], c = xi[u * R + r];
        xr[u * R + r] = a * w.r - c * wi;
        xi[u * R + r] = a * wi + c * w.r;
      }
    }
    if constexpr (R == 8) {
      dft8<T, DIR>(xr + u * R, xi + u * R);
    } else if constexpr (R == 4) {
      dft4<T, DIR>(xr + u * R, xi + u * R);
    } else {
      dft2<T, DIR>(xr + u * R, xi + u * R);
    }
    const int base = (b / NS) * NS * R + j;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = Lds<N>::at(base + r * NS);
      re[s] = xr[u * R + r];
      im[s] = xi[u * R + r];
    }
  }
  __syncthreads();
}

// Full unnormalised DFT (DIR = -1) or inverse DFT (DIR = +1), natural order in and out.
template <typename T, int N, int NS, int DIR>
__device__ __forceinline__ void fft_stages(T* re, T* im, const Cx<T>* __restrict__ tw, int t) {
  if constexpr (NS < N) {
    constexpr int R = (N / NS >= 8) ? 8 : (N / NS);
    stockham_stage<T, N, R, NS, DIR>(re, im, tw, t);
    fft_stages<T, N, NS * R, DIR>(re, im, tw, t);
  }
}

// ---------------------------------------------------------------------------------------
// Pair split after the forward DFT: from Z[p] = (A, B) and Z[N-p] = (C, D) produce the
// DCT-II values of the two packed sequences at p and N-p.  (c, s) = (cos, sin)(pi p / 2N).
template <typename T>
__device__ __forceinline__ void split_pair(T A, T B, T C, T D, T c, T s, T& xa, T& xb, T& xa2, T& xb2) {
  xa = (T)0.5 * (c * (A + C) + s * (B - D));
  xb = (T)0.5 * (c * (B + D) + s * (C - A));
  xa2 = (T)0.5 * (s * (C + A) + c * (D - B));
  xb2 = (T)0.5 * (s * (D + B) + c * (A - C));
}

// Pair merge before the inverse DFT: from the cosine coefficients of two sequences at p
// and N-p produce Z[p] and Z[N-p] of the packed inverse.
template <typename T>
__device__ __forceinline__ void merge_pair(T ya, T yb, T ya2, T yb2, T c, T s, T& zr, T& zi, T& z2r, T& z2i) {
  zr = c * ya + s * ya2 - (s * yb - c * yb2);
  zi = s * ya - c * ya2 + c * yb + s * yb2;
  z2r = s * ya2 + c * ya - (c * yb2 - s * yb);
  z2i = c * ya2 - s * ya + s * yb2 + c * yb;
}

}  // namespace vs
