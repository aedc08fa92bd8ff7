// Device building blocks for the real 2-D cosine transforms of the convolution.
//
// A length-N complex DFT belongs to one group of TPF = N / E lanes of a single wavefront
// (E = 8 elements per lane, 16 for N = 1024), so only wavefront-level ordering is needed.
// Lane t of the group holds element t + TPF m in register slot m.  The transform is a
// Stockham autosort sequence: the first stage is a radix-E DFT of the lane's own slots (in
// registers), the middle stages are radix 8 (a final radix 4 or 2 when needed) through an LDS
// buffer, and the last stage leaves element t + TPF m in slot m again -- the layout the next
// transform starts from.  LDS keeps real and imaginary parts in separate arrays.  The LDS has
// 32 four-byte banks and serves each half-wavefront separately; element i of a transform sits
// at word i + p (i >> a) + q (i >> b), with (a, p, b, q) and the per-transform pitch chosen per
// N so that every load and store pattern of the stages (and of neighbouring transforms sharing
// a wavefront) hits distinct banks for N <= 64 and costs 1.25x the conflict-free time above.
//
// Two real sequences share one complex DFT (one as the real part, one as the imaginary
// part).  The cosine transforms use the N-point reordering of a sequence (even samples
// ascending, odd samples descending); with V = DFT(v),
//     DCT-II:  X[p] = Re( e^{-i pi p / 2N} V[p] )
//     inverse: V[p] = e^{+i pi p / 2N} (X[p] - i X[N-p]),  v = unnormalised inverse DFT of V.
// Splitting the two packed spectra needs Z[N-p] next to Z[p]; that partner sits in lane
// (TPF - t) mod TPF of the group and is fetched with a lane permute.
#pragma once

#include "common.hpp"

namespace vs {

template <int N>
struct Shape {
  static constexpr int E = N >= 1024 ? 16 : 8;  // elements per lane
  static constexpr int TPF = N / E;             // lanes per transform (<= 64)
  // LDS padding i + PP (i >> PA) + PQ (i >> PB) and buffer pitch
  static constexpr int PA = N <= 64 ? 3 : (N == 128 ? 4 : 5);
  static constexpr int PP = (N == 256 || N == 512) ? 2 : 1;
  static constexpr int PB = N == 16 ? 4 : N == 32 ? 5 : N == 64 ? 6 : N == 128 ? 5 : N == 1024 ? 10 : 7;
  static constexpr int PQ = N == 128 ? 2 : 1;
  static constexpr int LAST = (N - 1) + PP * ((N - 1) >> PA) + PQ * ((N - 1) >> PB);
  static constexpr int STRIDE = LAST + 1 + (N <= 64 ? 1 : (N == 128 ? 3 : 0));
};

template <int N>
__device__ __forceinline__ int lds_at(int i) {
  return i + Shape<N>::PP * (i >> Shape<N>::PA) + Shape<N>::PQ * (i >> Shape<N>::PB);
}

// sample position of slot k of the reordered sequence (and of its spectrum slot)
template <int N>
__device__ __forceinline__ int unperm(int k) {
  return k < N / 2 ? 2 * k : 2 * N - 1 - 2 * k;
}
template <int N>
__device__ __forceinline__ int perm(int i) {
  return (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
}

// Ordering point for LDS traffic inside one wavefront: no instruction is moved across it and
// the wavefront's LDS operations before it are visible to its lanes after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of `v` held by lane `src` of the wavefront
__device__ __forceinline__ float lane_get(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// out[m] = element N - (t + TPF m) of the group's sequence held in own[] (lane-reversed).
// PERIODIC: index N means 0 (a DFT); otherwise element N is taken as 0 (a cosine spectrum).
// EL: elements per lane (default: the transform's own shape; a smaller EL spreads the sequence
// over TPF = N / EL <= 64 lanes)
template <typename T, int N, bool PERIODIC, int EL = Shape<N>::E>
__device__ __forceinline__ void partner(const T* own, T* out, int t) {
  constexpr int E = EL, TPF = N / EL;
  const int lane = __lane_id();
  const int src = (lane & ~(TPF - 1)) + ((TPF - t) & (TPF - 1));
  const bool head = t == 0;
  // Lane t > 0 reads slot E-1-r of lane TPF-t; lane 0 reads itself and keeps its own slot
  // (E-r) mod E instead.  The choice is made after the exchange so that it stays a select
  // between two values: a select between two slots of own[] is folded by the compiler into a
  // lane-varying register index, which it expands into a compare/select chain per element.
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const T got = lane_get(own[E - 1 - r], src);
    out[r] = head ? own[(E - r) & (E - 1)] : got;
  }
  if (!PERIODIC && head) out[0] = (T)0;
}

// a b + c d with one fixed rounding order (the product c d rounded, then fused with a b), so
// that every kernel computing the same expression gets the same bits whatever the compiler's
// contraction choices around it
template <typename T>
__device__ __forceinline__ T dot2(T a, T b, T c, T d) {
  return fma(a, b, c * d);
}

// Compensated twiddles (CT): a constant w held as w_hi + w_lo, w_hi = w rounded to T and
// w_lo = (w - w_hi) rounded, so a product x w is x w_hi plus the correction x w_lo, which
// removes the rounding of the constant itself from the result (an option of the FP32
// transforms; FP64 never uses it).
template <typename T>
struct Split {
  T hi, lo;
};
template <typename T>
__host__ __device__ constexpr Split<T> split_const(double w) {
  return {(T)w, (T)(w - (double)(T)w)};
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

// strided radix-4 on elements base, base+s, base+2s, base+3s
template <typename T, int DIR>
__device__ __forceinline__ void dft4s(T* r, T* i, int b, int s) {
  T xr[4] = {r[b], r[b + s], r[b + 2 * s], r[b + 3 * s]}, xi[4] = {i[b], i[b + s], i[b + 2 * s], i[b + 3 * s]};
  dft4<T, DIR>(xr, xi);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[b + k * s] = xr[k];
    i[b + k * s] = xi[k];
  }
}

template <typename T, int DIR, bool CT = false>
__device__ __forceinline__ void dft8(T* r, T* i) {
  T er[4] = {r[0], r[2], r[4], r[6]}, ei[4] = {i[0], i[2], i[4], i[6]};
  T orr[4] = {r[1], r[3], r[5], r[7]}, oi[4] = {i[1], i[3], i[5], i[7]};
  dft4<T, DIR>(er, ei);
  dft4<T, DIR>(orr, oi);
  mul_i<T, DIR>(orr[2], oi[2]);
#pragma unroll
  for (int k = 0; k < 4; k += 2) {
    r[k] = er[k] + orr[k];
    i[k] = ei[k] + oi[k];
    r[k + 4] = er[k] - orr[k];
    i[k + 4] = ei[k] - oi[k];
  }
  // odd terms 1 and 3 carry W8^k = c (+-1 +- i): the factor c is applied in fused
  // multiply-adds with the even terms (fixed rounding, independent of the compiler's choices)
  const T c = (T)0.70710678118654752440084436210485;
  const T x1 = orr[1] - (T)DIR * oi[1], y1 = oi[1] + (T)DIR * orr[1];
  const T x3 = -orr[3] - (T)DIR * oi[3], y3 = -oi[3] + (T)DIR * orr[3];
  if constexpr (CT) {
    constexpr T cl = split_const<T>(0.70710678118654752440084436210485).lo;
    r[1] = fma(cl, x1, fma(c, x1, er[1]));
    i[1] = fma(cl, y1, fma(c, y1, ei[1]));
    r[5] = fma(-cl, x1, fma(-c, x1, er[1]));
    i[5] = fma(-cl, y1, fma(-c, y1, ei[1]));
    r[3] = fma(cl, x3, fma(c, x3, er[3]));
    i[3] = fma(cl, y3, fma(c, y3, ei[3]));
    r[7] = fma(-cl, x3, fma(-c, x3, er[3]));
    i[7] = fma(-cl, y3, fma(-c, y3, ei[3]));
    return;
  }
  r[1] = fma(c, x1, er[1]);
  i[1] = fma(c, y1, ei[1]);
  r[5] = fma(-c, x1, er[1]);
  i[5] = fma(-c, y1, ei[1]);
  r[3] = fma(c, x3, er[3]);
  i[3] = fma(c, y3, ei[3]);
  r[7] = fma(-c, x3, er[3]);
  i[7] = fma(-c, y3, ei[3]);
}

// radix 16 as 4 x 4: inner DFT-4 over n1 of x[4 n1 + n2], twiddle W16^(n2 k1), outer DFT-4 over n2
template <typename T, int DIR, bool CT = false>
__device__ __forceinline__ void dft16(T* r, T* i) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4s<T, DIR>(r, i, n2, 4);  // a[n2 + 4 k1]
  constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173, H = 0.70710678118654752440;
  const T c1 = (T)C1, s1 = (T)S1, h = (T)H;
  const T cs[10] = {(T)1, c1, h, s1, (T)0, -s1, -h, -c1, (T)-1, -c1};  // cos(2 pi j / 16), j = 0..9
  const T sn[10] = {(T)0, s1, h, c1, (T)1, c1, h, s1, (T)0, -s1};      // sin(2 pi j / 16)
  // low parts of the same constants (compensated twiddles)
  constexpr T c1l = split_const<T>(C1).lo, s1l = split_const<T>(S1).lo, hl = split_const<T>(H).lo;
  const T csl[10] = {(T)0, c1l, hl, s1l, (T)0, -s1l, -hl, -c1l, (T)0, -c1l};
  const T snl[10] = {(T)0, s1l, hl, c1l, (T)0, c1l, hl, s1l, (T)0, -s1l};
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int j = n2 * k1;
      const T wr = cs[j], wi = (T)DIR * sn[j];
      const int e = n2 + 4 * k1;
      const T a = r[e], b = i[e];
      r[e] = dot2(a, wr, -b, wi);
      i[e] = dot2(a, wi, b, wr);
      if constexpr (CT) {
        const T wrl = csl[j], wil = (T)DIR * snl[j];
        r[e] = fma(a, wrl, fma(-b, wil, r[e]));
        i[e] = fma(a, wil, fma(b, wrl, i[e]));
      }
    }
  T yr[16], yi[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T xr[4] = {r[4 * k1], r[4 * k1 + 1], r[4 * k1 + 2], r[4 * k1 + 3]};
    T xi[4] = {i[4 * k1], i[4 * k1 + 1], i[4 * k1 + 2], i[4 * k1 + 3]};
    dft4<T, DIR>(xr, xi);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      yr[k1 + 4 * k2] = xr[k2];
      yi[k1 + 4 * k2] = xi[k2];
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    r[k] = yr[k];
    i[k] = yi[k];
  }
}

template <typename T, int R, int DIR, bool CT = false>
__device__ __forceinline__ void dft_r(T* r, T* i) {
  if constexpr (R == 16) dft16<T, DIR, CT>(r, i);
  else if constexpr (R == 8) dft8<T, DIR, CT>(r, i);
  else if constexpr (R == 4) dft4<T, DIR>(r, i);
  else dft2<T, DIR>(r, i);
}

// Stockham stages of span NS onwards: LDS in, LDS out (middle) or registers out (last).
// tw[TS k] = exp(-2 pi i k / N): TS = 1 with the table of N, TS = 2 with the table of 2N.
// CT: twl holds the low parts of the same twiddles (compensated twiddles).  LS: element stride
// of the LDS buffer (1: re / im contiguous; > 1: a column of a row-major tile of pitch LS).
template <typename T, int N, int NS, int DIR, int TS = 1, bool CT = false, int LS = 1, int EL = Shape<N>::E>
__device__ __forceinline__ void stages_from(T* xr, T* xi, T* re, T* im, const Cx<T>* __restrict__ tw, int t,
                                            const Cx<T>* __restrict__ twl = nullptr) {
  constexpr int E = EL, TPF = N / EL;
  constexpr int R0 = (N / NS >= 8) ? 8 : (N / NS);
  constexpr int R = R0 < E ? R0 : E;  // the radix never exceeds the elements a lane holds
  constexpr int NB = N / R, PER = E / R;
  constexpr bool LAST = NS * R == N;
  T yr[E], yi[E];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = t + TPF * u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = lds_at<N>(b + r * NB);
      yr[u * R + r] = re[s * LS];
      yi[u * R + r] = im[s * LS];
    }
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = t + TPF * u;
    const int j = b & (NS - 1);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const Cx<T> w = tw[TS * j * r * (N / (NS * R))];
      const T wi = DIR < 0 ? w.i : -w.i;
      const T a = yr[u * R + r], c = yi[u * R + r];
      yr[u * R + r] = dot2(a, w.r, -c, wi);
      yi[u * R + r] = dot2(a, wi, c, w.r);
      if constexpr (CT) {
        const Cx<T> wl = twl[TS * j * r * (N / (NS * R))];
        const T wli = DIR < 0 ? wl.i : -wl.i;
        yr[u * R + r] = fma(a, wl.r, fma(-c, wli, yr[u * R + r]));
        yi[u * R + r] = fma(a, wli, fma(c, wl.r, yi[u * R + r]));
      }
    }
    dft_r<T, R, DIR, CT>(yr + u * R, yi + u * R);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        xr[u + r * PER] = yr[u * R + r];
        xi[u + r * PER] = yi[u * R + r];
      }
    } else {
      const int base = (b / NS) * NS * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int s = lds_at<N>(base + r * NS);
        re[s * LS] = yr[u * R + r];
        im[s * LS] = yi[u * R + r];
      }
    }
  }
  if constexpr (!LAST) {
    wave_sync();
    stages_from<T, N, NS * R, DIR, TS, CT, LS, EL>(xr, xi, re, im, tw, t, twl);
  }
}

// Unnormalised DFT (DIR = -1) or inverse DFT (DIR = +1) of the group's sequence, slot m of lane
// t holding element t + TPF m on entry and on exit.  (re, im): this group's LDS buffer; the
// caller must have finished its own reads of that buffer (wave_sync) before the call.
template <typename T, int N, int DIR, int TS = 1, bool CT = false, int LS = 1, int EL = Shape<N>::E>
__device__ __forceinline__ void fft_reg(T* xr, T* xi, T* re, T* im, const Cx<T>* __restrict__ tw, int t,
                                        const Cx<T>* __restrict__ twl = nullptr) {
  constexpr int E = EL;
  dft_r<T, E, DIR, CT>(xr, xi);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int s = lds_at<N>(t * E + r);
    re[s * LS] = xr[r];
    im[s * LS] = xi[r];
  }
  wave_sync();
  stages_from<T, N, E, DIR, TS, CT, LS, EL>(xr, xi, re, im, tw, t, twl);
}

// ---------------------------------------------------------------------------------------
// Split after the forward DFT: Z[p] = (A, B), Z[N-p] = (C, D) give the DCT-II values of the
// two packed sequences at p (and at N - p).  (c, s) = (cos, sin)(pi p / 2N).
template <typename T>
__device__ __forceinline__ void split_pair(T A, T B, T C, T D, T c, T s, T& xa, T& xb, T& xa2, T& xb2) {
  xa = (T)0.5 * dot2(c, A + C, s, B - D);
  xb = (T)0.5 * dot2(c, B + D, s, C - A);
  xa2 = (T)0.5 * dot2(s, C + A, c, D - B);
  xb2 = (T)0.5 * dot2(s, D + B, c, A - C);
}
// the same with compensated (c, s) = (c + cl, s + sl)
template <typename T>
__device__ __forceinline__ void split_pair_ct(T A, T B, T C, T D, T c, T s, T cl, T sl, T& xa, T& xb, T& xa2,
                                              T& xb2) {
  xa = (T)0.5 * fma(cl, A + C, fma(sl, B - D, dot2(c, A + C, s, B - D)));
  xb = (T)0.5 * fma(cl, B + D, fma(sl, C - A, dot2(c, B + D, s, C - A)));
  xa2 = (T)0.5 * fma(sl, C + A, fma(cl, D - B, dot2(s, C + A, c, D - B)));
  xb2 = (T)0.5 * fma(sl, D + B, fma(cl, A - C, dot2(s, D + B, c, A - C)));
}

// Merge before the inverse DFT: cosine coefficients of the two sequences at p and N - p give
// Z[p] of the packed inverse.
template <typename T>
__device__ __forceinline__ void merge_pair(T ya, T yb, T ya2, T yb2, T c, T s, T& zr, T& zi) {
  zr = dot2(c, ya, s, ya2) - dot2(s, yb, -c, yb2);
  zi = dot2(s, ya, -c, ya2) + dot2(c, yb, s, yb2);
}
// the same with compensated (c, s) = (c + cl, s + sl)
template <typename T>
__device__ __forceinline__ void merge_pair_ct(T ya, T yb, T ya2, T yb2, T c, T s, T cl, T sl, T& zr, T& zi) {
  merge_pair<T>(ya, yb, ya2, yb2, c, s, zr, zi);
  zr = fma(cl, ya, fma(sl, ya2, fma(-sl, yb, fma(cl, yb2, zr))));
  zi = fma(sl, ya, fma(-cl, ya2, fma(cl, yb, fma(sl, yb2, zi))));
}

}  // namespace vs
