// Green's-function tabulation on the device, in FP64 (Sec. II-B Eq. Green, Appendix Theorem I,
// Sec. IV-F images).
//
// The point response of one slab (thickness t, conductivity k, adiabatic top, isothermal
// bottom) to a unit source on its top face has the 2-D Fourier transform tanh(s t) / (k s); by
// Theorem I its inverse is an order-0 inverse Hankel transform.  Writing
//     tanh(s t) / s = 1/s - 2 / (s (exp(2 s t) + 1))
// splits the response into the half-space part 1/(2 pi k r) and a smooth remainder
//     2 pi k f(r) = 1/r + R(r),   R(r) = -(1/t) int_0^inf J0(u r / 2t) / (exp(u) + 1) du.
// Far from the source the Hankel integral is summed over the poles of tanh instead:
//     2 pi k f(r) = (2/t) sum_{m>=0} K0((m + 1/2) pi r / t).
//
// Table entry K(a, b) = average of f over the cell at the origin seen from the centre of
// cell (a, b) (power is piecewise constant over cells).  Near cells: the 1/r part in closed
// form (corner antiderivative of 1/r) next to the origin, Gauss-Legendre further out; R by
// Gauss-Legendre of a Chebyshev interpolant in r^2 built from the Hankel integral.  Far cells:
// Gauss-Legendre of the pole sum with K0 from its integral exp(-x cosh u) (trapezoid rule).
// The side-wall images repeat with period 2n, so the table is summed over periods.
//
// lambda[p][q] = sum_{a, b in (-n, n]} K_per cos(pi q a / nx) cos(pi p b / ny) then diagonalises
// the mirrored convolution; it is stored transposed and divided by nx * ny, which is the
// normalisation the unnormalised inverse transforms of the solve expect.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace vs {

namespace {

constexpr int kCheb = 48;      // Chebyshev coefficients of R in r^2
constexpr int kJ0Pts = 64;     // trapezoid points of J0 over one period
constexpr int kHankelPanels = 22;

// Gauss-Legendre rules on [-1, 1] of orders 2, 4, 6, 12, 16, packed at offsets 0, 2, 6, 12, 24
// (nodes in gl[0..40), weights in gl[40..80)); computed on the device by Newton's method on
// the three-term Legendre recurrence.
constexpr int kGLTotal = 40;
__device__ inline int gl_offset(int q) { return q == 2 ? 0 : (q == 4 ? 2 : (q == 6 ? 6 : (q == 12 ? 12 : 24))); }

__global__ void gauss_legendre_kernel(double* __restrict__ gl) {
  const int orders[5] = {2, 4, 6, 12, 16};
  const int slot = threadIdx.x;  // one thread per node
  int q = 0, i = 0, acc = 0;
  for (int o = 0; o < 5; ++o) {
    if (slot < acc + orders[o]) {
      q = orders[o];
      i = slot - acc;
      break;
    }
    acc += orders[o];
  }
  if (q == 0) return;
  double x = cospi((i + 0.75) / (q + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int n = 2; n <= q; ++n) {
      const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (x * p1 - p0) / (x * x - 1.0);
    const double dx = p1 / dp;
    x -= dx;
    if (fabs(dx) < 1e-17) break;
  }
  {
    double p0 = 1.0, p1 = x;
    for (int n = 2; n <= q; ++n) {
      const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (x * p1 - p0) / (x * x - 1.0);
  }
  gl[slot] = x;
  gl[kGLTotal + slot] = 2.0 / ((1.0 - x * x) * dp * dp);
}

// J0(x) = (1/pi) int_0^pi cos(x sin th) d th, trapezoid rule over the period (spectral accuracy)
__device__ double bessel_j0(double x) {
  double acc = 0.0;
  for (int j = 0; j < kJ0Pts; ++j) acc += cos(x * sinpi((double)j / kJ0Pts));
  return acc / kJ0Pts;
}

// exp(x) K0(x) = int_0^inf exp(-x (cosh u - 1)) du, trapezoid rule with step 1/20
__device__ double bessel_k0_scaled(double x) {
  const double h = 0.05;
  double acc = 0.5;
  for (int j = 1; j < 4000; ++j) {
    const double e = x * (cosh(j * h) - 1.0);
    if (e > 46.0) break;
    acc += exp(-e);
  }
  return acc * h;
}

// 2 pi k f(r) from the pole sum, r > 0
__device__ double pole_sum(double r, double t) {
  double acc = 0.0;
  const double base = M_PI * r / t;
  for (int m = 0; m < 400; ++m) {
    const double x = (m + 0.5) * base;
    const double term = exp(-x) * bessel_k0_scaled(x);
    acc += term;
    if (term < 1e-19 * acc) break;
  }
  return 2.0 * acc / t;
}

// integral of 1/r over [x1, x2] x [y1, y2] via the corner antiderivative
__device__ double corner(double x, double y) {
  double v = 0.0;
  const double ax = fabs(x), ay = fabs(y);
  if (ax > 0.0) v += x * asinh(y / ax);
  if (ay > 0.0) v += y * asinh(x / ay);
  return v;
}
__device__ double cell_inv_r(double x0, double y0, double hx, double hy) {
  const double x1 = x0 - 0.5 * hx, x2 = x0 + 0.5 * hx, y1 = y0 - 0.5 * hy, y2 = y0 + 0.5 * hy;
  return corner(x2, y2) - corner(x1, y2) - corner(x2, y1) + corner(x1, y1);
}

__device__ double cheb_eval(const double* __restrict__ c, double s, double smax) {
  const double xi = 2.0 * s / smax - 1.0;
  double b1 = 0.0, b2 = 0.0;
  for (int k = kCheb - 1; k >= 1; --k) {
    const double b0 = 2.0 * xi * b1 - b2 + c[k];
    b2 = b1;
    b1 = b0;
  }
  return xi * b1 - b2 + 0.5 * c[0];
}

// cell-averaged 2 pi k f about a cell offset (a, b), un-periodised
__device__ double cell_response(long a, long b, double hx, double hy, double t, const double* rc, double smax,
                                const double* __restrict__ gl) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  const double x0 = a * hx, y0 = b * hy;
  const double rho = hypot(x0, y0);
  if (rho > 60.0 * t) return 0.0;  // below exp(-30 pi) of the peak
  const double hmax = fmax(hx, hy), hmin = fmin(hx, hy);
  if (rho < 1.5 * t + hmax) {
    double inv_r;
    if (a <= 2 && b <= 2) {
      inv_r = cell_inv_r(x0, y0, hx, hy) / (hx * hy);
    } else {
      const int off = gl_offset(12);
      inv_r = 0.0;
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
          const double x = x0 + 0.5 * hx * gl[off + i], y = y0 + 0.5 * hy * gl[off + j];
          inv_r += gl[kGLTotal + off + i] * gl[kGLTotal + off + j] / hypot(x, y);
        }
      inv_r *= 0.25;
    }
    double rem = 0.0;
    for (int i = 0; i < 16; ++i)
      for (int j = 0; j < 16; ++j) {
        const double x = x0 + 0.5 * hx * gl[24 + i], y = y0 + 0.5 * hy * gl[24 + j];
        rem += gl[kGLTotal + 24 + i] * gl[kGLTotal + 24 + j] * cheb_eval(rc, x * x + y * y, smax);
      }
    return inv_r + 0.25 * rem;
  }
  const double d = rho / hmin;
  const int q = d < 10.0 ? 12 : (d < 80.0 ? 6 : (d < 600.0 ? 4 : 2));
  const int off = gl_offset(q);
  double acc = 0.0;
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      const double x = x0 + 0.5 * hx * gl[off + i], y = y0 + 0.5 * hy * gl[off + j];
      acc += gl[kGLTotal + off + i] * gl[kGLTotal + off + j] * pole_sum(hypot(x, y), t);
    }
  return 0.25 * acc;
}

// R(r) at Chebyshev nodes in s = r^2 on [0, smax] by the Hankel integral, then coefficients.
__global__ void __launch_bounds__(64) remainder_cheb_kernel(double* __restrict__ coef, double t, double smax,
                                                                 const double* __restrict__ gl) {
  __shared__ double vals[kCheb];
  const int j = threadIdx.x;
  if (j < kCheb) {
    const double s = 0.5 * smax * (1.0 + cospi((j + 0.5) / kCheb));
    const double z = sqrt(s) / (2.0 * t);
    double acc = 0.0;
    for (int p = 0; p < kHankelPanels; ++p) {
      const double lo = 2.0 * p;
      for (int g = 0; g < 16; ++g) {
        const double u = lo + 1.0 + gl[24 + g];
        acc += gl[kGLTotal + 24 + g] * bessel_j0(u * z) / (exp(u) + 1.0);
      }
    }
    vals[j] = -acc / t;
  }
  __syncthreads();
  if (j < kCheb) {
    double c = 0.0;
    for (int i = 0; i < kCheb; ++i) c += vals[i] * cospi((double)j * (i + 0.5) / kCheb);
    coef[j] = 2.0 * c / kCheb;
  }
}

// K_per(a, b) for a in [0, nx], b in [0, ny]; out [ny + 1][nx + 1] in K/W
__global__ void __launch_bounds__(256) kper_kernel(double* __restrict__ out, int nx, int ny, double hx, double hy,
                                                   double t, double k, const double* __restrict__ rc, double smax,
                                                   int periods, const double* __restrict__ gl) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a > nx || b > ny) return;
  double acc = 0.0;
  for (int m = -periods; m <= periods; ++m)
    for (int n = -periods; n <= periods; ++n)
      acc += cell_response((long)a + 2L * nx * m, (long)b + 2L * ny * n, hx, hy, t, rc, smax, gl);
  out[(size_t)b * (nx + 1) + a] = acc / (2.0 * M_PI * k);
}

// cos(pi j / n) for j in [0, 2n)
__global__ void cos_table_kernel(double* __restrict__ c, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 2 * n) c[j] = cospi((double)j / n);
}

// A[b][q] = sum_a w_a K[b][a] cos(pi q a / nx), q in [0, nx), b in [0, ny]
__global__ void __launch_bounds__(256) dct1_x_kernel(const double* __restrict__ kper, double* __restrict__ A,
                                                     const double* __restrict__ cosx, int nx, int ny) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (q >= nx) return;
  const double* row = kper + (size_t)b * (nx + 1);
  double acc = row[0] + ((q & 1) ? -row[nx] : row[nx]);
  int idx = 0;
  for (int a = 1; a < nx; ++a) {
    idx += q;
    if (idx >= 2 * nx) idx -= 2 * nx;
    acc += 2.0 * row[a] * cosx[idx];
  }
  A[(size_t)b * nx + q] = acc;
}

// lamT[q][p] = scale * sum_b w_b A[b][q] cos(pi p b / ny); also the FP32 copy
__global__ void __launch_bounds__(256) dct1_y_kernel(const double* __restrict__ A, double* __restrict__ lam64T,
                                                     float* __restrict__ lam32T, double* __restrict__ lam_rowmajor,
                                                     const double* __restrict__ cosy, int nx, int ny, double scale) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= ny) return;
  double acc = A[q] + ((p & 1) ? -A[(size_t)ny * nx + q] : A[(size_t)ny * nx + q]);
  int idx = 0;
  for (int b = 1; b < ny; ++b) {
    idx += p;
    if (idx >= 2 * ny) idx -= 2 * ny;
    acc += 2.0 * A[(size_t)b * nx + q] * cosy[idx];
  }
  lam64T[(size_t)q * ny + p] = acc * scale;
  lam32T[(size_t)q * ny + p] = (float)(acc * scale);
  if (lam_rowmajor) lam_rowmajor[(size_t)p * nx + q] = acc;
}

// Column-pass coefficients.  For the packed column pair the split of the forward transform,
// the multiplication by lambda and the merge of the inverse combine, at spectral index p with
// (c, s) = (cos, sin)(pi p / 2n), into
//     alpha = (c^2 l[p] + s^2 l[n-p]) / 2,  beta = c s (l[p] - l[n-p]) / 2,  gamma = (s^2 l[p] + c^2 l[n-p]) / 2
// per column (alpha, gamma even and beta odd under p -> n - p, so p in [0, n/2] is stored).
// out[q][p] = (alpha, beta, gamma, 0) for column q; l = lamT[q][.] (already scaled).
// c_scaled != 0: the eigenvalues of the leakage-aware deterministic operator, l / (1 - c_scaled l)
// (c_scaled = 0 leaves l exactly as it is).
__global__ void __launch_bounds__(256) coef_kernel(const double* __restrict__ lamT, double* __restrict__ c64,
                                                   float* __restrict__ c32, int nx, int ny, double c_scaled) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  const int half = ny / 2;
  if (p > half) return;
  const double* l = lamT + (size_t)q * ny;
  auto lam = [&](int i) { return l[i] / (1.0 - c_scaled * l[i]); };
  double a, b, g;
  if (p == 0) {
    a = 0.5 * lam(0);
    b = 0.0;
    g = 0.0;
  } else {
    double sn, cs;
    sincospi(0.5 * p / ny, &sn, &cs);
    const double lp = lam(p), lq = lam(ny - p);
    a = 0.5 * (cs * cs * lp + sn * sn * lq);
    b = 0.5 * cs * sn * (lp - lq);
    g = 0.5 * (sn * sn * lp + cs * cs * lq);
  }
  const size_t o = ((size_t)q * (half + 1) + p) * 4;
  c64[o] = a;
  c64[o + 1] = b;
  c64[o + 2] = g;
  c64[o + 3] = 0.0;
  c32[o] = (float)a;
  c32[o + 1] = (float)b;
  c32[o + 2] = (float)g;
  c32[o + 3] = 0.0f;
}

// DFT twiddles exp(-2 pi i k / n) and quarter-wave pairs (cos, sin)(pi p / 2n), FP64 and FP32,
// and the FP32 low parts (FP64 value - FP32 value, rounded) for compensated twiddles
__global__ void twiddle_kernel(Cx<double>* tw64, Cx<float>* tw32, Cx<double>* qw64, Cx<float>* qw32,
                               Cx<float>* tw32lo, Cx<float>* qw32lo, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  auto lo = [](double v) { return (float)(v - (double)(float)v); };
  double s, c;
  sincospi(2.0 * k / n, &s, &c);
  tw64[k] = {c, -s};
  tw32[k] = {(float)c, (float)-s};
  tw32lo[k] = {lo(c), lo(-s)};
  sincospi(0.5 * k / n, &s, &c);
  qw64[k] = {c, s};
  qw32[k] = {(float)c, (float)s};
  qw32lo[k] = {lo(c), lo(s)};
}

// Package stack below the first layer (Table param; Sec. II-B's f_sp = f_silic + const): the
// first layer's cosine eigenvalues get the stack's extra impedance.  With Z the impedance
// T / q seen from the bottom face of layer 1 looking down (Z = 0 isothermal, 1/h convective,
// then up through each lower layer: Z <- (Z + tanh(s t) / (k s)) / (1 + k s tanh(s t) Z)), the
// stack's surface symbol minus layer 1's alone is, without cancellation,
//     dF(s) = Z sech^2(s t1) / (1 + k1 s tanh(s t1) Z),
// and the mirrored, cell-averaged operator's eigenvalue gains
//     dlambda[p][q] = (1 / (hx hy)) sum_{i, j} dF(|kappa|) S(kappa),
//     kappa = (pi (q + 2 nx j) / lx, pi (p + 2 ny i) / ly),  S = sinc(kx hx / 2) sinc(ky hy / 2)
// (the images' Poisson sum; |i|, |j| <= aliases, beyond which exp(-2 |kappa| t1) < 1e-21).
__global__ void __launch_bounds__(256) stack_lambda_kernel(double* __restrict__ lam64T, float* __restrict__ lam32T,
                                                           double* __restrict__ lam_rowmajor, StackSpec st, int nx,
                                                           int ny, double lx, double ly, double scale) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= ny) return;
  const double hx = lx / nx, hy = ly / ny;
  double acc = 0.0;
  for (int j = -st.aliases; j <= st.aliases; ++j) {
    const double kx = M_PI * (q + 2.0 * nx * j) / lx;
    const double ux = 0.5 * kx * hx;
    const double sx = ux == 0.0 ? 1.0 : sin(ux) / ux;
    for (int i = -st.aliases; i <= st.aliases; ++i) {
      const double ky = M_PI * (p + 2.0 * ny * i) / ly;
      const double uy = 0.5 * ky * hy;
      const double sy = uy == 0.0 ? 1.0 : sin(uy) / uy;
      const double s = hypot(kx, ky);
      double z = st.bottom_h > 0.0 ? 1.0 / st.bottom_h : 0.0;
      double dF;
      if (s == 0.0) {
        for (int l = st.n - 1; l >= 1; --l) z += st.t[l] / st.k[l];
        dF = z;
      } else {
        for (int l = st.n - 1; l >= 1; --l) {
          const double th = tanh(s * st.t[l]);
          z = (z + th / (st.k[l] * s)) / (1.0 + st.k[l] * s * th * z);
        }
        const double th1 = tanh(s * st.t[0]), ch = cosh(s * st.t[0]);
        dF = s * st.t[0] > 350.0 ? 0.0 : z / (ch * ch) / (1.0 + st.k[0] * s * th1 * z);
      }
      acc += dF * sx * sy;
    }
  }
  const double d = acc / (hx * hy);
  const size_t o = (size_t)q * ny + p;
  lam64T[o] += d * scale;
  lam32T[o] = (float)lam64T[o];
  if (lam_rowmajor) lam_rowmajor[(size_t)p * nx + q] += d;
}

}  // namespace

// number of 2L periods per side beyond which the kernel is below 1e-30 of its peak
static int periods_needed(double lx, double ly, double t) {
  const double lmin = lx < ly ? lx : ly;
  int m = 1;
  while (std::exp(-M_PI * (2 * m + 1) * lmin / (2.0 * t)) > 1e-30 && m < 64) ++m;
  return m;
}

hipError_t launch_green_table(const TableSpec& sp, double* kper, double* lam64T, float* lam32T, double* coef64,
                              float* coef32, double* lam_rowmajor, double* scratch, hipStream_t stream) {
  // scratch: Gauss-Legendre rules, kCheb + 2 nx + 2 ny + (ny + 1) nx doubles
  double* gl = scratch;
  double* coef = gl + 2 * kGLTotal;
  double* cosx = coef + kCheb;
  double* cosy = cosx + 2 * sp.nx;
  double* A = cosy + 2 * sp.ny;
  const double hx = sp.lx / sp.nx, hy = sp.ly / sp.ny;
  const double hmax = hx > hy ? hx : hy;
  const double rmax = 1.5 * sp.t + hmax + 0.5 * std::hypot(hx, hy);
  const double smax = 1.0001 * rmax * rmax;
  hipLaunchKernelGGL(gauss_legendre_kernel, dim3(1), dim3(64), 0, stream, gl);
  hipLaunchKernelGGL(remainder_cheb_kernel, dim3(1), dim3(64), 0, stream, coef, sp.t, smax, gl);
  const int periods = periods_needed(sp.lx, sp.ly, sp.t);
  hipLaunchKernelGGL(kper_kernel, dim3((sp.nx + 1 + 255) / 256, sp.ny + 1), dim3(256), 0, stream, kper, sp.nx, sp.ny,
                     hx, hy, sp.t, sp.k_ref, coef, smax, periods, gl);
  hipLaunchKernelGGL(cos_table_kernel, dim3((2 * sp.nx + 255) / 256), dim3(256), 0, stream, cosx, sp.nx);
  hipLaunchKernelGGL(cos_table_kernel, dim3((2 * sp.ny + 255) / 256), dim3(256), 0, stream, cosy, sp.ny);
  hipLaunchKernelGGL(dct1_x_kernel, dim3((sp.nx + 255) / 256, sp.ny + 1), dim3(256), 0, stream, kper, A, cosx, sp.nx,
                     sp.ny);
  hipLaunchKernelGGL(dct1_y_kernel, dim3((sp.ny + 255) / 256, sp.nx), dim3(256), 0, stream, A, lam64T, lam32T,
                     lam_rowmajor, cosy, sp.nx, sp.ny, 1.0 / ((double)sp.nx * sp.ny));
  if (sp.stack.n > 1 || sp.stack.bottom_h > 0.0)
    hipLaunchKernelGGL(stack_lambda_kernel, dim3((sp.ny + 255) / 256, sp.nx), dim3(256), 0, stream, lam64T, lam32T,
                       lam_rowmajor, sp.stack, sp.nx, sp.ny, sp.lx, sp.ly, 1.0 / ((double)sp.nx * sp.ny));
  hipLaunchKernelGGL(coef_kernel, dim3((sp.ny / 2 + 1 + 255) / 256, sp.nx), dim3(256), 0, stream, lam64T, coef64, coef32,
                     sp.nx, sp.ny, 0.0);
  return hipGetLastError();
}

hipError_t launch_det_coef(const TableSpec& sp, const double* lam64T, double c, double* coef64, float* coef32,
                           hipStream_t stream) {
  // lam64T holds lambda / (nx ny)
  const double c_scaled = c * (double)sp.nx * (double)sp.ny;
  hipLaunchKernelGGL(coef_kernel, dim3((sp.ny / 2 + 1 + 255) / 256, sp.nx), dim3(256), 0, stream, lam64T, coef64, coef32,
                     sp.nx, sp.ny, c_scaled);
  return hipGetLastError();
}

size_t green_table_scratch_doubles(int nx, int ny) {
  return (size_t)2 * kGLTotal + kCheb + 2 * nx + 2 * ny + (size_t)(ny + 1) * nx;
}

hipError_t launch_twiddles(int n, Cx<double>* tw64, Cx<float>* tw32, Cx<double>* qw64, Cx<float>* qw32,
                           Cx<float>* tw32lo, Cx<float>* qw32lo, hipStream_t stream) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, tw64, tw32, qw64, qw32, tw32lo,
                     qw32lo, n);
  return hipGetLastError();
}

}  // namespace vs
