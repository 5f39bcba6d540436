// Influence coefficients (Section 2.1, Eqs. 8-10) and their kernel spectrum
// (Eq. 13), both in FP64.
//
// K(di, dj) is the integral of (a^2 + b^2)^(-(1+k)/2) over the element
// [(di-1/2)Dx, (di+1/2)Dx] x [(dj-1/2)Dy, (dj+1/2)Dy].  Two rules:
//  * near the load (max(di, dj) <= 4) the element integral is written
//    through the corner function F(x, y) = int_0^x int_0^y, odd in each
//    argument:  K = F(p,m) - F(q,m) - F(p,n) + F(q,n) with p, q the element's
//    x-limits and m, n its y-limits.  In polar coordinates, with the
//    substitution tan(theta) = sinh(s), F(x, y) = [x^(1-k) J(asinh(y/x)) +
//    y^(1-k) J(asinh(x/y))] / (1 - k), J(S) = int_0^S cosh(s)^-k ds; J is
//    computed by composite 12-point Gauss-Legendre on panels of length <= 1/2
//    (the integrand is analytic within pi/2 of the real axis).  At k = 0 this
//    is Love's x asinh(y/x) + y asinh(x/y).
//  * elsewhere the integrand is analytic on the element: tensor
//    Gauss-Legendre, 12 x 12 up to ring 16 and 8 x 8 beyond.
// The corner form loses about 2 log10(ring) digits to cancellation, which is
// why it is only used near the load.
//
// Spectrum.  K is even in both offsets, so its DFT on the padded My x Mx grid
// is real and even:  Khat(ky,kx) = sum K(i,j) cos(2 pi i kx/Mx) cos(2 pi j ky/My).
// With Q(i,j) = K(i,j) c_i c_j for i, j >= 0 (c_0 = 1/2, else 1), the
// product of cosines splits into cos(a+b) + cos(a-b), so
// Khat(ky,kx) = 2 Re[Qhat(ky,kx) + Qhat(-ky,kx)].  Q is non-zero only in the
// first ny x nx block, which is exactly the input shape the pruned
// convolution sweeps handle, so the same row kernel and a forward-only
// column kernel compute it.
#include <math.h>

#include "conv_kernels.h"
#include "launch.h"

namespace bem {

struct GaussTables {
  double x12[12], w12[12], x8[8], w8[8];
};

// Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n.
static void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

__device__ double j_integral(double S, double k, const GaussTables& g) {
  int np = (int)ceil(S * 2.0);
  if (np < 1) np = 1;
  const double h = S / np;
  double sum = 0.0;
  for (int q = 0; q < np; ++q) {
    const double mid = (q + 0.5) * h;
    for (int i = 0; i < 12; ++i) sum += g.w12[i] * pow(cosh(mid + 0.5 * h * g.x12[i]), -k);
  }
  return 0.5 * h * sum;
}

__device__ double corner(double x, double y, double k, const GaussTables& g) {
  if (x == 0.0 || y == 0.0) return 0.0;
  const double sg = ((x < 0.0) != (y < 0.0)) ? -1.0 : 1.0;
  x = fabs(x);
  y = fabs(y);
  const double e = 1.0 - k;
  return sg * (pow(x, e) * j_integral(asinh(y / x), k, g) + pow(y, e) * j_integral(asinh(x / y), k, g)) / e;
}

template <int NG>
__device__ double tensor_gl(double ac, double bc, double dx, double dy, double k, const double* xg,
                            const double* wg) {
  const double s = -0.5 * (1.0 + k);
  double sum = 0.0;
  for (int i = 0; i < NG; ++i) {
    const double a = ac + 0.5 * dx * xg[i];
    double row = 0.0;
    for (int j = 0; j < NG; ++j) {
      const double b = bc + 0.5 * dy * xg[j];
      row += wg[j] * pow(a * a + b * b, s);
    }
    sum += wg[i] * row;
  }
  return 0.25 * dx * dy * sum;
}

__global__ void k_influence(double* __restrict__ Kq, int nx, int ny, double dx, double dy, double k,
                            GaussTables g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= ny) return;
  const int ring = i > j ? i : j;
  double v;
  if (ring <= 4) {
    const double p = (i + 0.5) * dx, q = (i - 0.5) * dx;
    const double m = (j + 0.5) * dy, n = (j - 0.5) * dy;
    v = corner(p, m, k, g) - corner(q, m, k, g) - corner(p, n, k, g) + corner(q, n, k, g);
  } else if (ring <= 16) {
    v = tensor_gl<12>(i * dx, j * dy, dx, dy, k, g.x12, g.w12);
  } else {
    v = tensor_gl<8>(i * dx, j * dy, dx, dy, k, g.x8, g.w8);
  }
  Kq[(size_t)j * nx + i] = v;
}

__global__ void k_twiddles(cplx<double>* __restrict__ t64, cplx<float>* __restrict__ t32, int M) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double s, c;
  sincospi(2.0 * (double)m / (double)M, &s, &c);   // exact rational argument
  t64[m] = {c, -s};
  t32[m] = {(float)c, (float)-s};
}

__global__ void k_wave_twiddles(cplx<double>* __restrict__ t64, cplx<float>* __restrict__ t32,
                                int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;   // m = k1 * 64 + l
  if (m >= L) return;
  const int k1 = m >> 6, l = m & 63;
  double s, c;
  sincospi(2.0 * (double)(l * k1) / (double)L, &s, &c);
  t64[m] = {c, -s};
  t32[m] = {(float)c, (float)-s};
}

// Q(i, j) = K(i, j) c_i c_j (see file header)
template <int PER>
struct QLoad {
  const double* Kq;
  int nx;
  double fa[PER], fb[PER];
  template <int NTHR>
  __device__ bool issue() { return true; }
  template <int NTHR>
  __device__ void fetch(int ya, int yb, bool hasb, int nxl) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const double cx = n == 0 ? 0.5 : 1.0;
      const size_t safe = (size_t)ya * nx;
      fa[q] = load_or0(Kq, (size_t)ya * nx + n, safe, n < nxl) * cx * (ya == 0 ? 0.5 : 1.0);
      fb[q] = load_or0(Kq, (size_t)yb * nx + n, safe, n < nxl && hasb) * cx;
    }
  }
  template <int NTHR>
  __device__ bool decide(double*, int) { return true; }
  template <int NTHR>
  __device__ void make(int, int, bool, int, double (&va)[PER], double (&vb)[PER]) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      va[q] = fa[q];
      vb[q] = fb[q];
    }
  }
  template <int NTHR>
  __device__ void commit(int, int, bool, int, const double (&)[PER], const double (&)[PER]) {}
  template <int NTHR>
  __device__ void finish(double*, int) {}
};

hipError_t launch_twiddles(cplx<double>* t64, cplx<float>* t32, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((M + 255) / 256), dim3(256), 0, s, t64, t32, M);
  return hipGetLastError();
}

hipError_t launch_wave_twiddles(cplx<double>* t64, cplx<float>* t32, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_wave_twiddles, dim3((L + 255) / 256), dim3(256), 0, s, t64, t32, L);
  return hipGetLastError();
}

hipError_t launch_influence(double* Kq, int nx, int ny, double dx, double dy, double k,
                            hipStream_t s) {
  GaussTables g;
  gauss_legendre(12, g.x12, g.w12);
  gauss_legendre(8, g.x8, g.w8);
  hipLaunchKernelGGL(k_influence, dim3((nx + 127) / 128, ny), dim3(128), 0, s, Kq, nx, ny, dx, dy,
                     k, g);
  return hipGetLastError();
}

hipError_t launch_spectrum(const Geom& g, const double* Kq, cplx<double>* S,
                           const cplx<double>* twx, const cplx<double>* twy, double* KT64,
                           float* KT32, double scale, hipStream_t s) {
  hipError_t e = dispatch_L(g.Lx, [&](auto LX) -> hipError_t {
    constexpr int L = decltype(LX)::value;
    constexpr int NT = row_threads(L);
    constexpr int PER = row_per<L, NT>();
    QLoad<PER> q{Kq, g.nx};
    hipLaunchKernelGGL((k_row_r2c<double, L, NT, QLoad<PER>>), dim3((g.ny + 1) / 2), dim3(NT), 0, s,
                       q, S, g.nx, g.ny, twx);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  const int W = col_width<double>(g.Ly, g.Lx);
  return dispatch_L(g.Ly, [&](auto LYc) -> hipError_t {
    constexpr int LY = decltype(LYc)::value;
    return dispatch_W(W, [&](auto Wc) -> hipError_t {
      constexpr int WW = decltype(Wc)::value;
      if constexpr (WW > col_width_lds<double>(LY)) {
        return hipErrorInvalidValue;
      } else {
        constexpr int NT = col_threads(WW, LY);
        hipLaunchKernelGGL((k_col_spectrum<LY, WW, NT>), dim3(g.Lx / WW), dim3(NT), 0, s, S, g.Lx,
                           g.ny, twy, KT64, KT32, g.kpitch, scale);
        return hipGetLastError();
      }
    });
  });
}

}  // namespace bem
