// C ABI layer: argument checking, handles, device memory, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bem.h"
#include "internal.h"

namespace bem {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_error(BEM_ENOMEM, "%s: out of device memory", what);
  return set_error(BEM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- material scalars (Section 2.1, Eqs. 2-4) -------------------------------
double beta_kn(double k, double nu) { return std::sqrt((1.0 + k) * (1.0 - k * nu / (1.0 - nu))); }

double alpha_kn(double k, double nu) {
  const double pi = 3.14159265358979323846;
  const double b = beta_kn(k, nu);
  const double num = std::pow(2.0, k) * b * std::sin(b * pi / 2.0) *
                     std::tgamma((3.0 + k + b) / 2.0) * std::tgamma((3.0 + k - b) / 2.0);
  const double den = std::sqrt(pi) * (1.0 + k) * std::cos(k * pi / 2.0) * std::tgamma(2.0 + k) *
                     std::tgamma(1.0 + k / 2.0) * std::tgamma((1.0 - k) / 2.0);
  return num / den;
}

static int next_pow2_at_least(int v) {
  int m = 1;
  while (m < v) m <<= 1;
  return m;
}

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace bem

using namespace bem;

extern "C" {

const char* bem_last_error(void) { return g_last_error.c_str(); }

int bem_influence_ex(int nx, int ny, double dx, double dy, double k, double nu, double E0,
                     double c0, bem_influence_t* out) {
  clear_error();
  if (!out) return set_error(BEM_EINVAL, "bem_influence: out is NULL");
  if (nx < 1 || ny < 1) return set_error(BEM_EINVAL, "bem_influence: nx, ny must be >= 1");
  if (nx > BEM_MAX_N || ny > BEM_MAX_N)
    return set_error(BEM_EUNSUPPORTED, "bem_influence: grid side above %d", BEM_MAX_N);
  if (!(is_finite(dx) && dx > 0 && is_finite(dy) && dy > 0))
    return set_error(BEM_EINVAL, "bem_influence: element sizes must be positive and finite");
  if (!(is_finite(k) && k > -1.0 && k < 1.0))
    return set_error(BEM_EINVAL, "bem_influence: k must satisfy -1 < k < 1 (Eq. 1)");
  if (!(is_finite(nu) && nu >= 0.0 && nu < 0.5))
    return set_error(BEM_EINVAL, "bem_influence: nu must be in [0, 0.5)");
  if (!(is_finite(E0) && E0 > 0 && is_finite(c0) && c0 > 0))
    return set_error(BEM_EINVAL, "bem_influence: E0 and c0 must be positive and finite");

  auto* h = new bem_influence_s();
  h->nx = nx;
  h->ny = ny;
  h->dx = dx;
  h->dy = dy;
  h->k = k;
  h->nu = nu;
  h->E0 = E0;
  h->c0 = c0;
  h->alpha = alpha_kn(k, nu);
  h->C = h->alpha * (1.0 - nu * nu) * std::pow(c0, k) / E0;
  const int Mx = next_pow2_at_least(std::max(2 * nx, 2 * kMinL));
  const int My = next_pow2_at_least(std::max(2 * ny, 2 * kMinL));
  h->g.nx = nx;
  h->g.ny = ny;
  h->g.Lx = Mx / 2;
  h->g.Ly = My / 2;
  h->g.kpitch = ((My / 2 + 1) + 63) / 64 * 64;
  (void)hipGetDevice(&h->device);

  int rc = influence_build(h);
  if (rc != BEM_OK) {
    influence_release(h);
    delete h;
    return rc;
  }
  *out = h;
  return BEM_OK;
}

int bem_influence(int nx, int ny, double dx, double k, double nu, bem_influence_t* out) {
  return bem_influence_ex(nx, ny, dx, dx, k, nu, 1.0, 1.0, out);
}

int bem_influence_free(bem_influence_t K) {
  clear_error();
  if (!K) return BEM_OK;
  influence_release(K);
  delete K;
  return BEM_OK;
}

int bem_influence_info(bem_influence_t K, bem_influence_info_t* info) {
  clear_error();
  if (!K || !info) return set_error(BEM_EINVAL, "bem_influence_info: NULL argument");
  info->nx = K->nx;
  info->ny = K->ny;
  info->Mx = 2 * K->g.Lx;
  info->My = 2 * K->g.Ly;
  info->dx = K->dx;
  info->dy = K->dy;
  info->k = K->k;
  info->nu = K->nu;
  info->E0 = K->E0;
  info->c0 = K->c0;
  info->alpha = K->alpha;
  info->C = K->C;
  info->K00 = K->K00;
  info->device_bytes = K->device_bytes;
  return BEM_OK;
}

int bem_influence_coeffs(bem_influence_t K, double* K_out) {
  clear_error();
  if (!K || !K_out) return set_error(BEM_EINVAL, "bem_influence_coeffs: NULL argument");
  const int nx = K->nx, ny = K->ny;
  std::vector<double> q((size_t)nx * ny);
  hipError_t e = hipMemcpy(q.data(), K->Kq, q.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "bem_influence_coeffs");
  const int W = 2 * nx - 1;
  for (int dj = -(ny - 1); dj <= ny - 1; ++dj)
    for (int di = -(nx - 1); di <= nx - 1; ++di)
      K_out[(size_t)(dj + ny - 1) * W + (di + nx - 1)] = q[(size_t)std::abs(dj) * nx + std::abs(di)];
  return BEM_OK;
}

int bem_convolve_dev(bem_influence_t K, int precision, const void* p, void* u, void* stream) {
  clear_error();
  if (!K || !p || !u) return set_error(BEM_EINVAL, "bem_convolve_dev: NULL argument");
  if (precision != BEM_FP64 && precision != BEM_MIXED)
    return set_error(BEM_EINVAL, "bem_convolve_dev: unknown precision %d", precision);
  return convolve_device(K, precision, p, u, (hipStream_t)stream);
}

int bem_convolve(bem_influence_t K, const double* p, double* u, void* stream) {
  clear_error();
  if (!K || !p || !u) return set_error(BEM_EINVAL, "bem_convolve: NULL argument");
  const size_t n = (size_t)K->nx * K->ny;
  for (size_t i = 0; i < n; ++i)
    if (!is_finite(p[i])) return set_error(BEM_EINVAL, "bem_convolve: non-finite pressure");
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_io(K);
  if (rc != BEM_OK) return rc;
  hipError_t e = hipMemcpyAsync(K->io64, p, n * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "bem_convolve upload");
  rc = convolve_device(K, BEM_FP64, K->io64, K->io64, s);
  if (rc != BEM_OK) return rc;
  e = hipMemcpyAsync(u, K->io64, n * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "bem_convolve download");
  return BEM_OK;
}

int bem_kernel_time(bem_influence_t K, int precision, int which, int reps, void* stream,
                    double* avg_ms) {
  clear_error();
  if (!K || !avg_ms) return set_error(BEM_EINVAL, "bem_kernel_time: NULL argument");
  if (precision != BEM_FP64 && precision != BEM_MIXED)
    return set_error(BEM_EINVAL, "bem_kernel_time: unknown precision %d", precision);
  if (which < 0 || which > 3 || reps < 1)
    return set_error(BEM_EINVAL, "bem_kernel_time: which in {0,1,2,3}, reps >= 1");
  return sweep_time(K, precision, which, reps, (hipStream_t)stream, avg_ms);
}

}  // extern "C"
