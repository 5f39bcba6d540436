// Influence handle: device memory and the build pipeline (coefficients,
// twiddles, kernel spectrum), plus the convolution entry point.
#include <hip/hip_runtime.h>

#include "../../include/bem.h"
#include "internal.h"

namespace bem {

int dev_alloc(bem_influence_s* h, void** p, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, what);
  }
  h->device_bytes += (long long)bytes;
  return BEM_OK;
}

template <>
SpecView<double> spec_view<double>(const bem_influence_s* h) {
  return {h->KT64, h->twx64, h->twy64, h->twly64, h->twlx64};
}
template <>
SpecView<float> spec_view<float>(const bem_influence_s* h) {
  return {h->KT32, h->twx32, h->twy32, h->twly32, h->twlx32};
}

int influence_build(bem_influence_s* h) {
  const Geom& g = h->g;
  const int Mx = 2 * g.Lx, My = 2 * g.Ly;
  const size_t nq = (size_t)h->nx * h->ny;
  const size_t nk = (size_t)(g.Lx + 1) * g.kpitch;
  int rc;
  if ((rc = dev_alloc(h, (void**)&h->Kq, nq * sizeof(double), "influence coefficients"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->KT64, nk * sizeof(double), "kernel spectrum"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->KT32, nk * sizeof(float), "kernel spectrum"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twx64, Mx * sizeof(cplx<double>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twy64, My * sizeof(cplx<double>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twx32, Mx * sizeof(cplx<float>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twy32, My * sizeof(cplx<float>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twly64, g.Ly * sizeof(cplx<double>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twly32, g.Ly * sizeof(cplx<float>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twlx64, g.Lx * sizeof(cplx<double>), "twiddles"))) return rc;
  if ((rc = dev_alloc(h, (void**)&h->twlx32, g.Lx * sizeof(cplx<float>), "twiddles"))) return rc;

  hipStream_t s = nullptr;
  hipError_t e;
  if ((e = hipMemsetAsync(h->KT64, 0, nk * sizeof(double), s)) != hipSuccess)
    return hip_fail(e, "spectrum clear");
  if ((e = hipMemsetAsync(h->KT32, 0, nk * sizeof(float), s)) != hipSuccess)
    return hip_fail(e, "spectrum clear");
  if ((e = launch_twiddles(h->twx64, h->twx32, Mx, s)) != hipSuccess) return hip_fail(e, "twiddles");
  if ((e = launch_twiddles(h->twy64, h->twy32, My, s)) != hipSuccess) return hip_fail(e, "twiddles");
  if ((e = launch_wave_twiddles(h->twly64, h->twly32, g.Ly, s)) != hipSuccess)
    return hip_fail(e, "twiddles");
  if ((e = launch_wave_twiddles(h->twlx64, h->twlx32, g.Lx, s)) != hipSuccess)
    return hip_fail(e, "twiddles");
  if ((e = launch_influence(h->Kq, h->nx, h->ny, h->dx, h->dy, h->k, s)) != hipSuccess)
    return hip_fail(e, "influence coefficients");

  // the spectrum is built in the handle's FP64 convolution scratch, which
  // the handle keeps (a free here would wait for the whole device)
  if ((rc = dev_alloc(h, (void**)&h->S64, (size_t)spec_rows(h->ny) * g.Lx * sizeof(cplx<double>),
                      "spectrum scratch")))
    return rc;
  const double scale = h->C / ((double)Mx * (double)My);
  e = launch_spectrum(g, h->Kq, h->S64, h->twx64, h->twy64, h->KT64, h->KT32, scale, s);
  hipError_t e2 = hipMemcpyAsync(&h->K00, h->Kq, sizeof(double), hipMemcpyDeviceToHost, s);
  hipError_t e3 = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "kernel spectrum");
  if (e2 != hipSuccess) return hip_fail(e2, "kernel spectrum");
  if (e3 != hipSuccess) return hip_fail(e3, "influence build");
  return BEM_OK;
}

void influence_release(bem_influence_s* h) {
  void* ptrs[] = {h->Kq, h->KT64, h->KT32, h->twx64, h->twy64, h->twx32, h->twy32,
                  h->twly64, h->twly32, h->twlx64, h->twlx32, h->S64, h->S32, h->io64, h->io32, h->epart};
  for (void* p : ptrs)
    if (p) hipFree(p);
  h->device_bytes = 0;
}

int ensure_io(bem_influence_s* h) {
  if (h->io64) return BEM_OK;
  return dev_alloc(h, (void**)&h->io64, (size_t)h->nx * h->ny * sizeof(double), "convolution buffer");
}

int convolve_device(bem_influence_s* h, int precision, const void* p, void* u, hipStream_t s) {
  const size_t ns = (size_t)spec_rows(h->ny) * h->g.Lx;
  hipError_t e;
  if (precision == BEM_FP64) {
    if (!h->S64) {
      int rc = dev_alloc(h, (void**)&h->S64, ns * sizeof(cplx<double>), "convolution scratch");
      if (rc) return rc;
    }
    e = launch_conv<double>(h->g, spec_view<double>(h), (const double*)p, (double*)u, h->S64, s);
  } else {
    if (!h->S32) {
      int rc = dev_alloc(h, (void**)&h->S32, ns * sizeof(cplx<float>), "convolution scratch");
      if (rc) return rc;
    }
    e = launch_conv<float>(h->g, spec_view<float>(h), (const float*)p, (float*)u, h->S32, s);
  }
  if (e != hipSuccess) return hip_fail(e, "convolution launch");
  return BEM_OK;
}

int sweep_time(bem_influence_s* h, int precision, int which, int reps, hipStream_t s, double* ms) {
  const size_t n = (size_t)h->nx * h->ny;
  const size_t ns = (size_t)spec_rows(h->ny) * h->g.Lx;
  int rc;
  hipError_t e;
  if (precision == BEM_FP64) {
    if ((rc = ensure_io(h))) return rc;
    if (!h->S64 && (rc = dev_alloc(h, (void**)&h->S64, ns * sizeof(cplx<double>), "scratch")))
      return rc;
  } else {
    if (!h->io32 && (rc = dev_alloc(h, (void**)&h->io32, n * sizeof(float), "scratch"))) return rc;
    if (!h->S32 && (rc = dev_alloc(h, (void**)&h->S32, ns * sizeof(cplx<float>), "scratch")))
      return rc;
  }
  // defined inputs: zero field and spectrum
  if (precision == BEM_FP64) {
    e = hipMemsetAsync(h->io64, 0, n * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(h->S64, 0, ns * sizeof(cplx<double>), s);
  } else {
    e = hipMemsetAsync(h->io32, 0, n * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(h->S32, 0, ns * sizeof(cplx<float>), s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel timing setup");
  if (which == 3 && !h->epart &&
      (rc = dev_alloc(h, (void**)&h->epart, 4096 * sizeof(double), "scratch")))
    return rc;
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "event");
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    hipEventDestroy(a);
    return hip_fail(e, "event");
  }
  // one untimed launch, then `reps` timed back-to-back launches
  for (int r = -1; r < reps && e == hipSuccess; ++r) {
    if (r == 0) e = hipEventRecord(a, s);
    if (e != hipSuccess) break;
    if (which == 3)
      e = precision == BEM_FP64
              ? launch_col_energy<double>(h->g, spec_view<double>(h), h->S64, nullptr, h->epart, s)
              : launch_col_energy<float>(h->g, spec_view<float>(h), h->S32, nullptr, h->epart, s);
    else
      e = precision == BEM_FP64
              ? launch_sweep<double>(h->g, spec_view<double>(h), which, h->io64, h->io64, h->S64, s)
              : launch_sweep<float>(h->g, spec_view<float>(h), which, h->io32, h->io32, h->S32, s);
  }
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "kernel timing");
  *ms = (double)t / reps;
  return BEM_OK;
}

}  // namespace bem
