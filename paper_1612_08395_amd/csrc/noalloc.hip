// Allocation-free convolution entry point: bem_convolve_dev with its row
// spectrum in a fixed device array of this library instead of the handle's
// lazily allocated buffer, for callers that must not allocate device memory.
//
// The array lives in the code object: every GPU the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol); the device
// address comes from hipGetSymbolAddress, taken once per device on the first
// call made with that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bem.h"
#include "internal.h"

static_assert(BEM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");

// Row spectrum of the allocation-free convolution (spec_rows(ny) x Lx complex
// values); one copy per device, for the life of the process.
static __device__ __align__(256) unsigned char scratch[BEM_NOALLOC_SCRATCH_BYTES];

namespace bem {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "bem_convolve_dev_noalloc: scratch address");
    if (!ptr) return set_error(BEM_EDEVICE, "bem_convolve_dev_noalloc: scratch address is NULL");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return BEM_OK;
}

}  // namespace
}  // namespace bem

using namespace bem;

extern "C" int bem_convolve_dev_noalloc(bem_influence_t K, int precision, const void* p, void* u,
                                        void* stream) {
  clear_error();
  if (!K || !p || !u) return set_error(BEM_EINVAL, "bem_convolve_dev_noalloc: NULL argument");
  if (precision != BEM_FP64 && precision != BEM_MIXED)
    return set_error(BEM_EINVAL, "bem_convolve_dev_noalloc: unknown precision %d", precision);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "bem_convolve_dev_noalloc: current device");
  if (dev != K->device)
    return set_error(BEM_EINVAL,
                     "bem_convolve_dev_noalloc: the handle belongs to device %d, device %d is "
                     "current",
                     K->device, dev);
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(BEM_EUNSUPPORTED, "bem_convolve_dev_noalloc: device index %d", dev);
  const size_t cs = precision == BEM_FP64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  const size_t need = (size_t)spec_rows(K->ny) * K->g.Lx * cs;
  if (need > (size_t)BEM_NOALLOC_SCRATCH_BYTES)
    return set_error(BEM_EUNSUPPORTED,
                     "bem_convolve_dev_noalloc: the %d x %d grid needs %zu scratch bytes in this "
                     "precision, above the fixed %d (use bem_convolve_dev)",
                     K->nx, K->ny, need, BEM_NOALLOC_SCRATCH_BYTES);
  void* S = nullptr;
  int rc = scratch_address(dev, &S);
  if (rc) return rc;
  const hipStream_t s = (hipStream_t)stream;
  // the row sweep writes every entry of the spectrum before the column sweep
  // reads it, so the array needs no clearing between calls
  e = precision == BEM_FP64
          ? launch_conv<double>(K->g, spec_view<double>(K), (const double*)p, (double*)u,
                                (cplx<double>*)S, s)
          : launch_conv<float>(K->g, spec_view<float>(K), (const float*)p, (float*)u,
                               (cplx<float>*)S, s);
  if (e != hipSuccess) return hip_fail(e, "bem_convolve_dev_noalloc: launch");
  return BEM_OK;
}
