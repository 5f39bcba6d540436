// Host-side launchers shared between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "common.h"

namespace bem {

// Problem geometry.  Mx = 2 Lx, My = 2 Ly (powers of two); the row spectrum
// has ny rows of Lx complex values (row pairs interleaved, spec_idx); the
// kernel spectrum has Lx + 1 rows of kpitch reals (ky in [0, Ly]).
struct Geom {
  int nx, ny, Lx, Ly, kpitch;
};

template <typename T>
struct SpecView {
  const T* KT;             // (Lx + 1) x kpitch, pre-scaled by C / (Mx My)
  const cplx<T>* twx;      // Mx-point twiddles
  const cplx<T>* twy;      // My-point twiddles
  const cplx<T>* twly;     // wave-FFT inter-step table [k1][lane] for length Ly (or null)
  const cplx<T>* twlx;     // the same table for length Lx (row sweeps)
};

// Workgroup sizes and column-group widths, shared by launchers and the
// footprint model.
constexpr int kMinL = 32;
constexpr int kMaxL = 4096;

__host__ __device__ constexpr int row_threads(int L) {
  return L >= 4096 ? 512 : (L >= 1024 ? 256 : (L / 4 < 64 ? 64 : L / 4));
}

template <typename T>
__host__ __device__ constexpr int col_width_lds(int LY) {
  // largest power of two W <= 16 with 2 W padded columns within ~150 KB LDS
  int w = 16;
  while (w > 1 && 2 * w * LdsLayout<T>::col_stride(LY) * (int)sizeof(cplx<T>) > 150 * 1024) w >>= 1;
  return w;
}

// Tuning knob: BEM_COL_WIDTH (1 = default, 2, 4, 8, 16) caps the column-group
// width of the LDS Stockham column kernels.
int col_width_cap();

// Tuning knob BEM_ROW_WAVE: 1 (default) = wave-FFT row sweeps for FP32 at
// Lx = 2048, 0 = LDS Stockham row sweeps everywhere.
int row_wave_enabled();
inline bool row_wave(const Geom& g) { return g.Lx == 2048 && row_wave_enabled(); }

template <typename T>
inline int col_width(int LY, int lx) {
  int w = col_width_lds<T>(LY);
  int wmax = 1;
  while (wmax * 2 <= 16 && lx / (wmax * 2) >= 256) wmax *= 2;
  if (w > wmax) w = wmax;
  const int cap = col_width_cap();
  return w < cap ? w : cap;
}

__host__ __device__ constexpr int col_threads(int W, int LY) {
  int t = (2 * W * LY) / 16;
  return t < 64 ? 64 : (t > 512 ? 512 : t);
}

// Call f(std::integral_constant<int, L>) for a runtime power of two L.
template <class F>
inline hipError_t dispatch_L(int L, F&& f) {
  switch (L) {
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    case 2048: return f(std::integral_constant<int, 2048>{});
    case 4096: return f(std::integral_constant<int, 4096>{});
    default: return hipErrorInvalidValue;
  }
}

template <class F>
inline hipError_t dispatch_W(int W, F&& f) {
  switch (W) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_twiddles(cplx<double>* t64, cplx<float>* t32, int M, hipStream_t s);
// wave-FFT table for length L = 64 P: t[k1 * 64 + l] = exp(-2 pi i l k1 / L)
hipError_t launch_wave_twiddles(cplx<double>* t64, cplx<float>* t32, int L, hipStream_t s);
hipError_t launch_influence(double* Kq, int nx, int ny, double dx, double dy, double k,
                            hipStream_t s);
hipError_t launch_spectrum(const Geom& g, const double* Kq, cplx<double>* S,
                           const cplx<double>* twx, const cplx<double>* twy, double* KT64,
                           float* KT32, double scale, hipStream_t s);

template <typename T>
hipError_t launch_col(const Geom& g, const SpecView<T>& K, cplx<T>* S, const int* done,
                      hipStream_t s);

// Forward column transform and spectral energy sum_k KT |T|^2 (one FP64
// partial per workgroup into part); col_energy_blocks gives how many.
template <typename T>
int col_energy_blocks(const Geom& g);
template <typename T>
hipError_t launch_col_energy(const Geom& g, const SpecView<T>& K, const cplx<T>* S,
                             const int* done, double* part, hipStream_t s);

// One sweep of the convolution on its own: 0 row R2C, 1 column, 2 row C2R,
// 3 column transform + spectral energy.
template <typename T>
hipError_t launch_sweep(const Geom& g, const SpecView<T>& K, int which, const T* p, T* u,
                        cplx<T>* S, hipStream_t s);

template <typename T>
hipError_t launch_conv(const Geom& g, const SpecView<T>& K, const T* p, T* u, cplx<T>* S,
                       hipStream_t s);

}  // namespace bem
