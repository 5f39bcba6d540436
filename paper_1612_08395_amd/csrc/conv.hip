// Plain convolution u = C K * p (Eq. 13 with zero padding), FP32 and FP64.
#include "col_wave.h"
#include "conv_kernels.h"
#include "launch.h"
#include "row_wave.h"

#include <stdlib.h>

#include <type_traits>

namespace bem {

// One column per workgroup by default: more, smaller workgroups share each
// CU and do not load, transform and store in step.  Measured against the
// widest group the LDS allowed (FP64 at 2048^2: 2 columns; FP32 and FP64 at
// 1024^2: 4): column sweep FP64 2048^2 99.3 -> 83.7 us, 1024^2 27.0 -> 20.9
// us, FP32 1024^2 17.7 -> 16.6 us; spectral energy FP64 2048^2 65.5 -> 58.9
// us; the FP64 2048^2 sweep 60.5 -> 65.9 solves/s.
int col_width_cap() {
  static const int cap = [] {
    const char* v = getenv("BEM_COL_WIDTH");
    const int c = v ? atoi(v) : 1;
    return (c == 1 || c == 2 || c == 4 || c == 8 || c == 16) ? c : 1;
  }();
  return cap;
}

// Tuning knob BEM_COL_WAVE: 0 = LDS Stockham column kernel, 1 (default) =
// wave-FFT kernel.
int col_wave_enabled() {
  static const int on = [] {
    const char* v = getenv("BEM_COL_WAVE");
    return v ? atoi(v) : 1;
  }();
  return on;
}

int row_wave_enabled() {
  static const int on = [] {
    const char* v = getenv("BEM_ROW_WAVE");
    return v ? atoi(v) : 1;
  }();
  return on;
}

// Tuning knob: BEM_COL_NC = 2 (default) or 4 columns per workgroup of the
// wave column kernel at Ly = 2048.  Two columns (4 waves, 68 KB of LDS) let
// two workgroups share a CU, which are not in step; with the row spectrum's
// interleaved row pairs each still moves 32-byte pieces.  Measured at 2048^2:
// 36.4 against 37.9 us per launch.  The spectral-energy kernel keeps four
// columns (no gain measured with two: 22.2 against 21.8 us).
int col_wave_nc() {
  static const int nc = [] {
    const char* v = getenv("BEM_COL_NC");
    return (v && atoi(v) == 4) ? 4 : 2;
  }();
  return nc;
}

template <typename T>
hipError_t launch_col(const Geom& g, const SpecView<T>& K, cplx<T>* S, const int* done,
                      hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    // wave-FFT column kernel (Ly = 2048): NC columns per workgroup
    if (col_wave_enabled() && g.Ly == 2048) {
      if (col_wave_nc() == 2 && g.Lx % 2 == 0) {
        hipLaunchKernelGGL((k_col_conv_w<2048, 2>), dim3(g.Lx / 2), dim3(256), 0, s, S, g.Lx, g.ny,
                           K.KT, g.kpitch, K.twy, K.twly, done);
        return hipGetLastError();
      }
      if (g.Lx % 4 == 0) {
        hipLaunchKernelGGL((k_col_conv_w<2048, 4>), dim3(g.Lx / 4), dim3(512), 0, s, S, g.Lx, g.ny,
                           K.KT, g.kpitch, K.twy, K.twly, done);
        return hipGetLastError();
      }
    }
    // Ly = 4096: quarter sequences on the same 2048-point wave FFTs
    if (col_wave_enabled() && g.Ly == 4096 && g.Lx % 2 == 0) {
      hipLaunchKernelGGL((k_col_conv_q<2>), dim3(g.Lx / 2), dim3(512), 0, s, S, g.Lx, g.ny, K.KT,
                         g.kpitch, K.twy, K.twly, done);
      return hipGetLastError();
    }
  }
  const int W = col_width<T>(g.Ly, g.Lx);
  return dispatch_L(g.Ly, [&](auto LYc) -> hipError_t {
    constexpr int LY = decltype(LYc)::value;
    return dispatch_W(W, [&](auto Wc) -> hipError_t {
      constexpr int WW = decltype(Wc)::value;
      if constexpr (WW > col_width_lds<T>(LY)) {
        return hipErrorInvalidValue;
      } else {
        constexpr int NT = col_threads(WW, LY);
        hipLaunchKernelGGL((k_col_conv<T, LY, WW, NT>), dim3(g.Lx / WW), dim3(NT), 0, s, S, g.Lx,
                           g.ny, K.KT, g.kpitch, K.twy, done);
        return hipGetLastError();
      }
    });
  });
}

template <typename T>
hipError_t launch_conv(const Geom& g, const SpecView<T>& K, const T* p, T* u, cplx<T>* S,
                       hipStream_t s) {
  hipError_t e = launch_row_r2c<T, true>(
      g, K, S, [&](auto PERc) { return PlainLoad<T, decltype(PERc)::value>{p, g.nx}; }, s);
  if (e != hipSuccess) return e;
  e = launch_col<T>(g, K, S, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_row_c2r<T, true>(
      g, K, S, [&](auto PERc) { return PlainStore<T, decltype(PERc)::value>{u, g.nx}; }, s);
}

template <typename T>
hipError_t launch_sweep(const Geom& g, const SpecView<T>& K, int which, const T* p, T* u,
                        cplx<T>* S, hipStream_t s) {
  if (which == 1) return launch_col<T>(g, K, S, nullptr, s);
  if (which == 0)
    return launch_row_r2c<T, true>(
        g, K, S, [&](auto PERc) { return PlainLoad<T, decltype(PERc)::value>{p, g.nx}; }, s);
  return launch_row_c2r<T, true>(
      g, K, S, [&](auto PERc) { return PlainStore<T, decltype(PERc)::value>{u, g.nx}; }, s);
}

// The wave kernels for FP32 at Ly = 2048 (4 columns per workgroup) and
// Ly = 4096 (2 columns), else the LDS Stockham kernel with the column width
// launch_col uses.
template <typename T>
static int energy_wave_width(const Geom& g) {
  if (!std::is_same<T, float>::value || !col_wave_enabled()) return 0;
  if (g.Ly == 2048 && g.Lx % 4 == 0) return 4;
  if (g.Ly == 4096 && g.Lx % 2 == 0) return 2;
  return 0;
}

template <typename T>
int col_energy_blocks(const Geom& g) {
  const int w = energy_wave_width<T>(g);
  return g.Lx / (w ? w : col_width<T>(g.Ly, g.Lx));
}

template <typename T>
hipError_t launch_col_energy(const Geom& g, const SpecView<T>& K, const cplx<T>* S,
                             const int* done, double* part, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    const int w = energy_wave_width<T>(g);
    if (g.Ly == 2048 && w == 4) {
      hipLaunchKernelGGL((k_col_energy_w<2048, 4>), dim3(g.Lx / 4), dim3(512), 0, s, S, g.Lx, g.ny,
                         K.KT, g.kpitch, K.twy, K.twly, done, part);
      return hipGetLastError();
    }
    if (g.Ly == 4096 && w == 2) {
      hipLaunchKernelGGL((k_col_energy_q<2>), dim3(g.Lx / 2), dim3(512), 0, s, S, g.Lx, g.ny, K.KT,
                         g.kpitch, K.twy, K.twly, done, part);
      return hipGetLastError();
    }
  }
  const int W = col_width<T>(g.Ly, g.Lx);
  return dispatch_L(g.Ly, [&](auto LYc) -> hipError_t {
    constexpr int LY = decltype(LYc)::value;
    return dispatch_W(W, [&](auto Wc) -> hipError_t {
      constexpr int WW = decltype(Wc)::value;
      if constexpr (WW > col_width_lds<T>(LY)) {
        return hipErrorInvalidValue;
      } else {
        constexpr int NT = col_threads(WW, LY);
        hipLaunchKernelGGL((k_col_energy<T, LY, WW, NT>), dim3(g.Lx / WW), dim3(NT), 0, s, S,
                           g.Lx, g.ny, K.KT, g.kpitch, K.twy, done, part);
        return hipGetLastError();
      }
    });
  });
}

template int col_energy_blocks<float>(const Geom&);
template int col_energy_blocks<double>(const Geom&);
template hipError_t launch_col_energy<float>(const Geom&, const SpecView<float>&,
                                             const cplx<float>*, const int*, double*, hipStream_t);
template hipError_t launch_col_energy<double>(const Geom&, const SpecView<double>&,
                                              const cplx<double>*, const int*, double*,
                                              hipStream_t);
template hipError_t launch_sweep<float>(const Geom&, const SpecView<float>&, int, const float*,
                                        float*, cplx<float>*, hipStream_t);
template hipError_t launch_sweep<double>(const Geom&, const SpecView<double>&, int, const double*,
                                         double*, cplx<double>*, hipStream_t);
template hipError_t launch_col<float>(const Geom&, const SpecView<float>&, cplx<float>*, const int*,
                                      hipStream_t);
template hipError_t launch_col<double>(const Geom&, const SpecView<double>&, cplx<double>*,
                                       const int*, hipStream_t);
template hipError_t launch_conv<float>(const Geom&, const SpecView<float>&, const float*, float*,
                                       cplx<float>*, hipStream_t);
template hipError_t launch_conv<double>(const Geom&, const SpecView<double>&, const double*,
                                        double*, cplx<double>*, hipStream_t);

}  // namespace bem
