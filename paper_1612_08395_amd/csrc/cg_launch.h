// Launchers of the conjugate-gradient kernels, instantiated per precision in
// cg_f32.hip and cg_f64.hip.
#pragma once
#include "cg_kernels.h"
#include "launch.h"
#include "row_wave.h"

namespace bem {

inline int ew_blocks(size_t n) {
  size_t b = (n + EW_THREADS - 1) / EW_THREADS;
  if (b < 1) b = 1;
  return (int)(b > EW_MAX_BLOCKS ? EW_MAX_BLOCKS : b);
}

// ev (optional): six events recorded after the six launches, in order.
inline hipError_t mark(const hipEvent_t* ev, int k, hipStream_t s) {
  return ev ? hipEventRecord(ev[k], s) : hipSuccess;
}

template <typename T, int MODE>
hipError_t launch_cg_iteration(const Geom& g, const SpecView<T>& K, const CgBufs<T>& b, int it,
                               const hipEvent_t* ev, hipStream_t s, const double* shift) {
  const int nrp = (g.ny + 1) / 2;
  const int nbc = col_energy_blocks<T>(g);
  hipError_t e;
  if (shift) {
    // iteration 0 after a solve of the same p at another d: the gap by a
    // shift instead of the first convolution (the three events follow it)
    hipLaunchKernelGGL((k_gap_shift<T, 256>), dim3(nrp), dim3(256), 0, s, b.g, b.hd, b.p, b.mask,
                       *shift, b.part, g.nx, g.ny);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int k = 0; k < 3; ++k)
      if ((e = mark(ev, k, s)) != hipSuccess) return e;
  } else {
    // R2C sweeps: Stockham (their prologues carry most of the work, and the
    // wave kernels' lower occupancy costs more than their cheaper transform
    // saves); C2R sweeps: wave kernels at Lx = 2048, except under load
    // control, whose epilogues do not fit the wave kernel's registers
    e = launch_row_r2c<T, false>(
        g, K, b.S,
        [&](auto PERc) {
          return UpdatePro<T, MODE, decltype(PERc)::value>{b.p,    b.t,    b.g, b.mask, b.sc,
                                                            b.part, g.nx, nrp, it,     nbc};
        },
        s);
    if (e != hipSuccess || (e = mark(ev, 0, s)) != hipSuccess) return e;
    if ((e = launch_col<T>(g, K, b.S, &b.sc->done, s)) != hipSuccess) return e;
    if ((e = mark(ev, 1, s)) != hipSuccess) return e;
    e = launch_row_c2r<T, MODE != CG_FORCE>(
        g, K, b.S,
        [&](auto PERc) {
          return GapEpi<T, MODE, decltype(PERc)::value>{b.g,    b.hd, b.p, b.mask, b.sc,
                                                         b.part, g.nx, nrp, it};
        },
        s);
    if (e != hipSuccess || (e = mark(ev, 2, s)) != hipSuccess) return e;
  }
  e = launch_row_r2c<T, false>(
      g, K, b.S,
      [&](auto PERc) {
        return DirPro<T, MODE, decltype(PERc)::value>{b.t,    b.g,  b.p, b.mask, b.sc,
                                                       b.part, g.nx, nrp, it};
      },
      s);
  if (e != hipSuccess || (e = mark(ev, 3, s)) != hipSuccess) return e;
  if constexpr (MODE != CG_FORCE) {
    // second convolution: only sum t (C K * t) is needed (Parseval); no
    // inverse transforms and no sixth launch (its event follows at once)
    if ((e = launch_col_energy<T>(g, K, b.S, &b.sc->done, b.part + kPartRT, s)) != hipSuccess)
      return e;
    if ((e = mark(ev, 4, s)) != hipSuccess) return e;
    return mark(ev, 5, s);
  } else {
    if ((e = launch_col<T>(g, K, b.S, &b.sc->done, s)) != hipSuccess) return e;
    if ((e = mark(ev, 4, s)) != hipSuccess) return e;
    e = launch_row_c2r<T, false>(
        g, K, b.S,
        [&](auto PERc) {
          return DotsEpi<T, MODE, decltype(PERc)::value>{b.g, b.t, b.mask, b.sc, b.part, g.nx,
                                                          it};
        },
        s);
    if (e != hipSuccess) return e;
    return mark(ev, 5, s);
  }
}

// Queue iterations it0 .. it0 + n - 1.  ev (optional): 6 n + 1 events, the
// first recorded before the first launch, then six per iteration.  shift
// (displacement control only, it0 = 0): iteration 0 takes its gap from the
// state's g shifted by *shift (k_gap_shift).
template <typename T>
hipError_t launch_cg_iterations(const Geom& g, const SpecView<T>& K, const CgBufs<T>& b, int mode,
                                int it0, int n, const hipEvent_t* ev, hipStream_t s,
                                const double* shift) {
  if (shift && (mode != CG_DISP || it0 != 0)) return hipErrorInvalidValue;
  hipError_t e = mark(ev, 0, s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    const hipEvent_t* evi = ev ? ev + 1 + 6 * i : nullptr;
    const double* sh = i == 0 ? shift : nullptr;
    switch (mode) {
      case CG_DISP: e = launch_cg_iteration<T, CG_DISP>(g, K, b, it0 + i, evi, s, sh); break;
      case CG_FIXED: e = launch_cg_iteration<T, CG_FIXED>(g, K, b, it0 + i, evi, s, nullptr); break;
      case CG_FORCE: e = launch_cg_iteration<T, CG_FORCE>(g, K, b, it0 + i, evi, s, nullptr); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_make_hd(const double* h, double d, T* hd, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_make_hd<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, h, d, hd, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cold_start(T* p, const T* hd, double inv_ck00, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cold_start<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, p, hd, inv_ck00,
                     n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prepare(T* t, T* p, uint8_t* mask, bool fixed_set, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, t, p, mask,
                     fixed_set ? 1 : 0, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const CgBufs<T>& b, int mode, size_t n, hipStream_t s) {
  if (mode == CG_FIXED)
    hipLaunchKernelGGL((k_finalize<T, CG_FIXED>), dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, b.p,
                       b.g, b.mask, b.sc, b.part, n);
  else if (mode == CG_FORCE)
    hipLaunchKernelGGL((k_finalize<T, CG_FORCE>), dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, b.p,
                       b.g, b.mask, b.sc, b.part, n);
  else
    hipLaunchKernelGGL((k_finalize<T, CG_DISP>), dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, b.p,
                       b.g, b.mask, b.sc, b.part, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_min_h(const double* h, size_t n, CgScal* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_min_h<T>, dim3(1), dim3(EW_THREADS), 0, s, h, n, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, double v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, p, (T)v, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_detach(const CgBufs<T>& b, double pcrit, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_detach<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, b.p, b.mask, pcrit,
                     b.sc, b.part, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_to_f64(const T* src, double* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_from_f64(const double* src, T* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_from_f64<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_u_from_gap(const T* g, const double* h, double d, double* u, size_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_u_from_gap<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, s, g, h, d, u, n);
  return hipGetLastError();
}

#define BEM_INSTANTIATE_CG(T)                                                                    \
  template hipError_t launch_cg_iterations<T>(const Geom&, const SpecView<T>&, const CgBufs<T>&, \
                                              int, int, int, const hipEvent_t*, hipStream_t,     \
                                              const double*);                                    \
  template hipError_t launch_fill<T>(T*, double, size_t, hipStream_t);                           \
  template hipError_t launch_min_h<T>(const double*, size_t, CgScal*, hipStream_t);              \
  template hipError_t launch_make_hd<T>(const double*, double, T*, size_t, hipStream_t);         \
  template hipError_t launch_cold_start<T>(T*, const T*, double, size_t, hipStream_t);           \
  template hipError_t launch_prepare<T>(T*, T*, uint8_t*, bool, size_t, hipStream_t);            \
  template hipError_t launch_finalize<T>(const CgBufs<T>&, int, size_t, hipStream_t);           \
  template hipError_t launch_detach<T>(const CgBufs<T>&, double, size_t, hipStream_t);          \
  template hipError_t launch_to_f64<T>(const T*, double*, size_t, hipStream_t);                  \
  template hipError_t launch_from_f64<T>(const double*, T*, size_t, hipStream_t);                \
  template hipError_t launch_u_from_gap<T>(const T*, const double*, double, double*, size_t,     \
                                           hipStream_t);

}  // namespace bem
