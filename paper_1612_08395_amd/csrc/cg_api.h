// Host-side view of the conjugate-gradient solver's device data: the scalar
// block, the partial-sum layout, the buffer set of one solve, the slot of a
// batched launch, and the launchers (defined in cg_launch.h and batch.h,
// instantiated per precision in cg_f32/cg_f64.hip and batch_f32/batch_f64.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "launch.h"

namespace bem {

struct CgScal {
  double tol;
  int max_iter, stall_limit;
  // K4, workgroup 0, slot it & 1
  double G_hist[2], best_hist[2];
  int stall_hist[2];
  // decision record (written once, when done is set)
  int done, status, iter, pad_;
  double G, rhs2, sum_p;
  // final sums of the elementwise kernels
  double fin_sum_p, fin_contact, fin_pen, fin_detach;
  unsigned int ticket[8];
  // load control: prescribed sum of p (F / (dx dy)); K4 history (slot
  // it & 1) of the mean gap over Ic, the load scale and |Ic|; values at the
  // stopping iteration
  double W;
  double gbar_hist[2], scale_hist[2], nc_hist[2];
  double gbar, scale;
};

enum { CG_DISP = 0, CG_FIXED = 1, CG_FORCE = 2 };

enum { CG_ST_OK = 0, CG_ST_NOCONV = 1, CG_ST_FLOOR = 2, CG_ST_NUMERIC = -5 };

// partial-sum slots inside the `part` allocation
constexpr int kMaxRowBlocks = 2048;
constexpr int kPartUpd = 0;                      // 3 values: sum|dp|, sum|p|, n_ol
constexpr int kPartGap = 3 * kMaxRowBlocks;      // 2 values: sum_Ic g^2, sum_Ic (h-d)^2
                                                 // load control, 4: sum_Ic e, sum_Ic e^2,
                                                 // |Ic|, sum_Ic u^2 (e = g - previous gbar)
constexpr int kPartDots = 7 * kMaxRowBlocks;     // 1 value: sum g t (K4); load control,
                                                 // 4 (K6): sum g t, sum r t, sum t, sum_Ic r
constexpr int kMaxColBlocks = 4096;
constexpr int kPartRT = 11 * kMaxRowBlocks;      // 1 value per column workgroup: sum t r
constexpr int kPartElem = kPartRT + kMaxColBlocks;   // elementwise kernels (3 values x 1024)
constexpr int kPartTotal = kPartElem + 3 * 1024;

template <typename T>
struct CgBufs {
  T* p;
  T* t;
  T* g;
  T* hd;
  uint8_t* mask;
  cplx<T>* S;
  double* part;
  CgScal* sc;
};

enum { BATCH_EMPTY = -1 };

// One solve of a batched launch (batch.h).
template <typename T>
struct BatchSlot {
  T* p;
  T* t;
  T* g;
  const T* hd;
  uint8_t* mask;
  cplx<T>* S;
  double* part;
  CgScal* sc;
  const T* KT;        // the slot's kernel spectrum (pre-scaled by C / (Mx My))
  int nx, ny;
  int it0;            // CG iteration index of the launch's first iteration
  int mode;           // CG_DISP, CG_FIXED or BATCH_EMPTY
};

// Whether a geometry runs on the batched kernels: the LDS Stockham sweeps
// (rows and columns up to 1024 points; the wave kernels of longer FP32
// sweeps are not batched).
inline bool batch_geometry(const Geom& g) {
  return g.Lx <= 1024 && g.Ly <= 1024 && g.Lx >= kMinL && g.Ly >= kMinL;
}

template <typename T>
hipError_t launch_cg_iterations(const Geom& g, const SpecView<T>& K, const CgBufs<T>& b, int mode,
                                int it0, int n, const hipEvent_t* ev, hipStream_t s,
                                const double* shift);
template <typename T>
hipError_t launch_make_hd(const double* h, double d, T* hd, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_cold_start(T* p, const T* hd, double inv_ck00, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_prepare(T* t, T* p, uint8_t* mask, bool fixed_set, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_finalize(const CgBufs<T>& b, int mode, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_min_h(const double* h, size_t n, CgScal* sc, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* p, double v, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_detach(const CgBufs<T>& b, double pcrit, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_to_f64(const T* src, double* dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_from_f64(const double* src, T* dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_u_from_gap(const T* g, const double* h, double d, double* u, size_t n,
                             hipStream_t s);

// Queue n CG iterations for the nslots slots of `slots` (device array).
// modes: bit (1 << CG_DISP) / (1 << CG_FIXED) set when a slot of that mode is
// present (a row kernel is launched once per mode present; the column
// kernels serve every mode).  K: the geometry's twiddles (any slot's handle).
template <typename T>
hipError_t launch_batch_iterations(const Geom& g, const SpecView<T>& K,
                                   const BatchSlot<T>* slots, int nslots, unsigned modes, int n,
                                   hipStream_t s);

}  // namespace bem
