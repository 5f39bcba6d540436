// Constrained conjugate-gradient contact solve on the device.
//
// The paper solves the inverse problem (pressure from the surface
// displacement prescribed in contact) with the constrained conjugate-gradient
// method it cites (Section 2.1); this is its displacement-controlled form.
// With g = u + h - d, Ic the set of elements carrying pressure:
//
//   u = C K * p ; g = u + h - d ; G = sum_Ic g^2          (convolution 1)
//   t = g + delta (G / G_old) t on Ic, 0 elsewhere
//   r = C K * t ; tau = sum g t / sum r t                  (convolution 2)
//   p <- p - tau t on Ic ; p <- max(p, 0) ;
//   Iol = {p = 0 and g < 0}: p <- -tau g there, delta = 0 (else delta = 1)
//
// Non-adhesive mode: Ic = {p > 0}, projection and overlap step as above.
// Fixed-set mode (adhesive contact, Section 3.1): Ic = the contact set A,
// no projection, no overlap step, delta = 1 after the first iteration.
//
// One iteration is six kernel launches; the vector work is fused into the
// row sweeps of the two convolutions:
//   K1 row R2C   prologue UpdatePro : update p from the previous tau, t, g
//   K2 column    (fused spectrum multiply)
//   K3 row C2R   epilogue GapEpi    : g = u + (h - d), G, convergence test
//   K4 row R2C   prologue DirPro    : new direction t
//   K5 column
//   K6 row C2R   epilogue DotsEpi   : sum g t, sum r t, tau (r is not stored)
// Since t = 0 off Ic, the sums of K6 need no mask.
//
// Reductions are FP64: per-thread sums, a fixed-order block reduction, one
// partial per workgroup, and the last workgroup to finish (ticket counter)
// adds the partials in index order -- bitwise reproducible, no floating
// point atomics.  Scalars live in CgScal in device memory; every kernel
// returns at once when `done` is set, so the host may queue several
// iterations and check the flag rarely.
#pragma once
#include "common.h"
#include "conv_kernels.h"

namespace bem {

struct CgScal {
  double G, G_old, rhs2, ratio, tau, delta;
  double sum_dp, sum_p, gt, rt, best_G, tol;
  double n_ol;
  double fin_sum_p, fin_contact, fin_pen, fin_detach;
  int first, done, status, iter, stall, max_iter, stall_limit, pad_;
  unsigned int ticket[8];
};

enum { CG_ST_OK = 0, CG_ST_NOCONV = 1, CG_ST_FLOOR = 2, CG_ST_NUMERIC = -5 };

// Reduce NV per-thread values over the grid; returns true in the last
// workgroup, where tot[] holds the grid totals (valid in every thread).
template <int NV, int NTHR>
__device__ __forceinline__ bool grid_reduce_last(const double (&acc)[NV], double* red,
                                                 double* part, unsigned int* ticket,
                                                 double (&tot)[NV]) {
  __shared__ int am_last;
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = block_sum<NTHR>(acc[v], red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      __hip_atomic_store(&part[blockIdx.x * NV + v], s[v], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned int t = atomicAdd(ticket, 1u);
    am_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double a = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += NTHR)
      a += __hip_atomic_load(&part[i * NV + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tot[v] = block_sum<NTHR>(a, red);
  }
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
}

template <typename T, bool FS>
struct UpdatePro {
  T* p;
  const T* t;
  const T* g;
  const uint8_t* mask;
  CgScal* sc;
  double* part;
  int nx;
  double tau, a_dp, a_p, a_ol;
  int first;
  __device__ bool skip() const { return sc->done != 0; }
  __device__ void begin() {
    first = sc->first;
    tau = sc->tau;
    a_dp = a_p = a_ol = 0.0;
  }
  __device__ T load(int y, int x) {
    const size_t i = (size_t)y * nx + x;
    const T po = p[i];
    if (first) {
      a_p += fabs((double)po);
      return po;
    }
    double pn = (double)po;
    if constexpr (FS) {
      if (mask[i]) pn = (double)po - tau * (double)t[i];
    } else {
      if (po > T(0)) pn = (double)po - tau * (double)t[i];
      if (pn < 0.0) pn = 0.0;
      const double gv = (double)g[i];
      if (pn == 0.0 && gv < 0.0) {
        pn = -tau * gv;
        a_ol += 1.0;
      }
    }
    const T pt = (T)pn;
    p[i] = pt;
    a_dp += fabs((double)pt - (double)po);
    a_p += fabs((double)pt);
    return pt;
  }
  template <int NTHR>
  __device__ void finish(double* red) {
    const double acc[3] = {a_dp, a_p, a_ol};
    double tot[3];
    if (grid_reduce_last<3, NTHR>(acc, red, part, &sc->ticket[0], tot) && threadIdx.x == 0) {
      sc->sum_dp = tot[0];
      sc->sum_p = tot[1];
      sc->n_ol = tot[2];
      if (first) {
        sc->delta = 0.0;
      } else {
        sc->delta = (FS || tot[2] == 0.0) ? 1.0 : 0.0;
        sc->iter += 1;
      }
    }
  }
};

template <typename T, bool FS>
struct GapEpi {
  T* g;
  const T* hd;
  const T* p;
  const uint8_t* mask;
  CgScal* sc;
  double* part;
  int nx;
  double a_G, a_r;
  __device__ bool skip() const { return sc->done != 0; }
  __device__ void begin() { a_G = a_r = 0.0; }
  __device__ void store(int y, int x, T u) {
    const size_t i = (size_t)y * nx + x;
    const double h = (double)hd[i];
    const T gv = (T)((double)u + h);
    g[i] = gv;
    const bool in = FS ? (mask[i] != 0) : (p[i] > T(0));
    if (in) {
      a_G += (double)gv * (double)gv;
      a_r += h * h;
    }
  }
  template <int NTHR>
  __device__ void finish(double* red) {
    const double acc[2] = {a_G, a_r};
    double tot[2];
    if (grid_reduce_last<2, NTHR>(acc, red, part, &sc->ticket[1], tot) && threadIdx.x == 0) {
      const double G = tot[0];
      sc->G = G;
      sc->rhs2 = tot[1];
      int done = 0, status = CG_ST_OK;
      if (!isfinite(G) || !isfinite(sc->sum_p)) {
        done = 1;
        status = CG_ST_NUMERIC;
      } else if (!sc->first && sqrt(G) <= sc->tol * sqrt(tot[1]) && sc->n_ol == 0.0 &&
                 sc->sum_dp <= sc->tol * sc->sum_p) {
        done = 1;
      } else if (sc->iter >= sc->max_iter) {
        done = 1;
        status = CG_ST_NOCONV;
      } else if (sc->stall_limit > 0) {
        if (G < sc->best_G) {
          sc->best_G = G;
          sc->stall = 0;
        } else if (++sc->stall >= sc->stall_limit) {
          done = 1;
          status = CG_ST_FLOOR;
        }
      }
      if (!done) {
        sc->ratio = (sc->G_old > 0.0) ? sc->delta * (G / sc->G_old) : 0.0;
        sc->G_old = G;
        sc->first = 0;
      }
      sc->status = status;
      sc->done = done;
    }
  }
};

template <typename T, bool FS>
struct DirPro {
  T* t;
  const T* g;
  const T* p;
  const uint8_t* mask;
  const CgScal* sc;
  int nx;
  double ratio;
  __device__ bool skip() const { return sc->done != 0; }
  __device__ void begin() { ratio = sc->ratio; }
  __device__ T load(int y, int x) {
    const size_t i = (size_t)y * nx + x;
    const bool in = FS ? (mask[i] != 0) : (p[i] > T(0));
    const T tn = in ? (T)((double)g[i] + ratio * (double)t[i]) : T(0);
    t[i] = tn;
    return tn;
  }
  template <int NTHR>
  __device__ void finish(double*) {}
};

template <typename T>
struct DotsEpi {
  const T* g;
  const T* t;
  CgScal* sc;
  double* part;
  int nx;
  double a_gt, a_rt;
  __device__ bool skip() const { return sc->done != 0; }
  __device__ void begin() { a_gt = a_rt = 0.0; }
  __device__ void store(int y, int x, T r) {
    const size_t i = (size_t)y * nx + x;
    const double tv = (double)t[i];
    a_gt += (double)g[i] * tv;
    a_rt += (double)r * tv;
  }
  template <int NTHR>
  __device__ void finish(double* red) {
    const double acc[2] = {a_gt, a_rt};
    double tot[2];
    if (grid_reduce_last<2, NTHR>(acc, red, part, &sc->ticket[2], tot) && threadIdx.x == 0) {
      sc->gt = tot[0];
      sc->rt = tot[1];
      sc->tau = (tot[1] != 0.0) ? tot[0] / tot[1] : 0.0;
    }
  }
};

// ---- elementwise kernels -----------------------------------------------------

constexpr int EW_THREADS = 256;
constexpr int EW_MAX_BLOCKS = 1024;

template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_make_hd(const double* __restrict__ h, double d,
                                                        T* __restrict__ hd, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    hd[i] = (T)(h[i] - d);
}

// cold start p = max(d - h, 0) / (C K(0,0)): each element closing its own gap
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_cold_start(T* __restrict__ p, const T* __restrict__ hd,
                                                           double inv_ck00, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS) {
    const double v = -(double)hd[i];
    p[i] = (T)(v > 0.0 ? v * inv_ck00 : 0.0);
  }
}

// Zero the direction; fixed-set mode: zero the pressure off the contact set;
// non-adhesive mode: clip a warm-start pressure to p >= 0.
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_prepare(T* __restrict__ t, T* __restrict__ p,
                                                        const uint8_t* __restrict__ mask, int clip,
                                                        size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS) {
    t[i] = T(0);
    if (mask && !mask[i]) p[i] = T(0);
    if (clip && p[i] < T(0)) p[i] = T(0);
  }
}

// Final sums: sum p (force / (dx dy)), contact count, penetrations off A
// (fixed-set mode) and the contact mask (non-adhesive mode: p > 0).
template <typename T, bool FS>
__global__ __launch_bounds__(EW_THREADS) void k_finalize(const T* __restrict__ p,
                                                         const T* __restrict__ g,
                                                         uint8_t* __restrict__ mask, CgScal* sc,
                                                         double* part, size_t n) {
  __shared__ double red[64];
  double sp = 0.0, nc = 0.0, npen = 0.0;
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS) {
    const T pv = p[i];
    sp += (double)pv;
    bool in;
    if constexpr (FS) {
      in = mask[i] != 0;
      if (!in && g[i] < T(0)) npen += 1.0;
    } else {
      in = pv > T(0);
      mask[i] = in ? 1 : 0;
    }
    nc += in ? 1.0 : 0.0;
  }
  const double acc[3] = {sp, nc, npen};
  double tot[3];
  if (grid_reduce_last<3, EW_THREADS>(acc, red, part, &sc->ticket[3], tot) && threadIdx.x == 0) {
    sc->fin_sum_p = tot[0];
    sc->fin_contact = tot[1];
    sc->fin_pen = tot[2];
  }
}

// Detachment (Section 3.1, Eq. 24): every element of A whose tensile stress
// exceeds p_crit (-p > p_crit) leaves A, all in the same round.
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_detach(T* __restrict__ p, uint8_t* __restrict__ mask,
                                                       double pcrit, CgScal* sc, double* part,
                                                       size_t n) {
  __shared__ double red[64];
  double cnt = 0.0;
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS) {
    if (mask[i] && -(double)p[i] > pcrit) {
      mask[i] = 0;
      p[i] = T(0);
      cnt += 1.0;
    }
  }
  const double acc[1] = {cnt};
  double tot[1];
  if (grid_reduce_last<1, EW_THREADS>(acc, red, part, &sc->ticket[4], tot) && threadIdx.x == 0)
    sc->fin_detach = tot[0];
}

template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_to_f64(const T* __restrict__ src,
                                                       double* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    dst[i] = (double)src[i];
}

template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_from_f64(const double* __restrict__ src,
                                                         T* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    dst[i] = (T)src[i];
}

// u = g - (h - d): displacement output from the last gap evaluation
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_u_from_gap(const T* __restrict__ g,
                                                           const double* __restrict__ h, double d,
                                                           double* __restrict__ u, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    u[i] = (double)g[i] - (h[i] - d);
}

}  // namespace bem
