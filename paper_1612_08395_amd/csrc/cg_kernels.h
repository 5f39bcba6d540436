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
// Load-control mode (non-adhesive, total force W prescribed, d unknown):
// g is shifted by its mean over Ic (gbar, which becomes the indentation),
// r by its mean over Ic, and p is rescaled to carry W after each update.
// The rescaling is deferred: K1 stores the unscaled update p' and its sum;
// K3 scales u by s = W / sum p' (linearity) and the next K1 scales p' by the
// same s on reading.  G = sum_Ic (g - gbar)^2 is formed from sums shifted by
// the previous gbar, which keeps the subtraction benign near convergence.
//
// One iteration is five kernel launches (six under load control); the
// vector work is fused into the row sweeps of the two convolutions:
//   K1 row R2C   prologue UpdatePro : update p from the previous tau, t, g
//   K2 column    (fused spectrum multiply)
//   K3 row C2R   epilogue GapEpi    : g = u + (h - d), sums for G
//   K4 row R2C   prologue DirPro    : convergence decision, new direction t,
//                                     sum g t
//   K5 column    forward transform and sum_k KT |T|^2 = sum t r (Parseval;
//                t is zero outside the grid), no inverse transforms
// r = C K * t enters only through tau, so the second convolution ends in the
// spectral domain: five launches per iteration.  Since t = 0 off Ic, the
// sums need no mask.  Load control needs the mean of r over Ic and keeps the
// sixth launch:
//   K5 column    (full, as K2)
//   K6 row C2R   epilogue DotsEpi   : sum g t, sum r t, sum t, sum_Ic r
//
// Reductions are FP64 and the iteration kernels use no atomics or fences:
// every reducing kernel writes one partial per workgroup (fixed-order block
// sum) into its own buffer, and the kernel that needs the total adds the
// partials again at its start, in index order, in every workgroup.  The
// result is bitwise reproducible, identical in all workgroups, and made
// visible by the kernel boundary.  The iteration index `it` is a kernel
// argument; K4 makes the convergence decision (every workgroup reaches the
// same one, workgroup 0 records it) and keeps G_old and the stagnation state
// in slots indexed by it & 1.  Every kernel returns at once when `done` is
// set, so the host may queue several iterations and check the flag rarely.
#pragma once
#include "cg_api.h"
#include "common.h"
#include "conv_kernels.h"

namespace bem {

// Block sums of NV values (result in every thread), one barrier pair.
template <int NV, int NTHR>
__device__ __forceinline__ void block_sum_n(double (&v)[NV], double* red) {
  constexpr int NW = NTHR / 64;
  static_assert(NV * NW <= 64, "reduction scratch");
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * NW + w] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[k * NW + i];
    v[k] = s;
  }
  __syncthreads();
}

// This workgroup's partials (plain stores; read by later kernels).  bid:
// the workgroup's index within its problem (blockIdx.x, or the index inside
// its slot in a batched launch).
template <int NV, int NTHR>
__device__ __forceinline__ void write_partials(double (&acc)[NV], double* red, double* part,
                                               int bid) {
  block_sum_n<NV, NTHR>(acc, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) part[bid * NV + k] = acc[k];
}

// Totals of the nb partials an earlier kernel wrote (same order everywhere).
template <int NV, int NTHR>
__device__ __forceinline__ void read_totals(const double* __restrict__ part, int nb, double* red,
                                            double (&tot)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = 0.0;
#pragma unroll 4
  for (int i = threadIdx.x; i < nb; i += NTHR)
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] += part[i * NV + k];
  block_sum_n<NV, NTHR>(tot, red);
}

// read_totals split in two: issue() loads this thread's first R partials
// into registers (before the caller issues its field loads, so that waiting
// for them does not wait for the fields), total() adds them, and any beyond
// R NTHR, in the same order as read_totals.  R NTHR should cover the usual
// partial count (one per row pair: 1024 at 2048^2).
template <int NV, int R = 4>
struct Partials {
  double v[R][NV];
  template <int NTHR>
  __device__ __forceinline__ void issue(const double* __restrict__ part, int nb) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + r * NTHR;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[r][k] = load_or0(part, (size_t)i * NV + k, 0, i < nb);
    }
  }
  template <int NTHR>
  __device__ __forceinline__ void total(const double* __restrict__ part, int nb, double* red,
                                        double (&tot)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < NV; ++k) tot[k] += v[r][k];
    for (int i = threadIdx.x + R * NTHR; i < nb; i += NTHR)
#pragma unroll
      for (int k = 0; k < NV; ++k) tot[k] += part[i * NV + k];
    block_sum_n<NV, NTHR>(tot, red);
  }
};

// Partials per thread for a row sweep with PER elements per thread and row:
// the wave row kernels (PER = 16) run 128 threads, the others 256 or 512.
__host__ __device__ constexpr int part_regs(int per) { return per >= 16 ? 8 : 4; }

// Last-workgroup reduction, used only by the once-per-solve elementwise
// kernels (agent-scope stores, fence, ticket).
template <int NV, int NTHR>
__device__ __forceinline__ bool grid_reduce_last(const double (&acc)[NV], double* red,
                                                 double* part, unsigned int* ticket,
                                                 double (&tot)[NV]) {
  __shared__ int am_last;
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = acc[v];
  block_sum_n<NV, NTHR>(s, red);
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
  for (int v = 0; v < NV; ++v) tot[v] = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += NTHR)
#pragma unroll
    for (int v = 0; v < NV; ++v)
      tot[v] += __hip_atomic_load(&part[i * NV + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum_n<NV, NTHR>(tot, red);
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
}

// K1 prologue: p update with the previous iteration's tau, t and g.
template <typename T, int MODE, int PER>
struct UpdatePro {
  static constexpr bool FS = MODE == CG_FIXED, FC = MODE == CG_FORCE;
  static constexpr int NVD = FC ? 4 : 1;
  T* p;
  T* t;                  // read on Ic; zeroed where an element leaves Ic
  const T* g;
  uint8_t* mask;         // fixed set: the set A (read); else Ic = {p > 0} (written)
  const CgScal* sc;
  double* part;
  int nx, nb, it;
  int nbc;               // column workgroups of K5 (sum t r partials)
  double tau, a_dp, a_p, a_ol;
  double sprev, gshift;  // load control: scale of the stored p, mean gap
  T pa[PER], pb[PER], ta[PER], tb[PER], ga[PER], gb[PER];
  bool ma[PER], mb[PER];
  Partials<NVD, part_regs(PER)> dots;
  Partials<1, part_regs(PER)> rts;
  template <int NTHR>
  __device__ bool issue() {
    if (sc->done) return false;
    // always issued (valid buffers; unused when it == 0) so that no branch
    // separates these loads from the field loads
    dots.template issue<NTHR>(part + kPartDots, nb);
    if constexpr (!FC) rts.template issue<NTHR>(part + kPartRT, nbc);
    return true;
  }
  // p and g (the mask in fixed-set mode) first; t only where the update
  // uses it, p > 0 (in the set), since t is 0 elsewhere: off Ic a lane reads
  // its row's first element instead, one cache line per wave.  (t and g are
  // unused when it == 0.)
  template <int NTHR>
  __device__ void fetch(int ya, int yb, bool hasb, int nxl) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const bool in = n < nxl, inb = in && hasb;
      const size_t ia = (size_t)ya * nx + n, ib = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      pa[q] = load_or0(p, ia, sf, in);
      pb[q] = load_or0(p, ib, sf, inb);
      ga[q] = gb[q] = T(0);
      ma[q] = mb[q] = false;
      if constexpr (FS) {
        ma[q] = load_or0(mask, ia, sf, in) != 0;
        mb[q] = load_or0(mask, ib, sf, inb) != 0;
      } else {
        ga[q] = load_or0(g, ia, sf, in);
        gb[q] = load_or0(g, ib, sf, inb);
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const size_t ia = (size_t)ya * nx + n, ib = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      ta[q] = load_or0(t, ia, sf, FS ? ma[q] : pa[q] > T(0));
      tb[q] = load_or0(t, ib, sf, FS ? mb[q] : pb[q] > T(0));
    }
  }
  template <int NTHR>
  __device__ bool decide(double* red, int bid) {
    a_dp = a_p = a_ol = 0.0;
    double tot[NVD];
    dots.template total<NTHR>(part + kPartDots, nb, red, tot);
    if constexpr (FC) {
      const int j = (it - 1) & 1;
      sprev = it > 0 ? sc->scale_hist[j] : 1.0;
      gshift = it > 0 ? sc->gbar_hist[j] : 0.0;
      const double nc = it > 0 ? sc->nc_hist[j] : 0.0;
      // sum_Ic (r - rbar) t = sum r t - rbar sum t   (t = 0 off Ic)
      const double den = tot[1] - (nc > 0.0 ? tot[3] / nc : 0.0) * tot[2];
      tau = (it > 0 && den != 0.0) ? tot[0] / den : 0.0;
    } else {
      double rt[1];
      rts.template total<NTHR>(part + kPartRT, nbc, red, rt);
      sprev = 1.0;
      gshift = 0.0;
      tau = (it > 0 && rt[0] != 0.0) ? tot[0] / rt[0] : 0.0;
    }
    return true;
  }
  __device__ __forceinline__ T upd(double po, T tv, T gv, bool in_set) {
    double pn = po;
    if constexpr (FS) {
      if (in_set) pn = po - tau * (double)tv;
    } else {
      const double gs = (double)gv - gshift;
      if (po > 0.0) pn = po - tau * (double)tv;
      if (pn < 0.0) pn = 0.0;
      if (pn == 0.0 && gs < 0.0) {
        pn = -tau * gs;
        a_ol += 1.0;
      }
    }
    const T pt = (T)pn;
    a_dp += fabs((double)pt - po);
    a_p += fabs((double)pt);
    return pt;
  }
  template <int NTHR>
  __device__ void make(int, int, bool hasb, int nxl, T (&va)[PER], T (&vb)[PER]) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      va[q] = pa[q];
      vb[q] = pb[q];
    }
    if (it == 0) {
#pragma unroll
      for (int q = 0; q < PER; ++q) a_p += fabs((double)va[q]) + fabs((double)vb[q]);
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      if (n < nxl) {
        va[q] = upd(sprev * (double)va[q], ta[q], ga[q], ma[q]);
        if (hasb) vb[q] = upd(sprev * (double)vb[q], tb[q], gb[q], mb[q]);
      }
    }
  }
  template <int NTHR>
  __device__ void commit(int ya, int yb, bool hasb, int nxl, const T (&va)[PER],
                         const T (&vb)[PER]) {
    if (it == 0) return;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      if (n < nxl) {
        p[(size_t)ya * nx + n] = va[q];
        if (hasb) p[(size_t)yb * nx + n] = vb[q];
        if constexpr (!FS) {
          // contact flags for the rest of the iteration (1 byte instead of p)
          mask[(size_t)ya * nx + n] = va[q] > T(0) ? 1 : 0;
          if (hasb) mask[(size_t)yb * nx + n] = vb[q] > T(0) ? 1 : 0;
          // t is zero off Ic and only written on it (DirPro): an element
          // leaving Ic gets its zero here
          if (pa[q] > T(0) && !(va[q] > T(0))) t[(size_t)ya * nx + n] = T(0);
          if (hasb && pb[q] > T(0) && !(vb[q] > T(0))) t[(size_t)yb * nx + n] = T(0);
        }
      }
    }
  }
  template <int NTHR>
  __device__ void finish(double* red, int bid) {
    double acc[3] = {a_dp, a_p, a_ol};
    write_partials<3, NTHR>(acc, red, part + kPartUpd, bid);
  }
};

// K3 epilogue: g = u + (h - d) and the partial sums for G and its scale on
// Ic.  Load control: u is first scaled by s = W / sum p (K1's partials) and
// the sums are of e = g - (previous gbar), with |Ic| and sum_Ic u^2.
template <typename T, int MODE, int PER>
struct GapEpi {
  static constexpr bool FS = MODE == CG_FIXED, FC = MODE == CG_FORCE;
  static constexpr int NV = FC ? 4 : 2;
  T* g;
  const T* hd;
  const T* p;
  const uint8_t* mask;
  const CgScal* sc;
  double* part;
  int nx, nb, it;
  T ha[PER], hb[PER];
  bool ca[PER], cb[PER];
  double acc[NV];
  double s, gref;
  Partials<3, part_regs(PER)> pu;
  template <int NTHR>
  __device__ bool begin(double*) {
    if (sc->done) return false;
    if constexpr (FC) pu.template issue<NTHR>(part + kPartUpd, nb);
    return true;
  }
  template <int NTHR>
  __device__ void prefetch(int ya, int yb, bool hasb, int nxl) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const bool in = n < nxl, inb = in && hasb;
      const size_t a = (size_t)ya * nx + n, b = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      ha[q] = load_or0(hd, a, sf, in);
      hb[q] = load_or0(hd, b, sf, inb);
      // Ic: the fixed set A, or the flags {p > 0} the update kept current
      ca[q] = load_or0(mask, a, sf, in) != 0;
      cb[q] = load_or0(mask, b, sf, inb) != 0;
    }
  }
  // after the loads are issued: the reductions the epilogue needs
  template <int NTHR>
  __device__ void ready(double* red) {
    if constexpr (FC) {
      double up[3];
      pu.template total<NTHR>(part + kPartUpd, nb, red, up);
      s = sc->W / up[1];
      gref = it > 0 ? sc->gbar_hist[(it - 1) & 1] : 0.0;
    }
  }
  __device__ __forceinline__ void one(size_t i, T u, T h, bool c) {
    if constexpr (FC) {
      const double us = s * (double)u;
      const T gv = (T)(us + (double)h);
      g[i] = gv;
      if (c) {
        const double e = (double)gv - gref;
        acc[0] += e;
        acc[1] += e * e;
        acc[2] += 1.0;
        acc[3] += us * us;
      }
    } else {
      const T gv = (T)((double)u + (double)h);
      g[i] = gv;
      if (c) {
        acc[0] += (double)gv * (double)gv;
        acc[1] += (double)h * (double)h;
      }
    }
  }
  template <int NTHR>
  __device__ void consume(int ya, int yb, bool hasb, int nxl, const T (&va)[PER],
                          const T (&vb)[PER]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      if (n < nxl) {
        one((size_t)ya * nx + n, va[q], ha[q], ca[q]);
        if (hasb) one((size_t)yb * nx + n, vb[q], hb[q], cb[q]);
      }
    }
  }
  template <int NTHR>
  __device__ void finish(double* red, int bid) {
    write_partials<NV, NTHR>(acc, red, part + kPartGap, bid);
  }
};

// K4 prologue: convergence decision (stopping test at the current iterate,
// iteration limit, non-finite values, MIXED stagnation), then t.
template <typename T, int MODE, int PER>
struct DirPro {
  static constexpr bool FS = MODE == CG_FIXED, FC = MODE == CG_FORCE;
  static constexpr int NVG = FC ? 4 : 2;
  // at L = 4096 the uncapped kernel takes 130 VGPRs (3 waves per SIMD, one
  // 8-wave workgroup per CU); capped at 128 it does not spill, except under
  // load control, which keeps the compiler's choice
  static constexpr int kMinWaves = FC ? 1 : 4;
  T* t;
  const T* g;
  const T* p;
  const uint8_t* mask;
  CgScal* sc;
  double* part;
  int nx, nb, it;
  double ratio, gbar, a_gt;
  T ga[PER], gb[PER], ta[PER], tb[PER];
  bool ca[PER], cb[PER];
  Partials<3, part_regs(PER)> pu;
  Partials<NVG, part_regs(PER)> pg;
  template <int NTHR>
  __device__ bool issue() {
    if (sc->done) return false;
    pu.template issue<NTHR>(part + kPartUpd, nb);
    pg.template issue<NTHR>(part + kPartGap, nb);
    return true;
  }
  // The contact flags first; g and t only where an element is in Ic (t is 0
  // elsewhere): off Ic a lane reads its row's first element instead, one
  // cache line per wave, which cuts the field reads from 12 to about 1 +
  // 8 x (contact fraction) bytes per element.
  template <int NTHR>
  __device__ void fetch(int ya, int yb, bool hasb, int nxl) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const bool in = n < nxl, inb = in && hasb;
      const size_t a = (size_t)ya * nx + n, b = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      // Ic: the fixed set A, or the flags {p > 0} the update kept current
      ca[q] = load_or0(mask, a, sf, in) != 0;
      cb[q] = load_or0(mask, b, sf, inb) != 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const size_t a = (size_t)ya * nx + n, b = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      ga[q] = load_or0(g, a, sf, ca[q]);
      gb[q] = load_or0(g, b, sf, cb[q]);
      ta[q] = load_or0(t, a, sf, ca[q]);
      tb[q] = load_or0(t, b, sf, cb[q]);
    }
  }
  template <int NTHR>
  __device__ bool decide(double* red, int bid) {
    double up[3], gp[NVG];
    pu.template total<NTHR>(part + kPartUpd, nb, red, up);
    pg.template total<NTHR>(part + kPartGap, nb, red, gp);
    const double sum_dp = up[0], sum_p = up[1], n_ol = up[2];
    double G, rhs2, scale = 1.0, nc = 0.0;
    gbar = 0.0;
    if constexpr (FC) {
      const double gref = it > 0 ? sc->gbar_hist[(it - 1) & 1] : 0.0;
      nc = gp[2];
      gbar = nc > 0.0 ? gref + gp[0] / nc : gref;
      G = nc > 0.0 ? fmax(gp[1] - gp[0] * gp[0] / nc, 0.0) : 0.0;
      rhs2 = gp[3];
      scale = sc->W / sum_p;
    } else {
      G = gp[0];
      rhs2 = gp[1];
    }
    const double G_old = it > 0 ? sc->G_hist[(it - 1) & 1] : 1.0;
    double best = it > 0 ? sc->best_hist[(it - 1) & 1] : 1e300;
    int stall = it > 0 ? sc->stall_hist[(it - 1) & 1] : 0;
    int done = 0, status = CG_ST_OK;
    if (!isfinite(G) || !isfinite(sum_p) || !isfinite(scale)) {
      done = 1;
      status = CG_ST_NUMERIC;
    } else if (it > 0 && sqrt(G) <= sc->tol * sqrt(rhs2) && n_ol == 0.0 &&
               sum_dp <= sc->tol * sum_p) {
      done = 1;
    } else if (it >= sc->max_iter) {
      done = 1;
      status = CG_ST_NOCONV;
    } else if (sc->stall_limit > 0) {
      // the window grows with the solve: while the contact set still moves,
      // G can stay above its running minimum for hundreds of iterations far
      // above the rounding floor (4096^2 grids at k = -0.3)
      if (G < best) {
        best = G;
        stall = 0;
      } else if (++stall >= max(sc->stall_limit, it / 2)) {
        done = 1;
        status = CG_ST_FLOOR;
      }
    }
    if (bid == 0 && threadIdx.x == 0) {
      if constexpr (FC) {
        sc->gbar_hist[it & 1] = gbar;
        sc->scale_hist[it & 1] = scale;
        sc->nc_hist[it & 1] = nc;
      }
      if (done) {
        sc->status = status;
        sc->iter = it;
        sc->G = G;
        sc->rhs2 = rhs2;
        sc->sum_p = sum_p;
        sc->gbar = gbar;
        sc->scale = scale;
        sc->done = 1;
      } else {
        sc->G_hist[it & 1] = G;
        sc->best_hist[it & 1] = best;
        sc->stall_hist[it & 1] = stall;
      }
    }
    if (done) return false;
    const double delta = (it == 0) ? 0.0 : ((FS || n_ol == 0.0) ? 1.0 : 0.0);
    ratio = (G_old > 0.0) ? delta * (G / G_old) : 0.0;
    return true;
  }
  template <int NTHR>
  __device__ void make(int, int, bool, int, T (&va)[PER], T (&vb)[PER]) {
    double gt = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      va[q] = ca[q] ? (T)((double)ga[q] - gbar + ratio * (double)ta[q]) : T(0);
      vb[q] = cb[q] ? (T)((double)gb[q] - gbar + ratio * (double)tb[q]) : T(0);
      // sum g t with the stored (rounded) t; t = 0 off Ic
      gt += (double)ga[q] * (double)va[q] + (double)gb[q] * (double)vb[q];
    }
    a_gt = gt;
  }
  template <int NTHR>
  __device__ void commit(int ya, int yb, bool hasb, int nxl, const T (&va)[PER],
                         const T (&vb)[PER]) {
    // only on Ic: off Ic t stays zero (the prepare kernel clears it, and
    // UpdatePro zeroes each element that leaves Ic)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      if (n < nxl) {
        if (ca[q]) t[(size_t)ya * nx + n] = va[q];
        if (hasb && cb[q]) t[(size_t)yb * nx + n] = vb[q];
      }
    }
  }
  template <int NTHR>
  __device__ void finish(double* red, int bid) {
    if constexpr (!FC) {
      double acc[1] = {a_gt};
      write_partials<1, NTHR>(acc, red, part + kPartDots, bid);
    }
  }
};

// K6 epilogue (load control only): sum g t and sum r t (t = 0 off Ic, so no mask is needed).
// Load control: g is shifted by gbar, and sum t, sum_Ic r (Ic = {p > 0})
// give the shift of r by its mean over Ic.
template <typename T, int MODE, int PER>
struct DotsEpi {
  static constexpr bool FC = MODE == CG_FORCE;
  static constexpr int NV = FC ? 4 : 2;
  const T* g;
  const T* t;
  const uint8_t* mask;   // Ic = {p > 0}, kept current by UpdatePro
  const CgScal* sc;
  double* part;
  int nx, it;
  T ga_[PER], gb_[PER], ta_[PER], tb_[PER];
  bool ca[PER], cb[PER];
  double acc[NV];
  double gbar;
  template <int NTHR>
  __device__ bool begin(double*) {
    if (sc->done) return false;
    gbar = FC ? sc->gbar_hist[it & 1] : 0.0;
    return true;
  }
  template <int NTHR>
  __device__ void prefetch(int ya, int yb, bool hasb, int nxl) {
    // the flags first, then g and t on Ic only (t is 0 elsewhere, so every
    // sum is over Ic)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const bool in = n < nxl, inb = in && hasb;
      const size_t a = (size_t)ya * nx + n, b = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      ca[q] = load_or0(mask, a, sf, in) != 0;
      cb[q] = load_or0(mask, b, sf, inb) != 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const size_t a = (size_t)ya * nx + n, b = (size_t)yb * nx + n, sf = (size_t)ya * nx;
      ga_[q] = load_or0(g, a, sf, ca[q]);
      ta_[q] = load_or0(t, a, sf, ca[q]);
      gb_[q] = load_or0(g, b, sf, cb[q]);
      tb_[q] = load_or0(t, b, sf, cb[q]);
    }
  }
  template <int NTHR>
  __device__ void ready(double*) {}
  template <int NTHR>
  __device__ void consume(int, int, bool, int, const T (&va)[PER], const T (&vb)[PER]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      acc[0] += ((double)ga_[q] - gbar) * (double)ta_[q] + ((double)gb_[q] - gbar) * (double)tb_[q];
      acc[1] += (double)va[q] * (double)ta_[q] + (double)vb[q] * (double)tb_[q];
      if constexpr (FC) {
        acc[2] += (double)ta_[q] + (double)tb_[q];
        acc[3] += (ca[q] ? (double)va[q] : 0.0) + (cb[q] ? (double)vb[q] : 0.0);
      }
    }
  }
  template <int NTHR>
  __device__ void finish(double* red, int bid) {
    write_partials<NV, NTHR>(acc, red, part + kPartDots, bid);
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

// First iteration of a warm-started displacement-controlled solve within a
// sweep over d (same h): the state's g = C K * p + h - d_old belongs to the
// unchanged p, so the new gap is g + (d_old - d_new) and the iteration's
// first convolution can be skipped.  One workgroup per row pair writes the
// partial sums that the update prologue (sum |p|; nothing is updated at
// iteration 0) and the gap epilogue (sum over Ic of g^2 and of (h - d)^2)
// would have written.
template <typename T, int NTHR>
__global__ __launch_bounds__(NTHR) void k_gap_shift(T* __restrict__ g, const T* __restrict__ hd,
                                                    const T* __restrict__ p,
                                                    const uint8_t* __restrict__ mask,
                                                    double delta, double* __restrict__ part,
                                                    int nx, int ny) {
  __shared__ double red[64];
  const int ya = 2 * blockIdx.x;
  const int rows = ya + 1 < ny ? 2 : 1;
  double acc[3] = {0.0, 0.0, 0.0};   // sum |p|, sum_Ic g^2, sum_Ic (h - d)^2
  for (int r = 0; r < rows; ++r) {
    const size_t base = (size_t)(ya + r) * nx;
    for (int n = threadIdx.x; n < nx; n += NTHR) {
      const size_t i = base + n;
      const T gv = (T)((double)g[i] + delta);
      g[i] = gv;
      acc[0] += fabs((double)p[i]);
      if (mask[i]) {
        const double h = (double)hd[i];
        acc[1] += (double)gv * (double)gv;
        acc[2] += h * h;
      }
    }
  }
  block_sum_n<3, NTHR>(acc, red);
  if (threadIdx.x == 0) {
    part[kPartUpd + blockIdx.x * 3 + 0] = 0.0;
    part[kPartUpd + blockIdx.x * 3 + 1] = acc[0];
    part[kPartUpd + blockIdx.x * 3 + 2] = 0.0;
    part[kPartGap + blockIdx.x * 2 + 0] = acc[1];
    part[kPartGap + blockIdx.x * 2 + 1] = acc[2];
  }
}

// Zero the direction; fixed-set mode: zero the pressure off the contact set;
// non-adhesive mode: clip a warm-start pressure to p >= 0.
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_prepare(T* __restrict__ t, T* __restrict__ p,
                                                        uint8_t* __restrict__ mask, int fixed_set,
                                                        size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS) {
    t[i] = T(0);
    if (fixed_set) {
      if (!mask[i]) p[i] = T(0);
    } else {
      // the loop's contact flags: Ic = {p > 0}, kept current by UpdatePro
      T pv = p[i];
      if (pv < T(0)) p[i] = pv = T(0);
      mask[i] = pv > T(0) ? 1 : 0;
    }
  }
}

// Final sums: sum p (force / (dx dy)), contact count, penetrations off A
// (fixed-set mode) and the contact mask (non-adhesive mode: p > 0).
template <typename T, int MODE>
__global__ __launch_bounds__(EW_THREADS) void k_finalize(T* __restrict__ p,
                                                         const T* __restrict__ g,
                                                         uint8_t* __restrict__ mask, CgScal* sc,
                                                         double* part, size_t n) {
  constexpr bool FS = MODE == CG_FIXED, FC = MODE == CG_FORCE;
  __shared__ double red[64];
  double sp = 0.0, nc = 0.0, npen = 0.0;
  const double scale = FC ? sc->scale : 1.0;
  auto elem = [&](size_t i, T pv, bool m, T gv) {
    if constexpr (FC) {
      // load control: apply the scale of the stopping iteration
      pv = (T)(scale * (double)pv);
      p[i] = pv;
    }
    sp += (double)pv;
    bool in;
    if constexpr (FS) {
      in = m;
      if (!in && gv < T(0)) npen += 1.0;
    } else {
      in = pv > T(0);
      mask[i] = in ? 1 : 0;
    }
    nc += in ? 1.0 : 0.0;
  };
  // U elements per thread in flight at once (their loads first), visited in
  // the order of the plain grid-stride loop, so the sums are the same
  constexpr int U = 4;
  const size_t stride = (size_t)gridDim.x * EW_THREADS;
  size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    T pv[U], gv[U];
    bool mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pv[u] = p[i + u * stride];
      mv[u] = FS ? mask[i + u * stride] != 0 : false;
      gv[u] = FS ? g[i + u * stride] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) elem(i + u * stride, pv[u], mv[u], gv[u]);
  }
  for (; i < n; i += stride) elem(i, p[i], FS ? mask[i] != 0 : false, FS ? g[i] : T(0));
  const double acc[3] = {sp, nc, npen};
  double tot[3];
  if (grid_reduce_last<3, EW_THREADS>(acc, red, part + kPartElem, &sc->ticket[3], tot) && threadIdx.x == 0) {
    sc->fin_sum_p = tot[0];
    sc->fin_contact = tot[1];
    sc->fin_pen = tot[2];
  }
}

// p = v everywhere (load control: cold start carrying any load; the first
// iteration rescales it)
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_fill(T* __restrict__ p, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    p[i] = v;
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
  if (grid_reduce_last<1, EW_THREADS>(acc, red, part + kPartElem, &sc->ticket[4], tot) && threadIdx.x == 0)
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
// sc->gbar = min h (load control at zero load: the surfaces just touch).
// One workgroup of EW_THREADS.
template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_min_h(const double* __restrict__ h, size_t n,
                                                      CgScal* sc) {
  __shared__ double red[EW_THREADS / 64];
  double m = INFINITY;
  for (size_t i = threadIdx.x; i < n; i += EW_THREADS) m = fmin(m, h[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < EW_THREADS / 64; ++w) m = fmin(m, red[w]);
    sc->gbar = m;
  }
}

template <typename T>
__global__ __launch_bounds__(EW_THREADS) void k_u_from_gap(const T* __restrict__ g,
                                                           const double* __restrict__ h, double d,
                                                           double* __restrict__ u, size_t n) {
  for (size_t i = blockIdx.x * (size_t)EW_THREADS + threadIdx.x; i < n;
       i += (size_t)gridDim.x * EW_THREADS)
    u[i] = (double)g[i] - (h[i] - d);
}

}  // namespace bem
