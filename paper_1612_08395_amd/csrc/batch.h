// Batched conjugate-gradient iterations: one launch of each CG kernel runs
// that kernel for several independent contact solves of one padded geometry
// (Lx, Ly), the serving loop's continuous batching.  Each solve (a slot) has
// its own grid (nx <= Lx, ny <= Ly), kernel spectrum, fields, partial sums and
// scalar block; the workgroups of a launch are split evenly over the slots
// (slot = blockIdx.x / blocks-per-slot) and run exactly the per-problem code
// of the single-solve kernels with the workgroup index inside the slot, so a
// slot's arithmetic, reduction order and results are those of the same solve
// run alone.  Slots whose mode differs from the launch's return at once, as
// do the workgroups past a slot's row pairs and every workgroup of a
// converged slot.
#pragma once
#include "cg_kernels.h"
#include "launch.h"

namespace bem {

// rb: workgroups per slot of the row kernels (Ly / 2 >= every slot's row
// pairs); nbc: column workgroups per slot; itl: iteration within the chunk.
template <typename T, int L, int NTHR, int MODE>
__global__ __launch_bounds__(NTHR, (min_waves_of<UpdatePro<T, MODE, row_per<L, NTHR>()>>::value))
void kb_update(const BatchSlot<T>* __restrict__ slots, int rb, int nbc, int itl,
               const cplx<T>* __restrict__ tw) {
  const BatchSlot<T> sd = slots[blockIdx.x / rb];
  const int bid = blockIdx.x % rb, nrp = (sd.ny + 1) / 2;
  if (sd.mode != MODE || bid >= nrp) return;
  UpdatePro<T, MODE, row_per<L, NTHR>()> pro{sd.p,    sd.t,  sd.g, sd.mask,       sd.sc,
                                             sd.part, sd.nx, nrp,  sd.it0 + itl, nbc};
  row_r2c_body<T, L, NTHR>(pro, sd.S, sd.nx, sd.ny, tw, bid);
}

template <typename T, int L, int NTHR, int MODE>
__global__ __launch_bounds__(NTHR) void kb_gap(const BatchSlot<T>* __restrict__ slots, int rb,
                                               int itl, const cplx<T>* __restrict__ tw) {
  const BatchSlot<T> sd = slots[blockIdx.x / rb];
  const int bid = blockIdx.x % rb, nrp = (sd.ny + 1) / 2;
  if (sd.mode != MODE || bid >= nrp) return;
  GapEpi<T, MODE, row_per<L, NTHR>()> epi{sd.g,    sd.hd, sd.p, sd.mask,
                                          sd.sc,   sd.part, sd.nx, nrp, sd.it0 + itl};
  row_c2r_body<T, L, NTHR>(sd.S, sd.nx, sd.ny, tw, epi, bid);
}

template <typename T, int L, int NTHR, int MODE>
__global__ __launch_bounds__(NTHR, (min_waves_of<DirPro<T, MODE, row_per<L, NTHR>()>>::value))
void kb_direction(const BatchSlot<T>* __restrict__ slots, int rb, int itl,
                  const cplx<T>* __restrict__ tw) {
  const BatchSlot<T> sd = slots[blockIdx.x / rb];
  const int bid = blockIdx.x % rb, nrp = (sd.ny + 1) / 2;
  if (sd.mode != MODE || bid >= nrp) return;
  DirPro<T, MODE, row_per<L, NTHR>()> pro{sd.t,    sd.g,  sd.p, sd.mask,      sd.sc,
                                          sd.part, sd.nx, nrp,  sd.it0 + itl};
  row_r2c_body<T, L, NTHR>(pro, sd.S, sd.nx, sd.ny, tw, bid);
}

template <typename T, int LY, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void kb_column(const BatchSlot<T>* __restrict__ slots, int nbc,
                                                  int lx, int kpitch,
                                                  const cplx<T>* __restrict__ tw) {
  const BatchSlot<T> sd = slots[blockIdx.x / nbc];
  if (sd.mode == BATCH_EMPTY || sd.sc->done) return;
  col_conv_body<T, LY, W, NTHR>(sd.S, lx, sd.ny, sd.KT, kpitch, tw, blockIdx.x % nbc, nbc);
}

template <typename T, int LY, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void kb_energy(const BatchSlot<T>* __restrict__ slots, int nbc,
                                                  int lx, int kpitch,
                                                  const cplx<T>* __restrict__ tw) {
  const BatchSlot<T> sd = slots[blockIdx.x / nbc];
  if (sd.mode == BATCH_EMPTY || sd.sc->done) return;
  col_energy_body<T, LY, W, NTHR>(sd.S, lx, sd.ny, sd.KT, kpitch, tw, sd.part + kPartRT,
                                  blockIdx.x % nbc, nbc);
}

// Batched iterations (declared in cg_api.h).
template <typename T>
hipError_t launch_batch_iterations(const Geom& g, const SpecView<T>& K,
                                   const BatchSlot<T>* slots, int nslots, unsigned modes, int n,
                                   hipStream_t s) {
  if (!batch_geometry(g) || nslots < 1) return hipErrorInvalidValue;
  const int rb = g.Ly / 2;
  const int W = col_width<T>(g.Ly, g.Lx);
  const int nbc = g.Lx / W;
  return dispatch_L(g.Lx, [&](auto LXc) -> hipError_t {
    constexpr int LX = decltype(LXc)::value;
    constexpr int NT = row_threads(LX);
    return dispatch_L(g.Ly, [&](auto LYc) -> hipError_t {
      constexpr int LY = decltype(LYc)::value;
      return dispatch_W(W, [&](auto Wc) -> hipError_t {
        constexpr int WW = decltype(Wc)::value;
        if constexpr (WW > col_width_lds<T>(LY) || LX > 1024 || LY > 1024) {
          return hipErrorInvalidValue;
        } else {
          constexpr int CT = col_threads(WW, LY);
          const dim3 rows(nslots * rb), cols(nslots * nbc);
          hipError_t e = hipSuccess;
          for (int i = 0; i < n && e == hipSuccess; ++i) {
            if (modes & (1u << CG_DISP))
              hipLaunchKernelGGL((kb_update<T, LX, NT, CG_DISP>), rows, dim3(NT), 0, s, slots, rb,
                                 nbc, i, K.twx);
            if (modes & (1u << CG_FIXED))
              hipLaunchKernelGGL((kb_update<T, LX, NT, CG_FIXED>), rows, dim3(NT), 0, s, slots,
                                 rb, nbc, i, K.twx);
            hipLaunchKernelGGL((kb_column<T, LY, WW, CT>), cols, dim3(CT), 0, s, slots, nbc,
                               g.Lx, g.kpitch, K.twy);
            if (modes & (1u << CG_DISP))
              hipLaunchKernelGGL((kb_gap<T, LX, NT, CG_DISP>), rows, dim3(NT), 0, s, slots, rb, i,
                                 K.twx);
            if (modes & (1u << CG_FIXED))
              hipLaunchKernelGGL((kb_gap<T, LX, NT, CG_FIXED>), rows, dim3(NT), 0, s, slots, rb,
                                 i, K.twx);
            if (modes & (1u << CG_DISP))
              hipLaunchKernelGGL((kb_direction<T, LX, NT, CG_DISP>), rows, dim3(NT), 0, s, slots,
                                 rb, i, K.twx);
            if (modes & (1u << CG_FIXED))
              hipLaunchKernelGGL((kb_direction<T, LX, NT, CG_FIXED>), rows, dim3(NT), 0, s, slots,
                                 rb, i, K.twx);
            hipLaunchKernelGGL((kb_energy<T, LY, WW, CT>), cols, dim3(CT), 0, s, slots, nbc, g.Lx,
                               g.kpitch, K.twy);
            e = hipGetLastError();
          }
          return e;
        }
      });
    });
  });
}

}  // namespace bem
