// Row sweeps of Eq. 13 on wave FFTs, FP32, Lx = 64 P with P = 32.
//
// Same arithmetic as k_row_r2c / k_row_c2r (conv_kernels.h): two real rows
// packed as one complex row, the Mx-point transform of a row that is zero on
// [Lx, Mx) split into the Lx-point transforms of its even bins (DFT of z)
// and odd bins (DFT of z w^n).  Here a workgroup of two waves owns one row
// pair and each half is one wave-level FFT (wave_fft.h): wave 0 the even
// bins, wave 1 the odd bins.  Compared with the LDS Stockham passes this
// keeps the data in registers apart from one transpose, so the transform
// costs about half the VALU and LDS work.
//
// LDS: one region of P x 66 complex values per wave.  The row pair passes
// through region 0 in natural order on the way in (R2C) or out (C2R); each
// wave's spectrum half sits in its own region in natural frequency order for
// the untangling (R2C) or the Hermitian completion (C2R).  The prologue /
// epilogue functors are those of the Stockham sweeps, with NTHR = 128.
#pragma once
#include <type_traits>

#include "conv_kernels.h"
#include "launch.h"
#include "wave_fft.h"

namespace bem {

constexpr int kRowWaveThreads = 128;

template <int L, class Pro>
__global__ __launch_bounds__(kRowWaveThreads, 2) void k_row_r2c_w(Pro pro_arg,
                                                               cplx<float>* __restrict__ S, int nx,
                                                               int ny,
                                                               const cplx<float>* __restrict__ tw,
                                                               const cplx<float>* __restrict__ twl) {
  constexpr int NTHR = kRowWaveThreads;
  constexpr int P = L / 64;
  constexpr int REG = wave_region<P>();
  constexpr int PER = L / NTHR;
  static_assert(P == 32 && PER * NTHR == L, "row wave FFT shape");
  __shared__ cplx<float> lds[2 * REG];
  __shared__ double red[64];
  Pro pro = pro_arg;
  if (!pro.template issue<NTHR>()) return;
  const int ya = 2 * blockIdx.x, yb = ya + 1;
  const bool hasb = yb < ny;
  pro.template fetch<NTHR>(ya, yb, hasb, nx);
  if (!pro.template decide<NTHR>(red, blockIdx.x)) return;
  float va[PER], vb[PER];
  pro.template make<NTHR>(ya, yb, hasb, nx, va, vb);
#pragma unroll
  for (int q = 0; q < PER; ++q) lds[threadIdx.x + q * NTHR] = {va[q], vb[q]};
  pro.template commit<NTHR>(ya, yb, hasb, nx, va, vb);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cplx<float> v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = lds[lane + 64 * m];
  if (wv) {
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = cmul(v[m], tw[lane + 64 * m]);
  }
  __syncthreads();   // region 0 becomes wave 0's transpose region
  cplx<float>* reg = lds + wv * REG;
  wave_fft_fwd<float, P>(v, reg, twl, lane);
  // the half spectrum in natural order (the transpose reads of this wave
  // precede these writes in its LDS instruction order)
#pragma unroll
  for (int r = 0; r < P; ++r) reg[wave_freq<P>(lane, r)] = v[r];
  __syncthreads();
  // untangle A (row a) and B (row b) from Z[k] and conj Z[Mx - k]: even k
  // from the even half E, odd k from the odd half O; slot 0 packs A[0], A[Lx]
  const cplx<float>* E = lds;
  const cplx<float>* O = lds + REG;
  cplx<float> Z[PER], Zp[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int k = threadIdx.x + j * NTHR, kp = k >> 1;
    if (k & 1) {
      Z[j] = O[kp];
      Zp[j] = O[L - 1 - kp];
    } else {
      Z[j] = E[kp];
      Zp[j] = E[(L - kp) & (L - 1)];
    }
  }
  if (threadIdx.x == 0) Zp[0] = E[L / 2];   // k = 0: Z[Lx] for the packed slot
  cplx<float>* Sp = S + spec_idx(ya, 0, L);   // the pair's block, rows interleaved
  const float half = 0.5f;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int k = threadIdx.x + j * NTHR;
    cplx<float> a, b;
    if (k == 0) {
      a = {Z[j].x, Zp[j].x};
      b = {Z[j].y, Zp[j].y};
    } else {
      a = {half * (Z[j].x + Zp[j].x), half * (Z[j].y - Zp[j].y)};
      b = {half * (Z[j].y + Zp[j].y), half * (Zp[j].x - Z[j].x)};
    }
    store_pair(Sp + 2 * k, a, b);
  }
  pro.template finish<NTHR>(red, blockIdx.x);
}

template <int L, class Epi>
__global__ __launch_bounds__(kRowWaveThreads, 2) void k_row_c2r_w(const cplx<float>* __restrict__ S,
                                                               int nx, int ny,
                                                               const cplx<float>* __restrict__ tw,
                                                               const cplx<float>* __restrict__ twl,
                                                               Epi epi_arg) {
  constexpr int NTHR = kRowWaveThreads;
  constexpr int P = L / 64;
  constexpr int REG = wave_region<P>();
  constexpr int PER = L / NTHR;
  static_assert(P == 32 && PER * NTHR == L, "row wave FFT shape");
  __shared__ cplx<float> lds[2 * REG];
  __shared__ double red[64];
  Epi epi = epi_arg;
  if (!epi.template begin<NTHR>(red)) return;
  const int ya = 2 * blockIdx.x, yb = ya + 1;
  const bool hasb = yb < ny;
  const cplx<float>* Sp = S + spec_idx(ya, 0, L);   // the pair's block, rows interleaved
  cplx<float> Av[PER], Bv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const cpair<float> ab = load_pair(Sp + 2 * (threadIdx.x + j * NTHR));
    Av[j] = ab.a;
    Bv[j] = hasb ? ab.b : ab.a;
  }
  // the epilogue's loads stay in flight during the transform
  epi.template prefetch<NTHR>(ya, yb, hasb, nx);
  epi.template ready<NTHR>(red);
  // Hermitian completion: Z = A + i B at k and conj(A) + i conj(B) at Mx - k,
  // scattered into the even half (region 0) and the odd half (region 1)
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int k = threadIdx.x + j * NTHR;
    const cplx<float> A = Av[j];
    const cplx<float> B = cscale(Bv[j], hasb ? 1.f : 0.f);
    if (k == 0) {
      lds[0] = {A.x, B.x};
      lds[L / 2] = {A.y, B.y};
    } else {
      const int km = 2 * L - k;
      lds[(k & 1) * REG + (k >> 1)] = {A.x - B.y, A.y + B.x};
      lds[(km & 1) * REG + (km >> 1)] = {A.x + B.y, B.x - A.y};
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cplx<float>* reg = lds + wv * REG;
  cplx<float> v[P];
#pragma unroll
  for (int r = 0; r < P; ++r) v[r] = reg[wave_freq<P>(lane, r)];
  wave_lds_sync();
  wave_fft_inv<float, P>(v, reg, twl, lane);
  // time domain: even half e[n] as is, odd half as conj(w^n) o[n]
  if (wv) {
#pragma unroll
    for (int m = 0; m < P; ++m) reg[lane + 64 * m] = cmulc(v[m], tw[lane + 64 * m]);
  } else {
#pragma unroll
    for (int m = 0; m < P; ++m) reg[lane + 64 * m] = v[m];
  }
  __syncthreads();
  float va[PER], vb[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int n = threadIdx.x + q * NTHR;
    const cplx<float> z = cadd(lds[n], lds[REG + n]);
    const bool in = n < nx;
    va[q] = in ? z.x : 0.f;
    vb[q] = in ? z.y : 0.f;
  }
  epi.template consume<NTHR>(ya, yb, hasb, nx, va, vb);
  epi.template finish<NTHR>(red, blockIdx.x);
}

// Row sweep launchers: the wave kernels when WAVE is set (FP32, Lx = 2048,
// unless BEM_ROW_WAVE=0), else the Stockham kernels.  make(std::integral_constant<int, PER>)
// returns the prologue / epilogue functor for PER elements per thread and
// row.  A wave row kernel runs 8 waves per CU (its LDS use per row pair is
// that of the Stockham kernel, over 2 waves instead of 4), so a prologue or
// epilogue with much work of its own can run slower there despite the
// cheaper transform; the caller chooses.
template <typename T, bool WAVE, class Make>
hipError_t launch_row_r2c(const Geom& g, const SpecView<T>& K, cplx<T>* S, Make&& make,
                          hipStream_t s) {
  const int nrp = (g.ny + 1) / 2;
  if constexpr (WAVE && std::is_same<T, float>::value) {
    if (row_wave(g)) {
      constexpr int PER = 2048 / kRowWaveThreads;
      auto pro = make(std::integral_constant<int, PER>());
      hipLaunchKernelGGL((k_row_r2c_w<2048, decltype(pro)>), dim3(nrp), dim3(kRowWaveThreads), 0,
                         s, pro, S, g.nx, g.ny, K.twx, K.twlx);
      return hipGetLastError();
    }
  }
  return dispatch_L(g.Lx, [&](auto LX) -> hipError_t {
    constexpr int L = decltype(LX)::value;
    constexpr int NT = row_threads(L);
    constexpr int PER = row_per<L, NT>();
    auto pro = make(std::integral_constant<int, PER>());
    hipLaunchKernelGGL((k_row_r2c<T, L, NT, decltype(pro)>), dim3(nrp), dim3(NT), 0, s, pro, S,
                       g.nx, g.ny, K.twx);
    return hipGetLastError();
  });
}

template <typename T, bool WAVE, class Make>
hipError_t launch_row_c2r(const Geom& g, const SpecView<T>& K, const cplx<T>* S, Make&& make,
                          hipStream_t s) {
  const int nrp = (g.ny + 1) / 2;
  if constexpr (WAVE && std::is_same<T, float>::value) {
    if (row_wave(g)) {
      constexpr int PER = 2048 / kRowWaveThreads;
      auto epi = make(std::integral_constant<int, PER>());
      hipLaunchKernelGGL((k_row_c2r_w<2048, decltype(epi)>), dim3(nrp), dim3(kRowWaveThreads), 0,
                         s, S, g.nx, g.ny, K.twx, K.twlx, epi);
      return hipGetLastError();
    }
  }
  return dispatch_L(g.Lx, [&](auto LX) -> hipError_t {
    constexpr int L = decltype(LX)::value;
    constexpr int NT = row_threads(L);
    constexpr int PER = row_per<L, NT>();
    auto epi = make(std::integral_constant<int, PER>());
    hipLaunchKernelGGL((k_row_c2r<T, L, NT, decltype(epi)>), dim3(nrp), dim3(NT), 0, s, S, g.nx,
                       g.ny, K.twx, epi);
    return hipGetLastError();
  });
}

}  // namespace bem
