// Fused column sweep (column FFT x kernel spectrum x inverse FFT) on wave
// FFTs, FP32, Ly = 64 P with P in {32, 64}.
//
// A workgroup owns NC adjacent spectrum columns and runs 2 NC waves: for
// column j, wave 2j transforms the even-bin half (DFT of x) and wave 2j+1
// the odd-bin half (DFT of x w^n) of the My-point pruned transform (see
// conv_kernels.h).  Steps: (1) the NC columns are staged through LDS with
// coalesced row-segment loads; (2) each wave takes its column in the time
// layout (lane l, register m = row l + 64 m); (3) forward wave FFT; (4)
// multiply by the kernel spectrum at each register's frequency; column 0
// (packed DC / Nyquist) pairs bins k and -k through LDS; (5) inverse wave
// FFT; (6) the odd-half wave hands conj(w^n) o[n] to its partner through
// LDS, the even-half wave adds it; (7) coalesced row-segment stores.
// Workgroup barriers only around the shared staging and combine steps; the
// transposes use each wave's private region.
#pragma once
#include "conv_kernels.h"
#include "wave_fft.h"

namespace bem {

// Column cc of a workgroup's group is staged in the even region 2 cc, offset
// by 8 cc elements: the regions are a multiple of 32 banks apart, and the
// staging copy hands adjacent lanes adjacent columns of one row, which
// without the offset would all hit the same bank.
template <int P>
__device__ __forceinline__ int col_stage_base(int cc) {
  return 2 * cc * wave_region<P>() + 8 * cc;
}

// The forward lane-pair step, the multiplication by the real kernel weights
// and the inverse lane-pair step of a P = 32 wave FFT, in one exchange.
// Lane (k1, h), register r holds E (h = 0) or O (h = 1) of frequencies f_lo =
// k1 + 32 r and f_hi = f_lo + 1024; with w = w_64^r and K_lo, K_hi the
// weights there,
//   X_lo = E + w O, X_hi = E - w O,  Y = K X,
//   h = 0 keeps Y_lo + Y_hi        = A E + D (w O),
//   h = 1 keeps (Y_lo - Y_hi) w^-1 = A O + D (conj(w) E),
// A = K_lo + K_hi, D = K_lo - K_hi: each lane needs its partner's value and
// weight only.  The weight of register r is Kc[kq + r dk].
__device__ __forceinline__ void pair_multiply_pair(cplx<float> (&v)[32],
                                                   const float* __restrict__ Kc, int kq, int dk,
                                                   int lane) {
  const float sg = (lane & 1) ? -1.f : 1.f;
  // all weights in flight at once (loaded inside the loop below, each would
  // be waited for before the next is issued)
  float kw[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    kw[r] = Kc[kq];
    kq += dk;
  }
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const float ko = kw[r];
    const float kp = lane_xor1(ko);
    const float A = ko + kp, D = sg * (ko - kp);
    const cplx<float> b = {lane_xor1(v[r].x), lane_xor1(v[r].y)};
    // b w (h = 0) or b conj(w) (h = 1), w = exp(-2 pi i r / 64)
    cplx<float> tb = b;
    const int t = 2 * r;
    if (t == 32) {
      tb = {sg * b.y, -sg * b.x};
    } else if (t != 0) {
      const float cs = (float)cos128(t), sn = sg * (float)(-sin128(t));
      tb = {b.x * cs - b.y * sn, b.x * sn + b.y * cs};
    }
    v[r] = {A * v[r].x + D * tb.x, A * v[r].y + D * tb.y};
  }
}

template <int LY, int NC>
__global__ __launch_bounds__(128 * NC) void k_col_conv_w(cplx<float>* __restrict__ S, int lx,
                                                         int ny, const float* __restrict__ KT,
                                                         int kpitch,
                                                         const cplx<float>* __restrict__ tw,
                                                         const cplx<float>* __restrict__ twl,
                                                         const int* __restrict__ done) {
  constexpr int P = LY / 64;
  constexpr int REG = wave_region<P>();
  constexpr int NT = 128 * NC;
  static_assert(LY + 8 * (NC - 1) <= REG, "staged column fits its region");
  __shared__ cplx<float> lds[2 * NC * REG];
  if (done && *done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jc = wv >> 1, parity = wv & 1;
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * NC;
  const int c = c0 + jc;
  cplx<float>* reg = lds + wv * REG;

  // (1) stage the NC columns (rows < LY; zero beyond ny) into the even regions
  using Stage = ColStage<float, LY, NC, NT>;
  {
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j) lds[col_stage_base<P>(Stage::col(j)) + Stage::row(j)] = st.x[j];
  }
  __syncthreads();
  // (2) time layout
  cplx<float> v[P];
  const cplx<float>* src = lds + col_stage_base<P>(jc);
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = src[lane + 64 * m];
  __syncthreads();
  if (parity) {
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = cmul(v[m], tw[lane + 64 * m]);
  }
  // (3) forward transform up to its lane-pair step
  wave_fft_fwd_core<float, P>(v, reg, twl, lane);
  // (4) spectrum multiply; K(ky) is even: K(ky) = K(2 LY - ky)
  if constexpr (P == 32) {
    if (c != 0) {
      // lane (k1, h): the folded spectrum index runs as kq0 + 64 r (h = 0)
      // or kq0 - 64 r (h = 1)
      const int k1 = lane >> 1, h = lane & 1;
      pair_multiply_pair(v, KT + (size_t)c * kpitch, h ? LY - 2 * k1 - parity : 2 * k1 + parity,
                         h ? -64 : 64, lane);
    } else {
      // packed column 0: Z'[k] = ((K0+K1)/2) Z[k] + ((K0-K1)/2) conj(Z[-k]);
      // bins k and -k of one parity half sit in different lanes, so swap
      // via the wave's LDS region
      wave_fwd_pair<float>(v, lane);
      const float* K0 = KT;
      const float* K1 = KT + (size_t)lx * kpitch;
#pragma unroll
      for (int r = 0; r < P; ++r) reg[wave_freq<P>(lane, r)] = v[r];
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int f = wave_freq<P>(lane, r);
        const int fp = parity ? (LY - 1 - f) : ((LY - f) & (LY - 1));
        const cplx<float> z1 = reg[fp];
        const int ky = 2 * f + parity;
        const int kq = ky <= LY ? ky : 2 * LY - ky;
        const float a = 0.5f * (K0[kq] + K1[kq]), b = 0.5f * (K0[kq] - K1[kq]);
        v[r] = {a * v[r].x + b * z1.x, a * v[r].y - b * z1.y};
      }
      wave_lds_sync();
      wave_inv_pair<float>(v, lane);
    }
  } else {
    if (c != 0) {
      const float* Kc = KT + (size_t)c * kpitch;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int ky = 2 * wave_freq<P>(lane, r) + parity;
        const int kq = ky <= LY ? ky : 2 * LY - ky;
        v[r] = cscale(v[r], Kc[kq]);
      }
    } else {
      const float* K0 = KT;
      const float* K1 = KT + (size_t)lx * kpitch;
#pragma unroll
      for (int r = 0; r < P; ++r) reg[wave_freq<P>(lane, r)] = v[r];
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int f = wave_freq<P>(lane, r);
        const int fp = parity ? (LY - 1 - f) : ((LY - f) & (LY - 1));
        const cplx<float> z1 = reg[fp];
        const int ky = 2 * f + parity;
        const int kq = ky <= LY ? ky : 2 * LY - ky;
        const float a = 0.5f * (K0[kq] + K1[kq]), b = 0.5f * (K0[kq] - K1[kq]);
        v[r] = {a * v[r].x + b * z1.x, a * v[r].y - b * z1.y};
      }
      wave_lds_sync();
    }
  }
  // (5) inverse transform after its lane-pair step
  wave_fft_inv_core<float, P>(v, reg, twl, lane);
  // (6) combine the two halves: y[n] = e[n] + conj(w^n) o[n]
  if (parity) {
#pragma unroll
    for (int m = 0; m < P; ++m) reg[lane + 64 * m] = cmulc(v[m], tw[lane + 64 * m]);
  }
  __syncthreads();
  if (!parity) {
    const cplx<float>* o = reg + REG;
    cplx<float>* dst = lds + col_stage_base<P>(jc);
#pragma unroll
    for (int m = 0; m < P; ++m) dst[lane + 64 * m] = cadd(v[m], o[lane + 64 * m]);
  }
  __syncthreads();
  // (7) all LDS reads of the thread, then the stores of rows < ny
  cplx<float> y[Stage::CNT];
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j) y[j] = lds[col_stage_base<P>(Stage::col(j)) + Stage::row(j)];
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j)
    if (Stage::row(j) < ny) S[Stage::at(j, lx, c0)] = y[j];
}

}  // namespace bem

namespace bem {

// Forward wave-FFT column transform and the spectral energy
// sum_k KT(k) |T(k)|^2 (see k_col_energy): the first half of k_col_conv_w,
// then, per register, the weight of its frequency instead of the multiply.
// One FP64 partial per workgroup into part[blockIdx.x].
template <int LY, int NC>
__global__ __launch_bounds__(128 * NC) void k_col_energy_w(const cplx<float>* __restrict__ S,
                                                           int lx, int ny,
                                                           const float* __restrict__ KT,
                                                           int kpitch,
                                                           const cplx<float>* __restrict__ tw,
                                                           const cplx<float>* __restrict__ twl,
                                                           const int* __restrict__ done,
                                                           double* __restrict__ part) {
  constexpr int P = LY / 64;
  constexpr int REG = wave_region<P>();
  constexpr int NT = 128 * NC;
  static_assert(LY + 8 * (NC - 1) <= REG, "staged column fits its region");
  __shared__ cplx<float> lds[2 * NC * REG];
  __shared__ double red[NT / 64];
  if (done && *done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jc = wv >> 1, parity = wv & 1;
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * NC;
  const int c = c0 + jc;
  cplx<float>* reg = lds + wv * REG;
  {
    using Stage = ColStage<float, LY, NC, NT>;
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j) lds[col_stage_base<P>(Stage::col(j)) + Stage::row(j)] = st.x[j];
  }
  __syncthreads();
  cplx<float> v[P];
  const cplx<float>* src = lds + col_stage_base<P>(jc);
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = src[lane + 64 * m];
  __syncthreads();
  if (parity) {
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = cmul(v[m], tw[lane + 64 * m]);
  }
  wave_fft_fwd<float, P>(v, reg, twl, lane);
  double e = 0.0;
  if (c != 0) {
    const float* Kc = KT + (size_t)c * kpitch;
    if constexpr (P == 32) {
      const int k1 = lane >> 1, h = lane & 1;
      int kq = h ? LY - 2 * k1 - parity : 2 * k1 + parity;
      const int dk = h ? -64 : 64;
      float kw[P];   // all weights in flight at once
#pragma unroll
      for (int r = 0; r < P; ++r) {
        kw[r] = Kc[kq];
        kq += dk;
      }
#pragma unroll
      for (int r = 0; r < P; ++r) e += energy_term(v[r], kw[r]);
    } else {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int ky = 2 * wave_freq<P>(lane, r) + parity;
        e += energy_term(v[r], Kc[ky <= LY ? ky : 2 * LY - ky]);
      }
    }
  } else {
    // packed column 0: the partner bin -ky sits in another lane
#pragma unroll
    for (int r = 0; r < P; ++r) reg[wave_freq<P>(lane, r)] = v[r];
    wave_lds_sync();
    const float* K1 = KT + (size_t)lx * kpitch;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int f = wave_freq<P>(lane, r);
      const cplx<float> zm = reg[parity ? (LY - 1 - f) : ((LY - f) & (LY - 1))];
      const int ky = 2 * f + parity;
      const int kq = ky <= LY ? ky : 2 * LY - ky;
      e += energy_packed(v[r], zm, KT[kq], K1[kq]);
    }
  }
  e = block_sum<NT>(e, red);
  if (threadIdx.x == 0) part[blockIdx.x] = e;
}

// Column sweeps at Ly = 4096 (My = 8192) on the same 2048-point wave FFTs.
// Each of the two My/2-point halves of the pruned transform (even bins: DFT
// of x; odd bins: DFT of x w_My^n, n < 4096) is split once more by decimation
// in frequency into the 2048-point DFTs of
//   y0[n] = x[n] + x[n + 2048]                 (bins 2 j of the half)
//   y1[n] = (x[n] - x[n + 2048]) w_4096^n      (bins 2 j + 1),
// so a column takes four waves: quarter q = 2 half + par transforms y_half
// of the parity-par half and holds the My-point bins ky = 4 f + 2 half + par
// (f: its 2048-point frequency).  The inverse runs the same steps backwards;
// with a, b, c, d the inverse quarters (q = 0, 2, 1, 3) after their
// twiddles 1, conj(w_4096^n), conj(w_8192^n), conj(w_8192^3n),
//   out[n]        = a + b + c + d
//   out[n + 2048] = (a - b) + i (c - d),   n < 2048.
// The twiddles come from the My-point table (w_4096^n = w_8192^2n) and the
// wave table of Ly = 4096 read at every other k1.  Two columns per
// workgroup (eight waves, 133 KB of LDS); column cc is staged in regions
// 4 cc and 4 cc + 1.

// Column cc is staged across regions 4 cc and 4 cc + 1, offset by 16 cc
// elements: a half-wave of the staging copy holds rows 0..15 of both columns
// (row pairs, spec_idx order), which then fall on disjoint LDS banks.
template <int NC>
__device__ __forceinline__ int quarter_stage_base(int cc) {
  return 4 * cc * wave_region<32>() + 16 * cc;
}

// Quarter input for wave (par, half), n = lane + 64 m, from the staged column:
//   par = 0: y0 = xa + xb,              y1 = (xa - xb) w^2n
//   par = 1: y0 = (xa - i xb) w^n,      y1 = (xa + i xb) w^3n
// with xa = x[n], xb = x[n + 2048], w = w_8192 (w^2048 = -i folds the odd
// half's pre-twiddle of xb into the combination), i.e. one twiddle
// w^((par + 2 half) n) per value.
__device__ __forceinline__ void quarter_input(cplx<float> (&v)[32], const cplx<float>* src,
                                              const cplx<float>* __restrict__ tw, int lane,
                                              int par, int half) {
  const int e = par + 2 * half;
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    const int n = lane + 64 * m;
    const cplx<float> xa = src[n], xb = src[n + 2048];
    cplx<float> y;
    if (par == 0)
      y = half ? csub(xa, xb) : cadd(xa, xb);
    else
      y = half ? cplx<float>{xa.x - xb.y, xa.y + xb.x} : cplx<float>{xa.x + xb.y, xa.y - xb.x};
    v[m] = e ? cmul(y, tw[e * n]) : y;
  }
}

// Packed column 0 (DC in re, Nyquist in im): the partner bin -ky of a bin
// sits in another wave of the column, so the column's spectrum passes
// through its four LDS regions in natural order (arr[ky], ky < 8192).  All
// waves of the workgroup take part in the barriers.
__device__ __forceinline__ int quarter_bin(int lane, int r, int par, int half) {
  return 4 * wave_freq<32>(lane, r) + 2 * half + par;
}
__device__ __forceinline__ int fold8192(int ky) { return ky <= 4096 ? ky : 8192 - ky; }

template <int NC>
__global__ __launch_bounds__(256 * NC) void k_col_conv_q(cplx<float>* __restrict__ S, int lx,
                                                         int ny, const float* __restrict__ KT,
                                                         int kpitch,
                                                         const cplx<float>* __restrict__ tw,
                                                         const cplx<float>* __restrict__ twl,
                                                         const int* __restrict__ done) {
  constexpr int LY = 4096, P = 32, REG = wave_region<P>();
  constexpr int NT = 256 * NC;
  static_assert(LY + 16 * (NC - 1) <= 2 * REG && 8192 <= 4 * REG, "column regions");
  __shared__ cplx<float> lds[4 * NC * REG];
  if (done && *done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jc = wv >> 2, q = wv & 3, par = q & 1, half = q >> 1;
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * NC;
  const int c = c0 + jc;
  cplx<float>* reg = lds + wv * REG;
  using Stage = ColStage<float, LY, NC, NT>;
  {
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j)
      lds[quarter_stage_base<NC>(Stage::col(j)) + Stage::row(j)] = st.x[j];
  }
  __syncthreads();
  cplx<float> v[P];
  quarter_input(v, lds + quarter_stage_base<NC>(jc), tw, lane, par, half);
  __syncthreads();   // the regions become transpose space
  wave_fft_fwd_core<float, P, 128>(v, reg, twl, lane);
  const int k1 = lane >> 1, h = lane & 1;
  if (c != 0) {
    const int kq0 = 4 * k1 + 2 * half + par;
    pair_multiply_pair(v, KT + (size_t)c * kpitch, h ? LY - kq0 : kq0, h ? -128 : 128, lane);
  }
  if (c0 == 0) {
    cplx<float>* arr = lds + 4 * jc * REG;
    __syncthreads();   // every forward transpose of the workgroup is done
    if (c == 0) {
      wave_fwd_pair<float>(v, lane);
#pragma unroll
      for (int r = 0; r < P; ++r) arr[quarter_bin(lane, r, par, half)] = v[r];
    }
    __syncthreads();
    if (c == 0) {
      const float* K1 = KT + (size_t)lx * kpitch;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int ky = quarter_bin(lane, r, par, half);
        const cplx<float> z1 = arr[(8192 - ky) & 8191];
        const int kq = fold8192(ky);
        const float a = 0.5f * (KT[kq] + K1[kq]), b = 0.5f * (KT[kq] - K1[kq]);
        v[r] = {a * v[r].x + b * z1.x, a * v[r].y - b * z1.y};
      }
    }
    __syncthreads();   // before the inverse transposes reuse the regions
    if (c == 0) wave_inv_pair<float>(v, lane);
  }
  wave_fft_inv_core<float, P, 128>(v, reg, twl, lane);
  // own quarter times its twiddle conj(w_8192^(par n + 2 half n))
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int n = lane + 64 * m;
    reg[n] = cmulc(v[m], tw[(par + 2 * half) * n]);
  }
  __syncthreads();
  cplx<float> y[Stage::CNT];
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j) {
    const int cc = Stage::col(j), row = Stage::row(j), nn = row & 2047;
    const cplx<float>* R = lds + 4 * cc * REG;
    const cplx<float> a = R[nn], cq = R[REG + nn], b = R[2 * REG + nn], d = R[3 * REG + nn];
    if (row < 2048) {
      y[j] = {a.x + b.x + cq.x + d.x, a.y + b.y + cq.y + d.y};
    } else {
      // (a - b) + i (c - d)
      y[j] = {a.x - b.x - (cq.y - d.y), a.y - b.y + (cq.x - d.x)};
    }
  }
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j)
    if (Stage::row(j) < ny) S[Stage::at(j, lx, c0)] = y[j];
}

// Forward quarter transforms and the spectral energy sum_k KT(k) |T(k)|^2
// (see k_col_energy).  One FP64 partial per workgroup into part[blockIdx.x].
template <int NC>
__global__ __launch_bounds__(256 * NC) void k_col_energy_q(const cplx<float>* __restrict__ S,
                                                           int lx, int ny,
                                                           const float* __restrict__ KT,
                                                           int kpitch,
                                                           const cplx<float>* __restrict__ tw,
                                                           const cplx<float>* __restrict__ twl,
                                                           const int* __restrict__ done,
                                                           double* __restrict__ part) {
  constexpr int LY = 4096, P = 32, REG = wave_region<P>();
  constexpr int NT = 256 * NC;
  static_assert(LY + 16 * (NC - 1) <= 2 * REG && 8192 <= 4 * REG, "column regions");
  __shared__ cplx<float> lds[4 * NC * REG];
  __shared__ double red[NT / 64];
  if (done && *done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jc = wv >> 2, q = wv & 3, par = q & 1, half = q >> 1;
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * NC;
  const int c = c0 + jc;
  cplx<float>* reg = lds + wv * REG;
  {
    using Stage = ColStage<float, LY, NC, NT>;
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j)
      lds[quarter_stage_base<NC>(Stage::col(j)) + Stage::row(j)] = st.x[j];
  }
  __syncthreads();
  cplx<float> v[P];
  quarter_input(v, lds + quarter_stage_base<NC>(jc), tw, lane, par, half);
  __syncthreads();
  wave_fft_fwd_core<float, P, 128>(v, reg, twl, lane);
  wave_fwd_pair<float>(v, lane);
  double e = 0.0;
  const int k1 = lane >> 1, h = lane & 1;
  if (c != 0) {
    const float* Kc = KT + (size_t)c * kpitch;
    const int kq0 = 4 * k1 + 2 * half + par;
    int kq = h ? LY - kq0 : kq0;
    const int dk = h ? -128 : 128;
    float kw[P];   // all weights in flight at once
#pragma unroll
    for (int r = 0; r < P; ++r) {
      kw[r] = Kc[kq];
      kq += dk;
    }
#pragma unroll
    for (int r = 0; r < P; ++r) e += energy_term(v[r], kw[r]);
  }
  if (c0 == 0) {
    cplx<float>* arr = lds + 4 * jc * REG;
    __syncthreads();
    if (c == 0) {
#pragma unroll
      for (int r = 0; r < P; ++r) arr[quarter_bin(lane, r, par, half)] = v[r];
    }
    __syncthreads();
    if (c == 0) {
      const float* K1 = KT + (size_t)lx * kpitch;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int ky = quarter_bin(lane, r, par, half);
        const int kq = fold8192(ky);
        e += energy_packed(v[r], arr[(8192 - ky) & 8191], KT[kq], K1[kq]);
      }
    }
  }
  e = block_sum<NT>(e, red);
  if (threadIdx.x == 0) part[blockIdx.x] = e;
}

}  // namespace bem

