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
      // The forward lane-pair step, the multiply and the inverse lane-pair
      // step in one exchange.  Lane (k1, h), register r holds E (h = 0) or O
      // (h = 1) of frequencies f_lo = k1 + 32 r and f_hi = f_lo + 1024; with
      // w = w_64^r and K_lo, K_hi the kernel spectrum there,
      //   X_lo = E + w O, X_hi = E - w O,  Y = K X,
      //   h = 0 keeps Y_lo + Y_hi        = A E + D (w O),
      //   h = 1 keeps (Y_lo - Y_hi) w^-1 = A O + D (conj(w) E),
      // A = K_lo + K_hi, D = K_lo - K_hi: each lane needs its partner's
      // value and kernel weight only.  The folded spectrum index runs as
      // kq0 + 64 r (h = 0) or kq0 - 64 r (h = 1).
      const float* Kc = KT + (size_t)c * kpitch;
      const int k1 = lane >> 1, h = lane & 1;
      const float sg = h ? -1.f : 1.f;
      int kq = h ? LY - 2 * k1 - parity : 2 * k1 + parity;
      const int dk = h ? -64 : 64;
      // all weights in flight at once (loaded inside the loop below, each
      // would be waited for before the next is issued)
      float kw[P];
#pragma unroll
      for (int r = 0; r < P; ++r) {
        kw[r] = Kc[kq];
        kq += dk;
      }
#pragma unroll
      for (int r = 0; r < P; ++r) {
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
    if (Stage::row(j) < ny) S[(size_t)Stage::row(j) * lx + c0 + Stage::col(j)] = y[j];
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

}  // namespace bem
