// Wave-level FFT of length L = 64 P (P = 32 or 64) for the column sweep of
// Eq. 13: one wave64 owns one sequence, P points per lane, with a single
// LDS transpose per direction.
//
// With n = l + 64 m (lane l, register m) and k = k1 + P k2:
//   forward  A[l][k1] = sum_m x[l + 64 m] w_P^(m k1)          (registers)
//            B[l][k1] = A[l][k1] w_L^(l k1)                     (twiddle)
//            X[k1 + P k2] = sum_l B[l][k1] w_64^(l k2)          (after transpose)
// The 64-point transform over l runs in registers after the transpose: for
// P = 64 each lane owns one k1 and all 64 values of l; for P = 32 two lanes
// share a k1, each owning half of l (l = 2i + h), and a radix-2 step
// between the two lanes (DPP quad permutation) finishes it.  The output
// stays in this permuted order: lane (k1, h), register k2 holds frequency
// f = k1 + 32 (k2 + 32 h) (P = 32) or f = k1 + 64 k2 (P = 64).  The
// spectrum multiplication does not care about order, and the inverse runs
// the transposed algorithm (same stages in reverse, conjugate twiddles), so
// it reads the permuted order and returns y[l + 64 m] in natural order.
//
// Register DFTs (split radix) use constant twiddles (cosines of pi t / 64,
// exact quadrant symmetry); the inter-step twiddle w_L^(l k1) comes from a per-length table
// laid out [k1][lane], each entry rounded once from FP64.
#pragma once
#include "common.h"
#include "fft_lds.h"

namespace bem {

template <typename T, int P, int DIR>
__device__ __forceinline__ void reg_dft(cplx<T> (&v)[P]) {
  split_radix_dft<T, DIR, P>(v);
}

// v[k1] *= w_L^(lane k1) (DIR = -1) or its conjugate (DIR = +1).  twl is a
// table laid out [k1][lane]: twl[k1 * 64 + l] = exp(-2 pi i l k1 / L), each
// entry computed in FP64 and rounded once (coalesced across the wave).  With
// KS = 128 the table is that of length 2L, read at every other k1 (the same
// values: l (2 k1) / 2L = l k1 / L).
template <typename T, int P, int DIR, int KS = 64>
__device__ __forceinline__ void twiddle_lk1(cplx<T> (&v)[P], const cplx<T>* __restrict__ twl,
                                            int lane) {
#pragma unroll
  for (int k1 = 1; k1 < P; ++k1) {
    const cplx<T> w = twl[k1 * KS + lane];
    v[k1] = (DIR < 0) ? cmul(v[k1], w) : cmulc(v[k1], w);
  }
}

// Value of the partner lane (lane ^ 1): DPP quad permutation [1, 0, 3, 2].
// Every lane has a source, so the move needs no initialised old value (with
// update_dpp(0, ...) the compiler materialises the zero in an extra move).
__device__ __forceinline__ int lane_xor1_bits(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
}
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(lane_xor1_bits(__float_as_int(v)));
}
__device__ __forceinline__ double lane_xor1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor1_bits((int)(b & 0xffffffff));
  const int hi = lane_xor1_bits((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row pitch (complex elements) of a wave's transpose region: 64 values and
// padding.  For P = 32 the transposed access (lane (k1, h) at row k1, column
// 2 i + h) spreads a half-wave over distinct banks only with a pitch of 66
// (132 dwords, 4 mod 32); with 65 the lanes (k1, 1) and (k1 + 1, 0) share
// banks.  For P = 64 (lane l at row l) 65 suffices.
template <int P>
__host__ __device__ constexpr int wave_pitch() { return P == 32 ? 66 : 65; }

// LDS words per wave region (complex elements): P rows of wave_pitch
template <int P>
__host__ __device__ constexpr int wave_region() { return P * wave_pitch<P>(); }

// The transpose regions are private to a wave, so a wave-level ordering
// point suffices between writing a region and reading other lanes' values:
// LDS instructions of one wave execute in order, and the fences stop the
// compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Frequency index held by (lane, register r) after the forward transform.
template <int P>
__device__ __forceinline__ int wave_freq(int lane, int r) {
  if constexpr (P == 32) return (lane >> 1) + 32 * r + 1024 * (lane & 1);
  else return lane + 64 * r;
}

// Forward transform up to (not including) the lane-pair step of P = 32:
// register DFT, twiddle, transpose, register DFT.  `reg` is this wave's
// private LDS region (wave_region<P>()).
template <typename T, int P, int KS = 64>
__device__ __forceinline__ void wave_fft_fwd_core(cplx<T> (&v)[P], cplx<T>* reg,
                                                  const cplx<T>* __restrict__ twl, int lane) {
  static_assert(P == 32 || P == 64, "wave FFT sizes");
  constexpr int PT = wave_pitch<P>();
  reg_dft<T, P, -1>(v);
  twiddle_lk1<T, P, -1, KS>(v, twl, lane);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) reg[k1 * PT + lane] = v[k1];
  wave_lds_sync();
  if constexpr (P == 32) {
    const int k1 = lane >> 1, h = lane & 1;
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = reg[k1 * PT + 2 * i + h];
  } else {
#pragma unroll
    for (int i = 0; i < 64; ++i) v[i] = reg[lane * PT + i];
  }
  wave_lds_sync();
  reg_dft<T, P, -1>(v);
}

// Lane-pair step of the forward transform, P = 32 (h = 0: E, h = 1: O):
// X_lo = E + w O, X_hi = E - w O with w = w_64^k2.  The O lane multiplies
// by w before the exchange; each lane then adds (E) or subtracts (O) its own
// value from what it receives.
template <typename T>
__device__ __forceinline__ void wave_fwd_pair(cplx<T> (&v)[32], int lane) {
  const bool hi = lane & 1;
  const T sg = hi ? T(-1) : T(1);
#pragma unroll
  for (int k2 = 0; k2 < 32; ++k2) {
    const cplx<T> wv = mul_wn<T, -1>(v[k2], k2, 64);
    const cplx<T> x = hi ? wv : v[k2];
    const cplx<T> o = {lane_xor1(x.x), lane_xor1(x.y)};
    v[k2] = {o.x + sg * x.x, o.y + sg * x.y};
  }
}

// Forward transform.
template <typename T, int P>
__device__ __forceinline__ void wave_fft_fwd(cplx<T> (&v)[P], cplx<T>* reg,
                                             const cplx<T>* __restrict__ twl, int lane) {
  wave_fft_fwd_core<T, P>(v, reg, twl, lane);
  if constexpr (P == 32) wave_fwd_pair<T>(v, lane);
}

// Lane-pair step of the inverse transform, P = 32: h = 0 keeps
// X_lo + X_hi, h = 1 keeps (X_lo - X_hi) w^(-k2).
template <typename T>
__device__ __forceinline__ void wave_inv_pair(cplx<T> (&v)[32], int lane) {
  const bool hi = lane & 1;
  const T sg = hi ? T(-1) : T(1);
#pragma unroll
  for (int k2 = 0; k2 < 32; ++k2) {
    const cplx<T> o = {lane_xor1(v[k2].x), lane_xor1(v[k2].y)};
    const cplx<T> sum = {o.x + sg * v[k2].x, o.y + sg * v[k2].y};
    const cplx<T> tw = mul_wn<T, +1>(sum, k2, 64);
    v[k2] = hi ? tw : sum;
  }
}

// Inverse transform after the lane-pair step: register DFT, transpose,
// conjugate twiddle, register DFT; returns y[lane + 64 m] in v[m].
template <typename T, int P, int KS = 64>
__device__ __forceinline__ void wave_fft_inv_core(cplx<T> (&v)[P], cplx<T>* reg,
                                                  const cplx<T>* __restrict__ twl, int lane) {
  constexpr int PT = wave_pitch<P>();
  reg_dft<T, P, +1>(v);
  if constexpr (P == 32) {
    const int k1 = lane >> 1, h = lane & 1;
#pragma unroll
    for (int i = 0; i < 32; ++i) reg[k1 * PT + 2 * i + h] = v[i];
  } else {
#pragma unroll
    for (int i = 0; i < 64; ++i) reg[lane * PT + i] = v[i];
  }
  wave_lds_sync();
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) v[k1] = reg[k1 * PT + lane];
  wave_lds_sync();
  twiddle_lk1<T, P, +1, KS>(v, twl, lane);
  reg_dft<T, P, +1>(v);
}

// Inverse (unnormalised) transform from the permuted frequency layout back
// to y[lane + 64 m] in v[m].
template <typename T, int P>
__device__ __forceinline__ void wave_fft_inv(cplx<T> (&v)[P], cplx<T>* reg,
                                             const cplx<T>* __restrict__ twl, int lane) {
  if constexpr (P == 32) wave_inv_pair<T>(v, lane);
  wave_fft_inv_core<T, P>(v, reg, twl, lane);
}

}  // namespace bem
