// In-LDS Stockham FFT for power-of-two lengths: radix-8 passes, with one
// radix-2 or radix-4 pass where log2(L) is not a multiple of 3.
//
// The transform of Eq. 13 is the only place the method needs an FFT; these
// routines carry it.  A workgroup transforms NSEQ independent sequences of
// length L that sit in LDS at seq * STRIDE, element i at lds_idx<T>(i).  Each pass
// reads R points spaced L/R apart into registers, applies the twiddles
// w^(r k), does an R-point DFT and writes the R results Ns apart (Stockham
// auto-sort: natural order in and out, one LDS buffer, two barriers a pass).
//
// Twiddles come from a table tw[m] = exp(-2 pi i m / (2L)), m < 2L, computed
// once in FP64 from exact rational arguments and rounded once to T, so every
// twiddle carries a single rounding.  DIR = -1 forward (exp(-i...)),
// DIR = +1 inverse (exp(+i...), unnormalised).
#pragma once
#include "common.h"

namespace bem {

// multiply by -i (forward) or +i (inverse)
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

template <int DIR, typename T>
__device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cplx<T>* v) {
  cplx<T> s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
  cplx<T> s1 = cadd(v[1], v[3]), d1 = rot90<DIR>(csub(v[1], v[3]));
  v[0] = cadd(s0, s1);
  v[2] = csub(s0, s1);
  v[1] = cadd(d0, d1);
  v[3] = csub(d0, d1);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  // w8^k, w8 = exp(DIR i pi / 4)
  cplx<T> o1 = {h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x)};
  cplx<T> o2 = rot90<DIR>(o[2]);
  cplx<T> o3 = {h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// cos(pi t / 64), t = 0..32
__host__ __device__ constexpr double cos_q(int t) {
  constexpr double c[33] = {
      1.0, 0.9987954562051724, 0.9951847266721969, 0.989176509964781,
      0.9807852804032304, 0.970031253194544, 0.9569403357322088, 0.9415440651830208,
      0.9238795325112867, 0.9039892931234433, 0.881921264348355, 0.8577286100002721,
      0.8314696123025452, 0.8032075314806449, 0.773010453362737, 0.7409511253549591,
      0.7071067811865476, 0.6715589548470183, 0.6343932841636455, 0.5956993044924335,
      0.5555702330196023, 0.5141027441932217, 0.4713967368259978, 0.4275550934302822,
      0.38268343236508984, 0.33688985339222005, 0.29028467725446233, 0.24298017990326398,
      0.19509032201612833, 0.14673047445536175, 0.09801714032956077, 0.049067674327418126,
      0.0};
  return c[t];
}

// cos / sin of 2 pi t / 128 for any integer t, from the quadrant table
__host__ __device__ constexpr double cos128(int t) {
  t &= 127;
  return t <= 32 ? cos_q(t) : t <= 64 ? -cos_q(64 - t) : t <= 96 ? -cos_q(t - 64) : cos_q(128 - t);
}
__host__ __device__ constexpr double sin128(int t) { return cos128(t - 32); }

// y * w_N^j with w_N = exp(DIR 2 pi i / N), N <= 128, N | 128
template <typename T, int DIR>
__device__ __forceinline__ cplx<T> mul_wn(cplx<T> y, int j, int N) {
  const int t = (j * (128 / N)) & 127;
  if (t == 0) return y;
  if (t == 64) return {-y.x, -y.y};
  if (t == 32) return rot90<DIR>(y);
  if (t == 96) return rot90<-DIR>(y);
  const T c = (T)cos128(t), s = (T)(DIR * sin128(t));
  return {y.x * c - y.y * s, y.x * s + y.y * c};
}

// In-register DFT of N points, natural order in and out, by the split-radix
// decimation in time: with U the N/2-point DFT of the even samples and Z, Z'
// the N/4-point DFTs of x[4n + 1] and x[4n + 3],
//   X[k]          = U[k] + (w^k Z[k] + w^3k Z'[k])
//   X[k + N/2]    = U[k] - (w^k Z[k] + w^3k Z'[k])
//   X[k + N/4]    = U[k + N/4] + rot(w^k Z[k] - w^3k Z'[k])
//   X[k + 3N/4]   = U[k + N/4] - rot(w^k Z[k] - w^3k Z'[k])
// for k < N/4, w = exp(DIR 2 pi i / N), rot = multiplication by DIR i.
// Every index is a constant after unrolling; for N = 32 this takes 423
// VALU instructions against 452 for radix 2.
template <typename T, int DIR, int N>
__device__ __forceinline__ void split_radix_dft(cplx<T> (&x)[N]) {
  if constexpr (N == 2) {
    dft2<DIR>(x[0], x[1]);
  } else if constexpr (N == 4) {
    dft4<DIR>(x);
  } else if constexpr (N > 4) {
    cplx<T> u[N / 2], z[N / 4], zp[N / 4];
#pragma unroll
    for (int n = 0; n < N / 2; ++n) u[n] = x[2 * n];
#pragma unroll
    for (int n = 0; n < N / 4; ++n) {
      z[n] = x[4 * n + 1];
      zp[n] = x[4 * n + 3];
    }
    split_radix_dft<T, DIR, N / 2>(u);
    split_radix_dft<T, DIR, N / 4>(z);
    split_radix_dft<T, DIR, N / 4>(zp);
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
      const cplx<T> a = mul_wn<T, DIR>(z[k], k, N);
      const cplx<T> b = mul_wn<T, DIR>(zp[k], 3 * k, N);
      const cplx<T> sm = cadd(a, b), df = rot90<DIR>(csub(a, b));
      x[k] = cadd(u[k], sm);
      x[k + N / 2] = csub(u[k], sm);
      x[k + N / 4] = cadd(u[k + N / 4], df);
      x[k + 3 * N / 4] = csub(u[k + N / 4], df);
    }
  }
}

template <int DIR, int R, typename T>
__device__ __forceinline__ void dft(cplx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else split_radix_dft<T, DIR, R>(*reinterpret_cast<cplx<T>(*)[R]>(v));
}

// One Stockham pass: radix R, sub-transform length NS before the pass.
template <typename T, int L, int R, int NS, int DIR, int NSEQ, int NTHR, int STRIDE>
__device__ __forceinline__ void stockham_pass(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  constexpr int NB = L / R;
  constexpr int TOT = NB * NSEQ;
  constexpr int BPT = (TOT + NTHR - 1) / NTHR;
  constexpr int TWS = (2 * L) / (NS * R);  // table stride of w_{NS R}
  cplx<T> v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int f = threadIdx.x + b * NTHR;
    if (TOT % NTHR == 0 || f < TOT) {
      const int s = f / NB, j = f % NB;
      const int k = j % NS;
      cplx<T>* base = lds + s * STRIDE;
      // j < NB and r NB share no bits
      const int pj = lds_idx<T>(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = base[LdsLayout<T>::join(pj, lds_idx<T>(r * NB))];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[r * k * TWS];
          v[b][r] = (DIR < 0) ? cmul(v[b][r], w) : cmulc(v[b][r], w);
        }
      }
      dft<DIR, R>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int f = threadIdx.x + b * NTHR;
    if (TOT % NTHR == 0 || f < TOT) {
      const int s = f / NB, j = f % NB;
      const int k = j % NS;
      cplx<T>* base = lds + s * STRIDE;
      const int o = (j - k) * R + k;
      // k < NS, r NS < R NS and (j - k) R (a multiple of R NS) share no bits
      const int po = lds_idx<T>(o);
#pragma unroll
      for (int r = 0; r < R; ++r) base[LdsLayout<T>::join(po, lds_idx<T>(r * NS))] = v[b][r];
    }
  }
  __syncthreads();
}

// Passes of radix R from sub-transform length NS up to L.
template <typename T, int L, int R, int NS, int DIR, int NSEQ, int NTHR, int STRIDE>
__device__ __forceinline__ void radix_passes(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < L) {
    stockham_pass<T, L, R, NS, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
    radix_passes<T, L, R, NS * R, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  }
}

// Radix of the main passes.  Radix 16 (three passes instead of four at L =
// 2048) was measured slower for FP32 on gfx950: 18.1 -> 19.2 us for the
// 2048^2 row R2C sweep and 292 -> 358 us for the 4096^2 column sweep.
template <typename T>
__host__ __device__ constexpr int main_radix() { return 8; }

// Full transform of NSEQ sequences of length L: one pass of the radix that
// log2(L) leaves over (2, 4 or 8), then passes of the main radix.  Caller
// must __syncthreads() after writing the input; the routine ends with a
// barrier.
template <typename T, int L, int DIR, int NSEQ, int NTHR, int STRIDE>
__device__ __forceinline__ void fft_lds(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  constexpr int m = ilog2(L);
  static_assert((1 << m) == L, "power-of-two length");
  constexpr int RM = main_radix<T>();
  constexpr int rem = m % ilog2(RM);
  if constexpr (rem == 0) {
    radix_passes<T, L, RM, 1, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  } else {
    constexpr int R0 = 1 << rem;
    stockham_pass<T, L, R0, 1, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
    radix_passes<T, L, RM, R0, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  }
}

}  // namespace bem
