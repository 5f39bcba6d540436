// In-LDS Stockham FFT for power-of-two lengths, radix 8 with one radix-2 or
// radix-4 pass where log2(L) is not a multiple of 3.
//
// The transform of Eq. 13 is the only place the method needs an FFT; these
// routines carry it.  A workgroup transforms NSEQ independent sequences of
// length L that sit in LDS at seq * STRIDE (padded with lds_pad).  Each pass
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

template <int DIR, int R, typename T>
__device__ __forceinline__ void dft(cplx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v);
  else dft8<DIR>(v);
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
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = base[lds_pad(j + r * NB)];
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
#pragma unroll
      for (int r = 0; r < R; ++r) base[lds_pad(o + r * NS)] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename T, int L, int NS, int DIR, int NSEQ, int NTHR, int STRIDE>
__device__ __forceinline__ void radix8_passes(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < L) {
    stockham_pass<T, L, 8, NS, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
    radix8_passes<T, L, NS * 8, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  }
}

// Full transform of NSEQ sequences of length L.  Caller must __syncthreads()
// after writing the input; the routine ends with a barrier.
template <typename T, int L, int DIR, int NSEQ, int NTHR, int STRIDE>
__device__ __forceinline__ void fft_lds(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  constexpr int m = ilog2(L);
  static_assert((1 << m) == L, "power-of-two length");
  if constexpr (m % 3 == 1) {
    stockham_pass<T, L, 2, 1, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
    radix8_passes<T, L, 2, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  } else if constexpr (m % 3 == 2) {
    stockham_pass<T, L, 4, 1, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
    radix8_passes<T, L, 4, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  } else {
    radix8_passes<T, L, 1, DIR, NSEQ, NTHR, STRIDE>(lds, tw);
  }
}

}  // namespace bem
