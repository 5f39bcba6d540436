// Shared device-side helpers of the BEM library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bem {

template <typename T>
struct __align__(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

// LDS index padding: one spare slot every 32 elements breaks the power-of-two
// strides of the Stockham write pattern across the LDS banks.
// Guarded load without control flow: reads a[ok ? i : safe] (safe must be a
// valid index) and returns zero where !ok.  A load under an `if` becomes a
// branch whose value the compiler waits for inside it, which serialises the
// loads of a thread; this form keeps them all in flight.
template <typename T>
__device__ __forceinline__ T load_or0(const T* __restrict__ a, size_t i, size_t safe, bool ok) {
  const T v = a[ok ? i : safe];
  return ok ? v : T(0);
}

// Layout of a sequence in LDS for the Stockham passes (element i of a
// sequence sits at idx(i); sequences are stride apart).  LDS serves a 64-bit
// access 32 lanes at a time over 64 banks, a 128-bit access 16 lanes at a
// time.  join(idx(a), idx(b)) = idx(a | b) when a and b share no bits, which
// the passes use to address a butterfly's R points from one base.
//  FP32: one padding element per 32 (join is an addition, so the R points
//   share one address register with immediate offsets).
//  FP64: an XOR swizzle, i with bits 4 and 5 (5 and 6, ...) folded into its
//   low 4 bits: a permutation of every power-of-two length, linear over
//   GF(2).  The radix-8/4 passes at 2048 and 4096 points then hit 1.125
//   lanes per bank on average instead of 1.5 with padding (measured: FP64
//   column sweep at 2048^2 125 -> 118 us); for FP32 the XOR addressing costs
//   more VALU than the conflicts it removes (1.375 -> 1.125).
//  The stride offsets put the halves of a row pair or adjacent staged
//  columns on different banks.
template <typename T>
struct LdsLayout;
template <>
struct LdsLayout<float> {
  __host__ __device__ static constexpr int idx(int i) { return i + (i >> 5); }
  __host__ __device__ static constexpr int join(int a, int b) { return a + b; }
  __host__ __device__ static constexpr int row_stride(int n) { return n + (n >> 5) + 1; }
  __host__ __device__ static constexpr int col_stride(int n) { return n + (n >> 5) + 1; }
};
template <>
struct LdsLayout<double> {
  __host__ __device__ static constexpr int idx(int i) { return i ^ (((i >> 4) ^ (i >> 5)) & 15); }
  __host__ __device__ static constexpr int join(int a, int b) { return a ^ b; }
  __host__ __device__ static constexpr int row_stride(int n) { return n + 8; }
  __host__ __device__ static constexpr int col_stride(int n) { return n + 4; }
};
template <typename T>
__host__ __device__ constexpr int lds_idx(int i) { return LdsLayout<T>::idx(i); }

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// Row spectrum layout: the two rows of a row pair are interleaved per
// column, spectrum column c of row y at ((y >> 1) lx + c) 2 + (y & 1).  A row
// sweep (one workgroup per row pair) then writes and reads its pair as one
// contiguous block, and a column sweep over W adjacent columns moves 2 W
// complex values per row pair in one piece instead of W per row.  Holds
// spec_rows(ny) rows (ny rounded up to even).
__host__ __device__ __forceinline__ size_t spec_idx(int y, int c, int lx) {
  return ((size_t)(y >> 1) * lx + c) * 2 + (y & 1);
}
__host__ __device__ constexpr int spec_rows(int ny) { return ny + (ny & 1); }

// Both rows of a pair at one spectrum column, p = S + spec_idx(2 j, c, lx):
// one 16-byte access for float (32 bytes for double).  A row sweep stores
// the pair whole; for an odd ny the padding row's slot is written and never
// read as data.
template <typename T>
struct __align__(4 * sizeof(T)) cpair {
  cplx<T> a, b;
};
template <typename T>
__device__ __forceinline__ void store_pair(cplx<T>* p, cplx<T> a, cplx<T> b) {
  *reinterpret_cast<cpair<T>*>(p) = cpair<T>{a, b};
}
template <typename T>
__device__ __forceinline__ cpair<T> load_pair(const cplx<T>* p) {
  return *reinterpret_cast<const cpair<T>*>(p);
}

// Block-wide FP64 sum; every thread passes its value, the result is valid in
// every thread.  Fixed combination order (wave shuffles, then waves in index
// order), so the result is bitwise reproducible.  `red` holds >= 16 doubles.
template <int NTHR>
__device__ __forceinline__ double block_sum(double v, double* red) {
  static_assert(NTHR % 64 == 0 && NTHR <= 1024, "block size");
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  constexpr int NW = NTHR / 64;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  __syncthreads();
  return s;
}

}  // namespace bem
