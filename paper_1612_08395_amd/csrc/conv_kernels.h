// Zero-padded 2-D FFT convolution u = C K * p of Eq. 13, as three sweeps.
//
// Layout.  The field is ny x nx (row index y, x contiguous).  The padded
// transform is My x Mx (powers of two, My >= 2ny, Mx >= 2nx), half lengths
// Ly = My/2 and Lx = Mx/2.  Only the first ny rows and nx columns of the
// padded input are non-zero and only those outputs are kept, which the
// sweeps exploit:
//
//  * row sweep (R2C): two real rows a, b are packed as one complex row
//    z = a + i b.  Because z is zero on [Mx/2, Mx), its Mx-point DFT splits
//    into two Lx-point DFTs (even bins: DFT(z); odd bins: DFT(z w^n),
//    w = exp(-2 pi i / Mx)).  The real-row spectra A, B (bins 0..Lx) are
//    untangled from Z[k] and conj(Z[Mx - k]).  Bins 0 and Lx of a real row
//    are real, so slot 0 stores (A[0], A[Lx]): the spectrum S has exactly
//    Lx complex columns, its row pairs interleaved per column (spec_idx in
//    common.h).
//  * column sweep: for each spectrum column, the My-point DFT of the ny
//    non-zero values (same even/odd split), multiplication by the real,
//    even kernel spectrum, inverse DFT, and only outputs y < ny kept
//    (again two Ly-point transforms).  Column 0 carries the real DC and
//    Nyquist columns packed as re/im; it is multiplied by
//    ((K0+K1)/2) Z[k] + ((K0-K1)/2) conj(Z[-k]).
//  * row sweep (C2R): Hermitian completion of the two rows' spectra,
//    Lx-point inverse DFTs of the even and odd bins, outputs x < nx kept.
//
// The kernel spectrum is stored transposed, KT[kx * kpitch + ky] for
// kx in [0, Lx], ky in [0, Ly] (the other half of ky by evenness), and is
// pre-multiplied by C / (Mx My), so no other scaling is applied.
//
// Prologue / epilogue functors fuse the conjugate-gradient vector work into
// the row sweeps: a prologue supplies the value at (y, x) (and may update
// state there), an epilogue consumes u at (y, x).  Both may accumulate FP64
// partial sums; finish() reduces them per workgroup.
#pragma once
#include <type_traits>

#include "common.h"
#include "fft_lds.h"

namespace bem {

// Functor interface of the row sweeps.  Each thread handles the elements
// n = threadIdx.x + q NTHR (q < PER) of the workgroup's two rows ya, yb.
//  prologue (R2C), called in this order so that the field loads are in
//    flight while scalars are reduced:
//    issue<NTHR>() -> false: the whole workgroup returns; else issues the
//      loads of any partial sums the prologue needs;
//    fetch<NTHR>(ya, yb, hasb, nx): issues the field loads;
//    decide<NTHR>(red, bid) -> false: the whole workgroup returns (reduces the
//      partial sums; every workgroup reaches the same decision);
//    make<NTHR>(ya, yb, hasb, nx, va, vb): values to transform (zero for
//      n >= nx); commit<NTHR>(...): writes back updated state;
//    finish<NTHR>(red, bid): per-workgroup partial sums (bid: the
//      workgroup's index within its problem).
//  epilogue (C2R): begin (may issue loads of partial sums), prefetch<NTHR>
//    (ya, yb, hasb, nx) (issued before the transform so the loads overlap
//    it), ready<NTHR>(red) (reductions the epilogue needs), consume<NTHR>(...,
//    va, vb) with the convolution outputs, finish.
template <typename T, int PER>
struct PlainLoad {
  const T* in;
  int nx;
  T fa[PER], fb[PER];
  template <int NTHR>
  __device__ bool issue() { return true; }
  template <int NTHR>
  __device__ void fetch(int ya, int yb, bool hasb, int nx_) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      const size_t safe = (size_t)ya * nx;
      fa[q] = load_or0(in, (size_t)ya * nx + n, safe, n < nx_);
      fb[q] = load_or0(in, (size_t)yb * nx + n, safe, n < nx_ && hasb);
    }
  }
  template <int NTHR>
  __device__ bool decide(double*, int) { return true; }
  template <int NTHR>
  __device__ void make(int, int, bool, int, T (&va)[PER], T (&vb)[PER]) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      va[q] = fa[q];
      vb[q] = fb[q];
    }
  }
  template <int NTHR>
  __device__ void commit(int, int, bool, int, const T (&)[PER], const T (&)[PER]) {}
  template <int NTHR>
  __device__ void finish(double*, int) {}
};

template <typename T, int PER>
struct PlainStore {
  T* out;
  int nx;
  template <int NTHR>
  __device__ bool begin(double*) { return true; }
  template <int NTHR>
  __device__ void prefetch(int, int, bool, int) {}
  template <int NTHR>
  __device__ void ready(double*) {}
  template <int NTHR>
  __device__ void consume(int ya, int yb, bool hasb, int nx_, const T (&va)[PER],
                          const T (&vb)[PER]) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int n = threadIdx.x + q * NTHR;
      if (n < nx_) {
        out[(size_t)ya * nx + n] = va[q];
        if (hasb) out[(size_t)yb * nx + n] = vb[q];
      }
    }
  }
  template <int NTHR>
  __device__ void finish(double*, int) {}
};

template <int L, int NTHR>
__host__ __device__ constexpr int row_per() { return (L + NTHR - 1) / NTHR; }

// Waves per SIMD a row sweep asks the compiler to leave room for: a
// prologue may set kMinWaves (else 1, no register cap).  With 8-wave
// workgroups (L = 4096), 4 waves per SIMD (at most 128 VGPRs) is what lets
// two workgroups share a CU, as their LDS allows.
template <class F, class = void>
struct min_waves_of {
  static constexpr int value = 1;
};
template <class F>
struct min_waves_of<F, std::void_t<decltype(F::kMinWaves)>> {
  static constexpr int value = F::kMinWaves;
};

// Row sweep R2C of row pair bid (rows 2 bid, 2 bid + 1) of one problem.
template <typename T, int L, int NTHR, class Pro>
__device__ __forceinline__ void row_r2c_body(Pro& pro, cplx<T>* __restrict__ S, int nx, int ny,
                                             const cplx<T>* __restrict__ tw, int bid) {
  constexpr int STR = LdsLayout<T>::row_stride(L);
  constexpr int PER = row_per<L, NTHR>();
  __shared__ cplx<T> lds[2 * STR];
  __shared__ double red[64];
  if (!pro.template issue<NTHR>()) return;
  const int ya = 2 * bid, yb = ya + 1;
  const bool hasb = yb < ny;
  pro.template fetch<NTHR>(ya, yb, hasb, nx);
  if (!pro.template decide<NTHR>(red, bid)) return;
  T va[PER], vb[PER];
  pro.template make<NTHR>(ya, yb, hasb, nx, va, vb);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int n = threadIdx.x + q * NTHR;
    if (PER * NTHR == L || n < L) {
      const cplx<T> z = {va[q], vb[q]};
      lds[lds_idx<T>(n)] = z;
      lds[STR + lds_idx<T>(n)] = cmul(z, tw[n]);
    }
  }
  pro.template commit<NTHR>(ya, yb, hasb, nx, va, vb);
  __syncthreads();
  fft_lds<T, L, -1, 2, NTHR, STR>(lds, tw);
  const cplx<T>* E = lds;
  const cplx<T>* O = lds + STR;
  // the pair's block of the row spectrum: row a at even, row b at odd slots
  cplx<T>* Sp = S + spec_idx(ya, 0, L);
  const T half = T(0.5);
  for (int k = threadIdx.x; k < L; k += NTHR) {
    cplx<T> a, b;
    if (k == 0) {
      const cplx<T> z0 = E[lds_idx<T>(0)], zl = E[lds_idx<T>(L / 2)];
      a = {z0.x, zl.x};
      b = {z0.y, zl.y};
    } else {
      const int kp = k >> 1;
      cplx<T> Z, Zp;
      if ((k & 1) == 0) {
        Z = E[lds_idx<T>(kp)];
        Zp = E[lds_idx<T>(L - kp)];
      } else {
        Z = O[lds_idx<T>(kp)];
        Zp = O[lds_idx<T>(L - 1 - kp)];
      }
      a = {half * (Z.x + Zp.x), half * (Z.y - Zp.y)};
      b = {half * (Z.y + Zp.y), half * (Zp.x - Z.x)};
    }
    store_pair(Sp + 2 * k, a, b);
  }
  pro.template finish<NTHR>(red, bid);
}

template <typename T, int L, int NTHR, class Pro>
__global__ __launch_bounds__(NTHR, min_waves_of<Pro>::value) void k_row_r2c(
    Pro pro_arg, cplx<T>* __restrict__ S, int nx, int ny, const cplx<T>* __restrict__ tw) {
  Pro pro = pro_arg;
  row_r2c_body<T, L, NTHR>(pro, S, nx, ny, tw, blockIdx.x);
}

// Guarded load of a complex value without control flow (see load_or0).
template <typename T>
__device__ __forceinline__ cplx<T> cload_or0(const cplx<T>* __restrict__ a, size_t i, size_t safe,
                                             bool ok) {
  const cplx<T> v = a[ok ? i : safe];
  return {ok ? v.x : T(0), ok ? v.y : T(0)};
}

// Staging of a group of W adjacent spectrum columns c0.. through LDS.
// Element f = threadIdx.x + j NTHR of the group is (row parity f % 2, column
// (f / 2) % W, row pair f / 2W): consecutive elements are consecutive in the
// row spectrum (spec_idx), 2 W values per row pair.  Rows n < LY.  load()
// issues every load of the thread before any value is used, with rows >= ny
// read as zero: the same copy written as a loop with the row guard as a
// branch waits for each load before issuing the next, which leaves one load
// per thread in flight.
template <typename T, int LY, int W, int NTHR>
struct ColStage {
  static constexpr int TOT = W * LY;
  static constexpr int CNT = (TOT + NTHR - 1) / NTHR;
  cplx<T> x[CNT];
  __device__ __forceinline__ static bool valid(int j) {
    return TOT % NTHR == 0 || (int)threadIdx.x + j * NTHR < TOT;
  }
  __device__ __forceinline__ static int col(int j) {
    return (((int)threadIdx.x + j * NTHR) >> 1) % W;
  }
  __device__ __forceinline__ static int row(int j) {
    const int f = (int)threadIdx.x + j * NTHR;
    return 2 * ((f >> 1) / W) + (f & 1);
  }
  __device__ __forceinline__ static size_t at(int j, int lx, int c0) {
    return spec_idx(row(j), c0 + col(j), lx);
  }
  __device__ __forceinline__ void load(const cplx<T>* __restrict__ S, int lx, int ny, int c0) {
#pragma unroll
    for (int j = 0; j < CNT; ++j) {
      const bool ok = valid(j) && row(j) < ny;
      x[j] = cload_or0(S, at(j, lx, c0), spec_idx(0, c0, lx), ok);
    }
  }
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that XCD x works on the contiguous block range
// [x nb/8, (x+1) nb/8): adjacent column groups, which share the 128-byte
// lines of the row spectrum, then run on the same XCD and their partial-line
// reads and writes meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Multiply the transformed columns held in LDS by the kernel spectrum.
template <typename T, int LY, int W, int NTHR, int STR>
__device__ __forceinline__ void col_multiply(cplx<T>* lds, int c0, int lx, const T* __restrict__ KT,
                                             int kpitch) {
  for (int f = threadIdx.x; f < 2 * W * LY; f += NTHR) {
    const int s = f / LY, kp = f % LY;
    const int c = s >> 1;
    if (c0 + c == 0) continue;
    const int ky = 2 * kp + (s & 1);
    const int kq = ky <= LY ? ky : 2 * LY - ky;
    const T kv = KT[(size_t)(c0 + c) * kpitch + kq];
    cplx<T>* a = lds + s * STR + lds_idx<T>(kp);
    *a = cscale(*a, kv);
  }
  if (c0 == 0) {
    // packed DC (re) / Nyquist (im) column: sequences 0 (even bins), 1 (odd)
    const T* K0 = KT;
    const T* K1 = KT + (size_t)lx * kpitch;
    const T half = T(0.5);
    for (int f = threadIdx.x; f <= LY; f += NTHR) {
      // f in [0, LY/2]: even pair (f, LY - f); f in (LY/2, LY]: odd pair
      int seq, i0, i1, ky;
      if (f <= LY / 2) {
        seq = 0;
        i0 = f;
        i1 = (LY - f) & (LY - 1);
        ky = 2 * f;
      } else {
        seq = 1;
        i0 = f - LY / 2 - 1;
        i1 = LY - 1 - i0;
        ky = 2 * i0 + 1;
      }
      if (seq == 1 && i0 >= LY / 2) continue;
      const int kq = ky <= LY ? ky : 2 * LY - ky;
      const T a = half * (K0[kq] + K1[kq]), b = half * (K0[kq] - K1[kq]);
      cplx<T>* p0 = lds + seq * STR + lds_idx<T>(i0);
      cplx<T>* p1 = lds + seq * STR + lds_idx<T>(i1);
      const cplx<T> z0 = *p0, z1 = *p1;
      *p0 = {a * z0.x + b * z1.x, a * z0.y - b * z1.y};
      if (i1 != i0) *p1 = {a * z1.x + b * z0.x, a * z1.y - b * z0.y};
    }
  }
}

// Column sweep of column group xcd_block(bid, nblk) of one problem.
template <typename T, int LY, int W, int NTHR>
__device__ __forceinline__ void col_conv_body(cplx<T>* __restrict__ S, int lx, int ny,
                                              const T* __restrict__ KT, int kpitch,
                                              const cplx<T>* __restrict__ tw, int bid, int nblk) {
  constexpr int STR = LdsLayout<T>::col_stride(LY);
  __shared__ cplx<T> lds[2 * W * STR];
  const int c0 = xcd_block(bid, nblk) * W;
  using Stage = ColStage<T, LY, W, NTHR>;
  {
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j)
      if (Stage::valid(j)) {
        const int c = Stage::col(j), n = Stage::row(j);
        lds[(2 * c) * STR + lds_idx<T>(n)] = st.x[j];
        lds[(2 * c + 1) * STR + lds_idx<T>(n)] = cmul(st.x[j], tw[n]);
      }
  }
  __syncthreads();
  fft_lds<T, LY, -1, 2 * W, NTHR, STR>(lds, tw);
  col_multiply<T, LY, W, NTHR, STR>(lds, c0, lx, KT, kpitch);
  __syncthreads();
  fft_lds<T, LY, +1, 2 * W, NTHR, STR>(lds, tw);
  // combine the halves for every element first, then store (rows < ny)
  cplx<T> y[Stage::CNT];
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j) {
    const int c = Stage::col(j), n = Stage::row(j);
    if (Stage::valid(j)) {
      const cplx<T> e = lds[(2 * c) * STR + lds_idx<T>(n)];
      const cplx<T> o = lds[(2 * c + 1) * STR + lds_idx<T>(n)];
      y[j] = cadd(e, cmulc(o, tw[n]));
    }
  }
#pragma unroll
  for (int j = 0; j < Stage::CNT; ++j)
    if (Stage::valid(j) && Stage::row(j) < ny)
      S[Stage::at(j, lx, c0)] = y[j];
}

template <typename T, int LY, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void k_col_conv(cplx<T>* __restrict__ S, int lx, int ny,
                                                   const T* __restrict__ KT, int kpitch,
                                                   const cplx<T>* __restrict__ tw,
                                                   const int* __restrict__ done) {
  if (done && *done) return;
  col_conv_body<T, LY, W, NTHR>(S, lx, ny, KT, kpitch, tw, blockIdx.x, gridDim.x);
}

// Spectral energy of the packed half spectrum.  After the forward column
// transform, the full padded spectrum T(kx, ky) of a real field is known from
// columns kx = 1 .. Lx-1 (each also stands for Mx - kx) and from the packed
// column 0, whose transform is Z = A + i B with A (kx = 0) and B (kx = Lx)
// Hermitian in ky: A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i.
// Returns sum_k KT(k) |T(k)|^2 for this thread's share.
template <typename T>
__device__ __forceinline__ double energy_term(cplx<T> z, T kt) {
  return 2.0 * (double)kt * ((double)z.x * (double)z.x + (double)z.y * (double)z.y);
}
template <typename T>
__device__ __forceinline__ double energy_packed(cplx<T> z, cplx<T> zm, T k0, T k1) {
  const double ax = 0.5 * ((double)z.x + (double)zm.x), ay = 0.5 * ((double)z.y - (double)zm.y);
  const double bx = 0.5 * ((double)z.y + (double)zm.y), by = 0.5 * ((double)zm.x - (double)z.x);
  return (double)k0 * (ax * ax + ay * ay) + (double)k1 * (bx * bx + by * by);
}

// Forward column transform and the spectral energy sum_k KT(k) |T(k)|^2.
// With KT = C Khat / (Mx My), Parseval gives sum_x t(x) (C K * t)(x) for
// the zero-padded field t whose row spectrum is S; so this replaces the
// inverse transforms of a convolution whose only use is that inner product.
// One FP64 partial per workgroup into part[blockIdx.x].
template <typename T, int LY, int W, int NTHR>
__device__ __forceinline__ void col_energy_body(const cplx<T>* __restrict__ S, int lx, int ny,
                                                const T* __restrict__ KT, int kpitch,
                                                const cplx<T>* __restrict__ tw,
                                                double* __restrict__ part, int bid, int nblk) {
  constexpr int STR = LdsLayout<T>::col_stride(LY);
  __shared__ cplx<T> lds[2 * W * STR];
  __shared__ double red[64];
  const int c0 = xcd_block(bid, nblk) * W;
  {
    using Stage = ColStage<T, LY, W, NTHR>;
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j)
      if (Stage::valid(j)) {
        const int c = Stage::col(j), n = Stage::row(j);
        lds[(2 * c) * STR + lds_idx<T>(n)] = st.x[j];
        lds[(2 * c + 1) * STR + lds_idx<T>(n)] = cmul(st.x[j], tw[n]);
      }
  }
  __syncthreads();
  fft_lds<T, LY, -1, 2 * W, NTHR, STR>(lds, tw);
  double e = 0.0;
  for (int f = threadIdx.x; f < 2 * W * LY; f += NTHR) {
    const int s = f / LY, kp = f % LY;
    const int c = s >> 1;
    if (c0 + c == 0) continue;
    const int ky = 2 * kp + (s & 1);
    const int kq = ky <= LY ? ky : 2 * LY - ky;
    e += energy_term(lds[s * STR + lds_idx<T>(kp)], KT[(size_t)(c0 + c) * kpitch + kq]);
  }
  if (c0 == 0) {
    // column 0: sequences 0 (even ky) and 1 (odd ky); partner of ky is -ky
    for (int f = threadIdx.x; f < 2 * LY; f += NTHR) {
      const int s = f / LY, kp = f % LY;
      const int kpp = s ? LY - 1 - kp : (LY - kp) & (LY - 1);
      const int ky = 2 * kp + s;
      const int kq = ky <= LY ? ky : 2 * LY - ky;
      e += energy_packed(lds[s * STR + lds_idx<T>(kp)], lds[s * STR + lds_idx<T>(kpp)], KT[kq],
                         KT[(size_t)lx * kpitch + kq]);
    }
  }
  e = block_sum<NTHR>(e, red);
  if (threadIdx.x == 0) part[bid] = e;
}

template <typename T, int LY, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void k_col_energy(const cplx<T>* __restrict__ S, int lx, int ny,
                                                     const T* __restrict__ KT, int kpitch,
                                                     const cplx<T>* __restrict__ tw,
                                                     const int* __restrict__ done,
                                                     double* __restrict__ part) {
  if (done && *done) return;
  col_energy_body<T, LY, W, NTHR>(S, lx, ny, KT, kpitch, tw, part, blockIdx.x, gridDim.x);
}

// Row sweep C2R of row pair bid of one problem.
template <typename T, int L, int NTHR, class Epi>
__device__ __forceinline__ void row_c2r_body(const cplx<T>* __restrict__ S, int nx, int ny,
                                             const cplx<T>* __restrict__ tw, Epi& epi, int bid) {
  constexpr int STR = LdsLayout<T>::row_stride(L);
  constexpr int PER = row_per<L, NTHR>();
  __shared__ cplx<T> lds[2 * STR];
  __shared__ double red[64];
  if (!epi.template begin<NTHR>(red)) return;
  const int ya = 2 * bid, yb = ya + 1;
  const bool hasb = yb < ny;
  // the pair's block of the row spectrum (row b at odd slots; row a stands in
  // for an absent b)
  const cplx<T>* Sp = S + spec_idx(ya, 0, L);
  // all loads first (no control flow between them), then the LDS scatter
  constexpr int KPER = (L + NTHR - 1) / NTHR;
  cplx<T> Av[KPER], Bv[KPER];
#pragma unroll
  for (int j = 0; j < KPER; ++j) {
    const int k = threadIdx.x + j * NTHR;
    const int ks = k < L ? k : 0;
    const cpair<T> ab = load_pair(Sp + 2 * ks);
    Av[j] = ab.a;
    Bv[j] = hasb ? ab.b : ab.a;
  }
  // the epilogue's own loads, issued after the spectrum (in-order completion)
  // so that they stay in flight during the transform
  epi.template prefetch<NTHR>(ya, yb, hasb, nx);
  epi.template ready<NTHR>(red);
#pragma unroll
  for (int j = 0; j < KPER; ++j) {
    const int k = threadIdx.x + j * NTHR;
    if (KPER * NTHR != L && k >= L) break;
    const cplx<T> A = Av[j];
    // zero row b without a branch (a select here becomes one, with a wait
    // for every load in flight); Bv is finite data of a valid row
    const cplx<T> B = cscale(Bv[j], hasb ? T(1) : T(0));
    if (k == 0) {
      lds[lds_idx<T>(0)] = {A.x, B.x};        // Z[0]  = A[0]  + i B[0]
      lds[lds_idx<T>(L / 2)] = {A.y, B.y};    // Z[Lx] = A[Lx] + i B[Lx]
    } else {
      const cplx<T> Z = {A.x - B.y, A.y + B.x};    // A + i B
      const cplx<T> Zm = {A.x + B.y, B.x - A.y};   // conj(A) + i conj(B) = Z[Mx - k]
      const int km = 2 * L - k;
      lds[(k & 1) * STR + lds_idx<T>(k >> 1)] = Z;
      lds[(km & 1) * STR + lds_idx<T>(km >> 1)] = Zm;
    }
  }
  __syncthreads();
  fft_lds<T, L, +1, 2, NTHR, STR>(lds, tw);
  T va[PER], vb[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int n = threadIdx.x + q * NTHR;
    cplx<T> z = {T(0), T(0)};
    if (n < nx) z = cadd(lds[lds_idx<T>(n)], cmulc(lds[STR + lds_idx<T>(n)], tw[n]));
    va[q] = z.x;
    vb[q] = z.y;
  }
  epi.template consume<NTHR>(ya, yb, hasb, nx, va, vb);
  epi.template finish<NTHR>(red, bid);
}

template <typename T, int L, int NTHR, class Epi>
__global__ __launch_bounds__(NTHR) void k_row_c2r(const cplx<T>* __restrict__ S, int nx, int ny,
                                                  const cplx<T>* __restrict__ tw, Epi epi_arg) {
  Epi epi = epi_arg;
  row_c2r_body<T, L, NTHR>(S, nx, ny, tw, epi, blockIdx.x);
}

// Forward column transform of the (FP64) row spectrum of Q, and the real,
// even kernel spectrum Khat(ky, kx) = 2 Re[Qhat(ky, kx) + Qhat(-ky, kx)]
// written scaled, in FP64 and rounded to FP32.
template <int LY, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void k_col_spectrum(const cplx<double>* __restrict__ S, int lx,
                                                       int ny, const cplx<double>* __restrict__ tw,
                                                       double* __restrict__ KT64,
                                                       float* __restrict__ KT32, int kpitch,
                                                       double scale) {
  constexpr int STR = LdsLayout<double>::col_stride(LY);
  __shared__ cplx<double> lds[2 * W * STR];
  const int c0 = blockIdx.x * W;
  {
    using Stage = ColStage<double, LY, W, NTHR>;
    Stage st;
    st.load(S, lx, ny, c0);
#pragma unroll
    for (int j = 0; j < Stage::CNT; ++j)
      if (Stage::valid(j)) {
        const int c = Stage::col(j), n = Stage::row(j);
        lds[(2 * c) * STR + lds_idx<double>(n)] = st.x[j];
        lds[(2 * c + 1) * STR + lds_idx<double>(n)] = cmul(st.x[j], tw[n]);
      }
  }
  __syncthreads();
  fft_lds<double, LY, -1, 2 * W, NTHR, STR>(lds, tw);
  for (int f = threadIdx.x; f < W * (LY + 1); f += NTHR) {
    const int c = f / (LY + 1), ky = f % (LY + 1);
    const int kn = (2 * LY - ky) & (2 * LY - 1);
    const cplx<double> yk = lds[(2 * c + (ky & 1)) * STR + lds_idx<double>(ky >> 1)];
    const cplx<double> yn = lds[(2 * c + (kn & 1)) * STR + lds_idx<double>(kn >> 1)];
    const int cg = c0 + c;
    const double v = 2.0 * (yk.x + yn.x) * scale;
    KT64[(size_t)cg * kpitch + ky] = v;
    KT32[(size_t)cg * kpitch + ky] = (float)v;
    if (cg == 0) {
      const double w = 2.0 * (yk.y + yn.y) * scale;
      KT64[(size_t)lx * kpitch + ky] = w;
      KT32[(size_t)lx * kpitch + ky] = (float)w;
    }
  }
}

}  // namespace bem
