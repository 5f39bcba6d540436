// Internal declarations of the C ABI layer (not part of the public header).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bem.h"
#include "cg_api.h"
#include "launch.h"

struct bem_influence_s {
  int nx, ny;
  double dx, dy, k, nu, E0, c0;
  double alpha, C, K00;
  int device;
  bem::Geom g;
  long long device_bytes = 0;
  // FP64 influence coefficients, quarter 0 <= di < nx, 0 <= dj < ny
  double* Kq = nullptr;
  // kernel spectrum (Lx + 1) x kpitch, pre-scaled by C / (Mx My)
  double* KT64 = nullptr;
  float* KT32 = nullptr;
  // twiddles exp(-2 pi i m / M)
  bem::cplx<double>* twx64 = nullptr;
  bem::cplx<double>* twy64 = nullptr;
  bem::cplx<float>* twx32 = nullptr;
  bem::cplx<float>* twy32 = nullptr;
  bem::cplx<double>* twly64 = nullptr;  // wave-FFT table for length Ly (Ly = 64 P)
  bem::cplx<float>* twly32 = nullptr;
  bem::cplx<double>* twlx64 = nullptr;  // the same for length Lx (row sweeps)
  bem::cplx<float>* twlx32 = nullptr;
  // lazily allocated scratch of the convolution entry points
  bem::cplx<double>* S64 = nullptr;
  bem::cplx<float>* S32 = nullptr;
  double* io64 = nullptr;
  float* io32 = nullptr;
  double* epart = nullptr;   // partials of the spectral-energy sweep (timing hook)
};

// Solver state: device buffers of one solve and its warm-start data.
struct bem_state_s {
  bem_influence_s* K = nullptr;
  size_t n = 0;
  int precision = -1;  // precision of the T buffers below (-1: none yet)
  void* p = nullptr;
  void* t = nullptr;
  void* g = nullptr;
  void* hd = nullptr;
  void* S = nullptr;
  uint8_t* mask = nullptr;
  double* h64 = nullptr;
  double* out64 = nullptr;
  double* part = nullptr;
  bem::CgScal* sc = nullptr;
  bem::CgScal* sc_host = nullptr;  // pinned
  bool has_p = false, has_mask = false, pending_import = false, import_mask = false;
  // g = C K * p + h - g_d for the current p (set by a displacement-controlled
  // solve; a sweep's next step at another d starts from it, same h)
  bool g_valid = false;
  double g_d = 0.0;
  long long device_bytes = 0;
  int last_iters[3] = {0, 0, 0};  // iterations of the previous CG solve, per mode
};

namespace bem {

// solve.cpp: typed buffers for a precision; Eq. 24 parameter checks; status
// mapping and combination.
int ensure_precision(bem_state_s* st, int precision, hipStream_t s);
int check_params(const bem_influence_s* K, const bem_params* P, bool* adhesive, double* pcrit);
int status_code(int cg_status);
int worse(int a, int b);

int set_error(int code, const char* fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char* what);

// A solve on the gap profile the state already holds from its previous
// solve, as the next step of a sweep (solve.cpp; serving sessions).
int solve_same_h(bem_influence_t K, const bem_params* prm, bem_state_t st, double* p_out,
                 unsigned char* c_out, bem_result* res, hipStream_t s);

// Bytes of a solver state's partial-sum buffer (solve.cpp; footprint model).
long long state_partial_bytes();

// Solver clock (clock.cpp): events for a chunk of n CG iterations starting at
// it0 (nullptr when the calling thread's clock is off), and the outcome of
// that chunk once the host has synchronised.
const hipEvent_t* clock_chunk(int it0, int n);
void clock_chunk_done(bool done, int final_it);
// the chunk just opened (clock_chunk returned events for it) starts with a
// gap shift: its iteration 0 has no update, first-convolution or gap launches
// (their events are not timed)
void clock_chunk_shifted();
double alpha_kn(double k, double nu);
bool is_finite(double v);

int influence_build(bem_influence_s* h);
void influence_release(bem_influence_s* h);
int ensure_io(bem_influence_s* h);
int convolve_device(bem_influence_s* h, int precision, const void* p, void* u, hipStream_t s);
int sweep_time(bem_influence_s* h, int precision, int which, int reps, hipStream_t s, double* ms);

int dev_alloc(bem_influence_s* h, void** p, size_t bytes, const char* what);

template <typename T>
SpecView<T> spec_view(const bem_influence_s* h);

}  // namespace bem
