// Contact solves: solver state, the host side of the device CG loop, the
// adhesive detach / re-solve loop (Section 3.1), sweeps, Eq. 24.
//
// The host never takes part in an iteration: it queues a chunk of CG
// iterations (five kernels each, six under force control), copies the
// scalar block back and looks at the device-side `done` flag.  Kernels queued after convergence
// return at once, so results do not depend on the chunking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <system_error>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/bem.h"
#include "cg_api.h"
#include "internal.h"

using namespace bem;


namespace {

constexpr int kPartials = kPartTotal;
}  // namespace

namespace bem {
long long state_partial_bytes() { return (long long)kPartials * sizeof(double); }
}  // namespace bem

namespace {

int salloc(bem_state_s* st, void** p, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, what);
  }
  st->device_bytes += (long long)bytes;
  return BEM_OK;
}

void free_typed(bem_state_s* st) {
  for (void** q : {&st->p, &st->t, &st->g, &st->hd, &st->S}) {
    if (*q) hipFree(*q);
    *q = nullptr;
  }
  st->precision = -1;
}

size_t tsize(int precision) { return precision == BEM_FP64 ? sizeof(double) : sizeof(float); }

}  // namespace

// Make the T buffers match `precision`, carrying a warm-start pressure over.
int bem::ensure_precision(bem_state_s* st, int precision, hipStream_t s) {
  if (st->precision == precision) return BEM_OK;
  hipError_t e;
  if (st->has_p && st->precision >= 0) {
    e = st->precision == BEM_FP64
            ? launch_to_f64<double>((const double*)st->p, st->out64, st->n, s)
            : launch_to_f64<float>((const float*)st->p, st->out64, st->n, s);
    if (e != hipSuccess) return hip_fail(e, "precision change");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "precision change");
    st->pending_import = true;
    st->import_mask = st->has_mask;
  }
  free_typed(st);
  const size_t ts = tsize(precision);
  const size_t cs = 2 * ts;
  int rc;
  if ((rc = salloc(st, &st->p, st->n * ts, "pressure"))) return rc;
  if ((rc = salloc(st, &st->t, st->n * ts, "direction"))) return rc;
  if ((rc = salloc(st, &st->g, st->n * ts, "gap"))) return rc;
  if ((rc = salloc(st, &st->hd, st->n * ts, "gap profile"))) return rc;
  if ((rc = salloc(st, &st->S, (size_t)spec_rows(st->K->ny) * st->K->g.Lx * cs, "row spectrum")))
    return rc;
  st->precision = precision;
  return BEM_OK;
}

namespace {

template <typename T>
CgBufs<T> bufs(bem_state_s* st) {
  return {(T*)st->p, (T*)st->t, (T*)st->g, (T*)st->hd, st->mask, (cplx<T>*)st->S, st->part,
          st->sc};
}

struct SolveCfg {
  double tol;
  int max_iter;
  int stall_limit;
  double W = 0.0;  // load control: prescribed sum of p
};

}  // namespace

int bem::status_code(int st) {
  switch (st) {
    case CG_ST_NOCONV: return BEM_ENOCONV;
    case CG_ST_FLOOR: return BEM_EFLOOR;
    case CG_ST_NUMERIC: return BEM_ENUMERIC;
    default: return BEM_OK;
  }
}

namespace {

// Run one CG solve to convergence on the device.  Returns the status code;
// *iters receives the iterations of this solve.
// shift (displacement control): iteration 0 takes its gap from the state's g
// shifted by *shift instead of the first convolution.
template <typename T>
int run_cg(bem_state_s* st, int mode, const SolveCfg& cfg, int* iters, double* resid,
           hipStream_t s, const double* shift = nullptr) {
  const bool fixed_set = mode == CG_FIXED;
  CgScal* h = st->sc_host;
  std::memset(h, 0, sizeof(CgScal));
  h->tol = cfg.tol;
  h->max_iter = cfg.max_iter;
  h->stall_limit = cfg.stall_limit;
  h->W = cfg.W;
  hipError_t e = hipMemcpyAsync(st->sc, h, sizeof(CgScal), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "solver scalars");
  if ((e = launch_prepare<T>((T*)st->t, (T*)st->p, st->mask, fixed_set, st->n, s)) != hipSuccess)
    return hip_fail(e, "solver prepare");
  const Geom& g = st->K->g;
  const SpecView<T> K = spec_view<T>(st->K);
  const CgBufs<T> b = bufs<T>(st);
  // First chunk sized from the previous solve of this state (warm-started
  // sweeps converge in similar counts), then small doubling chunks.
  int& last = st->last_iters[mode];
  int chunk = last > 0 ? std::min(std::max(last + 2, 4), 64) : 4;
  int next = 4;
  int it = 0;
  for (;;) {
    const hipEvent_t* ev = clock_chunk(it, chunk);
    const double* sh = it == 0 ? shift : nullptr;
    if (sh && ev) clock_chunk_shifted();   // ev: this chunk has a clock segment
    if ((e = launch_cg_iterations<T>(g, K, b, mode, it, chunk, ev, s, sh)) != hipSuccess)
      return hip_fail(e, "CG iteration launch");
    it += chunk;
    if ((e = hipMemcpyAsync(h, st->sc, sizeof(CgScal), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e, "solver scalars");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "CG iteration");
    clock_chunk_done(h->done != 0, h->iter);
    if (h->done) break;
    // the device stops itself at max_iter; this only guards the host loop
    if (it > cfg.max_iter + 256) return set_error(BEM_EDEVICE, "CG loop did not report completion");
    chunk = next;
    next = std::min(next * 2, 32);
  }
  *iters = h->iter;
  last = h->iter;
  *resid = h->rhs2 > 0 ? std::sqrt(h->G / h->rhs2) : std::sqrt(h->G);
  return status_code(h->status);
}

template <typename T>
int finalize(bem_state_s* st, int mode, hipStream_t s) {
  hipError_t e = launch_finalize<T>(bufs<T>(st), mode, st->n, s);
  if (e == hipSuccess) e = hipMemcpyAsync(st->sc_host, st->sc, sizeof(CgScal), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "final sums");
  return BEM_OK;
}

}  // namespace

int bem::worse(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  return std::max(a, b);
}

namespace {

// Apply an imported (or precision-converted) pressure / contact set.
template <typename T>
int apply_import(bem_state_s* st, hipStream_t s) {
  if (!st->pending_import) return BEM_OK;
  hipError_t e = launch_from_f64<T>(st->out64, (T*)st->p, st->n, s);
  if (e != hipSuccess) return hip_fail(e, "state import");
  st->pending_import = false;
  st->has_p = true;
  if (!st->import_mask) {
    int rc = finalize<T>(st, CG_DISP, s);  // contact set = {p > 0}
    if (rc) return rc;
  }
  st->has_mask = true;
  return BEM_OK;
}

template <typename T>
int solve_typed(bem_state_s* st, const double* h_dev, const bem_params& P, bool adhesive,
                double pcrit, double* p_out, unsigned char* c_out, double* u_out, bool outs_host,
                bem_result* res, hipStream_t s, bool sweep_step) {
  bem_influence_s* K = st->K;
  const size_t n = st->n;
  // the previous solve's g may seed this one (sweep steps only: same h)
  const bool g_ok = sweep_step && st->g_valid && !st->pending_import;
  const double g_d = st->g_d;
  st->g_valid = false;
  int rc = apply_import<T>(st, s);
  if (rc) return rc;
  SolveCfg cfg;
  cfg.tol = P.tol > 0 ? P.tol : (P.precision == BEM_FP64 ? 1e-12 : 1e-6);
  cfg.max_iter = P.max_iter > 0 ? P.max_iter : 20000;
  cfg.stall_limit = P.stall_limit > 0 ? P.stall_limit
                                      : (P.stall_limit < 0 ? 0 : (P.precision == BEM_MIXED ? 50 : 0));
  hipError_t e;
  int status = BEM_OK, iters_total = 0, rounds = 0, it = 0;
  double resid = 0.0;
  const double inv_ck00 = 1.0 / (K->C * K->K00);

  auto non_adhesive = [&](double d) -> int {
    hipError_t ee = launch_make_hd<T>(h_dev, d, (T*)st->hd, n, s);
    if (ee != hipSuccess) return hip_fail(ee, "gap profile");
    const bool warm = st->has_p;
    if (!st->has_p) {
      ee = launch_cold_start<T>((T*)st->p, (const T*)st->hd, inv_ck00, n, s);
      if (ee != hipSuccess) return hip_fail(ee, "cold start");
      st->has_p = true;
    }
    // g = C K * p + h - g_d  ->  g + (g_d - d) = C K * p + h - d
    const double shift = g_d - d;
    int r = run_cg<T>(st, CG_DISP, cfg, &it, &resid, s, (g_ok && warm) ? &shift : nullptr);
    if (r < 0) return r;
    status = worse(status, r);
    iters_total += it;
    int f = finalize<T>(st, CG_DISP, s);
    if (f) return f;
    st->has_mask = true;
    st->g_valid = true;
    st->g_d = d;
    return BEM_OK;
  };

  // load control: d unknown (returned as the mean gap shift), hd = h
  double d_found = P.d;
  auto force_control = [&](double F) -> int {
    hipError_t ee = launch_make_hd<T>(h_dev, 0.0, (T*)st->hd, n, s);
    if (ee != hipSuccess) return hip_fail(ee, "gap profile");
    if (F == 0.0) {  // no load: no pressure, the surfaces just touch
      if ((ee = launch_fill<T>((T*)st->p, 0.0, n, s)) != hipSuccess) return hip_fail(ee, "zero load");
      if ((ee = launch_min_h<T>(h_dev, n, st->sc, s)) != hipSuccess) return hip_fail(ee, "zero load");
      st->has_p = false;
      int f = finalize<T>(st, CG_DISP, s);
      if (f) return f;
      d_found = st->sc_host->gbar;
      st->has_mask = true;
      return BEM_OK;
    }
    if (!st->has_p) {  // any positive field: the first iteration scales it to F
      if ((ee = launch_fill<T>((T*)st->p, 1.0, n, s)) != hipSuccess) return hip_fail(ee, "cold start");
      st->has_p = true;
    }
    SolveCfg fc = cfg;
    fc.W = F / (K->dx * K->dy);
    int r = run_cg<T>(st, CG_FORCE, fc, &it, &resid, s);
    if (r < 0) return r;
    status = worse(status, r);
    iters_total += it;
    int f = finalize<T>(st, CG_FORCE, s);
    if (f) return f;
    d_found = st->sc_host->gbar;
    st->has_mask = true;
    return BEM_OK;
  };

  if (P.control == BEM_CTRL_FORCE) {
    rc = force_control(P.F);
    if (rc) return rc;
  } else if (!adhesive) {
    rc = non_adhesive(P.d);
    if (rc) return rc;
  } else {
    if (!st->has_mask) {
      rc = non_adhesive(std::max(P.d, P.d_preload));
      if (rc) return rc;
    }
    if ((e = launch_make_hd<T>(h_dev, P.d, (T*)st->hd, n, s)) != hipSuccess)
      return hip_fail(e, "gap profile");
    st->g_valid = false;   // the fixed-set solves change p
    for (;;) {
      int r = run_cg<T>(st, CG_FIXED, cfg, &it, &resid, s);
      if (r < 0) return r;
      status = worse(status, r);
      iters_total += it;
      if ((e = launch_detach<T>(bufs<T>(st), pcrit, n, s)) != hipSuccess)
        return hip_fail(e, "detachment");
      if ((e = hipMemcpyAsync(st->sc_host, st->sc, sizeof(CgScal), hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
        return hip_fail(e, "detachment");
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "detachment");
      if (st->sc_host->fin_detach == 0.0) break;
      ++rounds;
      if (iters_total >= cfg.max_iter * 8) {
        status = worse(status, BEM_ENOCONV);
        break;
      }
    }
    rc = finalize<T>(st, CG_FIXED, s);
    if (rc) return rc;
  }

  const CgScal* h = st->sc_host;
  // a solve that ends with no pressure anywhere leaves nothing to warm-start from
  if (h->fin_contact == 0.0) st->has_p = false;
  if (res) {
    res->d = d_found;
    res->F = K->dx * K->dy * h->fin_sum_p;
    res->n_contact = (long long)h->fin_contact;
    res->area = (double)res->n_contact * K->dx * K->dy;
    res->n_penetrating = adhesive ? (long long)h->fin_pen : 0;
    res->residual = resid;
    res->p_crit = adhesive ? pcrit : 0.0;
    res->iters = iters_total;
    res->detach_rounds = rounds;
    res->status = status;
  }
  // outputs
  const hipMemcpyKind kd = outs_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (p_out) {
    const double* src;
    if (std::is_same<T, double>::value) {
      src = (const double*)st->p;
    } else {
      if ((e = launch_to_f64<T>((const T*)st->p, st->out64, n, s)) != hipSuccess)
        return hip_fail(e, "pressure output");
      src = st->out64;
    }
    if ((e = hipMemcpyAsync(p_out, src, n * sizeof(double), kd, s)) != hipSuccess)
      return hip_fail(e, "pressure output");
  }
  if (c_out && (e = hipMemcpyAsync(c_out, st->mask, n, kd, s)) != hipSuccess)
    return hip_fail(e, "contact output");
  if (u_out) {
    if (p_out && !std::is_same<T, double>::value) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "output");
    }
    // load control: g = u + h (no d in it)
    const double dg = P.control == BEM_CTRL_FORCE ? 0.0 : P.d;
    if ((e = launch_u_from_gap<T>((const T*)st->g, h_dev, dg, st->out64, n, s)) != hipSuccess)
      return hip_fail(e, "displacement output");
    if ((e = hipMemcpyAsync(u_out, st->out64, n * sizeof(double), kd, s)) != hipSuccess)
      return hip_fail(e, "displacement output");
  }
  if (outs_host && (e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "outputs");
  return status;
}

// ---- corrected c1 of Table 1 and its natural cubic spline in ln c1 --------
const double kTabK[19] = {-0.9, -0.8, -0.7, -0.6, -0.5, -0.4, -0.3, -0.2, -0.1, 0.0,
                          0.1,  0.2,  0.3,  0.4,  0.5,  0.6,  0.7,  0.8,  0.9};
const double kTabC1[19] = {0.14, 0.31, 0.495, 0.71, 0.96, 1.24, 1.58, 1.97, 2.43, 2.97,
                           3.66, 4.52, 5.62,  7.10, 9.15, 12.25, 17.50, 27.65, 58.00};

double c1_table(double k) {
  if (!(k > -1.0 && k < 1.0)) return std::nan("");
  for (int i = 0; i < 19; ++i)
    if (std::fabs(k - kTabK[i]) < 1e-12) return kTabC1[i];
  const int n = 19;
  double y[19], M[19], a[19], b[19], c[19], r[19];
  for (int i = 0; i < n; ++i) y[i] = std::log(kTabC1[i]);
  const double hh = 0.1;
  // natural spline: M0 = Mn-1 = 0; h (M[i-1] + 4 M[i] + M[i+1]) = 6 (y[i+1] - 2y[i] + y[i-1]) / h
  for (int i = 1; i < n - 1; ++i) {
    a[i] = 1.0;
    b[i] = 4.0;
    c[i] = 1.0;
    r[i] = 6.0 * (y[i + 1] - 2.0 * y[i] + y[i - 1]) / (hh * hh);
  }
  // Thomas algorithm on rows 1..n-2
  for (int i = 2; i < n - 1; ++i) {
    const double w = a[i] / b[i - 1];
    b[i] -= w * c[i - 1];
    r[i] -= w * r[i - 1];
  }
  M[0] = M[n - 1] = 0.0;
  M[n - 2] = r[n - 2] / b[n - 2];
  for (int i = n - 3; i >= 1; --i) M[i] = (r[i] - c[i] * M[i + 1]) / b[i];
  int i = (int)std::floor((k - kTabK[0]) / hh);
  i = std::max(0, std::min(n - 2, i));
  const double x0 = kTabK[i], x1 = kTabK[i + 1];
  const double A = (x1 - k) / hh, B = (k - x0) / hh;
  const double v = A * y[i] + B * y[i + 1] +
                   ((A * A * A - A) * M[i] + (B * B * B - B) * M[i + 1]) * hh * hh / 6.0;
  return std::exp(v);
}

double p_crit_eq24(double k, double nu, double gamma, double dx, double E0, double c0) {
  const double c1 = c1_table(k);
  return std::sqrt(2.0 * E0 * gamma /
                   (alpha_kn(k, nu) * (1.0 - nu * nu) * c1 * std::pow(c0, k) * std::pow(dx, 1.0 - k)));
}

}  // namespace

int bem::check_params(const bem_influence_s* K, const bem_params* P, bool* adhesive,
                      double* pcrit) {
  if (!P) return set_error(BEM_EINVAL, "bem_solve: params is NULL");
  if (P->precision != BEM_FP64 && P->precision != BEM_MIXED)
    return set_error(BEM_EINVAL, "bem_solve: unknown precision %d", P->precision);
  if (P->control != BEM_CTRL_INDENT && P->control != BEM_CTRL_FORCE)
    return set_error(BEM_EINVAL, "bem_solve: unknown control");
  if (!is_finite(P->d)) return set_error(BEM_EINVAL, "bem_solve: non-finite indentation");
  if (P->control == BEM_CTRL_FORCE && (!is_finite(P->F) || P->F < 0.0))
    return set_error(BEM_EINVAL, "bem_solve: force control needs a finite force F >= 0");
  if (!is_finite(P->gamma) || P->gamma < 0.0 || !is_finite(P->p_crit) || !is_finite(P->tol) ||
      !is_finite(P->d_preload))
    return set_error(BEM_EINVAL, "bem_solve: invalid adhesion or tolerance parameter");
  *adhesive = P->gamma > 0.0 || P->p_crit > 0.0;
  *pcrit = 0.0;
  if (*adhesive && P->control == BEM_CTRL_FORCE)
    return set_error(BEM_EUNSUPPORTED, "bem_solve: force control is for non-adhesive contact");
  if (*adhesive) {
    if (std::fabs(K->dx - K->dy) > 1e-12 * K->dx)
      return set_error(BEM_EUNSUPPORTED,
                       "bem_solve: adhesion needs square elements (Eqs. 21-24 assume dx = dy)");
    *pcrit = P->p_crit > 0.0 ? P->p_crit : p_crit_eq24(K->k, K->nu, P->gamma, K->dx, K->E0, K->c0);
  }
  return BEM_OK;
}

namespace {

int solve_common(bem_influence_t K, const double* h_dev, const bem_params* prm, bem_state_t state,
                 double* p_out, unsigned char* c_out, double* u_out, bool outs_host,
                 bem_result* res, hipStream_t s, bool sweep_step = false) {
  bool adhesive;
  double pcrit;
  int rc = check_params(K, prm, &adhesive, &pcrit);
  if (rc) return rc;
  bem_state_t tmp = nullptr;
  if (!state) {
    rc = bem_state_create(K, &tmp);
    if (rc) return rc;
    state = tmp;
  }
  if (state->K != K) {
    if (tmp) bem_state_free(tmp);
    return set_error(BEM_EINVAL, "bem_solve: state belongs to another influence handle");
  }
  rc = ensure_precision(state, prm->precision, s);
  if (rc == BEM_OK) {
    rc = prm->precision == BEM_FP64
             ? solve_typed<double>(state, h_dev, *prm, adhesive, pcrit, p_out, c_out, u_out,
                                   outs_host, res, s, sweep_step)
             : solve_typed<float>(state, h_dev, *prm, adhesive, pcrit, p_out, c_out, u_out,
                                  outs_host, res, s, sweep_step);
  }
  if (tmp) bem_state_free(tmp);
  return rc;
}

// The steps i = first, first + stride, ... of a sweep, warm-started from one
// to the next in `state` on stream s.  With stride 1 this is the sweep of
// Section 3.1: with adhesion, a step whose value is below the previous
// step's is a pull-off step, every other step a loading (non-adhesive) solve.
int sweep_steps(bem_influence_t K, const double* h_dev, const bem_params* prm,
                const double* d_list, int n_steps, int first, int stride, bem_state_t state,
                bem_result* res, hipStream_t s) {
  int worst = BEM_OK;
  const bool adhesive = prm->gamma > 0.0 || prm->p_crit > 0.0;
  state->g_valid = false;   // g may belong to another gap profile
  for (int i = first; i < n_steps; i += stride) {
    bem_params P = *prm;
    if (prm->control == BEM_CTRL_FORCE)
      P.F = d_list[i];
    else
      P.d = d_list[i];
    const bool unloading = adhesive && i > 0 && d_list[i] < d_list[i - 1];
    if (adhesive && !unloading) {
      P.gamma = 0.0;
      P.p_crit = 0.0;
    }
    const int r =
        solve_common(K, h_dev, &P, state, nullptr, nullptr, nullptr, true, &res[i], s, true);
    if (r < 0) return r;
    worst = worse(worst, r);
  }
  return worst;
}

// Carry src's warm-start data (pressure, contact set) into dst, a state of
// the same handle, on stream s.
int state_copy(bem_state_s* dst, const bem_state_s* src, hipStream_t s) {
  if (src->precision < 0 || !src->has_p) return BEM_OK;
  int rc = ensure_precision(dst, src->precision, s);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(dst->p, src->p, src->n * tsize(src->precision),
                                hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dst->mask, src->mask, src->n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "state copy");
  dst->has_p = src->has_p;
  dst->has_mask = src->has_mask;
  dst->g_valid = false;   // g is not copied
  dst->pending_import = dst->import_mask = false;
  std::copy(src->last_iters, src->last_iters + 3, dst->last_iters);
  return BEM_OK;
}

int upload_h(bem_state_t st, const double* h, hipStream_t s) {
  for (size_t i = 0; i < st->n; ++i)
    if (!is_finite(h[i])) return set_error(BEM_EINVAL, "bem_solve: non-finite gap profile");
  hipError_t e = hipMemcpyAsync(st->h64, h, st->n * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "gap profile upload");
  return BEM_OK;
}

}  // namespace

// A solve on the gap profile the state already holds (the previous solve's),
// as the next step of a sweep (see sweep_steps); host outputs.
int bem::solve_same_h(bem_influence_t K, const bem_params* prm, bem_state_t st, double* p_out,
                      unsigned char* c_out, bem_result* res, hipStream_t s) {
  clear_error();
  if (!K || !prm || !st) return set_error(BEM_EINVAL, "solve_same_h: NULL argument");
  return solve_common(K, st->h64, prm, st, p_out, c_out, nullptr, true, res, s, true);
}

extern "C" {

void bem_params_init(bem_params* prm) {
  if (!prm) return;
  std::memset(prm, 0, sizeof(*prm));
  prm->control = BEM_CTRL_INDENT;
  prm->precision = BEM_FP64;
}

int bem_state_create(bem_influence_t K, bem_state_t* out) {
  clear_error();
  if (!K || !out) return set_error(BEM_EINVAL, "bem_state_create: NULL argument");
  auto* st = new bem_state_s();
  st->K = K;
  st->n = (size_t)K->nx * K->ny;
  int rc;
  if ((rc = salloc(st, (void**)&st->mask, st->n, "contact set")) ||
      (rc = salloc(st, (void**)&st->h64, st->n * sizeof(double), "gap profile")) ||
      (rc = salloc(st, (void**)&st->out64, st->n * sizeof(double), "output staging")) ||
      (rc = salloc(st, (void**)&st->part, kPartials * sizeof(double), "partial sums")) ||
      (rc = salloc(st, (void**)&st->sc, sizeof(CgScal), "solver scalars"))) {
    bem_state_free(st);
    return rc;
  }
  hipError_t e = hipHostMalloc((void**)&st->sc_host, sizeof(CgScal), hipHostMallocDefault);
  if (e != hipSuccess) {
    bem_state_free(st);
    return hip_fail(e, "pinned scalars");
  }
  // hipMemset runs on the null stream and may return before it lands; the
  // state is then used on the caller's stream, possibly a non-blocking one
  // that does not order after the null stream, so wait for it here
  e = hipMemset(st->sc, 0, sizeof(CgScal));
  if (e == hipSuccess) e = hipMemset(st->mask, 0, st->n);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    bem_state_free(st);
    return hip_fail(e, "state init");
  }
  *out = st;
  return BEM_OK;
}

int bem_state_free(bem_state_t st) {
  if (!st) return BEM_OK;
  free_typed(st);
  for (void* q : {(void*)st->mask, (void*)st->h64, (void*)st->out64, (void*)st->part, (void*)st->sc})
    if (q) hipFree(q);
  if (st->sc_host) hipHostFree(st->sc_host);
  delete st;
  return BEM_OK;
}

int bem_state_reset(bem_state_t st) {
  clear_error();
  if (!st) return set_error(BEM_EINVAL, "bem_state_reset: NULL state");
  st->has_p = st->has_mask = st->pending_import = st->import_mask = st->g_valid = false;
  st->last_iters[0] = st->last_iters[1] = st->last_iters[2] = 0;
  return BEM_OK;
}

int bem_state_set(bem_state_t st, const double* p, const unsigned char* contact) {
  clear_error();
  if (!st) return set_error(BEM_EINVAL, "bem_state_set: NULL state");
  std::vector<double> zeros;
  if (!p) {
    zeros.assign(st->n, 0.0);
    p = zeros.data();
  }
  for (size_t i = 0; i < st->n; ++i)
    if (!is_finite(p[i])) return set_error(BEM_EINVAL, "bem_state_set: non-finite pressure");
  hipError_t e = hipMemcpy(st->out64, p, st->n * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess && contact) e = hipMemcpy(st->mask, contact, st->n, hipMemcpyHostToDevice);
  // a copy from pageable memory may return before the device write lands
  // (null stream; see bem_state_create)
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "bem_state_set");
  st->pending_import = true;
  st->import_mask = contact != nullptr;
  st->has_p = false;
  st->has_mask = false;
  return BEM_OK;
}

int bem_state_get(bem_state_t st, double* p, unsigned char* contact) {
  clear_error();
  if (!st) return set_error(BEM_EINVAL, "bem_state_get: NULL state");
  hipError_t e = hipSuccess;
  if (p) {
    if (st->pending_import) {
      e = hipMemcpy(p, st->out64, st->n * sizeof(double), hipMemcpyDeviceToHost);
    } else if (!st->has_p) {
      std::memset(p, 0, st->n * sizeof(double));
    } else {
      e = st->precision == BEM_FP64
              ? launch_to_f64<double>((const double*)st->p, st->out64, st->n, nullptr)
              : launch_to_f64<float>((const float*)st->p, st->out64, st->n, nullptr);
      if (e == hipSuccess) e = hipMemcpy(p, st->out64, st->n * sizeof(double), hipMemcpyDeviceToHost);
    }
  }
  if (e == hipSuccess && contact) e = hipMemcpy(contact, st->mask, st->n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "bem_state_get");
  return BEM_OK;
}

int bem_solve(bem_influence_t K, const double* h, const bem_params* prm, bem_state_t state,
              double* p_out, unsigned char* contact_out, double* u_out, bem_result* res,
              void* stream) {
  clear_error();
  if (!K || !h) return set_error(BEM_EINVAL, "bem_solve: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  bem_state_t tmp = nullptr;
  int rc;
  if (!state) {
    if ((rc = bem_state_create(K, &tmp))) return rc;
    state = tmp;
  }
  rc = upload_h(state, h, s);
  if (rc == BEM_OK)
    rc = solve_common(K, state->h64, prm, state, p_out, contact_out, u_out, true, res, s);
  if (tmp) bem_state_free(tmp);
  return rc;
}

int bem_solve_dev(bem_influence_t K, const double* h, const bem_params* prm, bem_state_t state,
                  double* p_out, unsigned char* contact_out, double* u_out, bem_result* res,
                  void* stream) {
  clear_error();
  if (!K || !h) return set_error(BEM_EINVAL, "bem_solve_dev: NULL argument");
  return solve_common(K, h, prm, state, p_out, contact_out, u_out, false, res, (hipStream_t)stream);
}

int bem_sweep(bem_influence_t K, const double* h, const bem_params* prm, const double* d_list,
              int n_steps, bem_state_t state, bem_result* res, void* stream) {
  clear_error();
  if (!K || !h || !prm || !d_list || !res || n_steps < 0)
    return set_error(BEM_EINVAL, "bem_sweep: invalid argument");
  for (int i = 0; i < n_steps; ++i)
    if (!is_finite(d_list[i])) return set_error(BEM_EINVAL, "bem_sweep: non-finite step value");
  hipStream_t s = (hipStream_t)stream;
  bem_state_t tmp = nullptr;
  int rc;
  if (!state) {
    if ((rc = bem_state_create(K, &tmp))) return rc;
    state = tmp;
  }
  rc = upload_h(state, h, s);
  if (rc == BEM_OK) rc = sweep_steps(K, state->h64, prm, d_list, n_steps, 0, 1, state, res, s);
  if (tmp) bem_state_free(tmp);
  return rc;
}

int bem_sweep_dev(bem_influence_t K, const double* h, const bem_params* prm, const double* d_list,
                  int n_steps, int chains, bem_state_t state, bem_result* res, void* stream) {
  clear_error();
  if (!K || !h || !prm || !d_list || !res || n_steps < 0 || chains < 1 || chains > 8)
    return set_error(BEM_EINVAL, "bem_sweep_dev: invalid argument (1 <= chains <= 8)");
  for (int i = 0; i < n_steps; ++i)
    if (!is_finite(d_list[i])) return set_error(BEM_EINVAL, "bem_sweep_dev: non-finite step value");
  if (state && state->K != K)
    return set_error(BEM_EINVAL, "bem_sweep_dev: state belongs to another influence handle");
  const bool adhesive = prm->gamma > 0.0 || prm->p_crit > 0.0;
  if (adhesive && chains > 1)
    return set_error(BEM_EUNSUPPORTED,
                     "bem_sweep_dev: an adhesive sweep depends on its path; chains must be 1");
  hipStream_t s0 = (hipStream_t)stream;
  chains = std::max(1, std::min(chains, n_steps));
  bem_state_t tmp = nullptr;
  int rc;
  if (!state) {
    if ((rc = bem_state_create(K, &tmp))) return rc;
    state = tmp;
  }
  if (chains == 1) {
    rc = sweep_steps(K, h, prm, d_list, n_steps, 0, 1, state, res, s0);
    if (tmp) bem_state_free(tmp);
    return rc;
  }
  // chain c > 0: a state and a non-blocking stream of its own, ordered
  // after the work already queued on the caller's stream
  std::vector<bem_state_t> st(chains, nullptr);
  std::vector<hipStream_t> ss(chains, nullptr);
  st[0] = state;
  ss[0] = s0;
  hipEvent_t ready = nullptr;
  hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ready, s0);
  rc = e == hipSuccess ? BEM_OK : hip_fail(e, "bem_sweep_dev: event");
  for (int c = 1; rc == BEM_OK && c < chains; ++c) {
    rc = bem_state_create(K, &st[c]);
    if (rc == BEM_OK) {
      e = hipStreamCreateWithFlags(&ss[c], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamWaitEvent(ss[c], ready, 0);
      if (e != hipSuccess) rc = hip_fail(e, "bem_sweep_dev: stream");
    }
  }
  if (rc == BEM_OK) {
    std::vector<int> rcs(chains, BEM_OK);
    std::vector<std::string> msgs(chains);
    const std::thread::id caller = std::this_thread::get_id();
    auto run = [&](int c) {
      if (std::this_thread::get_id() != caller) (void)hipSetDevice(K->device);
      rcs[c] = sweep_steps(K, h, prm, d_list, n_steps, c, chains, st[c], res, ss[c]);
      if (rcs[c] < 0) msgs[c] = bem_last_error();
      const hipError_t es = hipStreamSynchronize(ss[c]);
      if (es != hipSuccess && rcs[c] >= 0) {
        rcs[c] = BEM_EDEVICE;
        msgs[c] = std::string("bem_sweep_dev: ") + hipGetErrorString(es);
      }
    };
    // a chain whose thread cannot be started runs on this thread afterwards
    std::vector<std::thread> workers;
    std::vector<int> inline_chains;
    for (int c = 1; c < chains; ++c) {
      try {
        workers.emplace_back(run, c);
      } catch (const std::system_error&) {
        inline_chains.push_back(c);
      }
    }
    run(0);
    for (const int c : inline_chains) run(c);
    for (auto& w : workers) w.join();
    int worst = BEM_OK;
    const char* msg = nullptr;
    for (int c = 0; c < chains; ++c) {
      if (rcs[c] < 0 && !msg) msg = msgs[c].c_str();
      worst = worse(worst, rcs[c]);
    }
    if (msg) set_error(worst, "%s", msg);
    rc = worst;
    // the caller's state ends with the last step's pressure and contact set
    const int last = (n_steps - 1) % chains;
    if (rc >= 0 && last != 0) {
      const int r = state_copy(state, st[last], s0);
      rc = r ? r : rc;
      if (r == BEM_OK && (e = hipStreamSynchronize(s0)) != hipSuccess)
        rc = hip_fail(e, "bem_sweep_dev: state copy");
    }
  }
  for (int c = 1; c < chains; ++c) {
    if (ss[c]) (void)hipStreamDestroy(ss[c]);
    if (st[c]) bem_state_free(st[c]);
  }
  if (ready) (void)hipEventDestroy(ready);
  if (tmp) bem_state_free(tmp);
  return rc;
}

double bem_c1(double k) { return c1_table(k); }

double bem_p_crit(double k, double nu, double gamma, double dx, double E0, double c0) {
  if (!(k > -1.0 && k < 1.0) || !(nu >= 0.0 && nu < 0.5) || !(gamma >= 0.0) || !(dx > 0.0) ||
      !(E0 > 0.0) || !(c0 > 0.0))
    return std::nan("");
  return p_crit_eq24(k, nu, gamma, dx, E0, c0);
}

}  // extern "C"
