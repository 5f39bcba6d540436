/*
 * bem.h -- C ABI of the MI355X (gfx950) boundary element library for normal
 * non-adhesive and adhesive contact of power-law graded elastic half-spaces,
 * after Li & Popov, "Boundary element method for normal non-adhesive and
 * adhesive contacts of power-law graded elastic materials" (arXiv:1612.08395).
 *
 * Material (Section 2.1, Eq. 1): E(z) = E0 (z / c0)^k with -1 < k < 1 and a
 * constant Poisson ratio nu.  Surface: nx x ny rectangular elements of size
 * dx x dy carrying constant pressure, collocation at element centres.
 *
 * Conventions shared by every entry point
 *  - Arrays are row-major ny x nx (row index y, x contiguous), FP64 unless
 *    stated.  Host arrays are owned by the caller; they are read or written
 *    only during the call and never retained.
 *  - Device-pointer variants (suffix _dev) take pointers into the memory of
 *    the current HIP device; their element type is given per argument.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Host-array entry
 *    points return after the stream has finished their work; _dev entry
 *    points return once the work is queued.
 *  - Signs: pressure p > 0 is compressive; displacement u > 0 points into
 *    the half-space; h is the gap between the undeformed surfaces; the gap
 *    after deformation is g = u + h - d (contact: g = 0, separation: g > 0).
 *  - Every function returns an int status: 0 success, > 0 a warning (the
 *    outputs are valid), < 0 an error (outputs untouched unless stated).
 *    bem_last_error() returns a message for the calling thread.
 *  - Handles are library-owned, hold device memory of the device that was
 *    current when they were created, and are released with the matching
 *    _free call.  One handle may be used from several threads only if the
 *    calls do not overlap.
 */
#ifndef BEM_H
#define BEM_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BEM_OK = 0,
  BEM_ENOCONV = 1,       /* warning: iteration limit reached; outputs hold the last iterate */
  BEM_EFLOOR = 2,        /* warning: MIXED solve stopped at its FP32 rounding floor */
  BEM_EINVAL = -1,       /* invalid argument (range, size, non-finite input) */
  BEM_ENOMEM = -2,       /* device memory allocation failed */
  BEM_EDEVICE = -3,      /* HIP runtime error */
  BEM_EUNSUPPORTED = -4, /* valid request outside what this library implements */
  BEM_ENUMERIC = -5      /* non-finite value appeared during a solve */
};

/* Arithmetic of the convolution and vector updates.  Influence coefficients,
 * kernel spectrum generation, dot products / step lengths and force / area
 * sums are FP64 in both. */
enum { BEM_FP64 = 0, BEM_MIXED = 1 };

typedef struct bem_influence_s* bem_influence_t;

/* Largest supported grid side (padded transform 8192). */
#define BEM_MAX_N 4096

/*
 * bem_influence_ex -- build the influence operator of Section 2.1.
 *
 * Computes, in FP64 on the device, the influence coefficients of Eqs. 8-10,
 *   K(di, dj) = integral over [(di-1/2)dx, (di+1/2)dx] x [(dj-1/2)dy, (dj+1/2)dy]
 *               of (a^2 + b^2)^(-(1+k)/2) da db,
 * for 0 <= di < nx, 0 <= dj < ny, and the spectrum of K laid out on the
 * zero-padded My x Mx grid (Eq. 13; Mx, My = the smallest powers of two
 * >= max(2n, 64)), kept in FP64 and FP32 and pre-multiplied by
 *   C = alpha(k, nu) (1 - nu^2) c0^k / E0      (Eqs. 2-4, 12).
 * The paper computes this matrix once per calculation; reuse the handle.
 *
 * Errors: BEM_EINVAL if nx, ny < 1, dx, dy, E0, c0 <= 0 or non-finite,
 * k outside (-1, 1), nu outside [0, 0.5); BEM_EUNSUPPORTED if nx or ny
 * exceeds BEM_MAX_N; BEM_ENOMEM, BEM_EDEVICE.  *out is set only on success.
 */
int bem_influence_ex(int nx, int ny, double dx, double dy, double k, double nu, double E0,
                     double c0, bem_influence_t* out);

/* bem_influence -- square elements (dy = dx) and E0 = c0 = 1. */
int bem_influence(int nx, int ny, double dx, double k, double nu, bem_influence_t* out);

int bem_influence_free(bem_influence_t K);

/* Scalars of a handle: the prefactor C of Eq. 12, alpha of Eq. 3, K(0, 0),
 * the padded transform sizes and the device bytes the handle holds. */
typedef struct {
  int nx, ny, Mx, My;
  double dx, dy, k, nu, E0, c0;
  double alpha, C, K00;
  long long device_bytes;
} bem_influence_info_t;
int bem_influence_info(bem_influence_t K, bem_influence_info_t* info);

/*
 * bem_influence_coeffs -- copy the influence coefficients to the host.
 * K_out: (2ny - 1) x (2nx - 1) FP64, row-major, offset (di, dj) at row
 * dj + ny - 1, column di + nx - 1 (K is even in both offsets, Eq. 10).
 */
int bem_influence_coeffs(bem_influence_t K, double* K_out);

/*
 * bem_convolve -- surface displacement from pressure, Eqs. 7 / 12 / 13:
 *   u(i, j) = C * sum_{i', j'} K(i - i', j - j') p(i', j'),
 * the non-periodic half-space sum, evaluated as a zero-padded FFT product
 * in FP64.  p, u: host, ny x nx FP64 (may not alias).
 */
int bem_convolve(bem_influence_t K, const double* p, double* u, void* stream);

/*
 * bem_convolve_dev -- the same on device arrays, in the given precision:
 * precision BEM_FP64: p, u are double*; BEM_MIXED: float* (FP32 transforms).
 * p and u are ny x nx device arrays and may alias.  Uses a scratch buffer
 * owned by the handle: calls on one handle must not run concurrently on
 * different streams.
 */
int bem_convolve_dev(bem_influence_t K, int precision, const void* p, void* u, void* stream);

/*
 * bem_convolve_dev_noalloc -- bem_convolve_dev for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results, with the
 * row spectrum in a fixed array of BEM_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, so the call makes
 * no allocation of any kind.  The caller still passes p and u (device arrays
 * as for bem_convolve_dev).  The handle's device must be current.
 * Errors: BEM_EINVAL (NULL argument, bad precision, another device current),
 * BEM_EUNSUPPORTED when ny (rounded up to even) * Lx complex values of the
 * precision (Lx = Mx / 2,
 * bem_influence_info) exceed BEM_NOALLOC_SCRATCH_BYTES (16 MiB: up to
 * 1024 x 1024 in FP64, 2048 x 1024 in FP32), BEM_EDEVICE.
 * All calls on one device share the array: calls that overlap on a device
 * (other streams, other threads) race and must be ordered by the caller.
 */
#define BEM_NOALLOC_SCRATCH_BYTES (16 << 20)
int bem_convolve_dev_noalloc(bem_influence_t K, int precision, const void* p, void* u,
                             void* stream);

/* ---------------------------------------------------------------------------
 * Contact solves
 * ------------------------------------------------------------------------- */

typedef struct bem_state_s* bem_state_t;

enum { BEM_CTRL_INDENT = 0, BEM_CTRL_FORCE = 1 };

typedef struct {
  int control;       /* BEM_CTRL_INDENT: indentation d given; BEM_CTRL_FORCE:
                        normal force F given, d found (non-adhesive only) */
  int precision;     /* BEM_FP64 or BEM_MIXED */
  double d;          /* indentation: rigid-body approach of the indenter */
  double F;          /* prescribed normal force dx dy sum p (BEM_CTRL_FORCE),
                        >= 0 */
  double gamma;      /* work of adhesion gamma12 (Eq. 20); 0 = non-adhesive */
  double p_crit;     /* > 0: detachment stress used as given; <= 0: from gamma
                        by Eq. 24 with the corrected c1(k) of Table 1 */
  double d_preload;  /* adhesive solve without a contact set in the state:
                        the set is first made by a non-adhesive solve at
                        max(d, d_preload) (Section 3.1) */
  double tol;        /* relative tolerance; <= 0: 1e-12 (FP64), 1e-6 (MIXED) */
  int max_iter;      /* CG iteration limit per solve; <= 0: 20000 */
  int stall_limit;   /* stop after max(stall_limit, half the iterations so far)
                        iterations without a new smallest residual (MIXED
                        rounding floor); < 0: never; 0: default (50 for
                        MIXED, never for FP64) */
} bem_params;

/* Fills *prm with the defaults (indentation control, FP64, d = 0, no
 * adhesion). */
void bem_params_init(bem_params* prm);

typedef struct {
  double F;                  /* normal force dx dy sum p (FP64 sum) */
  double area;               /* contact area: contact elements * dx dy */
  double d;                  /* indentation of this solve (found, under force
                                control: the mean of u + h over the contact) */
  double residual;           /* final sqrt(sum_Ic g^2) / sqrt(sum_Ic (d-h)^2)
                                (force control: / sqrt(sum_Ic u^2)) */
  double p_crit;             /* detachment stress used (adhesive), else 0 */
  long long n_contact;       /* elements in contact */
  long long n_penetrating;   /* adhesive: elements off the contact set with g < 0 */
  int iters;                 /* CG iterations of this solve (all detach rounds) */
  int detach_rounds;         /* adhesive: rounds that removed elements */
  int status;                /* BEM_OK, BEM_ENOCONV, BEM_EFLOOR or BEM_ENUMERIC */
} bem_result;

/* Solver state: pressure, contact set and work buffers, device-resident.
 * A state carries the previous solve's pressure and contact set into the
 * next solve (warm start); a fresh state has neither. */
int bem_state_create(bem_influence_t K, bem_state_t* out);
int bem_state_free(bem_state_t st);
/* Import / export the warm-start data as host arrays (checkpoint / resume).
 * p: ny x nx FP64 (NULL on set = zeros); contact: ny x nx bytes, non-zero =
 * in contact (NULL on set: p > 0). */
int bem_state_set(bem_state_t st, const double* p, const unsigned char* contact);
int bem_state_get(bem_state_t st, double* p, unsigned char* contact);
/* Forget the warm-start data: the next solve starts cold, exactly as with a
 * fresh state (buffers are kept). */
int bem_state_reset(bem_state_t st);

/*
 * bem_solve -- one contact solve at indentation prm->d (or under the normal
 * force prm->F) for the gap profile h (host, ny x nx FP64, the gap between
 * the undeformed surfaces).
 *
 * Non-adhesive (gamma = 0 and p_crit <= 0): pressure p >= 0 with g = 0 where
 * p > 0 and g >= 0 elsewhere, by the constrained conjugate-gradient method
 * the paper uses for its inverse problem (Section 2.1), displacement
 * controlled.  The solution is unique; a warm start changes only the
 * iteration count.
 *
 * Force control (control = BEM_CTRL_FORCE, the problem statement of Section
 * 2.2 with F_N given): the same method in its load-controlled form (gap
 * shifted by its mean over the contact, pressure rescaled to carry F after
 * each update); res->d returns the indentation found.  Cold start: uniform
 * pressure.  F = 0: p = 0 and d = min h.  Non-adhesive only.
 *
 * Adhesive (gamma > 0 or p_crit > 0), one pull-off step of Section 3.1: with
 * the state's contact set A held fixed, u = d - h on A and p = 0 off A; then
 * every element of A with -p > p_crit detaches, all at once, and the solve is
 * repeated until no element violates the criterion (Eq. 24).  Adhesion
 * requires dx = dy (Eqs. 21-24 are for square elements), else
 * BEM_EUNSUPPORTED.
 *
 * state: NULL = a temporary state (cold start); otherwise used and updated.
 * p_out (FP64), contact_out (bytes, 1 = contact), u_out (FP64 surface
 * displacement): host ny x nx arrays or NULL.  res: may be NULL.
 * Returns BEM_OK, BEM_ENOCONV / BEM_EFLOOR (warnings; outputs hold the last
 * iterate), BEM_ENUMERIC, BEM_EINVAL (non-finite h or d, bad parameters),
 * BEM_EUNSUPPORTED (force control with adhesion; adhesion with dx != dy).
 */
int bem_solve(bem_influence_t K, const double* h, const bem_params* prm, bem_state_t state,
              double* p_out, unsigned char* contact_out, double* u_out, bem_result* res,
              void* stream);

/* bem_solve_dev -- as bem_solve with device arrays: h, p_out, u_out are
 * double*, contact_out unsigned char* (each output may be NULL).  h is read
 * in place (not copied); non-finite values in it surface as BEM_ENUMERIC. */
int bem_solve_dev(bem_influence_t K, const double* h, const bem_params* prm, bem_state_t state,
                  double* p_out, unsigned char* contact_out, double* u_out, bem_result* res,
                  void* stream);

/*
 * bem_sweep -- a sequence of solves at the indentations d_list[0..n_steps)
 * (under force control: at the normal forces d_list[0..n_steps)),
 * warm-started from step to step on the device (Section 3.1).  With
 * adhesion, a step whose d is below the previous step's is a pull-off step
 * (adhesive solve); every other step is a non-adhesive (loading) solve.
 * A displacement-controlled step that follows another on the same state
 * takes its first gap from the previous step's (h is the same, only d moves)
 * instead of a convolution; results are those of separate warm-started solves.
 * h: host ny x nx FP64.  res: n_steps results.  state: NULL = temporary.
 */
int bem_sweep(bem_influence_t K, const double* h, const bem_params* prm, const double* d_list,
              int n_steps, bem_state_t state, bem_result* res, void* stream);

/*
 * bem_sweep_dev -- the indentation sweep of bem_sweep (Sections 2.2, 3.1)
 * with the gap profile h on the device (ny x nx FP64, read in place, not
 * copied) and the steps split over `chains` (1..8) warm-start chains: chain
 * c solves steps c, c + chains, c + 2 chains, ..., each warm-started from
 * the chain's previous step, and the chains run
 * concurrently on the GPU (chain 0 on `stream` in `state`, chain c > 0 in a
 * state and on a non-blocking stream of its own, after the work already
 * queued on `stream`; one host thread per chain).  Each non-adhesive step
 * has one solution, so the chains change iteration counts, not results
 * (within the tolerance).  Kernels of one chain fill the gaps of another:
 * on a 2048^2 mixed sweep, 2 chains give about 10 % more solves/s than 1.
 * On return, `state` holds the last step's pressure and contact set.
 * chains = 1 is the sequential sweep of bem_sweep (adhesive sweeps, whose
 * pull-off steps depend on the path, need chains = 1: else
 * BEM_EUNSUPPORTED).  The solver clock records chain 0 only.
 */
int bem_sweep_dev(bem_influence_t K, const double* h, const bem_params* prm, const double* d_list,
                  int n_steps, int chains, bem_state_t state, bem_result* res, void* stream);

/* Corrected c1(k) of Table 1: the tabulated value at k = -0.9, ..., 0.9 and a
 * natural cubic spline of ln c1 over k in between (NaN outside (-1, 1)). */
double bem_c1(double k);

/* Detachment stress of Eq. 24 for square elements of side dx, with c1 from
 * bem_c1 (NaN on invalid arguments). */
double bem_p_crit(double k, double nu, double gamma, double dx, double E0, double c0);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent solves on one GPU
 * ------------------------------------------------------------------------- */

/* Device bytes of an influence handle and of one solver state for a grid,
 * as the server's admission control counts them. */
int bem_footprint(int nx, int ny, int precision, long long* influence_bytes,
                  long long* state_bytes);

typedef struct bem_server_s* bem_server_t;

typedef struct {
  int nx, ny;                 /* grid and material: the influence cache key */
  double dx, dy, k, nu, E0, c0;
  const double* h;            /* host ny x nx gap profile, copied at submit */
  bem_params prm;             /* indentation, adhesion, precision, tolerances */
  double* p_out;              /* optional host ny x nx pressure output; must stay valid
                                 until bem_server_poll reports the request done */
  unsigned char* contact_out; /* optional host ny x nx contact output (same rule) */
} bem_request;

typedef struct {
  long long completed, failed, queued;
  int running, peak_running;
  double p50_latency_s, p99_latency_s;  /* submit -> result, completed requests */
  double mean_wait_s;                   /* submit -> start */
  double solves_per_s;                  /* completed / (last completion - first submit) */
  long long device_bytes_reserved, cache_entries, cache_hits, cache_misses, evictions;
  long long batched;                    /* completed on the batched path */
  double mean_batch_slots;              /* mean solves per batched launch chunk */
  double engine_launch_s;               /* batched path's thread: queueing launches, */
  double engine_sync_s;                 /* waiting for the GPU, */
  double engine_step_s;                 /* stepping the solves between chunks (s) */
} bem_server_stats_t;

/*
 * bem_server_create_ex -- a request loop on the current device with a
 * device-memory budget for cached influence operators plus solver states
 * (bem_footprint); a queued request starts as soon as the budget admits it
 * (idle cache entries are evicted least-recently-used) and runs on the GPU
 * together with the requests already in progress.
 *  - Batched path (batch_slots > 0): displacement-controlled requests with
 *    nx, ny <= 256 are grouped by padded geometry and precision; each group
 *    runs up to batch_slots solves whose conjugate-gradient kernels share
 *    launches (one launch per kernel for all of them), admitting queued
 *    requests as slots free up between chunks of iterations.
 *  - Per-request path: every other request (larger grids, load control, or
 *    all requests when batch_slots = 0) is a bem_solve of its own on one of
 *    n_slots (1..16) worker threads, each with its own non-blocking stream.
 * Every request outside a session (below) is solved from a cold start with
 * the kernels and order of bem_solve, so its result does not depend on what
 * else runs.
 * batch_slots: 0..64.
 */
int bem_server_create_ex(long long budget_bytes, int n_slots, int batch_slots, bem_server_t* out);
/* bem_server_create -- bem_server_create_ex with batch_slots = 16. */
int bem_server_create(long long budget_bytes, int n_slots, bem_server_t* out);
/* Queue a request; *id identifies it.  BEM_ENOMEM if it can never fit the
 * budget, BEM_EINVAL for a bad grid. */
int bem_server_submit(bem_server_t srv, const bem_request* req, long long* id);
/*
 * Sessions: the solver state resident on the device across requests.  A
 * client that solves one indenter through a sequence of loads (a loading /
 * unloading curve, Section 3.1) opens a session and submits its requests to
 * it.  The server keeps one solver state for the session between its
 * requests and runs them one at a time, in submission order: each starts
 * from the previous request's pressure and contact set.  On the batched path
 * (see bem_server_create_ex) a request is then exactly bem_solve with that
 * state; on the per-request path a request whose gap profile is the same as
 * the previous request's also starts from that request's gap shifted to the
 * new indentation, exactly as the steps of bem_sweep.  Either way the
 * results are bitwise those of the corresponding library calls on one
 * state.  Loading steps are non-adhesive requests; pull-off steps are
 * adhesive requests, which hold the state's contact set fixed (bem_solve).
 *
 * bem_server_session_open: *session identifies the new session (> 0).
 * bem_server_submit_session: as bem_server_submit; the first request fixes
 *   the session's grid, material and precision, later ones must match
 *   (BEM_EINVAL otherwise, or for an unknown or closed session).  Requests
 *   of other clients keep running while one of the session's waits for its
 *   predecessor.  Poll them with bem_server_poll.
 * bem_server_session_close: no more requests; the state returns to the
 *   server's pool once the session's last request has completed.  An open
 *   session keeps its influence operator and state reserved in the budget.
 */
int bem_server_session_open(bem_server_t srv, long long* session);
int bem_server_submit_session(bem_server_t srv, long long session, const bem_request* req,
                              long long* id);
int bem_server_session_close(bem_server_t srv, long long session);
/* Returns 1 while the request is pending (wait = 0), else 0 with *res and
 * *status (the bem_solve status) filled in; the id is then released.  With
 * wait != 0 blocks until the request is done. */
int bem_server_poll(bem_server_t srv, long long id, int wait, bem_result* res, int* status);
int bem_server_stats(bem_server_t srv, bem_server_stats_t* out);
int bem_server_reset_stats(bem_server_t srv);
/* Stops the workers after their current solves; queued requests are dropped. */
int bem_server_free(bem_server_t srv);

/*
 * bem_kernel_time -- measurement hook: average duration (ms, from two HIP
 * events on `stream`) of `reps` back-to-back launches of one sweep of the
 * convolution of Eq. 13 on the handle's grid: which = 0 row R2C transform,
 * 1 column transform x kernel spectrum x inverse transform, 2 row C2R
 * transform, 3 column transform and spectral energy sum_k Khat |T|^2 (the
 * solver's second convolution, which only needs that inner product).  Runs on a zero field in the handle's scratch buffers (same
 * kernels and launch shapes as the solver's sweeps).  Synchronises `stream`.
 */
int bem_kernel_time(bem_influence_t K, int precision, int which, int reps, void* stream,
                    double* avg_ms);

/*
 * Solver clock -- measurement hook for the conjugate-gradient loop of the
 * contact solve (the constrained CG method of Section 2.1, which the paper
 * cites for its inverse problem after Eqs. 12-13).  Each iteration is
 * reported as six launch kinds:
 *   0 pressure update + row R2C,  1 column sweep,  2 row C2R + gap,
 *   3 direction + row R2C,        4 column transform of the direction with
 *   the spectral inner product sum t (C K * t)  (force control: full column
 *   sweep),  5 row C2R + dot products (force control only; otherwise no
 *   launch and a zero-length interval).
 * In a sweep, iteration 0 of a step that starts from the previous step's
 * gap has no kinds 0-2 but one gap-shift launch instead, reported as
 * `shifts` / `shift_ms` (it belongs to the iteration count).
 * After bem_clock_start, every bem_solve / bem_solve_dev / bem_sweep made BY
 * THE CALLING THREAD records a HIP event on its solver stream before the
 * first launch of each queued chunk and after every launch; no extra host
 * synchronisation is added.  bem_clock_stop resolves the events and returns,
 * per launch kind, the number of launches and their summed event-to-event
 * durations, counting only iterations the solver actually worked on; the
 * launches queued past convergence (which return at once) are summed
 * separately.  Durations include the command processor's dispatch gap
 * between back-to-back launches (about a microsecond).  Not for server
 * worker threads.  bem_clock_stop on a thread without a running clock
 * returns BEM_EINVAL.
 */
typedef struct {
  long long iterations;    /* CG iterations worked on */
  long long launches[6];   /* launches per kind that did work */
  double ms[6];            /* their summed durations (ms) */
  long long skipped;       /* launches queued past convergence */
  double skipped_ms;       /* their summed durations (ms) */
  long long shifts;        /* gap-shift launches (first iteration of a sweep step) */
  double shift_ms;         /* their summed durations (ms) */
} bem_clock_t;
int bem_clock_start(void);
int bem_clock_stop(bem_clock_t* out);

/* Message describing the last failure on the calling thread ("" if none). */
const char* bem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
