// Serving loop: continuous batching of independent contact solves on one GPU.
//
// Requests (grid, material, gap profile, solve parameters) are admitted as
// device memory frees up (footprint model of bem_footprint(); influence
// operators cached by (nx, ny, dx, dy, k, nu, E0, c0) with pooled solver
// states, idle entries evicted least-recently-used) and run on the GPU
// together, new requests starting while others are still in progress.
//
//  * Batched path: small requests (nx, ny <= 256, displacement control)
//    join the runner of their class (Lx, Ly, precision).  A runner owns up to batch_slots slots; each
//    CG kernel is one launch over all slots of the class (batch.h), so small
//    grids share launches instead of each paying its own.  Between chunks of
//    iterations the runner retires converged slots (final sums, outputs),
//    takes the next queued request of its class into a free slot, and steps
//    each adhesive slot through its preload and detach / re-solve rounds.
//  * Per-request path: every other request (larger grids, load control) is
//    a bem_solve of its own on one of n_slots worker threads, each with its
//    own non-blocking stream.
//
// Each request is solved from a cold start with the same kernels in the same
// order as bem_solve, so its result does not depend on what else runs.
//
// Sessions: a client that solves one indenter through a sequence of loads
// opens a session; the server keeps one solver state on the device for it
// between its requests (one at a time, in submission order), so each request
// starts from the previous one's pressure and contact set: on the batched
// path as bem_solve with that state, on the per-request path also from the
// previous gap when the profile is the same (a step of a sweep, as in
// bem_sweep).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/bem.h"
#include "cg_api.h"
#include "internal.h"

using namespace bem;

namespace {

using Clock = std::chrono::steady_clock;

double secs(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double>(t - t0).count();
}

using Key = std::tuple<int, int, double, double, double, double, double, double>;

struct Entry {
  Key key;
  bem_influence_t K = nullptr;
  // pooled states per precision (index BEM_FP64 / BEM_MIXED): a state's
  // typed buffers are sized for the precision of the solve that created it,
  // so it is only ever lent to requests of that precision
  std::vector<bem_state_t> free_states[2];
  int in_use = 0;
  long long bytes = 0;  // reserved: influence + pooled / lent states
  bool building = false;
  unsigned long long last_use = 0;
};

struct Session;

struct Req {
  long long id;
  bem_request r;
  std::vector<double> h;
  Clock::time_point t_submit, t_start, t_end;
  bem_result res;
  int rc = 0;
  bool done = false;
  long long need_infl = 0, need_state = 0;
  bem_state_t lent = nullptr;  // pooled state handed over at admission
  bool builder = false;        // this request created the cache entry
  Entry* entry = nullptr;      // batched path: admitted entry (prepared by a worker)
  Session* session = nullptr;  // the session this request belongs to, if any
};

// A session's resident solver state.  The first request fixes the grid,
// material and precision and is admitted like any request; the session then
// holds that entry (one in_use count) and the state until it is closed and
// its last request has completed.  busy and pending change under the server
// lock; h_prev only in the worker running the session's request.
struct Session {
  long long id = 0;
  bool keyed = false;
  Key key;
  int prec = 0;
  Entry* e = nullptr;
  bem_state_t st = nullptr;
  std::vector<double> h_prev;  // gap profile of the state's last solve
  int pending = 0;             // submitted and not yet completed
  bool busy = false;           // one of its requests is running
  bool closed = false;
};

}  // namespace

namespace {
struct Runner;
using ClassKey = std::tuple<int, int, int>;   // Lx, Ly, precision
}  // namespace

struct bem_server_s {
  long long budget = 0;
  int n_slots = 0;
  int batch_slots = 0;
  std::map<ClassKey, Runner*> runners;
  std::vector<Runner*> runner_list;    // creation order (engine thread, under the lock)
  std::thread engine;                  // the batched path's launch thread
  std::vector<hipStream_t> engine_streams;
  long long batched = 0;             // requests completed on the batched path
  double eng_launch = 0, eng_sync = 0, eng_step = 0;  // engine thread seconds
  double slot_chunks = 0, chunks = 0; // occupancy: active slots summed over chunks
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<long long, Req*> reqs;
  std::unordered_map<long long, Session*> sessions;
  long long next_session = 1;
  std::map<Key, Entry*> cache;
  long long used = 0;
  long long next_id = 1;
  unsigned long long tick = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  // statistics
  Clock::time_point t0;
  bool have_first = false;
  Clock::time_point t_first_submit, t_last_end;
  std::vector<double> latency, wait;
  long long completed = 0, failed = 0, evictions = 0, cache_hits = 0, cache_misses = 0;
  int running = 0, peak_running = 0;
};

namespace {

void free_entry(Entry* e) {
  for (auto& pool : e->free_states) {
    for (bem_state_t s : pool) bem_state_free(s);
    pool.clear();
  }
  if (e->K) bem_influence_free(e->K);
  e->K = nullptr;
}

// Try to reserve memory for `r`; evicts idle cache entries if needed.
// Called with the lock held.  Returns the entry (created if missing), or
// nullptr if the request has to wait.  A pooled state, if any, is lent to
// the request here, so two admissions never count on the same state.
Entry* admit(bem_server_s* S, Req* r) {
  const bem_request& q = r->r;
  Key key{q.nx, q.ny, q.dx, q.dy, q.k, q.nu, q.E0, q.c0};
  const int prec = q.prm.precision;
  auto it = S->cache.find(key);
  Entry* e = it == S->cache.end() ? nullptr : it->second;
  long long need = 0;
  if (!e) need += r->need_infl;
  if (!e || e->free_states[prec].empty()) need += r->need_state;
  while (S->used + need > S->budget) {
    // evict the least recently used idle entry other than this one
    Entry* victim = nullptr;
    for (auto& kv : S->cache) {
      Entry* c = kv.second;
      if (c == e || c->in_use > 0 || c->building) continue;
      if (!victim || c->last_use < victim->last_use) victim = c;
    }
    if (!victim) return nullptr;   // wait for running solves to finish
    S->cache.erase(victim->key);
    S->used -= victim->bytes;
    free_entry(victim);
    delete victim;
    S->evictions++;
  }
  if (!e) {
    e = new Entry();
    e->key = key;
    e->building = true;
    e->bytes = r->need_infl;
    S->cache[key] = e;
    S->used += r->need_infl;
    S->cache_misses++;
    r->builder = true;
  } else {
    S->cache_hits++;
  }
  if (e->free_states[prec].empty()) {
    e->bytes += r->need_state;
    S->used += r->need_state;
  } else {
    r->lent = e->free_states[prec].back();
    e->free_states[prec].pop_back();
  }
  e->in_use++;
  e->last_use = ++S->tick;
  return e;
}

// Bookkeeping of a finished request (lock held): the state returns to its
// entry's pool, statistics, wake the poller and the admission loops.
void release_session_locked(bem_server_s* S, Session* ss);

void complete_locked(bem_server_s* S, Req* r, Entry* e, bem_state_t state, int rc) {
  if (Session* ss = r->session) {
    // the session keeps the state and its hold on the entry; after a failed
    // request its next one starts cold
    if (rc < 0) {
      if (state) bem_state_reset(state);
      ss->h_prev.clear();
    }
    ss->st = state;
    ss->busy = false;
    ss->pending--;
    if (e) e->last_use = ++S->tick;
    if (ss->closed && ss->pending == 0) release_session_locked(S, ss);
  } else if (e) {
    if (state) e->free_states[r->r.prm.precision].push_back(state);
    e->in_use--;
    e->last_use = ++S->tick;
    if (!e->K && !e->building && e->in_use == 0) {  // failed build: drop the entry once unused
      S->cache.erase(e->key);
      S->used -= e->bytes;
      free_entry(e);
      delete e;
    }
  }
  r->rc = rc;
  r->t_end = Clock::now();
  r->done = true;
  S->running--;
  if (rc >= 0) {
    S->completed++;
    S->latency.push_back(secs(r->t_submit, r->t_end));
    S->wait.push_back(secs(r->t_submit, r->t_start));
    S->t_last_end = r->t_end;
  } else {
    S->failed++;
  }
  r->h.clear();
  r->h.shrink_to_fit();
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

// A closed session without pending requests (lock held): its state goes to
// the entry's pool, its hold on the entry ends.
void release_session_locked(bem_server_s* S, Session* ss) {
  if (Entry* e = ss->e) {
    if (ss->st) e->free_states[ss->prec].push_back(ss->st);
    e->in_use--;
    e->last_use = ++S->tick;
    if (!e->K && !e->building && e->in_use == 0) {  // failed build: drop the entry
      S->cache.erase(e->key);
      S->used -= e->bytes;
      free_entry(e);
      delete e;
    }
  }
  S->sessions.erase(ss->id);
  delete ss;
}

// Influence operator of an admitted request's entry: built here when the
// request created the entry, else waited for.  Returns BEM_OK or an error.
int entry_influence(bem_server_s* S, Req* r, Entry* e) {
  if (r->builder) {
    bem_influence_t K = nullptr;
    const bem_request& q = r->r;
    const int rc = bem_influence_ex(q.nx, q.ny, q.dx, q.dy, q.k, q.nu, q.E0, q.c0, &K);
    std::unique_lock<std::mutex> lk(S->mu);
    e->K = K;
    e->building = false;
    S->cv_done.notify_all();
    return rc;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return !e->building; });
  return e->K ? BEM_OK : BEM_EDEVICE;
}

// ---- batched path -------------------------------------------------------------

// Phases of a slot between chunks.
enum Phase {
  PH_FREE,
  PH_CG,          // a CG solve runs in the batch (mode DISP or FIXED)
  PH_FIN_DISP,    // final sums of the non-adhesive solve queued
  PH_DETACH,      // detachment of the fixed-set solve queued
  PH_FIN_FIXED,   // final sums of the adhesive step queued
  PH_OUT          // output copies queued
};

struct Slot {
  Req* r = nullptr;
  Entry* e = nullptr;
  bem_state_t st = nullptr;
  Phase ph = PH_FREE;
  int mode = BATCH_EMPTY, it0 = 0;
  bool adhesive = false;
  double pcrit = 0.0, tol = 0.0, resid = 0.0;
  int max_iter = 0, stall_limit = 0;
  int status = BEM_OK, iters = 0, rounds = 0;
};

struct Runner {
  bem_server_s* S = nullptr;
  int Lx = 0, Ly = 0, prec = 0, nslots = 0;
  std::deque<Req*> queue;         // this class's requests (server lock)
  // prepared by the worker threads (influence built, state typed, gap
  // profile on the device): the runner takes them into free slots
  std::deque<Req*> ready;
  int preparing = 0, active = 0;  // server lock
  hipStream_t stream = nullptr;
  CgScal* sc_dev = nullptr;       // one scalar block per slot
  CgScal* sc_host = nullptr;      // pinned mirror
  void* tab_dev = nullptr;        // BatchSlot<T>[nslots]
  void* tab_host = nullptr;       // pinned
  std::vector<Slot> slot;
  std::vector<int> fresh;         // slots filled at this round's admission
  int last_chunk_slots = 0;       // slots in this round's chunk
  hipEvent_t done_ev = nullptr;   // recorded after a round's launches
  bool in_flight = false;         // a round is queued on the stream
};

void runner_release(Runner* R) {
  if (R->done_ev) hipEventDestroy(R->done_ev);
  if (R->sc_dev) hipFree(R->sc_dev);
  if (R->tab_dev) hipFree(R->tab_dev);
  if (R->sc_host) hipHostFree(R->sc_host);
  if (R->tab_host) hipHostFree(R->tab_host);
}

int runner_alloc(Runner* R) {
  hipError_t e = hipEventCreateWithFlags(&R->done_ev, hipEventDisableTiming);
  const size_t tb = (size_t)R->nslots * std::max(sizeof(BatchSlot<float>), sizeof(BatchSlot<double>));
  if (e == hipSuccess) e = hipMalloc((void**)&R->sc_dev, R->nslots * sizeof(CgScal));
  if (e == hipSuccess) e = hipMalloc(&R->tab_dev, tb);
  if (e == hipSuccess) e = hipHostMalloc((void**)&R->sc_host, R->nslots * sizeof(CgScal), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&R->tab_host, tb, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(R->sc_dev, 0, R->nslots * sizeof(CgScal), R->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(R->stream);
  if (e != hipSuccess) return hip_fail(e, "batch runner");
  R->slot.assign(R->nslots, Slot());
  return BEM_OK;
}

template <typename T>
CgBufs<T> slot_bufs(Runner* R, int i) {
  bem_state_s* st = R->slot[i].st;
  return {(T*)st->p, (T*)st->t, (T*)st->g, (T*)st->hd, st->mask, (cplx<T>*)st->S, st->part,
          R->sc_dev + i};
}

// Scalars of a new CG solve of slot i (the bem_solve sequence: tolerances
// into a cleared block, then the prepare kernel).
template <typename T>
hipError_t slot_start_cg(Runner* R, int i, int mode) {
  Slot& sl = R->slot[i];
  CgScal* h = R->sc_host + i;
  std::memset(h, 0, sizeof(CgScal));
  h->tol = sl.tol;
  h->max_iter = sl.max_iter;
  h->stall_limit = sl.stall_limit;
  hipError_t e = hipMemcpyAsync(R->sc_dev + i, h, sizeof(CgScal), hipMemcpyHostToDevice, R->stream);
  if (e == hipSuccess)
    e = launch_prepare<T>((T*)sl.st->t, (T*)sl.st->p, sl.st->mask, mode == CG_FIXED, sl.st->n,
                          R->stream);
  sl.mode = mode;
  sl.it0 = 0;
  sl.ph = PH_CG;
  return e;
}

// Start a prepared request in slot i (influence, typed state and gap
// profile on the device already): cold start and the first CG solve, the
// bem_solve sequence.  Returns < 0 to fail the request.
template <typename T>
int slot_setup(Runner* R, int i) {
  Slot& sl = R->slot[i];
  Req* r = sl.r;
  bem_influence_s* K = sl.e->K;
  int rc = check_params(K, &r->r.prm, &sl.adhesive, &sl.pcrit);
  if (rc) return rc;
  const bem_params& P = r->r.prm;
  sl.tol = P.tol > 0 ? P.tol : (P.precision == BEM_FP64 ? 1e-12 : 1e-6);
  sl.max_iter = P.max_iter > 0 ? P.max_iter : 20000;
  sl.stall_limit = P.stall_limit > 0 ? P.stall_limit
                                     : (P.stall_limit < 0 ? 0 : (P.precision == BEM_MIXED ? 50 : 0));
  sl.status = BEM_OK;
  sl.iters = sl.rounds = 0;
  sl.resid = 0.0;
  bem_state_s* st = sl.st;
  st->g_valid = false;   // the batched kernels do not start from a shifted gap
  hipError_t e;
  if (sl.adhesive && st->has_mask) {
    // a pull-off step on the contact set the state holds (a session's
    // previous request): fixed-set solves at d at once
    e = launch_make_hd<T>(st->h64, P.d, (T*)st->hd, st->n, R->stream);
    if (e == hipSuccess) e = slot_start_cg<T>(R, i, CG_FIXED);
  } else {
    // an adhesive solve without a contact set first makes one non-adhesively
    // at max(d, d_preload) (Section 3.1); a state with a pressure (a
    // session's previous request) starts from it, else cold
    const double d0 = sl.adhesive ? std::max(P.d, P.d_preload) : P.d;
    e = launch_make_hd<T>(st->h64, d0, (T*)st->hd, st->n, R->stream);
    if (e == hipSuccess && !st->has_p)
      e = launch_cold_start<T>((T*)st->p, (const T*)st->hd, 1.0 / (K->C * K->K00), st->n,
                               R->stream);
    st->has_p = true;
    if (e == hipSuccess) e = slot_start_cg<T>(R, i, CG_DISP);
  }
  if (e != hipSuccess) return hip_fail(e, "batched solve setup");
  return BEM_OK;
}

// Worker-thread half of a batched request (outside the lock): influence
// operator, a state typed for the precision, and the gap profile on the
// device.  Then the request joins its runner's ready list, or fails.
void prepare_batched(bem_server_s* S, Runner* R, Req* r, hipStream_t s) {
  Entry* e = r->entry;
  Session* ss = r->session;
  // a session's state keeps its warm-start data; any other starts cold
  bem_state_t state = ss ? ss->st : r->lent;
  int rc = entry_influence(S, r, e);
  for (double v : r->h)
    if (rc == BEM_OK && !is_finite(v)) rc = set_error(BEM_EINVAL, "bem_solve: non-finite gap profile");
  if (rc == BEM_OK && !state) rc = bem_state_create(e->K, &state);
  if (rc == BEM_OK) {
    if (!ss) bem_state_reset(state);
    rc = ensure_precision(state, R->prec, s);
  }
  const bool same_h = ss && !ss->h_prev.empty() && ss->h_prev == r->h;
  if (rc == BEM_OK && !same_h) {
    hipError_t he = hipMemcpyAsync(state->h64, r->h.data(), state->n * sizeof(double),
                                   hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) rc = hip_fail(he, "gap profile upload");
  }
  if (ss) {
    if (rc == BEM_OK) {
      if (!same_h) ss->h_prev = r->h;
    } else {
      if (state) bem_state_reset(state);   // the next request starts cold
      ss->h_prev.clear();
    }
  }
  std::unique_lock<std::mutex> lk(S->mu);
  R->preparing--;
  if (rc == BEM_OK) {
    r->lent = state;
    R->ready.push_back(r);
    S->cv_work.notify_all();
  } else {
    complete_locked(S, r, e, state, rc);
  }
}

// Results and output copies of a finished slot (final sums in sc_host).
template <typename T>
hipError_t slot_outputs(Runner* R, int i) {
  Slot& sl = R->slot[i];
  Req* r = sl.r;
  bem_state_s* st = sl.st;
  const bem_influence_s* K = sl.e->K;
  const CgScal* h = R->sc_host + i;
  bem_result& res = r->res;
  res.d = r->r.prm.d;
  res.F = K->dx * K->dy * h->fin_sum_p;
  res.n_contact = (long long)h->fin_contact;
  res.area = (double)res.n_contact * K->dx * K->dy;
  res.n_penetrating = sl.adhesive ? (long long)h->fin_pen : 0;
  res.residual = sl.resid;
  res.p_crit = sl.adhesive ? sl.pcrit : 0.0;
  res.iters = sl.iters;
  res.detach_rounds = sl.rounds;
  res.status = sl.status;
  // a solve that ends with no pressure anywhere leaves nothing to warm-start from
  if (h->fin_contact == 0.0) st->has_p = false;
  hipError_t e = hipSuccess;
  const size_t n = st->n;
  if (r->r.p_out) {
    const void* src = st->p;
    if (!std::is_same<T, double>::value) {
      e = launch_to_f64<T>((const T*)st->p, st->out64, n, R->stream);
      src = st->out64;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(r->r.p_out, src, n * sizeof(double), hipMemcpyDeviceToHost, R->stream);
  }
  if (e == hipSuccess && r->r.contact_out)
    e = hipMemcpyAsync(r->r.contact_out, st->mask, n, hipMemcpyDeviceToHost, R->stream);
  sl.ph = PH_OUT;
  return e;
}

// After a chunk (scalars in sc_host): the next step of every slot.  Each
// step queues its kernels on the runner's stream; they complete before the
// next chunk's scalars are read.  Returns a HIP error, if any.
template <typename T>
hipError_t slot_advance(Runner* R, int i, int chunk, std::vector<std::pair<int, int>>& finished) {
  Slot& sl = R->slot[i];
  const CgScal* h = R->sc_host + i;
  hipError_t e = hipSuccess;
  switch (sl.ph) {
    case PH_CG:
      if (!h->done) {
        sl.it0 += chunk;
        if (sl.it0 > sl.max_iter + 256) {   // the device stops itself at max_iter
          set_error(BEM_EDEVICE, "batched CG loop did not report completion");
          finished.push_back({i, BEM_EDEVICE});
        }
        break;
      }
      sl.iters += h->iter;
      sl.resid = h->rhs2 > 0 ? std::sqrt(h->G / h->rhs2) : std::sqrt(h->G);
      {
        const int st = status_code(h->status);
        if (st < 0) {   // as bem_solve: a non-finite solve returns at once
          finished.push_back({i, st});
          break;
        }
        sl.status = worse(sl.status, st);
      }
      if (sl.mode == CG_DISP) {
        e = launch_finalize<T>(slot_bufs<T>(R, i), CG_DISP, sl.st->n, R->stream);
        sl.ph = PH_FIN_DISP;
      } else {
        e = launch_detach<T>(slot_bufs<T>(R, i), sl.pcrit, sl.st->n, R->stream);
        sl.ph = PH_DETACH;
      }
      sl.mode = BATCH_EMPTY;
      break;
    case PH_FIN_DISP:
      sl.st->has_mask = true;   // the contact set {p > 0} the final sums wrote
      if (sl.adhesive) {
        // the pull-off step: fixed-set solves at d on the preload's contact set
        e = launch_make_hd<T>(sl.st->h64, sl.r->r.prm.d, (T*)sl.st->hd, sl.st->n, R->stream);
        if (e == hipSuccess) e = slot_start_cg<T>(R, i, CG_FIXED);
      } else {
        e = slot_outputs<T>(R, i);
      }
      break;
    case PH_DETACH:
      if (h->fin_detach == 0.0) {
        e = launch_finalize<T>(slot_bufs<T>(R, i), CG_FIXED, sl.st->n, R->stream);
        sl.ph = PH_FIN_FIXED;
      } else {
        ++sl.rounds;
        if (sl.iters >= sl.max_iter * 8) {
          sl.status = worse(sl.status, BEM_ENOCONV);
          e = launch_finalize<T>(slot_bufs<T>(R, i), CG_FIXED, sl.st->n, R->stream);
          sl.ph = PH_FIN_FIXED;
        } else {
          e = slot_start_cg<T>(R, i, CG_FIXED);
        }
      }
      break;
    case PH_FIN_FIXED:
      e = slot_outputs<T>(R, i);
      break;
    case PH_OUT:
      finished.push_back({i, sl.status});
      break;
    case PH_FREE:
      break;
  }
  return e;
}

// One class's part of a round: start the solves admitted into its free
// slots, queue one chunk of iterations over its slots in a CG solve, and
// the copy of its scalar blocks, all on the class's stream.
template <typename T>
hipError_t class_launch(Runner* R, int chunk, std::vector<std::pair<int, int>>& finished) {
  for (int i : R->fresh) {
    const int rc = slot_setup<T>(R, i);
    if (rc < 0) {   // out of the chunk; retired below
      R->slot[i].ph = PH_FREE;
      R->slot[i].mode = BATCH_EMPTY;
      finished.push_back({i, rc});
    }
  }
  auto* tab = (BatchSlot<T>*)R->tab_host;
  unsigned modes = 0;
  int ncg = 0, last = -1;
  for (int i = 0; i < R->nslots; ++i) {
    Slot& sl = R->slot[i];
    BatchSlot<T>& b = tab[i];
    b = BatchSlot<T>{};
    b.mode = BATCH_EMPTY;
    if (sl.ph == PH_CG && sl.mode != BATCH_EMPTY) {
      const CgBufs<T> bb = slot_bufs<T>(R, i);
      b = BatchSlot<T>{bb.p, bb.t, bb.g, bb.hd, bb.mask, bb.S, bb.part, bb.sc,
                       spec_view<T>(sl.e->K).KT, sl.e->K->nx, sl.e->K->ny, sl.it0, sl.mode};
      modes |= 1u << sl.mode;
      ++ncg;
      last = i;
    }
  }
  hipError_t e = hipSuccess;
  if (ncg > 0) {
    const int used = last + 1;
    e = hipMemcpyAsync(R->tab_dev, tab, used * sizeof(BatchSlot<T>), hipMemcpyHostToDevice,
                       R->stream);
    if (e == hipSuccess)
      e = launch_batch_iterations<T>(R->slot[last].e->K->g, spec_view<T>(R->slot[last].e->K),
                                     (const BatchSlot<T>*)R->tab_dev, used, modes, chunk,
                                     R->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(R->sc_host, R->sc_dev, R->nslots * sizeof(CgScal), hipMemcpyDeviceToHost,
                       R->stream);
  R->last_chunk_slots = ncg;
  return e;
}

// After the round's synchronisation: the next step of each of the class's slots.
template <typename T>
hipError_t class_advance(Runner* R, int chunk, std::vector<std::pair<int, int>>& finished) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < R->nslots && e == hipSuccess; ++i) {
    bool done_already = false;
    for (auto& f : finished) done_already |= f.first == i;
    if (!done_already && R->slot[i].r) e = slot_advance<T>(R, i, chunk, finished);
  }
  return e;
}

// The batched path's launch thread.  Each class advances on its own: when
// its previous round has completed (event query), its slots take their next
// step, finished requests are retired, prepared requests of the class fill
// free slots, and its next round (setup of new slots, one chunk of
// iterations, the copy of its scalar blocks) is queued on its stream.
// Classes share the server's few engine streams round-robin (one per
// hardware queue); no class waits for another's rounds.
void engine_loop(bem_server_s* S) {
  (void)hipSetDevice(S->device);
  constexpr int kChunk = 8;
  std::vector<std::pair<int, int>> fin;
  for (;;) {
    std::vector<Runner*> rs;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        bool work = false;
        int preparing = 0;
        for (Runner* R : S->runner_list) {
          preparing += R->preparing;
          work |= R->in_flight || R->active > 0 || !R->ready.empty();
        }
        if (work) break;
        if (S->stop && preparing == 0) return;
        S->cv_work.wait(lk);
      }
      rs = S->runner_list;
    }
    bool progressed = false;
    for (Runner* R : rs) {
      // 1. a completed round: the next step of every slot, then retirement
      if (R->in_flight) {
        hipError_t e = hipEventQuery(R->done_ev);
        if (e == hipErrorNotReady) continue;
        R->in_flight = false;
        progressed = true;
        fin.clear();
        const Clock::time_point t0 = Clock::now();
        if (e == hipSuccess)
          e = R->prec == BEM_FP64 ? class_advance<double>(R, kChunk, fin)
                                  : class_advance<float>(R, kChunk, fin);
        if (e != hipSuccess) {   // the stream is unusable: fail the class's requests
          hip_fail(e, "batched solve");
          for (int i = 0; i < R->nslots; ++i)
            if (R->slot[i].r) fin.push_back({i, BEM_EDEVICE});
          (void)hipStreamSynchronize(R->stream);
        }
        std::unique_lock<std::mutex> lk(S->mu);
        S->eng_step += secs(t0, Clock::now());
        for (auto& f : fin) {
          Slot& sl = R->slot[f.first];
          if (!sl.r) continue;
          if (f.second >= 0) S->batched++;
          complete_locked(S, sl.r, sl.e, sl.st, f.second);
          sl = Slot();
        }
      }
      // 2. admission into free slots and the next round
      {
        std::unique_lock<std::mutex> lk(S->mu);
        R->fresh.clear();
        int active = 0;
        for (const Slot& sl : R->slot) active += sl.r != nullptr;
        for (int i = 0; i < R->nslots && !R->ready.empty(); ++i) {
          if (R->slot[i].r) continue;
          Req* r = R->ready.front();
          R->ready.pop_front();
          Slot& sl = R->slot[i];
          sl.r = r;
          sl.e = r->entry;
          sl.st = r->lent;
          R->fresh.push_back(i);
          ++active;
        }
        R->active = active;
        if (active == 0) continue;
      }
      fin.clear();
      const Clock::time_point t0 = Clock::now();
      hipError_t e = R->prec == BEM_FP64 ? class_launch<double>(R, kChunk, fin)
                                         : class_launch<float>(R, kChunk, fin);
      if (e == hipSuccess) e = hipEventRecord(R->done_ev, R->stream);
      progressed = true;
      std::unique_lock<std::mutex> lk(S->mu);
      S->eng_launch += secs(t0, Clock::now());
      if (R->last_chunk_slots > 0) {
        S->chunks += 1;
        S->slot_chunks += R->last_chunk_slots;
      }
      if (e != hipSuccess) {
        hip_fail(e, "batched solve");
        for (int i = 0; i < R->nslots; ++i)
          if (R->slot[i].r) fin.push_back({i, BEM_EDEVICE});
      }
      for (auto& f : fin) {   // setup failures (and launch errors) retire now
        Slot& sl = R->slot[f.first];
        if (!sl.r) continue;
        complete_locked(S, sl.r, sl.e, sl.st, f.second);
        sl = Slot();
        R->active--;
      }
      R->in_flight = e == hipSuccess;
    }
    if (!progressed) {
      // every class has a round on the GPU: wait a little before polling again
      const Clock::time_point t0 = Clock::now();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      std::unique_lock<std::mutex> lk(S->mu);
      S->eng_sync += secs(t0, Clock::now());
    }
  }
}

// Largest half-length of the padded transform served on the batched path
// (grids up to 256 x 256).  Measured on the serving stream with MIXED
// solves: at 64^2..128^2 one launch per CG kernel for all slots gave 1870
// against 1420 solves/s for independent solves on four streams, at
// 129^2..512^2 the two were equal (251 / 252), and above 512^2, where a
// single solve's kernels already fill the GPU, independent solves were
// faster (34 against 24 solves/s): their kernels overlap in different phases
// while a batch moves in lock-step.
constexpr int kBatchMaxL = 256;

// The class of a request on the batched path, or false for the per-request path.
bool batch_class(const bem_server_s* S, const bem_request& q, ClassKey* key) {
  if (S->batch_slots <= 0 || q.prm.control != BEM_CTRL_INDENT) return false;
  int Mx = 2 * kMinL, My = 2 * kMinL;
  while (Mx < 2 * q.nx) Mx <<= 1;
  while (My < 2 * q.ny) My <<= 1;
  Geom g{q.nx, q.ny, Mx / 2, My / 2, 0};
  if (!batch_geometry(g) || g.Lx > kBatchMaxL || g.Ly > kBatchMaxL) return false;
  *key = ClassKey{g.Lx, g.Ly, q.prm.precision};
  return true;
}

// The first request of `q` that can start now (lock held): requests start in
// queue order, except that one whose session is still busy with its
// predecessor is passed over; a session's later requests need no admission
// (its first one holds the entry and the state).  Returns nullptr when the
// first candidate does not fit the budget yet, so memory admission keeps the
// queue's order.
Req* take_startable(bem_server_s* S, std::deque<Req*>& q, Entry** entry) {
  for (auto qi = q.begin(); qi != q.end(); ++qi) {
    Req* c = *qi;
    Session* ss = c->session;
    if (ss && ss->busy) continue;
    Entry* ce = (ss && ss->e) ? ss->e : admit(S, c);
    if (!ce) return nullptr;
    if (ss) {
      ss->busy = true;
      if (!ss->e) {   // the session's first request: its admission is the session's
        ss->e = ce;
        ss->st = c->lent;
        c->lent = nullptr;
      }
    }
    q.erase(qi);
    *entry = ce;
    return c;
  }
  return nullptr;
}

void worker(bem_server_s* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[slot];
  for (;;) {
    Req* r = nullptr;
    Entry* e = nullptr;
    Runner* prep = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop) return;
        // batched requests first: admit and prepare one for a runner with
        // room (slots not yet running, ready or being prepared)
        for (auto& kv : S->runners) {
          Runner* R = kv.second;
          if (R->queue.empty() || R->active + (int)R->ready.size() + R->preparing >= R->nslots)
            continue;
          r = take_startable(S, R->queue, &e);
          if (!r) continue;
          r->entry = e;
          R->preparing++;
          prep = R;
          break;
        }
        if (r) break;
        // per-request path, in submission order
        r = take_startable(S, S->queue, &e);
        if (r) break;
        S->cv_work.wait(lk);
      }
      r->t_start = Clock::now();
      S->running++;
      S->peak_running = std::max(S->peak_running, S->running);
    }
    if (prep) {
      prepare_batched(S, prep, r, st);
      continue;
    }
    // build the influence operator if this request created the entry
    int rc = entry_influence(S, r, e);
    Session* ss = r->session;
    bem_state_t state = ss ? ss->st : r->lent;
    if (rc == BEM_OK && !state) rc = bem_state_create(e->K, &state);
    if (rc == BEM_OK && ss) {
      // warm start from the session's previous solve; from its gap as well
      // when the profile is the same
      if (!ss->h_prev.empty() && ss->h_prev == r->h)
        rc = solve_same_h(e->K, &r->r.prm, state, r->r.p_out, r->r.contact_out, &r->res, st);
      else
        rc = bem_solve(e->K, r->h.data(), &r->r.prm, state, r->r.p_out, r->r.contact_out,
                       nullptr, &r->res, st);
      if (rc < 0) {
        bem_state_reset(state);   // the next request starts cold
        ss->h_prev.clear();
      } else {
        ss->h_prev.swap(r->h);
      }
    } else if (rc == BEM_OK) {
      // every request is a fresh (cold-start) solve, as if solved alone
      bem_state_reset(state);
      rc = bem_solve(e->K, r->h.data(), &r->r.prm, state, r->r.p_out, r->r.contact_out, nullptr,
                     &r->res, st);
    }
    std::unique_lock<std::mutex> lk(S->mu);
    complete_locked(S, r, e, state, rc);
  }
}

double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

int bem_footprint(int nx, int ny, int precision, long long* influence_bytes,
                  long long* state_bytes) {
  if (nx < 1 || ny < 1 || nx > BEM_MAX_N || ny > BEM_MAX_N)
    return set_error(BEM_EINVAL, "bem_footprint: grid size");
  int Mx = 64, My = 64;
  while (Mx < 2 * nx) Mx <<= 1;
  while (My < 2 * ny) My <<= 1;
  const long long Lx = Mx / 2, Ly = My / 2;
  const long long kpitch = ((Ly + 1) + 63) / 64 * 64;
  const long long n = (long long)nx * ny;
  // coefficients, spectrum (FP64 + FP32), twiddles and the FP64 spectrum
  // scratch the handle keeps from its build
  if (influence_bytes)
    *influence_bytes = n * 8 + (Lx + 1) * kpitch * 12 + (long long)(Mx + My + Ly + Lx) * 24 +
                       (long long)(ny + (ny & 1)) * Lx * 16;
  const long long ts = precision == BEM_FP64 ? 8 : 4;
  if (state_bytes)
    *state_bytes = n * (1 + 8 + 8) + state_partial_bytes() + 512 + 4 * n * ts +
                   (long long)(ny + (ny & 1)) * Lx * 2 * ts;
  return BEM_OK;
}

int bem_server_create(long long budget_bytes, int n_slots, bem_server_t* out) {
  return bem_server_create_ex(budget_bytes, n_slots, 16, out);
}

int bem_server_create_ex(long long budget_bytes, int n_slots, int batch_slots, bem_server_t* out) {
  clear_error();
  if (!out || budget_bytes <= 0 || n_slots < 1 || n_slots > 16 || batch_slots < 0 ||
      batch_slots > 64)
    return set_error(BEM_EINVAL,
                     "bem_server_create: budget > 0, 1 <= n_slots <= 16, 0 <= batch_slots <= 64");
  auto* S = new bem_server_s();
  S->budget = budget_bytes;
  S->n_slots = n_slots;
  S->batch_slots = batch_slots;
  (void)hipGetDevice(&S->device);
  S->t0 = Clock::now();
  for (int i = 0; i < n_slots; ++i) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (hipStream_t q : S->streams) hipStreamDestroy(q);
      delete S;
      return hip_fail(e, "bem_server_create stream");
    }
    S->streams.push_back(s);
  }
  // the batched path: one launch thread over a few streams (one per hardware
  // queue of the default HIP configuration)
  for (int i = 0; batch_slots > 0 && i < 4; ++i) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (hipStream_t q : S->streams) hipStreamDestroy(q);
      for (hipStream_t q : S->engine_streams) hipStreamDestroy(q);
      delete S;
      return hip_fail(e, "bem_server_create stream");
    }
    S->engine_streams.push_back(s);
  }
  for (int i = 0; i < n_slots; ++i) S->workers.emplace_back(worker, S, i);
  if (batch_slots > 0) S->engine = std::thread(engine_loop, S);
  *out = S;
  return BEM_OK;
}

static int submit_impl(bem_server_t S, long long session, const bem_request* req, long long* id) {
  clear_error();
  if (!S || !req || !id || !req->h) return set_error(BEM_EINVAL, "bem_server_submit: NULL argument");
  const bem_request& q = *req;
  if (q.nx < 1 || q.ny < 1 || q.nx > BEM_MAX_N || q.ny > BEM_MAX_N)
    return set_error(BEM_EINVAL, "bem_server_submit: grid size");
  if (q.prm.precision != BEM_FP64 && q.prm.precision != BEM_MIXED)
    return set_error(BEM_EINVAL, "bem_server_submit: unknown precision %d", q.prm.precision);
  auto* r = new Req();
  r->r = q;
  r->h.assign(q.h, q.h + (size_t)q.nx * q.ny);
  r->r.h = nullptr;
  long long fi = 0, fs = 0;
  bem_footprint(q.nx, q.ny, q.prm.precision, &fi, &fs);
  r->need_infl = fi;
  r->need_state = fs;
  if (fi + fs > S->budget) {
    delete r;
    return set_error(BEM_ENOMEM, "bem_server_submit: request needs %lld bytes, budget %lld",
                     fi + fs, S->budget);
  }
  // the batched path: the runner of the request's class (made on first use)
  ClassKey key;
  Runner* R = nullptr;
  if (batch_class(S, q, &key)) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto it = S->runners.find(key);
      if (it != S->runners.end()) R = it->second;
    }
    if (!R) {
      auto* nr = new Runner();
      nr->S = S;
      nr->Lx = std::get<0>(key);
      nr->Ly = std::get<1>(key);
      nr->prec = std::get<2>(key);
      nr->nslots = S->batch_slots;
      const int rc = runner_alloc(nr);
      if (rc) {
        runner_release(nr);
        delete nr;
        delete r;
        return rc;
      }
      std::unique_lock<std::mutex> lk(S->mu);
      auto it = S->runners.find(key);
      if (it != S->runners.end()) {   // another submit made it meanwhile
        lk.unlock();
        runner_release(nr);
        delete nr;
        lk.lock();
        R = S->runners.find(key)->second;
      } else {
        nr->stream = S->engine_streams[S->runner_list.size() % S->engine_streams.size()];
        S->runners[key] = nr;
        S->runner_list.push_back(nr);
        R = nr;
      }
    }
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (session != 0) {
    auto si = S->sessions.find(session);
    if (si == S->sessions.end() || si->second->closed) {
      delete r;
      return set_error(BEM_EINVAL, "bem_server_submit_session: unknown or closed session %lld",
                       session);
    }
    Session* ss = si->second;
    const Key k{q.nx, q.ny, q.dx, q.dy, q.k, q.nu, q.E0, q.c0};
    if (ss->keyed && (k != ss->key || q.prm.precision != ss->prec)) {
      delete r;
      return set_error(BEM_EINVAL,
                       "bem_server_submit_session: grid, material and precision must be those "
                       "of the session's first request");
    }
    ss->keyed = true;
    ss->key = k;
    ss->prec = q.prm.precision;
    ss->pending++;
    r->session = ss;
  }
  r->id = S->next_id++;
  r->t_submit = Clock::now();
  if (!S->have_first) {
    S->have_first = true;
    S->t_first_submit = r->t_submit;
  }
  S->reqs[r->id] = r;
  if (R)
    R->queue.push_back(r);
  else
    S->queue.push_back(r);
  *id = r->id;
  S->cv_work.notify_all();
  return BEM_OK;
}

int bem_server_submit(bem_server_t S, const bem_request* req, long long* id) {
  return submit_impl(S, 0, req, id);
}

int bem_server_session_open(bem_server_t S, long long* session) {
  clear_error();
  if (!S || !session) return set_error(BEM_EINVAL, "bem_server_session_open: NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto* ss = new Session();
  ss->id = S->next_session++;
  S->sessions[ss->id] = ss;
  *session = ss->id;
  return BEM_OK;
}

int bem_server_submit_session(bem_server_t S, long long session, const bem_request* req,
                              long long* id) {
  if (session <= 0) {
    clear_error();
    return set_error(BEM_EINVAL, "bem_server_submit_session: invalid session %lld", session);
  }
  return submit_impl(S, session, req, id);
}

int bem_server_session_close(bem_server_t S, long long session) {
  clear_error();
  if (!S) return set_error(BEM_EINVAL, "bem_server_session_close: NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto si = S->sessions.find(session);
  if (si == S->sessions.end() || si->second->closed)
    return set_error(BEM_EINVAL, "bem_server_session_close: unknown or closed session %lld",
                     session);
  Session* ss = si->second;
  ss->closed = true;
  if (ss->pending == 0) release_session_locked(S, ss);
  S->cv_work.notify_all();
  return BEM_OK;
}

int bem_server_poll(bem_server_t S, long long id, int wait, bem_result* res, int* status) {
  clear_error();
  if (!S) return set_error(BEM_EINVAL, "bem_server_poll: NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return set_error(BEM_EINVAL, "bem_server_poll: unknown id %lld", id);
  Req* r = it->second;
  if (!r->done) {
    if (!wait) return 1;
    S->cv_done.wait(lk, [&] { return r->done; });
  }
  if (res) *res = r->res;
  if (status) *status = r->rc;
  S->reqs.erase(it);
  delete r;
  return BEM_OK;
}

int bem_server_stats(bem_server_t S, bem_server_stats_t* out) {
  clear_error();
  if (!S || !out) return set_error(BEM_EINVAL, "bem_server_stats: NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = S->completed;
  out->failed = S->failed;
  out->queued = (long long)S->queue.size();
  for (auto& kv : S->runners) out->queued += (long long)kv.second->queue.size();
  out->batched = S->batched;
  out->engine_launch_s = S->eng_launch;
  out->engine_sync_s = S->eng_sync;
  out->engine_step_s = S->eng_step;
  out->mean_batch_slots = S->chunks > 0 ? S->slot_chunks / S->chunks : 0.0;
  out->running = S->running;
  out->peak_running = S->peak_running;
  out->p50_latency_s = quantile(S->latency, 0.50);
  out->p99_latency_s = quantile(S->latency, 0.99);
  out->mean_wait_s = S->wait.empty() ? 0.0 : [&] {
    double a = 0;
    for (double w : S->wait) a += w;
    return a / S->wait.size();
  }();
  out->solves_per_s =
      (S->completed > 0 && S->have_first) ? S->completed / secs(S->t_first_submit, S->t_last_end) : 0.0;
  out->device_bytes_reserved = S->used;
  out->cache_entries = (long long)S->cache.size();
  out->cache_hits = S->cache_hits;
  out->cache_misses = S->cache_misses;
  out->evictions = S->evictions;
  return BEM_OK;
}

int bem_server_reset_stats(bem_server_t S) {
  if (!S) return set_error(BEM_EINVAL, "bem_server_reset_stats: NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  S->latency.clear();
  S->wait.clear();
  S->completed = S->failed = 0;
  S->have_first = false;
  S->peak_running = S->running;
  S->cache_hits = S->cache_misses = S->evictions = 0;
  S->batched = 0;
  S->chunks = S->slot_chunks = 0;
  S->eng_launch = S->eng_sync = S->eng_step = 0;
  return BEM_OK;
}

int bem_server_free(bem_server_t S) {
  if (!S) return BEM_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  for (auto& t : S->workers) t.join();
  if (S->engine.joinable()) S->engine.join();
  for (auto& kv : S->runners) {
    runner_release(kv.second);
    delete kv.second;
  }
  for (hipStream_t s : S->engine_streams) hipStreamDestroy(s);
  // session states go back to their entries' pools (freed with them)
  for (auto& kv : S->sessions) {
    Session* ss = kv.second;
    if (ss->st) {
      if (ss->e)
        ss->e->free_states[ss->prec].push_back(ss->st);
      else
        bem_state_free(ss->st);
    }
    delete ss;
  }
  S->sessions.clear();
  for (auto& kv : S->cache) {
    free_entry(kv.second);
    delete kv.second;
  }
  for (auto& kv : S->reqs) delete kv.second;
  for (hipStream_t s : S->streams) hipStreamDestroy(s);
  delete S;
  return BEM_OK;
}

}  // extern "C"
