// Serving loop: continuous batching of independent contact solves on one GPU.
//
// Requests (grid, material, gap profile, solve parameters) enter a FIFO
// queue.  n_slots worker threads, each with its own non-blocking HIP stream
// (default priority), take the queue head as soon as a slot is free and the
// device-memory budget admits it, so solves of different sizes, k and
// indenters run concurrently on the GPU and new requests start while others
// are still running.  Influence operators are cached by
// (nx, ny, dx, dy, k, nu, E0, c0) together with pooled solver states;
// entries that no running solve uses are evicted least-recently-used when
// the budget requires.  Admission uses the footprint model of
// bem_footprint(); a request that can never fit is rejected at submit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/bem.h"
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
};

}  // namespace

struct bem_server_s {
  long long budget = 0;
  int n_slots = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<long long, Req*> reqs;
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

void worker(bem_server_s* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[slot];
  for (;;) {
    Req* r = nullptr;
    Entry* e = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop) return;
        if (!S->queue.empty()) {
          e = admit(S, S->queue.front());
          if (e) {
            r = S->queue.front();
            S->queue.pop_front();
            break;
          }
        }
        S->cv_work.wait(lk);
      }
      r->t_start = Clock::now();
      S->running++;
      S->peak_running = std::max(S->peak_running, S->running);
    }
    // build the influence operator if this request created the entry
    int rc = BEM_OK;
    if (r->builder) {
      bem_influence_t K = nullptr;
      const bem_request& q = r->r;
      rc = bem_influence_ex(q.nx, q.ny, q.dx, q.dy, q.k, q.nu, q.E0, q.c0, &K);
      std::unique_lock<std::mutex> lk(S->mu);
      e->K = K;
      e->building = false;
      S->cv_done.notify_all();
    } else {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_done.wait(lk, [&] { return !e->building; });
      if (!e->K) rc = BEM_EDEVICE;
    }
    bem_state_t state = r->lent;
    if (rc == BEM_OK && !state) rc = bem_state_create(e->K, &state);
    if (rc == BEM_OK) {
      // every request is a fresh (cold-start) solve, as if solved alone
      bem_state_reset(state);
      rc = bem_solve(e->K, r->h.data(), &r->r.prm, state, r->r.p_out, r->r.contact_out, nullptr,
                     &r->res, st);
    }
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (state) e->free_states[r->r.prm.precision].push_back(state);
      e->in_use--;
      e->last_use = ++S->tick;
      if (!e->K && e->in_use == 0) {  // failed build: drop the entry once unused
        S->cache.erase(e->key);
        S->used -= e->bytes;
        free_entry(e);
        delete e;
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
  if (influence_bytes)
    *influence_bytes = n * 8 + (Lx + 1) * kpitch * 12 + (long long)(Mx + My + Ly + Lx) * 24;
  const long long ts = precision == BEM_FP64 ? 8 : 4;
  if (state_bytes)
    *state_bytes = n * (1 + 8 + 8) + state_partial_bytes() + 512 + 4 * n * ts +
                   (long long)ny * Lx * 2 * ts;
  return BEM_OK;
}

int bem_server_create(long long budget_bytes, int n_slots, bem_server_t* out) {
  clear_error();
  if (!out || budget_bytes <= 0 || n_slots < 1 || n_slots > 16)
    return set_error(BEM_EINVAL, "bem_server_create: budget > 0, 1 <= n_slots <= 16");
  auto* S = new bem_server_s();
  S->budget = budget_bytes;
  S->n_slots = n_slots;
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
  for (int i = 0; i < n_slots; ++i) S->workers.emplace_back(worker, S, i);
  *out = S;
  return BEM_OK;
}

int bem_server_submit(bem_server_t S, const bem_request* req, long long* id) {
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
  std::unique_lock<std::mutex> lk(S->mu);
  r->id = S->next_id++;
  r->t_submit = Clock::now();
  if (!S->have_first) {
    S->have_first = true;
    S->t_first_submit = r->t_submit;
  }
  S->reqs[r->id] = r;
  S->queue.push_back(r);
  *id = r->id;
  S->cv_work.notify_one();
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
