// Solver clock: HIP events around the launches of the conjugate-gradient
// loop, recorded on the solver's stream for the calling thread only.  The
// events are pooled per thread and resolved at bem_clock_stop, so the loop
// itself gains no host synchronisation.
#include <hip/hip_runtime.h>

#include <climits>
#include <vector>

#include "bem.h"
#include "internal.h"

namespace bem {
namespace {

struct Seg {
  size_t base;    // first event of the chunk in the pool
  int it0, n;     // iterations it0 .. it0 + n - 1
  int final_it;   // iteration at which the solver stopped; INT_MAX: not in
                  // this chunk; INT_MIN: chunk never completed (skip it)
  bool shifted;   // iteration it0 began with a gap shift (launches 0-2 absent)
};

struct Clock {
  bool on = false;
  bool bad_device = false;
  int device = -1;
  std::vector<hipEvent_t> pool;   // kept for the life of the thread
  size_t used = 0;
  std::vector<Seg> segs;
};

thread_local Clock tl_clock;

}  // namespace

const hipEvent_t* clock_chunk(int it0, int n) {
  Clock& c = tl_clock;
  if (!c.on || n <= 0) return nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (c.device < 0) c.device = dev;
  if (dev != c.device) {
    c.bad_device = true;
    return nullptr;
  }
  const size_t need = c.used + 6 * (size_t)n + 1;
  while (c.pool.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c.pool.push_back(e);
  }
  c.segs.push_back({c.used, it0, n, INT_MIN, false});
  const hipEvent_t* ev = c.pool.data() + c.used;
  c.used = need;
  return ev;
}

void clock_chunk_shifted() {
  Clock& c = tl_clock;
  if (c.on && !c.segs.empty()) c.segs.back().shifted = true;
}

void clock_chunk_done(bool done, int final_it) {
  Clock& c = tl_clock;
  if (!c.on || c.segs.empty()) return;
  c.segs.back().final_it = done ? final_it : INT_MAX;
}

}  // namespace bem

using namespace bem;

extern "C" {

int bem_clock_start(void) {
  clear_error();
  Clock& c = tl_clock;
  c.on = true;
  c.bad_device = false;
  c.used = 0;
  c.segs.clear();
  return BEM_OK;
}

int bem_clock_stop(bem_clock_t* out) {
  clear_error();
  Clock& c = tl_clock;
  if (!out) return set_error(BEM_EINVAL, "bem_clock_stop: NULL argument");
  if (!c.on) return set_error(BEM_EINVAL, "bem_clock_stop: no clock running on this thread");
  c.on = false;
  if (c.bad_device) return set_error(BEM_EINVAL, "bem_clock_stop: solves on more than one device");
  bem_clock_t r = {};
  for (const Seg& sg : c.segs) {
    if (sg.final_it == INT_MIN) continue;
    for (int i = 0; i < sg.n; ++i) {
      const int j = sg.it0 + i;
      if (j < sg.final_it) ++r.iterations;
      for (int k = 0; k < 6; ++k) {
        float ms = 0.f;
        const hipError_t e = hipEventElapsedTime(&ms, c.pool[sg.base + 6 * (size_t)i + k],
                                                 c.pool[sg.base + 6 * (size_t)i + k + 1]);
        if (e != hipSuccess) return hip_fail(e, "bem_clock_stop: event timing");
        // after a gap shift the first interval of iteration it0 is the shift
        // kernel (reported on its own) and the next two are empty
        if (sg.shifted && i == 0 && k <= 2) {
          if (k == 0) {
            ++r.shifts;
            r.shift_ms += ms;
          }
          continue;
        }
        // at the stopping iteration the direction kernel only takes the decision
        const bool worked = j < sg.final_it || (j == sg.final_it && k <= 2);
        if (worked) {
          ++r.launches[k];
          r.ms[k] += ms;
        } else {
          ++r.skipped;
          r.skipped_ms += ms;
        }
      }
    }
  }
  c.segs.clear();
  c.used = 0;
  *out = r;
  return BEM_OK;
}

}  // extern "C"
