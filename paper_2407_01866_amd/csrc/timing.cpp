// Opt-in phase timers for libimagegs: HIP event pairs recorded on the caller's stream around the
// phases of each entry point, summed when read.
#include "timing.hpp"

#include <vector>

namespace igs {
namespace {

struct Pair {
  hipEvent_t start, stop;
  int phase;
};

bool g_on = false;
std::vector<Pair> g_pool;    // created events, reused
size_t g_used = 0;           // pairs recorded since the last read
double g_ms[kNumPhases] = {};
int64_t g_calls[kNumPhases] = {};
constexpr size_t kMaxPairs = 65536;

}  // namespace

bool timing_on() { return g_on; }

void timing_enable(bool on) { g_on = on; }

int timing_begin(int phase, hipStream_t s) {
  if (!g_on || g_used >= kMaxPairs) return -1;
  if (g_used == g_pool.size()) {
    Pair p{};
    if (hipEventCreate(&p.start) != hipSuccess) return -1;
    if (hipEventCreate(&p.stop) != hipSuccess) {
      (void)hipEventDestroy(p.start);
      return -1;
    }
    g_pool.push_back(p);
  }
  Pair &p = g_pool[g_used];
  if (hipEventRecord(p.start, s) != hipSuccess) return -1;
  p.phase = phase;
  return (int)g_used++;
}

void timing_end(int token, hipStream_t s) {
  if (token < 0) return;
  (void)hipEventRecord(g_pool[(size_t)token].stop, s);
}

hipError_t timing_read(double *ms, int64_t *calls, bool reset) {
  for (size_t i = 0; i < g_used; ++i) {
    Pair &p = g_pool[i];
    hipError_t e = hipEventSynchronize(p.stop);
    if (e != hipSuccess) return e;
    float t = 0.f;
    e = hipEventElapsedTime(&t, p.start, p.stop);
    if (e != hipSuccess) return e;
    g_ms[p.phase] += t;
    g_calls[p.phase] += 1;
  }
  g_used = 0;
  for (int k = 0; k < kNumPhases; ++k) {
    ms[k] = g_ms[k];
    calls[k] = g_calls[k];
    if (reset) {
      g_ms[k] = 0.0;
      g_calls[k] = 0;
    }
  }
  return hipSuccess;
}

}  // namespace igs
