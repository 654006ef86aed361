// Opt-in phase timers (see igs_timing_enable in include/imagegs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace igs {

constexpr int kNumPhases = 7;
enum Phase {
  kPhaseBinning = 0,
  kPhaseRasterFwd = 1,
  kPhaseRasterBwd = 2,
  kPhaseLoss = 3,
  kPhaseAdam = 4,
  kPhaseGradReduce = 5,
  kPhaseRasterFit = 6
};

bool timing_on();
void timing_enable(bool on);
int timing_begin(int phase, hipStream_t s);  // returns a token, -1 when not timing
void timing_end(int token, hipStream_t s);
hipError_t timing_read(double *ms, int64_t *calls, bool reset);

// Times the enclosing scope as one phase.
struct PhaseTimer {
  int token;
  hipStream_t s;
  PhaseTimer(int phase, hipStream_t st) : token(timing_begin(phase, st)), s(st) {}
  ~PhaseTimer() { timing_end(token, s); }
};

}  // namespace igs
