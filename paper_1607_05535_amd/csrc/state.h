// Host-side state object shared by the runtime sources of libthor.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "kernels.h"

struct TimedLaunch {
  std::string family;
  hipEvent_t start, stop;
};

// Kernel families with a tuned workgroup size (wavefronts per workgroup).
enum { FAM_LARGE = 0, FAM_SLOW, FAM_HMOM, FAM_VERT, FAM_COUNT };
static const char *const kFamily[FAM_COUNT] = {"large", "slow", "hmom", "vert"};

struct thor_state {
  int precision = THOR_FP64;
  thor::Consts c{};
  // f[0] and f[1] are the same buffers with the state set and the Phi[t] set
  // exchanged; between large steps the state is in the *_t buffers of
  // f[parity], and every large step flips the parity.
  thor::Fields<double> f64[2]{};
  thor::Fields<float> f32[2]{};
  int parity = 0;
  int wpb[FAM_COUNT] = {4, 4, 4, 4};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::map<int, hipGraphExec_t> graphs;   // key: n_acoustic * 2 + parity
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  size_t next_event = 0;
  int64_t n_col = 0;
  int n_lev = 0;
  bool in_batch = false;   // members of an ensemble are stepped by thor_batch_step
};

