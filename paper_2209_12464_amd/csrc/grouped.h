// Grouped launches: one launch runs the same kernel for many independent
// problems of a batch.  Every kernel body takes its block index and block
// count as arguments; the single-problem kernel passes blockIdx.x and
// gridDim.x, the grouped kernel reads a table of per-problem arguments and
// the prefix sums of their block counts and gives each block the index and
// count it would have had in the problem's own launch, so the arithmetic
// (and every summation order) is the problem's own.
//
// On the host, each launcher either launches its kernel or, while a launch
// recorder is active on the calling thread, appends the launch (grouped
// launcher, argument bytes, block count) to the recorder instead; the batch
// executor replays recorded sequences as grouped launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <vector>

namespace rqlp {

// Launch the grouped form of one kernel: `args` points to `count` argument
// structs in device memory, `start` to count + 1 block offsets (device),
// `blocks` = start[count].
typedef void (*GroupedFn)(const void* args, const int* start, int count, unsigned blocks, hipStream_t s);

constexpr int kMaxRecArgs = 160;  // bytes of the largest argument struct

struct LaunchRec {
  GroupedFn fn;
  unsigned blocks;
  uint16_t size;
  uint8_t args[kMaxRecArgs];
};

struct LaunchRecorder {
  std::vector<LaunchRec> seq;
  std::vector<int> phase;  // phase index of each recorded launch
  int cur_phase = 0;
};

// The recorder of the calling thread (null: launchers launch).
LaunchRecorder*& launch_recorder();

// Record a launch when a recorder is active; returns true if recorded.
template <typename A>
inline bool record_launch(GroupedFn fn, const A& a, unsigned blocks) {
  LaunchRecorder* r = launch_recorder();
  if (!r) return false;
  static_assert(sizeof(A) <= kMaxRecArgs, "argument struct too large to record");
  LaunchRec x;
  x.fn = fn;
  x.blocks = blocks;
  x.size = (uint16_t)sizeof(A);
  std::memcpy(x.args, &a, sizeof(A));
  r->seq.push_back(x);
  r->phase.push_back(r->cur_phase);
  return true;
}

// Block b of a grouped launch belongs to the last item p with start[p] <= b.
__device__ inline int group_find(const int* __restrict__ start, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace rqlp
