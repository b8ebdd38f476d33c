// Autotuner of the tile shapes of the matrix-core products (tune.cpp).
//
// Each product launch site (dgemm, the residual pass, the BF16 plane
// product) asks tune_get for its configuration before choosing its own
// heuristic one. The tuner records the launches of one decomposition
// (tune_record: the key, the candidate configurations that are valid for
// that call's scratch sizes, and a closure that enqueues the same launch
// again), then replays every key not yet tuned once per candidate with the
// candidate forced, times them with HIP events, and stores the fastest.
#pragma once

#include <stdint.h>

#include <functional>
#include <vector>

#include "common.hpp"

namespace rsvd {

enum TuneKind : int {
  kTuneDma = 0,      // FP64 / in-register mixed streaming kernel (LDS-DMA)
  kTuneGeneric = 1,  // register-staged kernel (transposed A, unaligned rows)
  kTuneResid = 2,    // residual pass
  kTuneBf16 = 3      // BF16 plane product
};

struct TuneKey {
  int kind = 0, prec = 0, ta = 0;
  int64_t M = 0, N = 0, K = 0;
  bool operator<(const TuneKey& o) const;
  bool operator==(const TuneKey& o) const;
};

// kTuneDma: a = waves per workgroup (4 | 8), b = K splits
// kTuneGeneric: b = K splits
// kTuneResid: a = waves per workgroup (4 | 8), b = column tiles per workgroup (0: widest)
// kTuneBf16: a = 16-row fragments per wave (1 | 2), b = K splits, c = column groups
struct TuneCfg {
  int a = 0, b = 0, c = 0;
};

// The forced configuration while the tuner replays a candidate of this key,
// else the tuned one; false when there is neither.
bool tune_get(const TuneKey& k, TuneCfg* c);
// Changes whenever the table changes (captured graphs hold launch shapes).
uint64_t tune_generation();
bool tune_recording();
void tune_record(const TuneKey& k, std::vector<TuneCfg> candidates,
                 std::function<rsvd_status(hipStream_t)> again);

// Arguments of one rsvd_run.
struct TuneRun {
  const double* A;
  int64_t lda;
  const double* omega;
  int64_t ldo;
  double* S;
  double* U;
  int64_t ldu;
  double* V;
  int64_t ldv;
  rsvd_result* res;
  void* work;
  size_t work_bytes;
};
// Tune the products of one decomposition (recorded run, replays, final run);
// tuned (may be null) is incremented per key added to the table.
rsvd_status tune_plan(rsvd_plan_t plan, const TuneRun& a, int reps, hipStream_t s, int* tuned);

}  // namespace rsvd
