// Autotuner of the tile shapes of the matrix-core products and its C ABI
// (include/rsvd.h, "Autotuning").
//
// rsvd_tune runs one decomposition while the launch sites record themselves,
// replays each recorded key that is not in the table with every candidate
// configuration forced (one warm-up launch, then `reps` launches between two
// HIP events on the caller's stream), stores the fastest candidate in a
// process-wide table, and finally runs the decomposition once more so that
// the outputs are those of the tuned shapes (the replays overwrite
// intermediate buffers). Later launches of a tuned key, by any plan, use the
// table.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "tune.hpp"

namespace rsvd {

bool TuneKey::operator<(const TuneKey& o) const {
  return std::tie(kind, prec, ta, M, N, K) < std::tie(o.kind, o.prec, o.ta, o.M, o.N, o.K);
}
bool TuneKey::operator==(const TuneKey& o) const {
  return kind == o.kind && prec == o.prec && ta == o.ta && M == o.M && N == o.N && K == o.K;
}

namespace {

struct Recorded {
  TuneKey key;
  std::vector<TuneCfg> cands;
  std::function<rsvd_status(hipStream_t)> again;
};

std::mutex g_mu;
std::map<TuneKey, TuneCfg> g_table;
uint64_t g_gen = 0;
// tuner state (one tuning caller at a time, under g_tune_mu)
std::mutex g_tune_mu;
bool g_recording = false;
std::vector<Recorded> g_recs;
bool g_forcing = false;
TuneKey g_force_key;
TuneCfg g_force_cfg;

}  // namespace

bool tune_get(const TuneKey& k, TuneCfg* c) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_forcing && g_force_key == k) {
    *c = g_force_cfg;
    return true;
  }
  auto it = g_table.find(k);
  if (it == g_table.end()) return false;
  *c = it->second;
  return true;
}

uint64_t tune_generation() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_gen;
}

bool tune_recording() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_recording;
}

void tune_record(const TuneKey& k, std::vector<TuneCfg> candidates,
                 std::function<rsvd_status(hipStream_t)> again) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_recording || candidates.size() < 2) return;
  for (const Recorded& r : g_recs)
    if (r.key == k) return;  // the first launch of a key stands for all
  g_recs.push_back({k, std::move(candidates), std::move(again)});
}

namespace {

void set_force(bool on, const TuneKey& k = TuneKey(), const TuneCfg& c = TuneCfg()) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_forcing = on;
  g_force_key = k;
  g_force_cfg = c;
}

// Time every candidate of the recorded keys not yet in the table.
rsvd_status tune_recorded(int reps, hipStream_t s, int* tuned) {
  std::vector<Recorded> recs;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    recs.swap(g_recs);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return RSVD_EHIP;
  }
  rsvd_status st = RSVD_OK;
  for (const Recorded& r : recs) {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      if (g_table.count(r.key)) continue;
    }
    float best = 0.0f;
    int best_i = -1;
    for (size_t i = 0; i < r.cands.size() && st == RSVD_OK; i++) {
      set_force(true, r.key, r.cands[i]);
      st = r.again(s);  // warm-up (and first-touch of the scratch it uses)
      if (st != RSVD_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) st = RSVD_EHIP;
      for (int rep = 0; rep < reps && st == RSVD_OK; rep++) st = r.again(s);
      if (st == RSVD_OK && hipEventRecord(e1, s) != hipSuccess) st = RSVD_EHIP;
      float ms = 0.0f;
      if (st == RSVD_OK &&
          (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = RSVD_EHIP;
      if (st == RSVD_OK && (best_i < 0 || ms < best)) {
        best = ms;
        best_i = (int)i;
      }
    }
    set_force(false);
    if (st != RSVD_OK) break;
    if (best_i >= 0) {
      std::lock_guard<std::mutex> lk(g_mu);
      g_table[r.key] = r.cands[best_i];
      g_gen++;
      if (tuned) (*tuned)++;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

rsvd_status run_once(rsvd_plan_t plan, const TuneRun& a, hipStream_t s) {
  return rsvd_run(plan, a.A, a.lda, a.omega, a.ldo, a.S, a.U, a.ldu, a.V, a.ldv, a.res, a.work,
                  a.work_bytes, (void*)s);
}

rsvd_status tune_one(rsvd_plan_t plan, const TuneRun& a, int reps, hipStream_t s, int* tuned) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.clear();
    g_recording = true;
  }
  rsvd_status r = run_once(plan, a, s);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recording = false;
  }
  if (r == RSVD_OK && hipStreamSynchronize(s) != hipSuccess) r = RSVD_EHIP;
  if (r == RSVD_OK) r = tune_recorded(reps, s, tuned);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.clear();
  }
  if (r != RSVD_OK) return r;
  r = run_once(plan, a, s);
  if (r == RSVD_OK && hipStreamSynchronize(s) != hipSuccess) r = RSVD_EHIP;
  return r;
}

}  // namespace

rsvd_status tune_plan(rsvd_plan_t plan, const TuneRun& a, int reps, hipStream_t s, int* tuned) {
  if (!plan || reps < 1 || reps > 100) return RSVD_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return tune_one(plan, a, reps, s, tuned);
}

}  // namespace rsvd

using namespace rsvd;

extern "C" {

rsvd_status rsvd_tune(rsvd_plan_t plan, const double* A, int64_t lda, const double* omega,
                      int64_t ldo, double* S, double* U, int64_t ldu, double* V, int64_t ldv,
                      rsvd_result* res_dev, void* work, size_t work_bytes, int32_t reps,
                      int32_t* n_tuned, void* stream) {
  int tuned = 0;
  const TuneRun a{A, lda, omega, ldo, S, U, ldu, V, ldv, res_dev, work, work_bytes};
  const rsvd_status r = tune_plan(plan, a, reps, (hipStream_t)stream, &tuned);
  if (n_tuned) *n_tuned = tuned;
  return r;
}

int64_t rsvd_tune_entries(int64_t max, int32_t* kind, int64_t* mnk, int32_t* cfg) {
  std::lock_guard<std::mutex> lk(g_mu);
  int64_t i = 0;
  for (const auto& kv : g_table) {
    if (i < max) {
      if (kind) kind[i] = kv.first.kind * 100 + kv.first.prec * 10 + kv.first.ta;
      if (mnk) {
        mnk[3 * i] = kv.first.M;
        mnk[3 * i + 1] = kv.first.N;
        mnk[3 * i + 2] = kv.first.K;
      }
      if (cfg) {
        cfg[3 * i] = kv.second.a;
        cfg[3 * i + 1] = kv.second.b;
        cfg[3 * i + 2] = kv.second.c;
      }
    }
    i++;
  }
  return i;
}

rsvd_status rsvd_tune_set(int32_t kind, int32_t arith, int32_t trans, int64_t M, int64_t N,
                          int64_t K, int32_t a, int32_t b, int32_t c) {
  if (kind < kTuneDma || kind > kTuneBf16 || arith < 0 || arith > 3 || (trans != 0 && trans != 1) ||
      M < 1 || N < 1 || K < 1)
    return RSVD_EINVAL;
  // the launch sites validate a tiling against the call's scratch and fall
  // back to their heuristic when it does not fit; here only the ranges
  if ((kind == kTuneDma && (a != 4 && a != 8)) || (kind == kTuneResid && (a != 4 && a != 8)) ||
      (kind == kTuneBf16 && (a != 1 && a != 2)) || (kind == kTuneResid && (b > 17 || c > 1)) ||
      b < 0 ||
      b > 64 || c < 0 || c > 1024)
    return RSVD_EINVAL;
  TuneKey k;
  k.kind = kind;
  k.prec = arith;
  k.ta = trans;
  k.M = M;
  k.N = N;
  k.K = kind == kTuneBf16 ? bf16_pad(K) : K;
  TuneCfg cfg;
  cfg.a = a;
  cfg.b = b;
  cfg.c = c;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = cfg;
  g_gen++;
  return RSVD_OK;
}

void rsvd_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_gen++;
}

}  // extern "C"
