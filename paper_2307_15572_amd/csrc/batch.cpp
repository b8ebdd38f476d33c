// Batched decompositions of independent channels (include/rsvd.h, "Batched
// decompositions"): an LPT schedule of the channels over concurrent HIP
// streams, optionally captured once into a hipGraph and replayed.
//
// Small channels leave most of the 256 compute units idle in their latency-
// bound phases (QR of the panels, the Jacobi sweeps of the small SVD); running
// several channels on concurrent streams fills the device with independent
// work, while the large channels' streaming products fill it on their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"
#include "plan.hpp"
#include "tune.hpp"

struct rsvd_batch_s {
  int64_t count = 0;
  int lanes = 0;
  bool use_graph = false;
  std::vector<rsvd_plan_t> plans;
  std::vector<int32_t> lane_of;
  std::vector<std::vector<int64_t>> items;  // channels of each lane, in run order
  std::vector<size_t> lane_off, lane_bytes;
  size_t total = 0;
  // small SVDs grouped into one launch (jacobi_batch): values-only channels
  // keep their Jacobi matrix and state in compact slots; channels that want
  // vectors run in a workspace slice of their own and are resumed there
  std::vector<int64_t> deferred;          // channel ids, in table order
  std::vector<rsvd::JacChan> table;       // their Jacobi matrices and states
  std::vector<size_t> def_sig, def_scr;   // per deferred channel: values, ordering scratch
  std::vector<int> kind;                  // per channel: 0 whole, 1 compact, 2 own slice
  std::vector<size_t> own_off, own_bytes; // per channel: its own slice (kind 2)
  size_t off_bar = 0;                     // grid barrier of the grouped launch
  int64_t first_round_pairs = 0;
  rsvd::JacChan* dtable = nullptr;        // device copy of the table
  // device objects, created at the first run
  int device = -1;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
  bool graph_failed = false;
  bool graph_used = false;
};

namespace {

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of the own slices of channels that want vectors and have their
// small SVD grouped; channels beyond it run whole in their lane's slice.
constexpr size_t kOwnSliceBudget = (size_t)64 << 30;

void release(rsvd_batch_s* b) {
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamSynchronize(s);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  for (hipEvent_t e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  for (rsvd_plan_t p : b->plans) rsvd_destroy(p);
  if (b->dtable) (void)hipFree(b->dtable);
  b->dtable = nullptr;
  b->exec = nullptr;
  b->fork = nullptr;
  b->joins.clear();
  b->streams.clear();
  b->plans.clear();
}

rsvd_status ensure_device_objects(rsvd_batch_s* b) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSVD_EHIP;
  if (b->device >= 0) return dev == b->device ? RSVD_OK : RSVD_EINVAL;
  b->streams.assign(b->lanes, nullptr);
  b->joins.assign(b->lanes, nullptr);
  for (int i = 0; i < b->lanes; i++) {
    // default priority, non-blocking with respect to the null stream
    if (hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) != hipSuccess)
      return RSVD_EHIP;
    if (hipEventCreateWithFlags(&b->joins[i], hipEventDisableTiming) != hipSuccess)
      return RSVD_EHIP;
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return RSVD_EHIP;
  if (!b->table.empty()) {
    // the table holds workspace offsets, so one upload serves every run
    const size_t bytes = b->table.size() * sizeof(rsvd::JacChan);
    if (hipMalloc((void**)&b->dtable, bytes) != hipSuccess) return RSVD_EHIP;
    if (hipMemcpy(b->dtable, b->table.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
      return RSVD_EHIP;
  }
  b->device = dev;
  return RSVD_OK;
}

struct BatchArgs {
  const double* const* A;
  const int64_t* lda;
  double* const* S;
  double* const* U;
  const int64_t* ldu;
  double* const* V;
  const int64_t* ldv;
  rsvd_result* res;
  char* work;
};

// Host-side checks of one channel's arguments (those rsvd_run makes), done
// for every channel before anything is enqueued.
rsvd_status check_channel(const rsvd_plan_s& pl, const BatchArgs& a, int64_t c) {
  const rsvd_problem& p = pl.p;
  if (!a.A[c] || !a.S[c] || a.lda[c] < p.n) return RSVD_EINVAL;
  if (p.want_u && (!a.U || !a.ldu || !a.U[c] || a.ldu[c] < pl.kc)) return RSVD_EINVAL;
  if (p.want_v && (!a.V || !a.ldv || !a.V[c] || a.ldv[c] < pl.kc)) return RSVD_EINVAL;
  return RSVD_OK;
}

// Point the deferred channels' plans at their slots of this workspace (or
// clear them: work == nullptr).
void set_deferral(rsvd_batch_s* b, char* work) {
  for (size_t i = 0; i < b->deferred.size(); i++) {
    const int64_t c = b->deferred[i];
    rsvd_plan_s& pl = *b->plans[c];
    const bool compact = b->kind[c] == 1;
    pl.defer_M = work && compact ? reinterpret_cast<double*>(work + b->table[i].M_off) : nullptr;
    pl.defer_st =
        work && compact ? reinterpret_cast<rsvd::DevState*>(work + b->table[i].st_off) : nullptr;
    pl.defer_inplace = work && !compact;
  }
}

// Workspace of channel c's run: its own slice, or its lane's.
char* chan_work(const rsvd_batch_s* b, char* work, int64_t c, size_t* bytes) {
  if (b->kind[c] == 2) {
    *bytes = b->own_bytes[c];
    return work + b->own_off[c];
  }
  const int i = b->lane_of[c];
  *bytes = b->lane_bytes[i];
  return work + b->lane_off[i];
}

rsvd_status fork(rsvd_batch_s* b, hipStream_t origin) {
  if (hipEventRecord(b->fork, origin) != hipSuccess) return RSVD_EHIP;
  for (int i = 0; i < b->lanes; i++)
    if (b->streams[i] != origin && hipStreamWaitEvent(b->streams[i], b->fork, 0) != hipSuccess)
      return RSVD_EHIP;
  return RSVD_OK;
}

rsvd_status join(rsvd_batch_s* b, hipStream_t origin) {
  for (int i = 0; i < b->lanes; i++) {
    if (b->streams[i] == origin) continue;
    if (hipEventRecord(b->joins[i], b->streams[i]) != hipSuccess) return RSVD_EHIP;
    if (hipStreamWaitEvent(origin, b->joins[i], 0) != hipSuccess) return RSVD_EHIP;
  }
  return RSVD_OK;
}

// Fork from `origin`, run every lane's channels (enqueued interleaved so all
// lanes start early), join back into `origin`. Values-only channels stop
// before their small SVD; after the join their sweeps run in one grouped
// launch and their results are finished on `origin`.
rsvd_status enqueue_all(rsvd_batch_s* b, const BatchArgs& a, hipStream_t origin) {
  set_deferral(b, a.work);
  rsvd_status r = fork(b, origin);
  if (r != RSVD_OK) return r;
  size_t longest = 0;
  for (const auto& it : b->items) longest = std::max(longest, it.size());
  for (size_t pos = 0; pos < longest; pos++) {
    for (int i = 0; i < b->lanes; i++) {
      if (pos >= b->items[i].size()) continue;
      const int64_t c = b->items[i][pos];
      const rsvd_plan_s& pl = *b->plans[c];
      size_t bytes = 0;
      char* w = chan_work(b, a.work, c, &bytes);
      r = rsvd_run(b->plans[c], a.A[c], a.lda[c], nullptr, 0, a.S[c],
                   pl.p.want_u ? a.U[c] : nullptr, pl.p.want_u ? a.ldu[c] : 0,
                   pl.p.want_v ? a.V[c] : nullptr, pl.p.want_v ? a.ldv[c] : 0, a.res + c, w, bytes,
                   (void*)b->streams[i]);
      if (r != RSVD_OK && r != kStatusDeferred) return r;
    }
  }
  if ((r = join(b, origin)) != RSVD_OK) return r;
  if (b->deferred.empty()) return RSVD_OK;
  // the sweeps of every deferred channel in one launch
  r = rsvd::jacobi_batch(b->dtable, (int)b->deferred.size(), b->first_round_pairs, a.work,
                         reinterpret_cast<rsvd::GridBar*>(a.work + b->off_bar), origin);
  if (r != RSVD_OK) return r;
  // values-only channels: finished on the caller's stream
  for (size_t i = 0; i < b->deferred.size(); i++) {
    const int64_t c = b->deferred[i];
    if (b->kind[c] != 1) continue;
    r = finish_deferred(*b->plans[c], reinterpret_cast<double*>(a.work + b->table[i].M_off),
                        reinterpret_cast<rsvd::DevState*>(a.work + b->table[i].st_off),
                        reinterpret_cast<double*>(a.work + b->def_sig[i]),
                        reinterpret_cast<double*>(a.work + b->def_scr[i]), a.S[c], a.res + c, origin);
    if (r != RSVD_OK) return r;
  }
  // channels with vectors: resumed in their own slices on their lanes
  bool any = false;
  for (int64_t c : b->deferred) any = any || b->kind[c] == 2;
  if (!any) return RSVD_OK;
  if ((r = fork(b, origin)) != RSVD_OK) return r;
  for (size_t pos = 0; pos < longest; pos++) {
    for (int i = 0; i < b->lanes; i++) {
      if (pos >= b->items[i].size()) continue;
      const int64_t c = b->items[i][pos];
      if (b->kind[c] != 2) continue;
      const rsvd_plan_s& pl = *b->plans[c];
      r = resume_deferred(pl, a.A[c], a.lda[c], a.S[c], pl.p.want_u ? a.U[c] : nullptr,
                          pl.p.want_u ? a.ldu[c] : 0, pl.p.want_v ? a.V[c] : nullptr,
                          pl.p.want_v ? a.ldv[c] : 0, a.res + c, a.work + b->own_off[c],
                          b->streams[i]);
      if (r != RSVD_OK) return r;
    }
  }
  return join(b, origin);
}

std::vector<uintptr_t> make_key(const rsvd_batch_s* b, const BatchArgs& a) {
  std::vector<uintptr_t> k;
  k.reserve((size_t)b->count * 7 + 2);
  for (int64_t c = 0; c < b->count; c++) {
    const rsvd_problem& p = b->plans[c]->p;
    k.push_back((uintptr_t)a.A[c]);
    k.push_back((uintptr_t)a.lda[c]);
    k.push_back((uintptr_t)a.S[c]);
    k.push_back(p.want_u ? (uintptr_t)a.U[c] : 0);
    k.push_back(p.want_u ? (uintptr_t)a.ldu[c] : 0);
    k.push_back(p.want_v ? (uintptr_t)a.V[c] : 0);
    k.push_back(p.want_v ? (uintptr_t)a.ldv[c] : 0);
  }
  k.push_back((uintptr_t)a.res);
  k.push_back((uintptr_t)a.work);
  // captured launches hold the tile shapes in force when they were captured
  k.push_back((uintptr_t)rsvd::tune_generation());
  return k;
}

// Capture the fork / run / join sequence into b->exec. Returns false (and
// leaves no capture open) if the runtime refuses any part of it.
bool capture(rsvd_batch_s* b, const BatchArgs& a) {
  hipStream_t origin = b->streams[0];
  if (hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const rsvd_status r = enqueue_all(b, a, origin);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(origin, &g);
  bool ok = r == RSVD_OK && e == hipSuccess && g != nullptr;
  if (ok && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->exec = nullptr;
    ok = false;
  }
  if (g) (void)hipGraphDestroy(g);
  if (!ok) (void)hipGetLastError();
  return ok;
}

}  // namespace

extern "C" {

rsvd_status rsvd_batch_plan(const rsvd_problem* probs, int64_t count, int32_t lanes,
                            int32_t use_graph, rsvd_batch_t* out, size_t* workspace_bytes) {
  if (!probs || !out || count < 1 || lanes < 0 || lanes > 16) return RSVD_EINVAL;
  for (int64_t c = 0; c < count; c++)
    if (probs[c].adaptive) return RSVD_EINVAL;
  rsvd_batch_s* b = new (std::nothrow) rsvd_batch_s();
  if (!b) return RSVD_ENOMEM;
  b->count = count;
  int L = lanes > 0 ? lanes : 4;
  if (L > count) L = (int)count;
  b->lanes = L;
  b->use_graph = use_graph != 0;
  std::vector<size_t> ws((size_t)count);
  std::vector<double> cost((size_t)count);
  b->plans.reserve((size_t)count);
  for (int64_t c = 0; c < count; c++) {
    rsvd_plan_t p = nullptr;
    const rsvd_status r = rsvd_plan(&probs[c], &p, &ws[c]);
    if (r != RSVD_OK) {
      release(b);
      delete b;
      return r;
    }
    p->coop_share = L;
    b->plans.push_back(p);
    const rsvd_problem& q = p->p;
    cost[c] = (double)q.m * (double)q.n * (double)p->l *
              (double)(2 * q.power_iters + 2 + (q.want_residual ? 1 : 0));
  }
  // LPT: longest channel first, each to the least-loaded lane
  std::vector<int64_t> order((size_t)count);
  for (int64_t c = 0; c < count; c++) order[c] = c;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
  std::vector<double> load((size_t)L, 0.0);
  b->items.assign((size_t)L, {});
  b->lane_of.assign((size_t)count, 0);
  for (int64_t c : order) {
    int best = 0;
    for (int i = 1; i < L; i++)
      if (load[i] < load[best]) best = i;
    b->items[best].push_back(c);
    b->lane_of[c] = best;
    load[best] += cost[c];
  }
  // grouped small SVD: values-only channels in compact slots (kind 1), the
  // others in slices of their own within a budget (kind 2), widest first;
  // a single channel runs whole
  b->kind.assign((size_t)count, 0);
  b->own_off.assign((size_t)count, 0);
  b->own_bytes.assign((size_t)count, 0);
  std::vector<int64_t> dorder = order;
  std::stable_sort(dorder.begin(), dorder.end(),
                   [&](int64_t x, int64_t y) { return b->plans[x]->l > b->plans[y]->l; });
  if (count > 1) {
    size_t own_total = 0;
    for (int64_t c : dorder) {
      const rsvd_plan_s& pl = *b->plans[c];
      if (pl.adaptive) continue;
      if (b->deferred.size() >= rsvd::jacobi_batch_max_channels()) break;
      if (!pl.vectors) {
        b->kind[c] = 1;
      } else if (own_total + round256(ws[c]) <= kOwnSliceBudget) {
        b->kind[c] = 2;
        own_total += round256(ws[c]);
      } else {
        continue;
      }
      b->deferred.push_back(c);
    }
  }
  // lane slices: for the channels that run in them (whole or compact)
  b->lane_off.assign((size_t)L, 0);
  b->lane_bytes.assign((size_t)L, 0);
  size_t at = 0;
  for (int i = 0; i < L; i++) {
    size_t need = 0;
    for (int64_t c : b->items[i])
      if (b->kind[c] != 2) need = std::max(need, ws[c]);
    b->lane_off[i] = at;
    b->lane_bytes[i] = need;
    at += round256(need);
  }
  for (int64_t c : b->deferred) {
    if (b->kind[c] != 2) continue;
    b->own_off[c] = at;
    b->own_bytes[c] = ws[c];
    at += round256(ws[c]);
  }
  for (int64_t c : b->deferred) {
    const rsvd_plan_s& pl = *b->plans[c];
    const int64_t l = pl.l, Lp = rsvd::jacobi_padded(l);
    rsvd::JacChan ch{};
    ch.l = (int)l;
    ch.Lp = (int)Lp;
    const int ms = pl.p.max_sweeps > 0 ? pl.p.max_sweeps : 30;
    ch.max_sweeps = ms > 64 ? 64 : ms;
    if (b->kind[c] == 1) {
      ch.M_off = (int64_t)at;
      at += round256((size_t)Lp * Lp * sizeof(double));
      ch.st_off = (int64_t)at;
      at += round256(sizeof(rsvd::DevState));
      ch.P_off = -1;
      b->def_sig.push_back(at);
      at += round256((size_t)l * sizeof(double));
      b->def_scr.push_back(at);
      at += round256((size_t)2 * l * sizeof(double));
    } else {
      ch.M_off = (int64_t)(b->own_off[c] + pl.off_M);
      ch.st_off = (int64_t)(b->own_off[c] + pl.off_state);
      ch.P_off = (int64_t)(b->own_off[c] + pl.off_P);
      b->def_sig.push_back(0);
      b->def_scr.push_back(0);
    }
    b->table.push_back(ch);
    b->first_round_pairs += Lp / 32;
  }
  if (!b->deferred.empty()) {
    b->off_bar = at;
    at += round256(sizeof(rsvd::GridBar));
  }
  b->total = at;
  *out = b;
  if (workspace_bytes) *workspace_bytes = b->total;
  return RSVD_OK;
}

rsvd_status rsvd_batch_run(rsvd_batch_t plan, const double* const* A, const int64_t* lda,
                           double* const* S, double* const* U, const int64_t* ldu,
                           double* const* V, const int64_t* ldv, rsvd_result* res_dev,
                           void* work, size_t work_bytes, void* stream) {
  if (!plan || !A || !lda || !S || !res_dev || !work) return RSVD_EINVAL;
  rsvd_batch_s* b = plan;
  if (work_bytes < b->total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  BatchArgs a{A, lda, S, U, ldu, V, ldv, res_dev, (char*)work};
  for (int64_t c = 0; c < b->count; c++) {
    const rsvd_status r = check_channel(*b->plans[c], a, c);
    if (r != RSVD_OK) return r;
  }
  rsvd_status r = ensure_device_objects(b);
  if (r != RSVD_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  b->graph_used = false;
  if (b->use_graph && !b->graph_failed) {
    std::vector<uintptr_t> key = make_key(b, a);
    if (!b->exec || key != b->key) {
      if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
      }
      if (capture(b, a)) {
        b->key.swap(key);
      } else {
        b->graph_failed = true;
        b->key.clear();
      }
    }
    if (b->exec) {
      if (hipGraphLaunch(b->exec, s) != hipSuccess) return RSVD_EHIP;
      b->graph_used = true;
      return RSVD_OK;
    }
  }
  return enqueue_all(b, a, s);
}

rsvd_status rsvd_batch_tune(rsvd_batch_t plan, const double* const* A, const int64_t* lda,
                            double* const* S, double* const* U, const int64_t* ldu,
                            double* const* V, const int64_t* ldv, rsvd_result* res_dev,
                            void* work, size_t work_bytes, int32_t reps, int32_t* n_tuned,
                            void* stream) {
  if (!plan || !A || !lda || !S || !res_dev || !work) return RSVD_EINVAL;
  rsvd_batch_s* b = plan;
  if (work_bytes < b->total) return RSVD_ENOMEM;
  if (((uintptr_t)work & 255) != 0) return RSVD_EINVAL;
  BatchArgs a{A, lda, S, U, ldu, V, ldv, res_dev, (char*)work};
  for (int64_t c = 0; c < b->count; c++) {
    const rsvd_status r = check_channel(*b->plans[c], a, c);
    if (r != RSVD_OK) return r;
  }
  // channel by channel on the caller's stream, each in its run's workspace;
  // shapes already in the table are not timed again (whole runs: nothing is
  // deferred to the grouped launch here)
  set_deferral(b, nullptr);
  int tuned = 0;
  rsvd_status r = RSVD_OK;
  for (int64_t c = 0; c < b->count && r == RSVD_OK; c++) {
    const rsvd_plan_s& pl = *b->plans[c];
    size_t bytes = 0;
    char* w = chan_work(b, a.work, c, &bytes);
    const rsvd::TuneRun run{a.A[c], a.lda[c], nullptr, 0, a.S[c],
                            pl.p.want_u ? a.U[c] : nullptr, pl.p.want_u ? a.ldu[c] : 0,
                            pl.p.want_v ? a.V[c] : nullptr, pl.p.want_v ? a.ldv[c] : 0,
                            a.res + c, w, bytes};
    r = rsvd::tune_plan(b->plans[c], run, reps, (hipStream_t)stream, &tuned);
  }
  if (n_tuned) *n_tuned = tuned;
  return r;
}

rsvd_status rsvd_batch_info(rsvd_batch_t plan, int32_t* lane_of, int32_t* graph_replayed) {
  if (!plan) return RSVD_EINVAL;
  if (lane_of)
    for (int64_t c = 0; c < plan->count; c++) lane_of[c] = plan->lane_of[c];
  if (graph_replayed) *graph_replayed = plan->graph_used ? 1 : 0;
  return RSVD_OK;
}

void rsvd_batch_destroy(rsvd_batch_t plan) {
  if (!plan) return;
  release(plan);
  delete plan;
}

}  // extern "C"
