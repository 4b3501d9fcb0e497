// Batched stepping of many independent problems (parameter sweeps, uneven sizes).
//
// One iteration of a batch issues one launch per step kernel for all instances
// (work tables map a block to (instance, local block)) and one launch per size
// class of eigensolves (all pair matrices of the same n in one launch, all
// momentum blocks of the same n_op in another), with threads per workgroup
// chosen by the autotuner per class.  Pair projections run on a side stream,
// concurrently with the cluster update, the DFTs and the momentum projections.
// The iteration is captured twice in HIP
// graphs -- all eigensolves warm-started, and the periodic cold refresh -- and
// replayed.  Each instance keeps its own state and kept eigenvectors, so a
// problem can be stepped alone or in a batch interchangeably.
#include <algorithm>
#include <cstddef>
#include <map>
#include <tuple>
#include <vector>

#include "problem.h"
#include "sign_batched.h"

using namespace vemb;

struct vemb_batch {
  std::vector<vemb_problem*> probs;
  hipStream_t stream = nullptr;  // own non-blocking stream (capturable), default priority
  hipStream_t side = nullptr;    // pair projections, concurrent with the momentum branch
  hipEvent_t ev = nullptr, fork_ev = nullptr, join_ev = nullptr;
  int refresh = 64;
  StepArgs* d_args = nullptr;
  WorkItem* d_work[5] = {};
  int nwork[5] = {};
  PairPtrs* d_pair = nullptr;
  MomPtrs* d_mom = nullptr;
  std::vector<int> active;  // host copy of the instances' mask (1 stepped, 0 masked)
  struct Group {
    int kind, n, precision, count, tpb;
    int2* d_item;
    void* vstore_any;
    void* wscr;
    void* tscr;
    void* nscr;  // FP64 blocks above 64: scratch of the sign-function projection (else null)
  };
  std::vector<Group> groups;
  bool use_graph = true;
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // [cold]
  DeviceMemory mem;  // every device allocation of the batch
  // sampled kernel timing (vemb_batch_set_profiling): iterations whose batch iteration index is a
  // multiple of prof_every are enqueued directly with events around the timed launches
  int prof_every = 0;
  int64_t iter = 0;
  struct Mark { int id; hipEvent_t start, stop; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> free_events;
  double prof_ms[VEMB_BK_COUNT] = {};
  int64_t prof_n[VEMB_BK_COUNT] = {};
};

namespace {

template <typename T>
int balloc(vemb_batch* b, T** p, size_t count) {
  void* raw = b->mem.get(std::max<size_t>(count, 1) * sizeof(T));
  if (!raw) return fail(VEMB_E_NOMEM, "batch allocation");
  *p = static_cast<T*>(raw);
  return VEMB_OK;
}

// Mask (0) or unmask (1) instance i: the flags inside its device step arguments and projection pointers,
// written on the batch stream, so that later launches and graph replays see them.
int set_active(vemb_batch* b, int i, int active) {
  hipStream_t s = b->stream;
  const int v = active;
  char* a = reinterpret_cast<char*>(b->d_args + i) + offsetof(StepArgs, active);
  char* pp = reinterpret_cast<char*>(b->d_pair + i) + offsetof(PairPtrs, active);
  char* mp = reinterpret_cast<char*>(b->d_mom + i) + offsetof(MomPtrs, active);
  VEMB_TRY(hip_rc(hipMemcpyAsync(a, &v, sizeof(int), hipMemcpyHostToDevice, s), "mask"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(pp, &v, sizeof(int), hipMemcpyHostToDevice, s), "mask"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(mp, &v, sizeof(int), hipMemcpyHostToDevice, s), "mask"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "mask sync"));
  b->active[i] = active;
  return VEMB_OK;
}

hipEvent_t take_event(vemb_batch* b) {
  if (!b->free_events.empty()) {
    hipEvent_t e = b->free_events.back();
    b->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Events of one timed launch: `on` false leaves the launch untimed.
struct Timer {
  vemb_batch* b;
  bool on;
  int id = 0;
  hipEvent_t start = nullptr;
  void before(int kid, hipStream_t st) {
    if (!on) return;
    id = kid;
    start = take_event(b);
    if (start) hipEventRecord(start, st);
  }
  void after(hipStream_t st) {
    if (!on || !start) return;
    hipEvent_t stop = take_event(b);
    if (stop) {
      hipEventRecord(stop, st);
      b->marks.push_back({id, start, stop});
    }
    start = nullptr;
  }
};

struct SignHookCtx {
  Timer* timer;
  int id;
};
void sign_hook(void* ctx, int phase, hipStream_t st) {
  auto* c = static_cast<SignHookCtx*>(ctx);
  if (phase == 0)
    c->timer->before(c->id, st);
  else
    c->timer->after(st);
}

int enqueue_iteration(vemb_batch* b, int cold, bool timed = false) {
  hipStream_t s = b->stream;
  const int n_inst = (int)b->probs.size();
  const int max_sweeps = b->probs[0]->opt.max_sweeps;
  Timer tm{b, timed}, tm_side{b, timed};
  tm.before(VEMB_BK_PAIR_UPDATE, s);
  VEMB_TRY(hip_rc(launch_step_batched(0, b->d_args, b->d_work[0], b->nwork[0], s), "batched pair update"));
  tm.after(s);
  tm.before(VEMB_BK_PAIR_XSTEP, s);
  VEMB_TRY(hip_rc(launch_step_batched(1, b->d_args, b->d_work[1], b->nwork[1], s), "batched X step"));
  tm.after(s);
  // fork: pair projections on the side stream (they feed only the next iteration)
  VEMB_TRY(hip_rc(hipEventRecord(b->fork_ev, s), "fork"));
  VEMB_TRY(hip_rc(hipStreamWaitEvent(b->side, b->fork_ev, 0), "fork"));
  SignHookCtx side_ctx{&tm_side, VEMB_BK_SIGN_GEMM_REAL}, main_ctx{&tm, VEMB_BK_SIGN_GEMM_CPLX};
  const LaunchHook side_hook{sign_hook, &side_ctx}, main_hook{sign_hook, &main_ctx};
  for (const auto& g : b->groups)
    if (g.kind == 0) {
      if (!g.nscr) tm_side.before(VEMB_BK_PAIR_JACOBI, b->side);
      VEMB_TRY(hip_rc(g.nscr ? launch_projection_group_sign(0, g.n, g.count, g.d_item, b->d_pair, g.nscr, b->side,
                                                            timed ? &side_hook : nullptr, solve_precision(g.precision))
                             : launch_projection_group(0, g.n, g.count, solve_precision(g.precision), max_sweeps, cold,
                                                       g.tpb, g.d_item, b->d_pair, g.vstore_any, g.wscr, g.tscr,
                                                       b->side),
                      "batched pair projection"));
      if (!g.nscr) tm_side.after(b->side);
    }
  VEMB_TRY(hip_rc(hipEventRecord(b->join_ev, b->side), "join"));
  tm.before(VEMB_BK_CLUSTER, s);
  VEMB_TRY(hip_rc(launch_step_batched(2, b->d_args, nullptr, n_inst, s), "batched cluster update"));
  tm.after(s);
  tm.before(VEMB_BK_DFT_FWD, s);
  VEMB_TRY(hip_rc(launch_step_batched(3, b->d_args, b->d_work[3], b->nwork[3], s), "batched forward DFT"));
  tm.after(s);
  for (const auto& g : b->groups)
    if (g.kind == 1) {
      if (!g.nscr) tm.before(VEMB_BK_MOM_JACOBI, s);
      VEMB_TRY(hip_rc(g.nscr ? launch_projection_group_sign(1, g.n, g.count, g.d_item, b->d_mom, g.nscr, s,
                                                            timed ? &main_hook : nullptr, solve_precision(g.precision))
                             : launch_projection_group(1, g.n, g.count, solve_precision(g.precision), max_sweeps, cold,
                                                       g.tpb, g.d_item, b->d_mom, g.vstore_any, g.wscr, g.tscr, s),
                      "batched momentum projection"));
      if (!g.nscr) tm.after(s);
    }
  tm.before(VEMB_BK_DFT_INV, s);
  VEMB_TRY(hip_rc(launch_step_batched(4, b->d_args, b->d_work[4], b->nwork[4], s), "batched inverse DFT"));
  tm.after(s);
  VEMB_TRY(hip_rc(hipStreamWaitEvent(s, b->join_ev, 0), "join"));
  return VEMB_OK;
}

int drain_marks(vemb_batch* b) {
  if (b->marks.empty()) return VEMB_OK;
  VEMB_TRY(hip_rc(hipStreamSynchronize(b->stream), "profile sync"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(b->side), "profile sync"));
  for (auto& mk : b->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, mk.start, mk.stop) == hipSuccess) {
      b->prof_ms[mk.id] += ms;
      b->prof_n[mk.id] += 1;
    }
    b->free_events.push_back(mk.start);
    b->free_events.push_back(mk.stop);
  }
  b->marks.clear();
  return VEMB_OK;
}

int capture(vemb_batch* b, int cold, hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  VEMB_TRY(hip_rc(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture"));
  const int rc = enqueue_iteration(b, cold);
  const hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (rc != VEMB_OK) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  VEMB_TRY(hip_rc(e, "end capture"));
  const hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  return hip_rc(ie, "graph instantiate");
}

}  // namespace

extern "C" {

int vemb_batch_create(vemb_problem* const* problems, int count, int use_graph, vemb_batch** out) {
  if (!problems || count <= 0 || !out) return fail(VEMB_E_INVALID, "bad arguments to vemb_batch_create");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!problems[i]) return fail(VEMB_E_INVALID, "NULL problem in batch");
    if (problems[i]->opt.max_sweeps != problems[0]->opt.max_sweeps ||
        problems[i]->opt.warm_refresh != problems[0]->opt.warm_refresh)
      return fail(VEMB_E_INVALID, "problems of a batch must share max_sweeps and warm_refresh");
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return fail(VEMB_E_INVALID, "a problem appears twice in the batch");
    if (problems[i]->opt.adapt_every > 0)
      return fail(VEMB_E_UNSUPPORTED, "adaptive parameters (adapt_every) run on single problems only");
  }
  auto* b = new vemb_batch();
  object_created();
  b->probs.assign(problems, problems + count);
  b->active.assign(count, 1);
  b->use_graph = use_graph != 0;
  b->refresh = problems[0]->opt.warm_refresh;
  auto cleanup = [&](int rc) {
    vemb_batch_destroy(b);
    return rc;
  };
  int rc;
  if ((rc = hip_rc(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "batch stream")) ||
      (rc = hip_rc(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "batch stream")) ||
      (rc = hip_rc(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming), "batch event")) ||
      (rc = hip_rc(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming), "batch event")) ||
      (rc = hip_rc(hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming), "batch event")))
    return cleanup(rc);
  // per-instance arguments, pointers and work tables
  std::vector<StepArgs> args(count);
  std::vector<PairPtrs> pp(count);
  std::vector<MomPtrs> mp(count);
  std::vector<WorkItem> work[5];
  std::map<std::tuple<int, int, int>, std::vector<int2>> classes;  // (kind, n, precision) -> items
  for (int i = 0; i < count; ++i) {
    vemb_problem* p = problems[i];
    args[i] = p->a;
    args[i].active = 1;
    pp[i] = {p->a.rho, p->a.Lam, p->a.rho_t, p->a.feas, p->a.sweeps, p->a.Vpair, p->a.mu, 1};
    mp[i] = {p->a.Xh, p->a.sweeps + p->P, p->a.Vmom, 1};
    int grid[5][2];
    local_grids(p->a, grid);
    for (int w = 0; w < 5; ++w) {
      if (w == 2) continue;
      for (int by = 0; by < grid[w][1]; ++by)
        for (int bx = 0; bx < grid[w][0]; ++bx) work[w].push_back({i, bx, by, 0});
    }
    const int prec = p->opt.precision;
    for (int d = 0; d < p->P; ++d) classes[{0, p->a.n, prec}].push_back(make_int2(i, d));
    for (int k = 0; k < p->Ku; ++k) classes[{1, p->a.n_op, prec}].push_back(make_int2(i, k));
  }
  if ((rc = balloc(b, &b->d_args, count)) || (rc = balloc(b, &b->d_pair, count)) || (rc = balloc(b, &b->d_mom, count)))
    return cleanup(rc);
  hipStream_t s = b->stream;
  if ((rc = hip_rc(hipMemcpyAsync(b->d_args, args.data(), sizeof(StepArgs) * count, hipMemcpyHostToDevice, s), "args")) ||
      (rc = hip_rc(hipMemcpyAsync(b->d_pair, pp.data(), sizeof(PairPtrs) * count, hipMemcpyHostToDevice, s), "ptrs")) ||
      (rc = hip_rc(hipMemcpyAsync(b->d_mom, mp.data(), sizeof(MomPtrs) * count, hipMemcpyHostToDevice, s), "ptrs")))
    return cleanup(rc);
  for (int w = 0; w < 5; ++w) {
    if (w == 2) continue;
    b->nwork[w] = (int)work[w].size();
    if ((rc = balloc(b, &b->d_work[w], work[w].size())) ||
        (rc = hip_rc(hipMemcpyAsync(b->d_work[w], work[w].data(), sizeof(WorkItem) * work[w].size(),
                                    hipMemcpyHostToDevice, s), "work table")))
      return cleanup(rc);
  }
  for (auto& kv : classes) {
    const auto& items = kv.second;
    vemb_batch::Group g{};
    g.kind = std::get<0>(kv.first);
    g.n = std::get<1>(kv.first);
    g.precision = std::get<2>(kv.first);
    g.count = (int)items.size();
    g.vstore_any = g.kind == 0 ? (void*)problems[items[0].x]->a.Vpair : (void*)problems[items[0].x]->a.Vmom;
    if ((rc = balloc(b, &g.d_item, items.size())) ||
        (rc = hip_rc(hipMemcpyAsync(g.d_item, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, s),
                     "class table")))
      return cleanup(rc);
    if (g.n > 64) {  // sign-function projection on matrix cores (FP64, or FP32 for MIXED / FP32)
      char* w = nullptr;
      if ((rc = balloc(b, &w, sign_work_bytes(g.n, g.count, g.kind == 1)))) return cleanup(rc);
      g.nscr = w;
      g.tpb = 256;
    } else if (g.n > 64) {  // streamed solver scratch, complex-double sized
      double *w = nullptr, *t = nullptr;
      if ((rc = balloc(b, &w, (size_t)2 * g.count * g.n * g.n)) || (rc = balloc(b, &t, (size_t)2 * g.count * g.n * g.n)))
        return cleanup(rc);
      g.wscr = w;
      g.tscr = t;
      g.tpb = 256;
    } else {
      // a fixed opts->tpb is honoured; otherwise tune for the class's batch size
      const vemb_problem* first = problems[items[0].x];
      g.tpb = first->opt.tpb > 0 ? (g.kind == 0 ? first->tpb_pair : first->tpb_mom)
                                 : tuned_tpb(g.n, g.kind == 1, solve_precision(g.precision), g.count, s);
      if (g.tpb <= 0) return cleanup(g.tpb);
    }
    b->groups.push_back(g);
  }
  if ((rc = hip_rc(hipStreamSynchronize(s), "batch setup sync"))) return cleanup(rc);
  if (b->use_graph) {
    if ((rc = capture(b, 0, &b->exec[0])) || (rc = capture(b, 1, &b->exec[1]))) return cleanup(rc);
  }
  *out = b;
  return VEMB_OK;
}

int vemb_batch_step(vemb_batch* b, int iters) {
  if (!b || iters < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_batch_step");
  // order after work already queued on the problems' streams
  for (vemb_problem* p : b->probs) {
    VEMB_TRY(hip_rc(hipEventRecord(b->ev, p->stream), "batch order"));
    VEMB_TRY(hip_rc(hipStreamWaitEvent(b->stream, b->ev, 0), "batch order"));
  }
  for (int it = 0; it < iters; ++it) {
    // one graph serves all instances: start cold if any instance would alone
    bool cold = b->refresh < 0;
    for (size_t i = 0; i < b->probs.size(); ++i) {
      const vemb_problem* p = b->probs[i];
      if (b->active[i]) cold = cold || !p->v_valid || (b->refresh > 0 && p->t % b->refresh == 0);
    }
    const bool timed = b->prof_every > 0 && b->iter % b->prof_every == 0;
    if (b->use_graph && !timed)
      VEMB_TRY(hip_rc(hipGraphLaunch(b->exec[cold ? 1 : 0], b->stream), "graph launch"));
    else
      VEMB_TRY(enqueue_iteration(b, cold ? 1 : 0, timed));
    ++b->iter;
    for (size_t i = 0; i < b->probs.size(); ++i) {
      if (!b->active[i]) continue;  // a masked instance keeps its state and its iteration count
      vemb_problem* p = b->probs[i];
      p->v_valid = true;
      p->v_fp32 = solve_precision(p->opt.precision) != VEMB_FP64;
      ++p->t;
    }
  }
  // later work on a problem's own stream waits for the batch
  VEMB_TRY(hip_rc(hipEventRecord(b->ev, b->stream), "batch order"));
  for (vemb_problem* p : b->probs) VEMB_TRY(hip_rc(hipStreamWaitEvent(p->stream, b->ev, 0), "batch order"));
  return VEMB_OK;
}

int vemb_batch_dual_bounds(vemb_batch* b, double* lb, int* status) {
  if (!b || !lb) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(hip_rc(hipStreamSynchronize(b->stream), "batch sync"));
  int worst = VEMB_OK;
  for (size_t i = 0; i < b->probs.size(); ++i) {
    const int rc = vemb_dual_bound(b->probs[i], &lb[i]);
    if (status) status[i] = rc;
    if (rc != VEMB_OK) worst = rc;
    if (rc == VEMB_E_NUMERIC && b->active[i]) VEMB_TRY(set_active(b, (int)i, 0));
  }
  return worst;
}

int vemb_batch_primal_energies(vemb_batch* b, double* e, double* feas) {
  if (!b) return fail(VEMB_E_INVALID, "NULL batch");
  VEMB_TRY(hip_rc(hipStreamSynchronize(b->stream), "batch sync"));
  int worst = VEMB_OK;
  for (size_t i = 0; i < b->probs.size(); ++i) {
    const int rc = vemb_primal_energy(b->probs[i], e ? &e[i] : nullptr, feas ? &feas[i] : nullptr);
    if (rc != VEMB_OK) worst = rc;
    if (rc == VEMB_E_NUMERIC && b->active[i]) VEMB_TRY(set_active(b, (int)i, 0));
  }
  return worst;
}

int vemb_batch_set_active(vemb_batch* b, int index, int active) {
  if (!b || index < 0 || index >= (int)b->probs.size())
    return fail(VEMB_E_INVALID, "bad arguments to vemb_batch_set_active");
  return set_active(b, index, active ? 1 : 0);
}

int vemb_batch_get_active(const vemb_batch* b, int* active) {
  if (!b || !active) return fail(VEMB_E_INVALID, "NULL argument");
  for (size_t i = 0; i < b->probs.size(); ++i) active[i] = b->active[i];
  return VEMB_OK;
}

int vemb_batch_info(const vemb_batch* b, int* groups, int* launches_per_iteration) {
  if (!b) return fail(VEMB_E_INVALID, "NULL batch");
  if (groups) *groups = (int)b->groups.size();
  if (launches_per_iteration) {
    int l = 5;
    for (const auto& g : b->groups) l += g.nscr ? sign_launches(solve_precision(g.precision)) : 1;
    *launches_per_iteration = l;
  }
  return VEMB_OK;
}

int vemb_batch_set_profiling(vemb_batch* b, int every) {
  if (!b || every < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_batch_set_profiling");
  VEMB_TRY(drain_marks(b));
  for (int k = 0; k < VEMB_BK_COUNT; ++k) {
    b->prof_ms[k] = 0.0;
    b->prof_n[k] = 0;
  }
  b->prof_every = every;
  // events for the timings are created here, not between launches
  while (every > 0 && b->free_events.size() < 1024) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    b->free_events.push_back(e);
  }
  return VEMB_OK;
}

int vemb_batch_get_profile(vemb_batch* b, vemb_batch_profile* out) {
  if (!b || !out) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(drain_marks(b));
  for (int k = 0; k < VEMB_BK_COUNT; ++k) {
    out->ms[k] = b->prof_ms[k];
    out->launches[k] = b->prof_n[k];
  }
  return VEMB_OK;
}

int vemb_batch_sync(vemb_batch* b) {
  if (!b) return fail(VEMB_E_INVALID, "NULL batch");
  return hip_rc(hipStreamSynchronize(b->stream), "batch sync");
}

void vemb_batch_destroy(vemb_batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  for (auto& e : b->exec)
    if (e) hipGraphExecDestroy(e);
  if (b->side) hipStreamSynchronize(b->side);
  b->mem.release();
  for (auto& mk : b->marks) {
    hipEventDestroy(mk.start);
    hipEventDestroy(mk.stop);
  }
  for (hipEvent_t e : b->free_events) hipEventDestroy(e);
  if (b->ev) hipEventDestroy(b->ev);
  if (b->fork_ev) hipEventDestroy(b->fork_ev);
  if (b->join_ev) hipEventDestroy(b->join_ev);
  if (b->side) hipStreamDestroy(b->side);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
  object_destroyed();
}

}  // extern "C"
