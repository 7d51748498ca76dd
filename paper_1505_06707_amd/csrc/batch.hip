// Batched propagation of many independent 2D problems of uneven size
// (the split-operator step of Sec. II applied to each run).
//
// Runs with the same problem statement form a class that shares one plan's
// tables; one launch of a pass covers the lines of every run of a class
// (tdse.hip: a tile list over runs, run-major).  Per class the launch shape
// (threads per block, one block per tile or a persistent grid) is chosen by
// timing the candidates on scratch states.  The steady-state steps are
// replayed from a captured HIP graph with one independent branch per class;
// the step index comes from a per-class device counter that the branch
// advances, so one graph serves every chunk of steps.
#include <algorithm>
#include <cstring>
#include <map>

#include "internal.hpp"

struct sofft_plan;   // defined in plan.hip: a Plan

namespace sofft {
Plan& plan_of(sofft_plan* p);

namespace {

struct BatchClass {
  sofft_plan* plan = nullptr;  // tables shared by the runs of this shape
  std::vector<int> runs;       // global run indices
  int64_t points = 0;          // n_x n_y
  DevBuf ptrs;                 // device: [state pointers (nr)][f_mid row pointers (nr)]
  DevBuf counter;              // device int64: step offset of graph replays
  PassLaunch row, col;
  bool tuned = false;
  hipStream_t stream = nullptr;   // graph branch (default priority)
  hipEvent_t done = nullptr;
};

bool same_problem(const sofft_problem& a, const sofft_problem& b) {
  return a.ndim == b.ndim && a.dtype == b.dtype && a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2] &&
         a.L[0] == b.L[0] && a.L[1] == b.L[1] && a.L[2] == b.L[2] && a.R0[0] == b.R0[0] && a.R0[1] == b.R0[1] &&
         a.R0[2] == b.R0[2] && a.theta == b.theta && a.contour == b.contour && a.charge == b.charge && a.a2 == b.a2;
}

}  // namespace
}  // namespace sofft

using namespace sofft;

struct sofft_batch {
  int32_t nrun = 0;
  int32_t dtype = SOFFT_C128;
  std::vector<BatchClass> cls;
  int graph_steps = 32;             // steady steps per captured graph (0: plain launches)
  hipGraphExec_t exec = nullptr;    // captured chunk of graph_steps steps
  hipGraph_t graph = nullptr;
  int exec_steps = 0;
  bool exec_field = false;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;        // capture origin (the caller's stream may be the null stream)
  void* ws = nullptr;               // caller-owned workspace (sofft_batch_bind)
  size_t ws_bytes = 0;
  std::vector<double> host_partials;
  std::vector<void*> staging;
};

namespace sofft {
namespace {

void drop_graph(sofft_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->exec_steps = 0;
}

void destroy(sofft_batch* b) {
  drop_graph(b);
  for (BatchClass& c : b->cls) {
    dev_free(c.ptrs);
    dev_free(c.counter);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    if (c.done) (void)hipEventDestroy(c.done);
    sofft_plan_destroy(c.plan);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

sofft_status dev_alloc(DevBuf& d, size_t bytes) {
  if (d.p && d.bytes >= bytes) return SOFFT_OK;
  dev_free(d);
  if (hipMalloc(&d.p, bytes) != hipSuccess) {
    d.p = nullptr;
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return SOFFT_ENOMEM;
  }
  d.bytes = bytes;
  return SOFFT_OK;
}

constexpr int kNormBlocksRun = 64;
size_t r256(size_t b) { return (b + 255) / 256 * 256; }

// Layout of a batch's caller workspace: each class plan's workspace (its
// potential-phase table), the per-run norm partial sums, then the scratch
// states and pointer table the launch-shape timing runs on (the size of the
// largest class's runs).
struct BatchWs {
  std::vector<size_t> cls_off, cls_bytes;
  size_t partials = 0, tune = 0, tune_ptrs = 0, total = 0;
};
BatchWs batch_ws_layout(const sofft_batch* b) {
  BatchWs L;
  size_t off = 0, tune = 0, nrmax = 0;
  const size_t elem = b->dtype == SOFFT_C128 ? 16 : 8;
  for (const BatchClass& c : b->cls) {
    const size_t bytes = plan_ws_layout(plan_of(c.plan), 0).total;
    L.cls_off.push_back(off);
    L.cls_bytes.push_back(bytes);
    off += r256(bytes);
    tune = std::max(tune, c.runs.size() * size_t(c.points) * elem);
    nrmax = std::max(nrmax, c.runs.size());
  }
  L.partials = off;
  off += r256(size_t(b->nrun) * kNormBlocksRun * sizeof(double));
  L.tune = off;
  off += r256(tune);
  L.tune_ptrs = off;
  off += r256(nrmax * sizeof(void*));
  L.total = off;
  return L;
}

sofft_status batch_ws_check(const sofft_batch* b, BatchWs* out) {
  BatchWs L = batch_ws_layout(b);
  if (!b->ws || b->ws_bytes < L.total) {
    set_error("the batch needs a bound workspace of " + std::to_string(L.total) +
              " bytes (sofft_batch_workspace_size, sofft_batch_bind); bound: " + std::to_string(b->ws ? b->ws_bytes : 0));
    return SOFFT_EWORKSPACE;
  }
  *out = std::move(L);
  return SOFFT_OK;
}

PassRequest request(const BatchClass& c, bool row, bool half, int do_pot, double dt, bool field) {
  PassRequest rq;
  rq.row = row;
  rq.half_kinetic = half;
  rq.do_pot = do_pot;
  rq.dt = dt;
  rq.runs = static_cast<void* const*>(c.ptrs.p);
  rq.f_runs = field ? reinterpret_cast<const double* const*>(static_cast<void**>(c.ptrs.p) + c.runs.size()) : nullptr;
  rq.nruns = int(c.runs.size());
  rq.cfg = row ? c.row : c.col;
  return rq;
}

// Time one pass of a class with each candidate launch shape on scratch states
// and keep the fastest.  Candidates: 256, 512 and 1024 threads per block, each
// with one block per tile and with a persistent grid of the resident blocks.
sofft_status tune_class(BatchClass& c, double dt, void* scratch, void* scratch_ptrs, hipStream_t s) {
  Plan& p = plan_of(c.plan);
  const size_t elem = p.prob.dtype == SOFFT_C128 ? 16 : 8;
  const int nr = int(c.runs.size());
  sofft_status st;
  std::vector<void*> hp(nr);
  for (int r = 0; r < nr; ++r) hp[r] = static_cast<char*>(scratch) + size_t(r) * size_t(c.points) * elem;
  int cus = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto fail = [&](sofft_status code) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return code;
  };
  if (hipMemcpy(scratch_ptrs, hp.data(), nr * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(scratch, 0, size_t(nr) * size_t(c.points) * elem, s) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("batch tuning: HIP set-up failed");
    return fail(SOFFT_EHIP);
  }
  for (int pass = 0; pass < 2; ++pass) {
    const bool row = pass == 0;
    PassRequest rq = request(c, row, false, 1, dt, false);
    rq.runs = static_cast<void* const*>(scratch_ptrs);
    float best = 1e30f;
    PassLaunch pick{};
    for (int threads : {256, 512, 1024}) {
      int nb = 0, bt = 0;
      if (pass_residency(p, row, threads, &nb, &bt) != SOFFT_OK || nb <= 0) continue;
      for (int persistent = 0; persistent < 2; ++persistent) {
        rq.cfg.threads = threads;
        rq.cfg.grid = persistent ? nb * cus : 0;
        if ((st = launch_pass(p, rq, s)) != SOFFT_OK) return fail(st);   // warm-up
        const int reps = 3;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(SOFFT_EHIP);
        for (int k = 0; k < reps; ++k)
          if ((st = launch_pass(p, rq, s)) != SOFFT_OK) return fail(st);
        float ms = 0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          set_error("batch tuning: event timing failed");
          return fail(SOFFT_EHIP);
        }
        if (ms < best) {
          best = ms;
          pick = rq.cfg;
        }
      }
    }
    if (best >= 1e30f) {
      set_error("batch tuning: no launch shape fits");
      return fail(SOFFT_EUNSUPPORTED);
    }
    (row ? c.row : c.col) = pick;
  }
  c.tuned = true;
  (void)fail(SOFFT_OK);
  return SOFFT_OK;
}

// One step (row pass, column pass) of every class, on the stream of each class
// (capture) or on s.
sofft_status step_all(sofft_batch* b, double dt, bool field, int64_t step, bool half_row, bool half_col,
                      bool from_counter, hipStream_t s, bool per_class_stream) {
  for (BatchClass& c : b->cls) {
    hipStream_t cs = per_class_stream ? c.stream : s;
    PassRequest r = request(c, true, half_row, 1, dt, field);
    PassRequest k = request(c, false, half_col, 1, dt, field);
    r.step = k.step = step;
    if (from_counter) r.step_base = k.step_base = static_cast<const int64_t*>(c.counter.p);
    sofft_status st = launch_pass(plan_of(c.plan), r, cs);
    if (st == SOFFT_OK) st = launch_pass(plan_of(c.plan), k, cs);
    if (st != SOFFT_OK) return st;
  }
  return SOFFT_OK;
}

// Capture graph_steps steady steps: per class a chain of row/column passes
// reading the step offset from the class counter, then counter += steps.
// Captured from the batch's own stream (the null stream cannot be captured);
// the graph is then launched on the caller's stream.
sofft_status capture(sofft_batch* b, double dt, bool field) {
  drop_graph(b);
  hipStream_t s = b->cap;
  const int G = b->graph_steps;
  // Kernel attributes (LDS limits) are set outside the capture.
  for (BatchClass& c : b->cls) {
    int nb = 0, bt = 0;
    sofft_status st = pass_residency(plan_of(c.plan), true, c.row.threads, &nb, &bt);
    if (st == SOFFT_OK) st = pass_residency(plan_of(c.plan), false, c.col.threads, &nb, &bt);
    if (st != SOFFT_OK) return st;
  }
  SOFFT_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  sofft_status st = SOFFT_OK;
  if (hipEventRecord(b->fork, s) != hipSuccess) st = SOFFT_EHIP;
  for (BatchClass& c : b->cls) {
    if (st != SOFFT_OK) break;
    if (hipStreamWaitEvent(c.stream, b->fork, 0) != hipSuccess) {
      st = SOFFT_EHIP;
      break;
    }
    for (int k = 0; k < G && st == SOFFT_OK; ++k) {
      PassRequest r = request(c, true, false, 1, dt, field);
      PassRequest q = request(c, false, false, 1, dt, field);
      r.step = q.step = k;
      r.step_base = q.step_base = static_cast<const int64_t*>(c.counter.p);
      st = launch_pass(plan_of(c.plan), r, c.stream);
      if (st == SOFFT_OK) st = launch_pass(plan_of(c.plan), q, c.stream);
    }
    if (st == SOFFT_OK) st = launch_step_add(static_cast<int64_t*>(c.counter.p), G, false, c.stream);
    if (st == SOFFT_OK && (hipEventRecord(c.done, c.stream) != hipSuccess ||
                           hipStreamWaitEvent(s, c.done, 0) != hipSuccess))
      st = SOFFT_EHIP;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != SOFFT_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (st == SOFFT_EHIP || st == SOFFT_OK) set_error("batch graph capture failed");
    return st == SOFFT_OK ? SOFFT_EHIP : st;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->exec = nullptr;
    drop_graph(b);
    set_error("hipGraphInstantiate failed");
    return SOFFT_EHIP;
  }
  b->exec_steps = G;
  b->exec_field = field;
  return SOFFT_OK;
}

}  // namespace
}  // namespace sofft

extern "C" {

sofft_status sofft_batch_create(const sofft_problem* probs, int32_t nrun, sofft_batch** out) {
  if (!out) {
    set_error("out is null");
    return SOFFT_EINVAL;
  }
  *out = nullptr;
  if (!probs || nrun <= 0) {
    set_error("bad argument to sofft_batch_create");
    return SOFFT_EINVAL;
  }
  for (int r = 0; r < nrun; ++r) {
    if (probs[r].ndim != 2) {
      set_error("batched runs must be 2D");
      return SOFFT_EINVAL;
    }
    if (probs[r].dtype != probs[0].dtype) {
      set_error("batched runs must share one dtype");
      return SOFFT_EINVAL;
    }
  }
  sofft_batch* b = new sofft_batch();
  b->nrun = nrun;
  b->dtype = probs[0].dtype;
  for (int r = 0; r < nrun; ++r) {
    BatchClass* c = nullptr;
    for (BatchClass& k : b->cls)
      if (same_problem(plan_of(k.plan).prob, probs[r])) c = &k;
    if (!c) {
      b->cls.emplace_back();
      c = &b->cls.back();
      sofft_status st = sofft_plan_create(&probs[r], &c->plan);
      if (st != SOFFT_OK) {
        b->cls.pop_back();
        destroy(b);
        return st;
      }
      c->points = probs[r].n[0] * probs[r].n[1];
    }
    c->runs.push_back(r);
  }
  for (BatchClass& c : b->cls) {
    sofft_status st = dev_alloc(c.ptrs, 2 * c.runs.size() * sizeof(void*));
    if (st == SOFFT_OK) st = dev_alloc(c.counter, sizeof(int64_t));
    if (st == SOFFT_OK && (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
                           hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess)) {
      set_error("stream or event creation failed");
      st = SOFFT_EHIP;
    }
    if (st != SOFFT_OK) {
      destroy(b);
      return st;
    }
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    set_error("event or stream creation failed");
    destroy(b);
    return SOFFT_EHIP;
  }
  *out = b;
  return SOFFT_OK;
}

sofft_status sofft_batch_workspace_size(const sofft_batch* b, int64_t* bytes) {
  if (!b || !bytes) {
    set_error("bad argument to sofft_batch_workspace_size");
    return SOFFT_EINVAL;
  }
  *bytes = int64_t(batch_ws_layout(b).total);
  return SOFFT_OK;
}

sofft_status sofft_batch_bind(sofft_batch* b, void* workspace, int64_t bytes) {
  if (!b || bytes < 0 || (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)) {
    set_error("bad argument to sofft_batch_bind (the workspace must be 256-byte aligned)");
    return SOFFT_EINVAL;
  }
  const BatchWs L = batch_ws_layout(b);
  const bool fits = workspace && size_t(bytes) >= L.total;
  b->ws = workspace;
  b->ws_bytes = workspace ? size_t(bytes) : 0;
  for (size_t k = 0; k < b->cls.size(); ++k) {
    Plan& p = plan_of(b->cls[k].plan);
    p.ws = fits ? static_cast<char*>(workspace) + L.cls_off[k] : nullptr;
    p.ws_bytes = fits ? L.cls_bytes[k] : 0;
    p.vphase_ht = __builtin_nan("");
  }
  drop_graph(b);   // the captured passes read tables in the previous workspace
  return SOFFT_OK;
}

sofft_status sofft_batch_destroy(sofft_batch* b) {
  if (b) destroy(b);
  return SOFFT_OK;
}

sofft_status sofft_batch_set_graph_steps(sofft_batch* b, int32_t steps) {
  if (!b || steps < 0 || steps > 4096) {
    set_error("bad argument to sofft_batch_set_graph_steps");
    return SOFFT_EINVAL;
  }
  if (steps != b->graph_steps) drop_graph(b);
  b->graph_steps = steps;
  return SOFFT_OK;
}

sofft_status sofft_batch_set_launch_shape(sofft_batch* b, int32_t run, int32_t pass, int32_t threads,
                                          int32_t grid) {
  if (!b || run < 0 || run >= b->nrun || (pass != 0 && pass != 1) ||
      !(threads == 256 || threads == 512 || threads == 1024) || grid < 0) {
    set_error("bad argument to sofft_batch_set_launch_shape");
    return SOFFT_EINVAL;
  }
  for (BatchClass& c : b->cls)
    if (std::find(c.runs.begin(), c.runs.end(), run) != c.runs.end()) {
      (pass == 0 ? c.row : c.col) = PassLaunch{threads, grid};
      c.tuned = true;
    }
  drop_graph(b);
  return SOFFT_OK;
}

sofft_status sofft_batch_launch_shape(const sofft_batch* b, int32_t run, int32_t pass, int32_t* threads,
                                      int32_t* grid) {
  if (!b || run < 0 || run >= b->nrun || (pass != 0 && pass != 1) || !threads || !grid) {
    set_error("bad argument to sofft_batch_launch_shape");
    return SOFFT_EINVAL;
  }
  for (const BatchClass& c : b->cls)
    if (std::find(c.runs.begin(), c.runs.end(), run) != c.runs.end()) {
      const PassLaunch& l = pass == 0 ? c.row : c.col;
      *threads = l.threads;
      *grid = l.grid;
      return SOFFT_OK;
    }
  set_error("run not found");
  return SOFFT_EINVAL;
}

sofft_status sofft_batch_propagate(sofft_batch* b, void* const* psi, double dt, int64_t nsteps,
                                   const double* f_mid, double* norm2_host, void* stream) {
  if (!b || !psi || nsteps < 0 || !std::isfinite(dt)) {
    set_error("bad argument to sofft_batch_propagate");
    return SOFFT_EINVAL;
  }
  for (int r = 0; r < b->nrun; ++r)
    if (!psi[r]) {
      set_error("null state pointer in sofft_batch_propagate");
      return SOFFT_EINVAL;
    }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  sofft_status st;
  BatchWs WL;
  if ((st = batch_ws_check(b, &WL)) != SOFFT_OK) return st;
  const bool field = f_mid != nullptr;
  bool tables_changed = false;
  for (BatchClass& c : b->cls) {
    Plan& p = plan_of(c.plan);
    for (int d = 0; d < 2; ++d) {
      const bool had = p.ax[d].have_dt && p.ax[d].dt == dt;
      if ((st = ensure_dt(p.ax[d], dt)) != SOFFT_OK) return st;
      tables_changed |= !had;
    }
  }
  for (BatchClass& c : b->cls) {
    bool changed = false;
    if ((st = ensure_vphase(plan_of(c.plan), dt, s, &changed)) != SOFFT_OK) return st;
    tables_changed |= changed;
  }
  if (tables_changed) drop_graph(b);   // table addresses and dt-dependent arguments may have changed
  // State and field-row pointer tables of every class (ordered on s after the
  // work of earlier calls, which reads them).
  for (BatchClass& c : b->cls) {
    const size_t nr = c.runs.size();
    b->staging.assign(2 * nr, nullptr);
    for (size_t i = 0; i < nr; ++i) {
      b->staging[i] = psi[c.runs[i]];
      b->staging[nr + i] = field ? const_cast<double*>(f_mid + size_t(c.runs[i]) * size_t(nsteps)) : nullptr;
    }
    SOFFT_HIP_TRY(hipMemcpyAsync(c.ptrs.p, b->staging.data(), 2 * nr * sizeof(void*), hipMemcpyHostToDevice, s));
    SOFFT_HIP_TRY(hipStreamSynchronize(s));
  }
  if (nsteps > 0) {
    for (BatchClass& c : b->cls)
      if (!c.tuned) {
        if ((st = tune_class(c, dt, static_cast<char*>(b->ws) + WL.tune, static_cast<char*>(b->ws) + WL.tune_ptrs,
                             s)) != SOFFT_OK)
          return st;
        drop_graph(b);
      }
    // opening K_y/2
    for (BatchClass& c : b->cls)
      if ((st = launch_pass(plan_of(c.plan), request(c, false, true, 0, dt, false), s)) != SOFFT_OK) return st;
    // step 0: K_x/2 opens it; the last step's column pass closes with K_y/2
    if ((st = step_all(b, dt, field, 0, true, nsteps == 1, false, s, false)) != SOFFT_OK) return st;
    int64_t n = 1;
    const int64_t last = nsteps - 1;   // steps 1 .. last-1 are steady
    const int G = b->graph_steps;
    if (G > 0 && last - n >= G) {
      if (!b->exec || b->exec_steps != G || b->exec_field != field) {
        if ((st = capture(b, dt, field)) != SOFFT_OK) return st;
      }
      for (BatchClass& c : b->cls)
        if ((st = launch_step_add(static_cast<int64_t*>(c.counter.p), n, true, s)) != SOFFT_OK) return st;
      while (last - n >= G) {
        SOFFT_HIP_TRY(hipGraphLaunch(b->exec, s));
        n += G;
      }
    }
    for (; n < last; ++n)
      if ((st = step_all(b, dt, field, n, false, false, false, s, false)) != SOFFT_OK) return st;
    if (nsteps >= 2 && (st = step_all(b, dt, field, last, false, true, false, s, false)) != SOFFT_OK) return st;
    // closing K_x/2
    for (BatchClass& c : b->cls)
      if ((st = launch_pass(plan_of(c.plan), request(c, true, true, 0, dt, false), s)) != SOFFT_OK) return st;
  }
  if (norm2_host) {
    constexpr int kBlocks = kNormBlocksRun;
    double* part = reinterpret_cast<double*>(static_cast<char*>(b->ws) + WL.partials);
    int off = 0;
    for (BatchClass& c : b->cls) {
      const int nr = int(c.runs.size());
      if ((st = launch_norm2_runs(static_cast<void* const*>(c.ptrs.p), nr, c.points, b->dtype == SOFFT_C128,
                                  part + size_t(off) * kBlocks, s)) != SOFFT_OK)
        return st;
      off += nr;
    }
    b->host_partials.resize(size_t(b->nrun) * kBlocks);
    SOFFT_HIP_TRY(hipMemcpyAsync(b->host_partials.data(), part, b->host_partials.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    SOFFT_HIP_TRY(hipStreamSynchronize(s));
    off = 0;
    for (BatchClass& c : b->cls) {
      for (size_t i = 0; i < c.runs.size(); ++i) {
        double acc = 0.0;
        for (int k = 0; k < kBlocks; ++k) acc += b->host_partials[(size_t(off) + i) * kBlocks + k];
        norm2_host[c.runs[i]] = acc;
      }
      off += int(c.runs.size());
    }
  }
  return SOFFT_OK;
}

}  // extern "C"
