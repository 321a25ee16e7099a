// Resumable PCG solver (Sec. II) for one or several right-hand sides that
// share a pointing and a noise model, with optional FP32-operator inner
// solves under FP64 iterative refinement; mm_solve is its blocking form.
//
// The whole state machine runs on the device: a step enqueues (when the last
// poll saw a finished inner solve) one outer refinement step -- x += dx,
// r = b - A64 x, the outer stopping test, a gated re-initialisation of the
// inner PCG -- then k inner iterations whose kernels return at once for a
// right-hand side that is done, then an asynchronous copy of the per-RHS
// state to pinned host memory.  Polling only queries an event, so a serving
// loop can keep many solvers in flight on their own streams.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mm_internal.h"

using namespace mm;

namespace {

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

struct Layout {
  PcgArgs A;
  OuterArgs O;
  double* b64;
  double* b;
};

int32_t inner_hist_len(const mm_solve_opts& o) { return std::max<int32_t>(1, (o.fixed_iter > 0 ? o.fixed_iter : o.max_iter) + 1); }
// Operator variants chosen by the tuner, shared by every noise handle of the
// process: problems on one device whose sample counts round down to the same
// power of two, with the same storage, arithmetic, right-hand sides, values
// per pixel, band and noise kind, take the first such problem's choice.  A
// stream of similar problems (a server's requests, each with handles of its
// own) then times the variants once per size class instead of once per
// problem; the variants are within a few percent of each other inside one.
struct TuneClass {
  int device;
  int32_t log2n, dtype, arith, nrhs, ncomp, lambda, kind;
  bool operator==(const TuneClass& o) const {
    return device == o.device && log2n == o.log2n && dtype == o.dtype && arith == o.arith && nrhs == o.nrhs &&
           ncomp == o.ncomp && lambda == o.lambda && kind == o.kind;
  }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneClass, int32_t>> g_tune_cache;

TuneClass tune_class(const mm_pointing_s* pt, const mm_noise_s* nz, int arith, int nrhs) {
  int32_t log2n = -1;
  for (int64_t n = pt->n_samples; n > 0; n >>= 1) ++log2n;
  return TuneClass{nz->device, log2n, pt->dtype, arith, nrhs, pt->ncomp, nz->lambda, nz->kind};
}

int32_t outer_hist_len(const mm_solve_opts& o) { return std::max<int32_t>(1, o.max_outer + 1); }

size_t carve(Carver& cv, int32_t n_kept, int32_t ncomp, int32_t nrhs, const mm_solve_opts& o, Layout* L) {
  const size_t n3 = (size_t)ncomp * n_kept, nv = n3 * nrhs;
  PcgArgs& A = L->A;
  A.x = cv.take<double>(nv);
  A.r = cv.take<double>(nv);
  A.z = cv.take<double>(nv);
  A.p = cv.take<double>(nv);
  A.q = cv.take<double>(nv);
  L->b = cv.take<double>(nv);
  A.partials = cv.take<double>(2 * (size_t)kPcgBlocks * nrhs);
  A.st = cv.take<PcgState>(nrhs);
  A.hist_len = inner_hist_len(o);
  A.hist = cv.take<double>((size_t)A.hist_len * nrhs);
  A.vstride = (int64_t)n3;
  A.n_kept = n_kept;
  A.ncomp = ncomp;
  A.max_iter = o.max_iter;
  A.b = L->b;
  OuterArgs& O = L->O;
  O.xt = cv.take<double>(nv);
  O.rt = cv.take<double>(nv);
  L->b64 = cv.take<double>(nv);
  O.b64 = L->b64;
  O.partials = cv.take<double>(2 * (size_t)kPcgBlocks * nrhs);
  O.os = cv.take<OuterState>(nrhs);
  O.hist_len = outer_hist_len(o);
  O.hist = cv.take<double>((size_t)O.hist_len * nrhs);
  O.vstride = (int64_t)n3;
  O.max_outer = o.max_outer;
  return cv.used;
}

int check_opts(const mm_solve_opts& o) {
  if (!(o.tol >= 0.0) || o.max_iter < 0 || o.check_every < 1 || o.max_outer < 1 || !(o.inner_tol > 0.0))
    return fail(MM_EINVAL, "bad solve options");
  if (o.mixed && o.fixed_iter > 0) return fail(MM_EINVAL, "fixed_iter is not available with mixed precision");
  if (o.op_variant < 0 || o.op_variant >= kOpVariants) return fail(MM_EINVAL, "op_variant out of range");
  if (o.graph != 0 && o.graph != 1) return fail(MM_EINVAL, "graph must be 0 or 1");
  if (o.bj_start != 0 && o.bj_start != 1) return fail(MM_EINVAL, "bj_start must be 0 or 1");
  return MM_OK;
}

}  // namespace

struct mm_solver_s {
  const mm_pointing_s* pt = nullptr;
  const mm_noise_s* nz = nullptr;
  mm_solve_opts o{};
  hipStream_t s = nullptr;
  int32_t nrhs = 1;
  int64_t n3 = 0;
  Layout L{};
  bool mixed = false;
  int32_t variant = 0;         // band-Toeplitz operator variant
  bool outer_pending = false;  // the last poll saw a finished inner solve
  bool step_pending = false;   // a state copy is in flight
  void* ws = nullptr;          // the caller's workspace and the bytes the solver uses of it
  size_t ws_used = 0;
  hipEvent_t ev = nullptr;
  PcgState* h_st = nullptr;    // pinned mirrors
  OuterState* h_os = nullptr;
  std::vector<PcgState> st;    // last known
  std::vector<OuterState> os;
  // optional timing of iterations and of the A kernel
  bool timing = false;
  std::vector<hipEvent_t> tev;
  int32_t tev_used = 0;
  int64_t work_seen = 0;
  std::vector<double> iter_ms;
  double op_ms = 0.0;
  int32_t op_launches = 0;
  // recorded iteration chunk (opts.graph): graph_k iterations, replayed on s
  hipStream_t cs = nullptr;  // private stream the chunk is recorded on
  hipGraphExec_t gexec = nullptr;
  int32_t graph_k = -1;

  ~mm_solver_s() {
    drop_graph();
    if (cs) (void)hipStreamDestroy(cs);
    if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
    if (h_st) (void)hipHostFree(h_st);
    if (h_os) (void)hipHostFree(h_os);
  }

  int64_t work_total() const {
    // inner iterations that did work, summed over right-hand sides
    int64_t w = 0;
    for (int r = 0; r < nrhs; ++r) w += mixed ? (int64_t)os[r].inner_total + st[r].iter : st[r].iter;
    return w;
  }

  bool all_done() const {
    for (int r = 0; r < nrhs; ++r)
      if (!(mixed ? os[r].done : st[r].done)) return false;
    return true;
  }

  int step(int32_t k) {
    if (mixed && outer_pending) {
      // outer step for every right-hand side whose inner solve has ended
      if (int rc = launch_outer_add(L.O, L.A, nrhs, s)) return rc;
      RhsBatch rb;
      rb.nrhs = nrhs;
      rb.vstride = n3;
      rb.done = &L.O.os[0].skip;
      rb.done_stride = kOuterStride;
      if (int rc = apply_A_impl(pt, nz, L.O.xt, L.A.q, MM_F64, rb, s, variant)) return rc;
      if (int rc = launch_outer_end(L.O, L.A, nrhs, o.tol, o.max_outer, s)) return rc;
      if (int rc = launch_pcg_init(pt, L.A, nrhs, o.inner_tol, o.max_iter, 0, L.O.os, s)) return rc;
      outer_pending = false;
    }
    RhsBatch rb;
    rb.nrhs = nrhs;
    rb.vstride = n3;
    rb.done = &L.A.st[0].done;
    rb.done_stride = kPcgDoneStride;
    const int arith = mixed ? MM_F32 : MM_F64;
    if (o.graph && !timing && k > 0) {
      if (graph_k != k)
        if (int rc = record_chunk(k, rb, arith)) return rc;
      MM_HIP(hipGraphLaunch(gexec, s));
      tev_used = 0;
      return record_state();
    }
    if (timing && (int32_t)tev.size() < 2 * k + 1) {
      for (hipEvent_t e : tev) (void)hipEventDestroy(e);
      tev.assign(2 * (size_t)k + 1, nullptr);
      for (auto& e : tev) MM_HIP(hipEventCreate(&e));
    }
    for (int32_t i = 0; i < k; ++i) {
      if (timing) MM_HIP(hipEventRecord(tev[2 * i], s));
      if (int rc = apply_A_impl(pt, nz, L.A.p, L.A.q, arith, rb, s, variant)) return rc;
      if (timing) MM_HIP(hipEventRecord(tev[2 * i + 1], s));
      if (int rc = launch_pcg_iteration_tail(pt, L.A, nrhs, s)) return rc;
    }
    if (timing) MM_HIP(hipEventRecord(tev[2 * k], s));
    tev_used = timing ? k : 0;
    return record_state();
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    graph_k = -1;
  }

  // Record k iterations (the eager loop of step, launched on the private
  // stream cs under capture, so nothing runs) and instantiate the graph.
  // The launches clear memory with fill kernels, never with memset nodes.
  int record_chunk(int32_t k, const RhsBatch& rb, int arith) {
    drop_graph();
    if (!cs) MM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    MM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = MM_OK;
    for (int32_t i = 0; i < k && rc == MM_OK; ++i) {
      rc = apply_A_impl(pt, nz, L.A.p, L.A.q, arith, rb, cs, variant);
      if (rc == MM_OK) rc = launch_pcg_iteration_tail(pt, L.A, nrhs, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);  // always ends the capture
    if (rc != MM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != MM_OK ? rc : hip_fail(e, "iteration graph capture");
    }
    const hipError_t ei = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      gexec = nullptr;
      return hip_fail(ei, "iteration graph instantiate");
    }
    graph_k = k;
    return MM_OK;
  }

  // Autotuner: time each variant of the fused band-Toeplitz operator on
  // this problem (one warm-up and two timed launches on the current search
  // direction, into q, which is cleared afterwards) and keep the fastest.
  // The choice is remembered by the noise handle for this problem shape,
  // and across the process's handles for its size class (tune_class).
  int tune() {
    const int arith = mixed ? MM_F32 : MM_F64;
    for (const auto& t : nz->tuned)
      if (t.n_samples == pt->n_samples && t.n_kept == pt->n_kept && t.dtype == pt->dtype && t.arith == arith &&
          t.nrhs == nrhs && t.ncomp == pt->ncomp) {
        variant = t.variant;
        return MM_OK;
      }
    const TuneClass cls = tune_class(pt, nz, arith, nrhs);
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      for (const auto& c : g_tune_cache)
        if (c.first == cls) {
          variant = c.second;
          nz->tuned.push_back(
              mm_noise_s::Tuned{pt->n_samples, pt->n_kept, pt->dtype, arith, nrhs, variant, pt->ncomp});
          return MM_OK;
        }
    }
    RhsBatch rb;
    rb.nrhs = nrhs;
    rb.vstride = n3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MM_HIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      return hip_fail(e, "tuner event");
    }
    int rc = MM_OK;
    float best = 0.f;
    int32_t best_v = 0;
    for (int32_t v = 0; v < kOpVariants && rc == MM_OK; ++v) {
      if ((v & kOpCarry) && (v & kOpNoStaging)) continue;  // the carrying form never stages
      // the two-per-CU form: plain tiles, never staged
      if ((v & kOpHalfLds) && (v & (kOpCarry | kOpNoStaging))) continue;
      // the longer plan: plain tiles, never staged
      if ((v & kOpLongPlan) && (v & (kOpCarry | kOpNoStaging | kOpHalfLds))) continue;
      if ((rc = apply_A_impl(pt, nz, L.A.p, L.A.q, arith, rb, s, v))) break;
      if ((e = hipEventRecord(e0, s)) != hipSuccess) { rc = hip_fail(e, "tuner event"); break; }
      for (int r = 0; r < 2 && rc == MM_OK; ++r) rc = apply_A_impl(pt, nz, L.A.p, L.A.q, arith, rb, s, v);
      if (rc) break;
      if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_fail(e, "tuner event");
        break;
      }
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail(e, "tuner event"); break; }
      if (v == 0 || ms < best) {
        best = ms;
        best_v = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = launch_fill(L.A.q, n3 * nrhs, 0.0, s))) return rc;
    variant = best_v;
    nz->tuned.push_back(mm_noise_s::Tuned{pt->n_samples, pt->n_kept, pt->dtype, arith, nrhs, best_v, pt->ncomp});
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      bool have = false;
      for (const auto& c : g_tune_cache) have = have || c.first == cls;
      if (!have) g_tune_cache.emplace_back(cls, best_v);
    }
    return MM_OK;
  }

  // asynchronous copy of the per-RHS state to the pinned mirrors
  int record_state() {
    MM_HIP(hipMemcpyAsync(h_st, L.A.st, sizeof(PcgState) * nrhs, hipMemcpyDeviceToHost, s));
    if (mixed) MM_HIP(hipMemcpyAsync(h_os, L.O.os, sizeof(OuterState) * nrhs, hipMemcpyDeviceToHost, s));
    MM_HIP(hipEventRecord(ev, s));
    step_pending = true;
    return MM_OK;
  }

  int poll(int32_t* done) {
    if (step_pending) {
      const hipError_t q = hipEventQuery(ev);
      if (q == hipErrorNotReady) {
        *done = 0;
        return MM_OK;
      }
      if (q != hipSuccess) return hip_fail(q, "solver event");
      std::copy(h_st, h_st + nrhs, st.begin());
      if (mixed) std::copy(h_os, h_os + nrhs, os.begin());
      step_pending = false;
      if (timing && tev_used > 0) {
        // the first (work - work_seen) iterations of the last step did work
        const int64_t w = work_total() - work_seen;
        for (int32_t i = 0; i < tev_used && i < w; ++i) {
          float a = 0.f, it = 0.f;
          MM_HIP(hipEventElapsedTime(&a, tev[2 * i], tev[2 * i + 1]));
          MM_HIP(hipEventElapsedTime(&it, tev[2 * i], tev[2 * i + 2]));
          op_ms += a;
          op_launches += 1;
          iter_ms.push_back(it);
        }
        work_seen = work_total();
        tev_used = 0;
      }
      if (mixed) {
        for (int r = 0; r < nrhs; ++r)
          if (st[r].done && !os[r].done) outer_pending = true;
      }
    }
    *done = all_done() ? 1 : 0;
    return MM_OK;
  }

  void fill_info(int r, mm_solve_info* inf) const {
    *inf = mm_solve_info{};
    if (mixed) {
      inf->iters = os[r].inner_total;
      inf->outer_iters = os[r].iters;
      inf->converged = os[r].converged;
      inf->breakdown = os[r].breakdown;
      inf->rel_resid = os[r].rel;
      inf->true_rel_resid = os[r].rel;
    } else {
      inf->iters = st[r].iter;
      inf->outer_iters = 1;
      inf->converged = st[r].converged;
      inf->breakdown = st[r].breakdown;
      inf->rel_resid = st[r].rel;
    }
    inf->op_variant = variant;
    if (timing) {
      inf->op_ms = op_ms;
      inf->op_launches = op_launches;
      inf->iter_ms_p50 = percentile(iter_ms, 0.5);
      inf->iter_ms_p99 = percentile(iter_ms, 0.99);
    }
  }
};

extern "C" {

int mm_solve_opts_default(mm_solve_opts* o) {
  if (!o) return fail(MM_EINVAL, "null opts");
  o->tol = 1e-10;
  o->max_iter = 2000;
  o->fixed_iter = 0;
  o->check_every = 8;
  o->mixed = 0;
  o->max_outer = 10;
  o->inner_tol = 1e-5;
  o->timing = 0;
  o->autotune = 0;
  o->op_variant = 0;
  o->graph = 0;
  o->x0 = nullptr;
  o->bj_start = 1;
  return MM_OK;
}

int mm_solver_workspace_size(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const mm_solve_opts* opts,
                             size_t* bytes) {
  if (int rc = check_pointing(pt)) return rc;
  if (!nz || !bytes || n_rhs < 1) return fail(MM_EINVAL, "bad solver workspace query");
  mm_solve_opts o;
  mm_solve_opts_default(&o);
  if (opts) o = *opts;
  Carver cv(nullptr, 0);
  Layout L;
  *bytes = carve(cv, pt->n_kept, pt->ncomp, n_rhs, o, &L);
  return MM_OK;
}

int mm_solver_workspace_bound(int32_t n_kept_max, int32_t ncomp, int32_t n_rhs, const mm_solve_opts* opts,
                              size_t* bytes) {
  if (!bytes || n_kept_max < 0 || n_rhs < 1 || ncomp < 1 || ncomp > 3)
    return fail(MM_EINVAL, "bad solver workspace bound query");
  mm_solve_opts o;
  mm_solve_opts_default(&o);
  if (opts) o = *opts;
  Carver cv(nullptr, 0);
  Layout L;
  *bytes = carve(cv, n_kept_max, ncomp, n_rhs, o, &L);
  return MM_OK;
}

int mm_solve_workspace_size(mm_pointing_t pt, mm_noise_t nz, const mm_solve_opts* opts, size_t* bytes) {
  return mm_solver_workspace_size(pt, nz, 1, opts, bytes);
}

int mm_solver_create(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const void* tod, const mm_solve_opts* opts,
                     void* workspace, size_t ws_bytes, void* stream, mm_solver_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (n_rhs < 1) return fail(MM_EINVAL, "n_rhs must be >= 1");
  if (pt->n_samples && !tod) return fail(MM_EINVAL, "null timeline");
  if (!workspace) return fail(MM_EINVAL, "null workspace");
  if (pt->n_kept == 0) return fail(MM_EINVAL, "no kept pixels to solve for");
  mm_solve_opts o;
  mm_solve_opts_default(&o);
  if (opts) o = *opts;
  if (int rc = check_opts(o)) return rc;
  auto* sv = new (std::nothrow) mm_solver_s();
  if (!sv) return fail(MM_EINVAL, "out of host memory");
  sv->pt = pt;
  sv->nz = nz;
  sv->o = o;
  sv->s = reinterpret_cast<hipStream_t>(stream);
  sv->nrhs = n_rhs;
  sv->n3 = (int64_t)pt->ncomp * pt->n_kept;
  sv->mixed = o.mixed != 0;
  sv->timing = o.timing != 0;
  sv->st.assign(n_rhs, PcgState{});
  sv->os.assign(n_rhs, OuterState{});
  Carver cv(workspace, ws_bytes);
  carve(cv, pt->n_kept, pt->ncomp, n_rhs, o, &sv->L);
  sv->ws = workspace;
  sv->ws_used = cv.used;
  auto bail = [&](int rc) {
    delete sv;
    return rc;
  };
  if (!cv.fits()) return bail(fail(MM_ENOSPC, "solver workspace too small"));
  hipError_t e;
  if ((e = hipHostMalloc((void**)&sv->h_st, sizeof(PcgState) * n_rhs, hipHostMallocDefault)) != hipSuccess)
    return bail(hip_fail(e, "pinned state"));
  if ((e = hipHostMalloc((void**)&sv->h_os, sizeof(OuterState) * n_rhs, hipHostMallocDefault)) != hipSuccess)
    return bail(hip_fail(e, "pinned state"));
  if ((e = hipEventCreateWithFlags(&sv->ev, hipEventDisableTiming)) != hipSuccess)
    return bail(hip_fail(e, "solver event"));
  // zero the per-RHS states: their reduction tickets must start at 0
  if ((e = hipMemsetAsync(sv->L.A.st, 0, sizeof(PcgState) * n_rhs, sv->s)) != hipSuccess)
    return bail(hip_fail(e, "state init"));
  if ((e = hipMemsetAsync(sv->L.O.os, 0, sizeof(OuterState) * n_rhs, sv->s)) != hipSuccess)
    return bail(hip_fail(e, "state init"));
  const size_t esz = pt->dtype == MM_F64 ? 8 : 4;
  double* rhs_dst = sv->mixed ? sv->L.b64 : sv->L.b;
  for (int32_t r = 0; r < n_rhs; ++r) {
    const char* t = static_cast<const char*>(tod) + (size_t)r * esz * (size_t)pt->n_samples;
    if (int rc = rhs_impl(pt, nz, t, rhs_dst + r * sv->n3, MM_F64, sv->s)) return bail(rc);
  }
  // the mixed form refines from the block-Jacobi map M b unless the caller
  // gives a start vector or asks for x0 = 0
  const bool bj = sv->mixed && o.x0 == nullptr && o.bj_start != 0;
  const bool from_x0 = o.x0 != nullptr || bj;
  if (from_x0) {
    // start vector: x (FP64 solve) or xt (outer FP64 refinement) = x0, and
    // q = A64 x0 in FP64 arithmetic; then ||b - A x0||^2, ||b||^2
    double* xs = sv->mixed ? sv->L.O.xt : sv->L.A.x;
    if (bj) {
      for (int32_t r = 0; r < n_rhs; ++r)
        if (int rc = launch_apply_M(pt, rhs_dst + r * sv->n3, xs + r * sv->n3, sv->s)) return bail(rc);
    } else {
      MM_HIP(hipMemcpyAsync(xs, o.x0, sizeof(double) * sv->n3 * n_rhs, hipMemcpyDeviceToDevice, sv->s));
    }
    if (int rc = launch_fill(sv->L.A.q, sv->n3 * n_rhs, 0.0, sv->s)) return bail(rc);
    RhsBatch rb;
    rb.nrhs = n_rhs;
    rb.vstride = sv->n3;
    if (int rc = apply_A_impl(pt, nz, xs, sv->L.A.q, MM_F64, rb, sv->s, o.op_variant)) return bail(rc);
    if (int rc = launch_diff_norm(sv->L.A, n_rhs, rhs_dst, sv->L.A.q, sv->s)) return bail(rc);
  }
  if (sv->mixed) {
    sv->L.A.b = sv->L.O.rt;  // inner solves run on the outer residual
    if (int rc = launch_outer_init(sv->L.O, sv->L.A, n_rhs, sv->s, from_x0)) return bail(rc);
    if (int rc = launch_pcg_init(pt, sv->L.A, n_rhs, o.inner_tol, o.max_iter, 0, sv->L.O.os, sv->s))
      return bail(rc);
  } else {
    if (int rc = launch_pcg_init(pt, sv->L.A, n_rhs, o.tol, o.max_iter, o.fixed_iter, nullptr, sv->s, from_x0))
      return bail(rc);
  }
  sv->variant = o.op_variant;
  if (o.autotune && (nz->kind == 1 || nz->kind == 2))
    if (int rc = sv->tune()) return bail(rc);
  *out = sv;
  return MM_OK;
}

int mm_solver_step(mm_solver_t sv, int32_t k) {
  if (!sv || k < 0) return fail(MM_EINVAL, "bad solver step");
  return sv->step(k);
}

int mm_solver_poll(mm_solver_t sv, int32_t* done, int32_t* in_flight, mm_solve_info* info) {
  if (!sv || !done) return fail(MM_EINVAL, "bad solver poll");
  if (int rc = sv->poll(done)) return rc;
  if (in_flight) *in_flight = sv->step_pending ? 1 : 0;
  if (info)
    for (int r = 0; r < sv->nrhs; ++r) sv->fill_info(r, &info[r]);
  return MM_OK;
}

int mm_solver_finish(mm_solver_t sv, double* maps_out, double* x_out, mm_solve_info* info, double* history_host,
                     int32_t history_len) {
  if (!sv) return fail(MM_EINVAL, "null solver");
  const mm_pointing_s* pt = sv->pt;
  hipStream_t s = sv->s;
  MM_HIP(hipStreamSynchronize(s));
  int32_t done = 0;
  if (int rc = sv->poll(&done)) return rc;
  std::vector<double> true_rel(sv->nrhs, 0.0);
  const double* xf = sv->mixed ? sv->L.O.xt : sv->L.A.x;
  if (!sv->mixed) {
    // ||b - A x|| / ||b|| in FP64 arithmetic
    RhsBatch rb;
    rb.nrhs = sv->nrhs;
    rb.vstride = sv->n3;
    if (int rc = launch_fill(sv->L.A.q, sv->n3 * sv->nrhs, 0.0, s)) return rc;
    if (int rc = apply_A_impl(pt, sv->nz, sv->L.A.x, sv->L.A.q, MM_F64, rb, s, sv->variant)) return rc;
    if (int rc = launch_diff_norm(sv->L.A, sv->nrhs, sv->L.b, sv->L.A.q, s)) return rc;
    MM_HIP(hipMemcpyAsync(sv->h_st, sv->L.A.st, sizeof(PcgState) * sv->nrhs, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < sv->nrhs; ++r)
      true_rel[r] = sv->h_st[r].scratch1 > 0 ? std::sqrt(sv->h_st[r].scratch0 / sv->h_st[r].scratch1) : 0.0;
  }
  for (int r = 0; r < sv->nrhs; ++r) {
    if (maps_out)
      if (int rc = launch_expand(pt, xf + r * sv->n3, maps_out + r * (int64_t)pt->ncomp * pt->n_pix, s))
        return rc;
  }
  if (x_out) MM_HIP(hipMemcpyAsync(x_out, xf, sizeof(double) * sv->n3 * sv->nrhs, hipMemcpyDeviceToDevice, s));
  MM_HIP(hipStreamSynchronize(s));
  if (history_host && history_len > 0) {
    // right-hand side 0: inner residual history, or the outer one (mixed);
    // a plain copy, since the destination is pageable caller memory
    const double* h = sv->mixed ? sv->L.O.hist : sv->L.A.hist;
    const int32_t avail = sv->mixed ? std::min(sv->L.O.hist_len, sv->os[0].iters + 1)
                                    : std::min(sv->L.A.hist_len, sv->st[0].iter + 1);
    const int32_t n = std::min(history_len, avail);
    if (n > 0) MM_HIP(hipMemcpy(history_host, h, sizeof(double) * n, hipMemcpyDeviceToHost));
  }
  if (history_host && history_len > 0 && sv->mixed) history_host[0] = sv->os[0].bnorm > 0 ? 1.0 : 0.0;
  bool breakdown = false, converged = true;
  for (int r = 0; r < sv->nrhs; ++r) {
    mm_solve_info inf;
    sv->fill_info(r, &inf);
    if (!sv->mixed) inf.true_rel_resid = true_rel[r];
    breakdown = breakdown || inf.breakdown;
    converged = converged && inf.converged;
    if (info) info[r] = inf;
  }
  if (breakdown) return fail(MM_EBREAKDOWN, "PCG breakdown (p^T A p <= 0 or non-finite value)");
  if (!converged && !(sv->o.fixed_iter > 0 && !sv->mixed)) return MM_NOTCONVERGED;
  return MM_OK;
}

}  // extern "C"

namespace {

// Snapshot layout: this header, then the solver's workspace bytes.  The
// workspace holds no pointers (only vectors and scalar state), so a
// snapshot restores into any solver created for the same problem.
struct SnapHeader {
  uint64_t magic;
  int32_t version, nrhs, mixed, variant, outer_pending, ncomp, dtype, pad_;
  int64_t n3, n_kept, n_samples, ws_used;
};
constexpr uint64_t kSnapMagic = 0x4d4d534e41503031ull;  // "MMSNAP01"

SnapHeader snap_header(const mm_solver_s* sv) {
  SnapHeader h{};
  h.magic = kSnapMagic;
  h.version = 1;
  h.nrhs = sv->nrhs;
  h.mixed = sv->mixed ? 1 : 0;
  h.variant = sv->variant;
  h.outer_pending = sv->outer_pending ? 1 : 0;
  h.ncomp = sv->pt->ncomp;
  h.dtype = sv->pt->dtype;
  h.n3 = sv->n3;
  h.n_kept = sv->pt->n_kept;
  h.n_samples = sv->pt->n_samples;
  h.ws_used = (int64_t)sv->ws_used;
  return h;
}

}  // namespace

extern "C" {

int mm_solver_snapshot_size(mm_solver_t sv, size_t* bytes) {
  if (!sv || !bytes) return fail(MM_EINVAL, "bad snapshot size query");
  *bytes = sizeof(SnapHeader) + sv->ws_used;
  return MM_OK;
}

int mm_solver_snapshot(mm_solver_t sv, void* dst, size_t bytes) {
  if (!sv || !dst) return fail(MM_EINVAL, "bad snapshot arguments");
  if (bytes < sizeof(SnapHeader) + sv->ws_used) return fail(MM_ENOSPC, "snapshot buffer too small");
  MM_HIP(hipStreamSynchronize(sv->s));  // no step in flight
  int32_t done = 0;
  if (int rc = sv->poll(&done)) return rc;  // land the last state copy (outer_pending)
  const SnapHeader h = snap_header(sv);
  char* d = static_cast<char*>(dst);
  MM_HIP(hipMemcpy(d, &h, sizeof(h), hipMemcpyDefault));
  MM_HIP(hipMemcpy(d + sizeof(h), sv->ws, sv->ws_used, hipMemcpyDefault));
  return MM_OK;
}

int mm_solver_restore(mm_solver_t sv, const void* src, size_t bytes) {
  if (!sv || !src || bytes < sizeof(SnapHeader)) return fail(MM_EINVAL, "bad restore arguments");
  SnapHeader h{};
  MM_HIP(hipStreamSynchronize(sv->s));
  MM_HIP(hipMemcpy(&h, src, sizeof(h), hipMemcpyDefault));
  const SnapHeader mine = snap_header(sv);
  if (h.magic != kSnapMagic || h.version != 1) return fail(MM_EINVAL, "not a solver snapshot");
  if (h.nrhs != mine.nrhs || h.mixed != mine.mixed || h.ncomp != mine.ncomp || h.dtype != mine.dtype ||
      h.n3 != mine.n3 || h.n_kept != mine.n_kept || h.n_samples != mine.n_samples || h.ws_used != mine.ws_used)
    return fail(MM_EINVAL, "snapshot of a different problem (sizes, right-hand sides, form, dtype or options)");
  if (bytes < sizeof(SnapHeader) + (size_t)h.ws_used) return fail(MM_EINVAL, "truncated snapshot");
  MM_HIP(hipMemcpy(sv->ws, static_cast<const char*>(src) + sizeof(h), sv->ws_used, hipMemcpyDefault));
  sv->variant = h.variant;
  sv->outer_pending = h.outer_pending != 0;
  sv->tev_used = 0;
  // refresh the host mirrors from the restored device state
  if (int rc = sv->record_state()) return rc;
  MM_HIP(hipStreamSynchronize(sv->s));
  const bool pending = sv->outer_pending;
  int32_t done = 0;
  if (int rc = sv->poll(&done)) return rc;
  sv->outer_pending = sv->outer_pending || pending;
  sv->work_seen = sv->work_total();
  return MM_OK;
}

int mm_solver_destroy(mm_solver_t sv) {
  delete sv;
  return MM_OK;
}

int mm_batch_step(mm_solver_t* solvers, int32_t n, int32_t k) {
  if (!solvers || n < 1 || k < 0) return fail(MM_EINVAL, "bad batch step");
  const mm_solver_s* s0 = solvers[0];
  if (!s0) return fail(MM_EINVAL, "null solver in batch");
  int32_t slots = 0;
  for (int32_t i = 0; i < n; ++i) {
    const mm_solver_s* sv = solvers[i];
    if (!sv) return fail(MM_EINVAL, "null solver in batch");
    for (int32_t j = 0; j < i; ++j)
      if (solvers[j] == sv) return fail(MM_EINVAL, "solver listed twice in batch");
    if (sv->s != s0->s) return fail(MM_EINVAL, "batch members must share one stream");
    if (sv->mixed != s0->mixed || sv->pt->dtype != s0->pt->dtype || sv->pt->ncomp != s0->pt->ncomp)
      return fail(MM_EINVAL, "batch members must share the timeline dtype, precision mode and map form");
    if (sv->pt->device != s0->pt->device) return fail(MM_EINVAL, "batch members must share one device");
    slots += sv->nrhs;
  }
  if (slots > kMaxBatch) return fail(MM_EINVAL, "more than 16 right-hand sides in one batch");
  hipStream_t s = s0->s;
  const bool mixed = s0->mixed;
  const int dtype = s0->pt->dtype;
  const int ncomp = s0->pt->ncomp;
  const int arith = mixed ? MM_F32 : MM_F64;
  // stored weights only where every band-Toeplitz (or every template) slot has usable ones
  auto weights_ok = [&](int ar, bool tpl) {
    for (int32_t i = 0; i < n; ++i) {
      const mm_pointing_s* pt = solvers[i]->pt;
      const int kind = solvers[i]->nz->kind;
      if ((tpl ? kind == 3 : (kind == 1 || kind == 2)) &&
          !(pt->weights != nullptr && (ar == MM_F32 || pt->dtype == MM_F64)))
        return false;
    }
    return true;
  };
  const bool w_in = weights_ok(arith, false), w_out = weights_ok(MM_F64, false);
  const bool wt_in = weights_ok(arith, true), wt_out = weights_ok(MM_F64, true);

  PcgBatch pb;
  // inner / outer operator slots: band-Toeplitz, white, template-filtered
  OpBatch t_in, w_in_b, p_in, t_out, w_out_b, p_out;
  bool pending = false;
  auto add_op = [](OpBatch& b, const mm_solver_s* sv, int plan, const double* x, double* q, const int32_t* done) {
    const mm_pointing_s* pt = sv->pt;
    const mm_noise_s* nz = sv->nz;
    if (nz->kind == 3 && pt->n_kept == 0) return;  // no unknowns: nothing to gather or scatter
    OpSlot& o = b.s[b.n];
    o = OpSlot{};
    o.sample_k = pt->sample_k;
    o.psi = pt->psi;
    o.wts = pt->weights;
    o.x = x;
    o.q = q;
    o.done = done;
    int64_t items;
    if (nz->kind == 3) {
      o.tiles = pt->tiles;
      o.n_pt_tiles = pt->n_tiles;
      o.iv = nz->tpl;
      o.det_w = nz->det_w;
      items = pt->n_tiles > 0 ? nz->n_chunks : 0;
    } else if (nz->kind != 0) {
      o.tiles = nz->tiles[plan];
      o.ab = nz->abr[plan];  // the half-buffer tile's region-major weights
      o.tw = nz->tw[plan];
      o.lambda = nz->lambda;
      o.wrap = nz->kind == 2 ? 1 : 0;
      items = nz->n_tiles[plan];
    } else {
      o.tiles = pt->tiles;
      o.det_w = nz->det_w;
      items = pt->n_tiles;
    }
    b.off[b.n + 1] = b.off[b.n] + items;
    b.n += 1;
  };
  for (int32_t i = 0; i < n; ++i) {
    mm_solver_s* sv = solvers[i];
    pending = pending || sv->outer_pending;
    for (int32_t r = 0; r < sv->nrhs; ++r) {
      // right-hand sides already seen finished take no slot (the device
      // flags still guard those that finished since the last poll)
      if (mixed ? sv->os[r].done : sv->st[r].done) continue;
      const int64_t o3 = (int64_t)r * sv->n3;
      PcgSlot& p = pb.s[pb.n++];
      p.A = sv->L.A;
      p.A.x += o3; p.A.r += o3; p.A.z += o3; p.A.p += o3; p.A.q += o3; p.A.b += o3;
      p.A.partials += (int64_t)r * 2 * kPcgBlocks;
      p.A.st += r;
      p.A.hist += (int64_t)r * p.A.hist_len;
      p.O = sv->L.O;
      p.O.xt += o3; p.O.rt += o3; p.O.b64 += o3;
      p.O.partials += (int64_t)r * 2 * kPcgBlocks;
      p.O.os += r;
      p.O.hist += (int64_t)r * p.O.hist_len;
      p.minv = sv->pt->minv;
      p.tol = sv->o.tol;
      p.inner_tol = sv->o.inner_tol;
      p.A.max_iter = sv->o.max_iter;
      p.O.max_outer = sv->o.max_outer;
      const int plan_in = arith == MM_F64 ? 0 : 1;
      const int kind = sv->nz->kind;
      add_op(kind == 3 ? p_in : kind != 0 ? t_in : w_in_b, sv, plan_in, p.A.p, p.A.q, &p.A.st->done);
      add_op(kind == 3 ? p_out : kind != 0 ? t_out : w_out_b, sv, 0, p.O.xt, p.A.q, &p.O.os->skip);
    }
  }
  if (mixed && pending) {
    // one outer step for every slot whose inner solve has ended (the
    // device-side flags decide; the others are marked skip and stay put)
    if (int rc = launch_outer_add_batch(pb, s)) return rc;
    if (int rc = launch_toeplitz_batch(t_out, dtype, MM_F64, w_out, ncomp, s)) return rc;
    if (int rc = launch_white_batch(w_out_b, dtype, MM_F64, ncomp, s)) return rc;
    if (int rc = launch_templates_batch(p_out, dtype, MM_F64, wt_out, ncomp, s)) return rc;
    if (int rc = launch_outer_end_batch(pb, s)) return rc;
    for (int32_t i = 0; i < n; ++i) solvers[i]->outer_pending = false;
  }
  for (int32_t i = 0; i < k; ++i) {
    if (int rc = launch_toeplitz_batch(t_in, dtype, arith, w_in, ncomp, s)) return rc;
    if (int rc = launch_white_batch(w_in_b, dtype, arith, ncomp, s)) return rc;
    if (int rc = launch_templates_batch(p_in, dtype, arith, wt_in, ncomp, s)) return rc;
    if (int rc = launch_pcg_iteration_tail_batch(pb, s)) return rc;
  }
  for (int32_t i = 0; i < n; ++i) {
    solvers[i]->tev_used = 0;  // batched steps are not timed
    if (int rc = solvers[i]->record_state()) return rc;
  }
  return MM_OK;
}

int mm_solve(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* map_out, double* x_out,
             const mm_solve_opts* opts, mm_solve_info* info, double* history_host, int32_t history_len,
             void* workspace, size_t ws_bytes, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  mm_solve_opts o;
  mm_solve_opts_default(&o);
  if (opts) o = *opts;
  if (int rc = check_opts(o)) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (pt->n_kept == 0) {
    if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
    if (map_out) MM_HIP(hipMemsetAsync(map_out, 0, sizeof(double) * pt->ncomp * (size_t)pt->n_pix, s));
    MM_HIP(hipStreamSynchronize(s));
    if (info) {
      *info = mm_solve_info{};
      info->converged = 1;
    }
    return MM_OK;
  }
  mm_solver_t sv = nullptr;
  if (int rc = mm_solver_create(pt, nz, 1, tod, &o, workspace, ws_bytes, stream, &sv)) return rc;
  // upper bound on steps: every inner solve is capped, so is the outer loop
  // (an outer step costs one extra step)
  const int64_t per_inner = (int64_t)(o.fixed_iter > 0 ? o.fixed_iter : o.max_iter) / o.check_every + 3;
  const int64_t max_steps = per_inner * (o.mixed ? o.max_outer : 1) + 4;
  int32_t done = 0;
  int rc = MM_OK;
  for (int64_t i = 0; i < max_steps && !done; ++i) {
    if ((rc = sv->step(o.check_every))) break;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = hip_fail(e, "solve sync");
      break;
    }
    if ((rc = sv->poll(&done))) break;
  }
  if (rc == MM_OK) rc = mm_solver_finish(sv, map_out, x_out, info, history_host, history_len);
  mm_solver_destroy(sv);
  return rc;
}

}  // extern "C"

// The autotuner's class cache, copied out and added to by the caller.
extern "C" {

int mm_tune_cache_get(mm_tune_entry* out, int32_t cap, int32_t* n) {
  if (n == nullptr || cap < 0 || (cap > 0 && out == nullptr)) return fail(MM_EINVAL, "bad tune cache query");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  *n = (int32_t)g_tune_cache.size();
  for (int32_t i = 0; i < cap && i < *n; ++i) {
    const TuneClass& c = g_tune_cache[i].first;
    out[i] = mm_tune_entry{c.device, c.log2n, c.dtype, c.arith, c.nrhs, c.ncomp, c.lambda, c.kind,
                           g_tune_cache[i].second};
  }
  return MM_OK;
}

int mm_tune_cache_put(const mm_tune_entry* in, int32_t n) {
  if (n < 0 || (n > 0 && in == nullptr)) return fail(MM_EINVAL, "bad tune cache entries");
  auto dt = [](int32_t d) { return d == MM_F64 || d == MM_F32; };
  for (int32_t i = 0; i < n; ++i) {
    const mm_tune_entry& e = in[i];
    if (e.device < 0 || e.log2_samples < 0 || e.log2_samples > 62 || !dt(e.dtype) || !dt(e.arith) || e.n_rhs < 1 ||
        e.ncomp < 1 || e.ncomp > 3 || e.lambda < 1 || e.lambda > kMaxLambda || (e.noise_kind != 1 && e.noise_kind != 2) ||
        e.op_variant < 0 || e.op_variant >= kOpVariants)
      return fail(MM_EINVAL, "tune cache entry out of range");
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (int32_t i = 0; i < n; ++i) {
    const mm_tune_entry& e = in[i];
    const TuneClass c{e.device, e.log2_samples, e.dtype, e.arith, e.n_rhs, e.ncomp, e.lambda, e.noise_kind};
    bool have = false;
    for (auto& kv : g_tune_cache)
      if (kv.first == c) {
        kv.second = e.op_variant;
        have = true;
      }
    if (!have) g_tune_cache.emplace_back(c, e.op_variant);
  }
  return MM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free blocking solve (mm_solve_noalloc).  The solver's vectors,
// partial sums, states and histories live in `scratch`, a file-scope device
// array, instead of a caller workspace; the host side keeps its state copies
// on the stack and waits with stream synchronisations, so the call creates
// no device memory, pinned memory, event or graph.  Each GPU the library
// runs on holds its own copy of the array until the process ends; every
// call on that GPU shares it, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};

// The device address of this device's copy of `scratch` (the host-side name
// is only a stand-in): looked up once per device, with that device current.
int scratch_ptr(void** out) {
  int dev = 0;
  MM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return fail(MM_EINVAL, "device index beyond the allocation-free table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return fail(MM_EHIP, "no device address for the allocation-free scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MM_OK;
}

}  // namespace

extern "C" {

int mm_solve_noalloc(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* map_out, double* x_out,
                     const mm_solve_opts* opts, mm_solve_info* info, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  mm_solve_opts o;
  mm_solve_opts_default(&o);
  if (opts) o = *opts;
  if (int rc = check_opts(o)) return rc;
  if (o.autotune || o.timing || o.graph)
    return fail(MM_EINVAL, "mm_solve_noalloc: autotune, timing and graph need events or graphs; pass op_variant");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (pt->n_kept == 0) {
    if (map_out)
      if (int rc = launch_fill(map_out, (int64_t)pt->ncomp * pt->n_pix, 0.0, s)) return rc;
    MM_HIP(hipStreamSynchronize(s));
    if (info) {
      *info = mm_solve_info{};
      info->converged = 1;
    }
    return MM_OK;
  }
  if (pt->n_samples && !tod) return fail(MM_EINVAL, "null timeline");
  Layout L;
  {
    Carver cv(nullptr, 0);
    const size_t need = carve(cv, pt->n_kept, pt->ncomp, 1, o, &L);
    if (need > kNoAllocBytes)
      return fail(MM_ENOSPC, "mm_solve_noalloc: the problem needs " + std::to_string(need) +
                                 " bytes of solver state, more than the " + std::to_string(kNoAllocBytes) +
                                 " bytes of its scratch array (use mm_solve with a workspace)");
  }
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  Carver cv(ws, kNoAllocBytes);
  carve(cv, pt->n_kept, pt->ncomp, 1, o, &L);
  const bool mixed = o.mixed != 0;
  const int64_t n3 = (int64_t)pt->ncomp * pt->n_kept;
  // the states left by an earlier call start from zero (reduction tickets)
  if (int rc = launch_fill(reinterpret_cast<double*>(L.A.st), sizeof(PcgState) / sizeof(double), 0.0, s)) return rc;
  if (int rc = launch_fill(reinterpret_cast<double*>(L.O.os), sizeof(OuterState) / sizeof(double), 0.0, s))
    return rc;
  double* rhs_dst = mixed ? L.b64 : L.b;
  if (int rc = rhs_impl(pt, nz, tod, rhs_dst, MM_F64, s)) return rc;
  const bool bj = mixed && o.x0 == nullptr && o.bj_start != 0;
  const bool from_x0 = o.x0 != nullptr || bj;
  RhsBatch one;
  one.nrhs = 1;
  one.vstride = n3;
  if (from_x0) {
    double* xs = mixed ? L.O.xt : L.A.x;
    if (bj) {
      if (int rc = launch_apply_M(pt, rhs_dst, xs, s)) return rc;
    } else {
      MM_HIP(hipMemcpyAsync(xs, o.x0, sizeof(double) * n3, hipMemcpyDeviceToDevice, s));
    }
    if (int rc = launch_fill(L.A.q, n3, 0.0, s)) return rc;
    if (int rc = apply_A_impl(pt, nz, xs, L.A.q, MM_F64, one, s, o.op_variant)) return rc;
    if (int rc = launch_diff_norm(L.A, 1, rhs_dst, L.A.q, s)) return rc;
  }
  if (mixed) {
    L.A.b = L.O.rt;
    if (int rc = launch_outer_init(L.O, L.A, 1, s, from_x0)) return rc;
    if (int rc = launch_pcg_init(pt, L.A, 1, o.inner_tol, o.max_iter, 0, L.O.os, s)) return rc;
  } else {
    if (int rc = launch_pcg_init(pt, L.A, 1, o.tol, o.max_iter, o.fixed_iter, nullptr, s, from_x0)) return rc;
  }
  // iterate in chunks of check_every, reading the state back after each
  const int64_t per_inner = (int64_t)(o.fixed_iter > 0 ? o.fixed_iter : o.max_iter) / o.check_every + 3;
  const int64_t max_steps = per_inner * (mixed ? o.max_outer : 1) + 4;
  PcgState st{};
  OuterState os{};
  bool outer_pending = false, done = false;
  const int arith = mixed ? MM_F32 : MM_F64;
  for (int64_t i = 0; i < max_steps && !done; ++i) {
    if (mixed && outer_pending) {
      RhsBatch rb = one;
      rb.done = &L.O.os[0].skip;
      rb.done_stride = kOuterStride;
      if (int rc = launch_outer_add(L.O, L.A, 1, s)) return rc;
      if (int rc = apply_A_impl(pt, nz, L.O.xt, L.A.q, MM_F64, rb, s, o.op_variant)) return rc;
      if (int rc = launch_outer_end(L.O, L.A, 1, o.tol, o.max_outer, s)) return rc;
      if (int rc = launch_pcg_init(pt, L.A, 1, o.inner_tol, o.max_iter, 0, L.O.os, s)) return rc;
      outer_pending = false;
    }
    RhsBatch rb = one;
    rb.done = &L.A.st[0].done;
    rb.done_stride = kPcgDoneStride;
    for (int32_t k = 0; k < o.check_every; ++k) {
      if (int rc = apply_A_impl(pt, nz, L.A.p, L.A.q, arith, rb, s, o.op_variant)) return rc;
      if (int rc = launch_pcg_iteration_tail(pt, L.A, 1, s)) return rc;
    }
    MM_HIP(hipStreamSynchronize(s));
    MM_HIP(hipMemcpy(&st, L.A.st, sizeof(PcgState), hipMemcpyDeviceToHost));
    if (mixed) {
      MM_HIP(hipMemcpy(&os, L.O.os, sizeof(OuterState), hipMemcpyDeviceToHost));
      if (st.done && !os.done) outer_pending = true;
      done = os.done != 0;
    } else {
      done = st.done != 0;
    }
  }
  double true_rel = 0.0;
  const double* xf = mixed ? L.O.xt : L.A.x;
  if (!mixed) {
    // ||b - A x|| / ||b|| in FP64 arithmetic
    if (int rc = launch_fill(L.A.q, n3, 0.0, s)) return rc;
    if (int rc = apply_A_impl(pt, nz, L.A.x, L.A.q, MM_F64, one, s, o.op_variant)) return rc;
    if (int rc = launch_diff_norm(L.A, 1, L.b, L.A.q, s)) return rc;
    MM_HIP(hipStreamSynchronize(s));
    PcgState fin{};
    MM_HIP(hipMemcpy(&fin, L.A.st, sizeof(PcgState), hipMemcpyDeviceToHost));
    true_rel = fin.scratch1 > 0 ? std::sqrt(fin.scratch0 / fin.scratch1) : 0.0;
  }
  if (map_out)
    if (int rc = launch_expand(pt, xf, map_out, s)) return rc;
  if (x_out) MM_HIP(hipMemcpyAsync(x_out, xf, sizeof(double) * n3, hipMemcpyDeviceToDevice, s));
  MM_HIP(hipStreamSynchronize(s));
  mm_solve_info inf{};
  if (mixed) {
    inf.iters = os.inner_total;
    inf.outer_iters = os.iters;
    inf.converged = os.converged;
    inf.breakdown = os.breakdown;
    inf.rel_resid = os.rel;
    inf.true_rel_resid = os.rel;
  } else {
    inf.iters = st.iter;
    inf.outer_iters = 1;
    inf.converged = st.converged;
    inf.breakdown = st.breakdown;
    inf.rel_resid = st.rel;
    inf.true_rel_resid = true_rel;
  }
  inf.op_variant = o.op_variant;
  if (info) *info = inf;
  if (inf.breakdown) return fail(MM_EBREAKDOWN, "PCG breakdown (p^T A p <= 0 or non-finite value)");
  return (inf.converged || (o.fixed_iter > 0 && !mixed)) ? MM_OK : MM_NOTCONVERGED;
}

}  // extern "C"
