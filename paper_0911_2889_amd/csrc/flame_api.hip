// C ABI of the flame stepper: plan construction, workspace layout, launches.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fft_engine.hpp"
#include "flame.h"
#include "flame_dev.hpp"
#include "flame_kernels.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FLAME_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
// Workgroups of the persistent ensemble launch at most (its item table in the workspace).
constexpr int kMaxEnsItems = 4096;
// Steps per persistent launch at most, and the default bound of each of its waits.
constexpr int kEnsMaxSteps = 1000;
constexpr long long kEnsDefaultWaitUs = 2000000;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ilog2_exact(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

struct Sizes {
  int logn1, logn2;
  int tcol, tiles;       // column tile width and tile count
  int tq;                // tile width of the Q layout
  int rpairs, rgroups;   // row pairs per workgroup and row workgroups
  size_t wq_elems;       // elements of each of Q, A1, A2 (Wp and Wm share 2 wq_elems)
  int n_spec;            // diag spectral workgroups
  size_t part_elems;     // doubles of the partial-sum buffer
};

int check_desc(const flame_desc* d, Sizes* s) {
  if (!d) return fail(FLAME_ERR_INVALID_ARG, "null flame_desc");
  const int l1 = ilog2_exact(d->n1), l2 = ilog2_exact(d->n2);
  if (l1 < 0 || l2 < 0) return fail(FLAME_ERR_UNSUPPORTED_SIZE, "grid %d x %d: sizes must be powers of two", d->n1, d->n2);
  if (l1 < flame::kMinLog || l1 > flame::kMaxLog || l2 < flame::kMinLog || l2 > flame::kMaxLog)
    return fail(FLAME_ERR_UNSUPPORTED_SIZE, "grid %d x %d: sizes must lie in [16, 16384]", d->n1, d->n2);
  if (!(std::isfinite(d->gamma) && d->gamma >= 0.0)) return fail(FLAME_ERR_INVALID_ARG, "gamma must be finite and >= 0");
  if (!(std::isfinite(d->theta_pi) && d->theta_pi > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "theta_pi must be > 0");
  if (!(std::isfinite(d->t0) && d->t0 > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "t0 must be > 0");
  if (!(std::isfinite(d->dt) && d->dt > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "dt must be > 0");
  for (int a = 0; a < 2; ++a)
    if (!(std::isfinite(d->axis_scale[a]) && d->axis_scale[a] >= 0.0))
      return fail(FLAME_ERR_INVALID_ARG, "axis_scale must be finite and >= 0");
  if ((d->axis_scale[0] == 0.0) != (d->axis_scale[1] == 0.0))
    return fail(FLAME_ERR_INVALID_ARG, "axis_scale must be both zero (use theta_pi) or both positive");
  if (d->r0_law != 0 && d->r0_law != 1) return fail(FLAME_ERR_INVALID_ARG, "r0_law must be 0 (r0 = t) or 1 (table)");
  if (d->integrator != 0 && d->integrator != 1)
    return fail(FLAME_ERR_INVALID_ARG, "integrator must be 0 (IF-Euler) or 1 (IF-Heun)");
  if (s) {
    s->logn1 = l1;
    s->logn2 = l2;
    const int m = d->n2 / 4;
    s->tcol = flame::col_tile(l1);
    s->tiles = (m + s->tcol - 1) / s->tcol;
    s->rpairs = flame::row_pairs(l2);
    s->rgroups = (d->n1 / 2 + s->rpairs - 1) / s->rpairs;
    s->tq = flame::q_tile(l1);
    const int qcols = (m + s->tq - 1) / s->tq * s->tq;
    s->wq_elems = (size_t)std::max(s->tiles * s->tcol, qcols) * d->n1;
    const long long spec = (long long)m * (d->n1 / 2);
    s->n_spec = (int)std::min<long long>(1024, (spec + flame::kDiagThreads - 1) / flame::kDiagThreads);
    s->part_elems = (size_t)s->rgroups + 2 * (size_t)s->n_spec;
  }
  return FLAME_OK;
}

struct Layout {
  std::vector<Sizes> sizes;
  std::vector<size_t> off_w, off_q, off_a1, off_a2, off_part;
  size_t off_tw[flame::kMaxLog + 1];   // twiddles, 16 points per thread
  size_t off_tw8[flame::kMaxLog + 1];  // twiddles, 8 points per thread
  size_t off_tw6[flame::kMaxLog + 1];  // twiddles of the length-3N1/4 transform (product grid)
  size_t off_tw6_8[flame::kMaxLog + 1];
  size_t off_tw12[flame::kMaxLog + 1];  // length 3*2^l/4 in the 12-point plan (product grids)
  size_t off_dev;
  size_t off_dev_full;  // device flame table whose W is the adjoint scratch (physical-grid W for diagnostics)
  size_t off_counter;  // step index read by graph replays
  size_t off_diag;     // 4 doubles per flame: flame_diagnostics_host's device copy
  size_t off_ens_items, off_ens_arrive, off_ens_err;  // persistent ensemble launch
  size_t total;
};

int plan_layout(const flame_desc* descs, int nfl, Layout* L) {
  if (!descs || nfl <= 0) return fail(FLAME_ERR_INVALID_ARG, "need at least one flame descriptor");
  L->sizes.resize(nfl);
  size_t off = 0;
  bool need_tw[flame::kMaxLog + 1] = {}, need_tw6[flame::kMaxLog + 1] = {}, need_tw12[flame::kMaxLog + 1] = {};
  for (int f = 0; f < nfl; ++f) {
    int rc = check_desc(&descs[f], &L->sizes[f]);
    if (rc) return rc;
    need_tw[L->sizes[f].logn1] = need_tw[L->sizes[f].logn2] = true;
    need_tw6[L->sizes[f].logn1] = L->sizes[f].logn1 >= flame::kMinLogProduct;
    if (L->sizes[f].logn1 >= flame::kMinLogProduct) need_tw12[L->sizes[f].logn1] = true;
    if (L->sizes[f].logn2 >= flame::kMinLogRow12) need_tw12[L->sizes[f].logn2] = true;
  }
  for (int f = 0; f < nfl; ++f) {
    const Sizes& s = L->sizes[f];
    L->off_w.push_back(off);  // Wp and Wm interleaved
    off = align_up(off + 2 * s.wq_elems * sizeof(float2));
    L->off_q.push_back(off);
    off = align_up(off + s.wq_elems * sizeof(float2));
    L->off_a1.push_back(off);
    off = align_up(off + s.wq_elems * sizeof(float2));
    L->off_a2.push_back(off);
    off = align_up(off + s.wq_elems * sizeof(float2));
    L->off_part.push_back(off);
    off = align_up(off + s.part_elems * sizeof(double));
  }
  for (int l = 0; l <= flame::kMaxLog; ++l) {
    L->off_tw[l] = off;
    if (need_tw[l]) {
      const ff::PassPlan pp = ff::make_pass_plan(l, 16);
      off = align_up(off + (size_t)(pp.tw_size > 0 ? pp.tw_size : 1) * sizeof(float2));
    }
    L->off_tw8[l] = off;
    if (need_tw[l]) {
      const ff::PassPlan pp = ff::make_pass_plan(l, 8);
      off = align_up(off + (size_t)(pp.tw_size > 0 ? pp.tw_size : 1) * sizeof(float2));
    }
    L->off_tw6[l] = off;
    if (need_tw6[l]) off = align_up(off + (size_t)ff::twiddles6_size(l - 3, 16) * sizeof(float2));
    L->off_tw6_8[l] = off;
    if (need_tw6[l]) off = align_up(off + (size_t)ff::twiddles6_size(l - 3, 8) * sizeof(float2));
    L->off_tw12[l] = off;
    if (need_tw12[l]) off = align_up(off + (size_t)std::max(1, ff::make_plan12(l - 4).tw_size) * sizeof(float2));
  }
  L->off_dev = off;
  off = align_up(off + (size_t)nfl * sizeof(flame::FlameDev));
  L->off_dev_full = off;
  off = align_up(off + (size_t)nfl * sizeof(flame::FlameDev));
  L->off_counter = off;
  off = align_up(off + sizeof(long long));
  L->off_diag = off;
  off = align_up(off + 4 * sizeof(double) * (size_t)nfl);
  L->off_ens_items = off;
  off = align_up(off + sizeof(flame::EnsembleItem) * (size_t)kMaxEnsItems);
  L->off_ens_arrive = off;
  off = align_up(off + sizeof(unsigned) * flame::kEnsArriveStride * (size_t)nfl);
  L->off_ens_err = off;
  off = align_up(off + sizeof(int));
  L->total = off;
  return FLAME_OK;
}

struct Group {
  int logn1, logn2, first, count, tiles, rpairs;
  int col_pts = ff::kPts, row_pts = ff::kPts;  // points per thread of the step kernels
  bool product = false;                        // step on the 3N1/4-row product grid
  int nt = 0;                                  // non-temporal stores: 0 none, 1 Q and W, 2 W, 3 Q
  bool forced = false;                         // some flame of the group has a forcing bound
  int integrator = 0;                          // 0: IF-Euler (one pass per step); 1: IF-Heun (two passes)
  int passes() const { return integrator == 1 ? 2 : 1; }
  // the column kernel's variant in pass 0 or 1 of a step
  int col_var(int pass) const {
    const int ntv = nt_w() ? flame::VAR_NT : 0;
    if (integrator == 1) return (pass == 0 ? flame::VAR_HEUN_P : flame::VAR_HEUN_C) | ntv;
    return (forced ? flame::VAR_EULER_F : flame::VAR_EULER) | ntv;
  }
  bool nt_q() const { return nt == 1 || nt == 3; }  // the row kernel's stores of Q
  bool nt_w() const { return nt == 1 || nt == 2; }  // the column kernel's stores of Wp and Wm
  int rows() const { return product ? 3 * (1 << logn1) / 4 : (1 << logn1); }
  // phi points of the quadratic term's grid: the 12-point row kernel forms it on 3 N2/4
  int cols() const { return row_pts == 12 ? 3 * (1 << logn2) / 4 : (1 << logn2); }
  int rgroups() const { return (rows() / 2 + rpairs - 1) / rpairs; }
};

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) == hipSuccess && prev_ != dev) {
      if (hipSetDevice(dev) == hipSuccess) switched_ = true;
    }
  }
  ~DeviceGuard() {
    if (switched_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1;
  bool switched_ = false;
};

}  // namespace

struct flame_plan_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int nfl = 0;
  std::vector<flame_desc> descs;
  Layout layout;
  std::vector<flame::FlameDev> hdev;
  std::vector<std::vector<float2>> tw_host;   // host copies of the tables (16 points per thread)
  std::vector<std::vector<float2>> tw_host8;  // 8 points per thread
  std::vector<std::vector<float2>> tw_host6;  // length-3N1/4 transforms (16 and 8 points per thread)
  std::vector<std::vector<float2>> tw_host6_8;
  std::vector<std::vector<float2>> tw_host12;  // length 3*2^l/4, 12 points per thread
  flame::FlameDev* ddev = nullptr;
  flame::FlameDev* ddev_full = nullptr;       // same flames, W in the adjoint scratch
  std::vector<flame::FlameDev> hdev_full;
  std::vector<Group> groups;
  std::vector<int> group_of;
  std::vector<char> w_valid;
  long long n = 0;
  // per-kernel timing (flame_timing_begin / flame_timing_end)
  bool timing = false;
  hipEvent_t chain = nullptr;  // last event of the current chain of timed launches
  std::vector<hipEvent_t> ev_pool;
  std::vector<hipEvent_t> ev_used[4];
  // graph of graph_steps steps (one kernel chain per grid-size group)
  int graph_steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  long long* counter = nullptr;
  // persistent ensemble launch (flame_set_persistent)
  bool persistent = false;
  int ens_wgs = 0;                              // requested workgroups (0: all that fit)
  unsigned long long ens_limit = 0;             // bound of each wait, wall-clock ticks
  std::vector<flame::EnsembleItem> ens_items;   // the partition in use (empty: to be built)
  std::vector<int> ens_sig;                     // the group configuration it was built for
  flame::EnsembleItem* d_items = nullptr;
  unsigned* d_arrive = nullptr;
  int* d_err = nullptr;
  hipGraph_t ens_graph = nullptr;  // graph_steps steps of the persistent launch
  hipGraphExec_t ens_graph_exec = nullptr;
  ~flame_plan_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ens_graph_exec) (void)hipGraphExecDestroy(ens_graph_exec);
    if (ens_graph) (void)hipGraphDestroy(ens_graph);
    std::vector<hipEvent_t> all(ev_pool);
    for (auto& v : ev_used) all.insert(all.end(), v.begin(), v.end());
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    for (hipEvent_t e : all) (void)hipEventDestroy(e);
  }
};

namespace {

int check_plan(flame_plan p, int flame = 0) {
  if (!p) return fail(FLAME_ERR_INVALID_ARG, "null plan");
  if (flame < 0 || flame >= p->nfl) return fail(FLAME_ERR_INVALID_ARG, "flame index %d out of range [0, %d)", flame, p->nfl);
  return FLAME_OK;
}

// Every step index in [n_first, n_last] of flames [f0, f1) with a tabulated
// reference radius must have a table entry (the kernels index it by n).
// Steps n_first .. n_last (or diagnostics / adjoint at those indices) need
// table entries up to n_last; a Heun step n also reads entry n + 1 when
// `stepping` is set.
int check_r0(flame_plan p, int f0, int f1, long long n_first, long long n_last, bool stepping = false) {
  for (int f = f0; f < f1; ++f) {
    if (p->descs[f].r0_law != 1) continue;
    if (!p->hdev[f].r0tab) return fail(FLAME_ERR_INVALID_ARG, "flame %d: r0_law = 1 but no r0 table set", f);
    const long long last = n_last + (stepping && p->descs[f].integrator == 1 ? 1 : 0);
    if (n_first < 0 || last >= p->hdev[f].r0n)
      return fail(FLAME_ERR_INVALID_ARG, "flame %d: step index %lld is beyond its r0 table of %lld entries", f,
                  n_first < 0 ? n_first : last, p->hdev[f].r0n);
  }
  return FLAME_OK;
}

int last_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return FLAME_OK;
}

enum TimedKind { KIND_ROW = 0, KIND_COL = 1, KIND_OTHER = 2, KIND_GRAPH = 3 };

hipEvent_t take_event(flame_plan p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Times consecutive launches with a chain of events on the plan's stream:
// the event recorded after one launch also opens the next, so the intervals
// partition the stream time (each includes its launch gap).
class Timed {
 public:
  Timed(flame_plan p, int kind) : p_(p), kind_(kind) {
    if (!p_->timing) return;
    if (!p_->chain) {
      p_->chain = take_event(p_);
      if (p_->chain) (void)hipEventRecord(p_->chain, p_->stream);
    }
    start_ = p_->chain;
  }
  ~Timed() {
    if (!p_->timing || !start_) return;
    hipEvent_t stop = take_event(p_);
    if (!stop) return;
    (void)hipEventRecord(stop, p_->stream);
    p_->ev_used[kind_].push_back(start_);
    p_->ev_used[kind_].push_back(stop);
    p_->chain = stop;
  }

 private:
  flame_plan p_;
  int kind_;
  hipEvent_t start_ = nullptr;
};

// Start and stop events of one step-kernel launch while timing is on (null
// otherwise); the launch records them in its own dispatch, so the interval is
// the kernel's execution alone.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  KernelEvents(flame_plan p, int kind) {
    if (!p->timing) return;
    start = take_event(p);
    stop = take_event(p);
    if (!start || !stop) {
      start = stop = nullptr;
      return;
    }
    p->ev_used[kind].push_back(start);
    p->ev_used[kind].push_back(stop);
  }
};

// Ends a chain of timed launches (another command may follow on the stream).
void break_chain(flame_plan p) { p->chain = nullptr; }

int rebuild_w(flame_plan p, int flame) {
  const Sizes& s = p->layout.sizes[flame];
  {
    Timed tm(p, KIND_OTHER);
    if (p->groups[p->group_of[flame]].product)
      flame::launch_colp(s.logn1, flame::COL_FIRST, s.tiles, 1, p->stream, p->ddev + flame, p->n, nullptr,
                         p->groups[p->group_of[flame]].col_pts);
    else
      flame::launch_col(s.logn1, flame::COL_FIRST, s.tiles, 1, p->stream, p->ddev + flame, p->n);
  }
  p->w_valid[flame] = 1;
  return last_launch("column transform launch");
}

// The step's row count lives in the device flame table (the row kernel
// reads it); rewrite the group's entries after a change of grid. The
// intermediates of the old grid are stale.
int apply_rows(flame_plan p, int gi) {
  const Group& gr = p->groups[gi];
  for (int f = gr.first; f < gr.first + gr.count; ++f) {
    p->hdev[f].rows = gr.rows();
    p->hdev[f].cols = gr.cols();
    p->w_valid[f] = 0;
  }
  hipError_t e = hipMemcpyAsync(p->ddev + gr.first, p->hdev.data() + gr.first, sizeof(flame::FlameDev) * gr.count,
                                hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // the host table may change again
  if (e != hipSuccess) return hip_fail(e, "flame table update");
  return FLAME_OK;
}

// The step's kernels of one group, on the plan's stream unless `st` is given.
void launch_step_row(flame_plan p, const Group& gr, long long n, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                     hipStream_t st = nullptr) {
  flame::launch_row(gr.logn2, flame::ROW_STEP, gr.rgroups(), gr.count, st ? st : p->stream, p->ddev + gr.first, n,
                    nullptr, nullptr, gr.row_pts, e0, e1, gr.nt_q());
}

void launch_step_col(flame_plan p, const Group& gr, long long n, int pass, hipEvent_t e0 = nullptr,
                     hipEvent_t e1 = nullptr, hipStream_t st = nullptr) {
  if (gr.product)
    flame::launch_colp(gr.logn1, flame::COL_STEP, gr.tiles, gr.count, st ? st : p->stream, p->ddev + gr.first, n,
                       nullptr, gr.col_pts, e0, e1, gr.col_var(pass));
  else
    flame::launch_col(gr.logn1, flame::COL_STEP, gr.tiles, gr.count, st ? st : p->stream, p->ddev + gr.first, n,
                      nullptr, gr.col_pts, e0, e1, gr.col_var(pass));
}

// Destroy the step graph. A replay may still run on the plan's stream (or
// the runtime may still hold it), so the stream is drained first.
void drop_graph(flame_plan p) {
  if (!p->graph_exec && !p->graph) return;
  (void)hipStreamSynchronize(p->stream);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
}

// Destroy the persistent launch's graph (it bakes in the partition, the wait
// limit and graph_steps), after draining the plan's stream.
void drop_ens_graph(flame_plan p) {
  if (!p->ens_graph_exec && !p->ens_graph) return;
  (void)hipStreamSynchronize(p->stream);
  if (p->ens_graph_exec) (void)hipGraphExecDestroy(p->ens_graph_exec);
  if (p->ens_graph) (void)hipGraphDestroy(p->ens_graph);
  p->ens_graph_exec = nullptr;
  p->ens_graph = nullptr;
}

// graph_steps steps of every flame: for each grid-size group a chain
// row(0) -> col(0) -> row(1) -> ... ; chains of different groups carry no
// edges between them, so the groups run concurrently. Kernels read the step
// index as counter + s.
int build_graph(flame_plan p) {
  drop_graph(p);
  hipError_t e = hipGraphCreate(&p->graph, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
  std::vector<hipGraphNode_t> last(p->groups.size(), nullptr);
  // one pass of group gi at step offset s: row node, then column node, chained after the group's last node
  auto add_pass = [&](size_t gi, int s, int pass) -> int {
    const Group& gr = p->groups[gi];
    const flame::KernelLaunch rk = flame::row_step_kernel(gr.logn2, gr.row_pts, gr.nt_q());
    const flame::KernelLaunch ck =
        gr.product ? flame::colp_kernel_info(gr.logn1, flame::COL_STEP, gr.col_pts, gr.col_var(pass))
                   : flame::col_step_kernel(gr.logn1, gr.col_pts, gr.col_var(pass));
    if (!rk.func || !ck.func) return fail(FLAME_ERR_UNSUPPORTED_SIZE, "no step kernel for this grid");
    const flame::FlameDev* fl = p->ddev + gr.first;
    long long n = s;
    const long long* nb = p->counter;
    const float* in = nullptr;
    float* outp = nullptr;
    const float2* src = nullptr;
    void* rargs[] = {&fl, &n, &nb, &in, &outp};
    void* cargs[] = {&fl, &n, &nb, &src};
    hipKernelNodeParams rp{};
    rp.func = const_cast<void*>(rk.func);
    rp.gridDim = dim3(gr.rgroups(), gr.count);
    rp.blockDim = dim3(rk.threads);
    rp.sharedMemBytes = rk.lds;
    rp.kernelParams = rargs;
    hipGraphNode_t rn;
    e = hipGraphAddKernelNode(&rn, p->graph, last[gi] ? &last[gi] : nullptr, last[gi] ? 1 : 0, &rp);
    if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (row)");
    hipKernelNodeParams cp{};
    cp.func = const_cast<void*>(ck.func);
    cp.gridDim = dim3(gr.tiles, gr.count);
    cp.blockDim = dim3(ck.threads);
    cp.sharedMemBytes = ck.lds;
    cp.kernelParams = cargs;
    hipGraphNode_t cn;
    e = hipGraphAddKernelNode(&cn, p->graph, &rn, 1, &cp);
    if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (col)");
    last[gi] = cn;
    return FLAME_OK;
  };
  // groups with more points per step first: their chains are the longest, and
  // the replay starts them first (on the 256-flame ensemble 2-3 % faster than
  // the order of first appearance)
  std::vector<size_t> order(p->groups.size());
  for (size_t gi = 0; gi < order.size(); ++gi) order[gi] = gi;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    const Group &ga = p->groups[a], &gb = p->groups[b];
    return (long long)ga.count << (ga.logn1 + ga.logn2) > (long long)gb.count << (gb.logn1 + gb.logn2);
  });
  for (int s = 0; s < p->graph_steps; ++s)
    for (const size_t gi : order)
      for (int pass = 0; pass < p->groups[gi].passes(); ++pass) {
        const int rc = add_pass(gi, s, pass);
        if (rc) return rc;
      }
  e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return FLAME_OK;
}

// ------------------------------------------------------------------------
// Workspace of flame_step_noalloc: a static device array (one copy per GPU,
// held until the process ends). Host code never passes the array's name to
// a kernel or copy: its device address comes from hipGetSymbolAddress, once
// per device, and is kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)FLAME_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FLAME_ERR_INVALID_ARG, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(FLAME_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FLAME_OK;
}

// One twiddle table: passes q = 1 .. npass-1 of a Stockham plan hold
// exp(-2 pi i r k / (ns_q R_q)) at off_q + (r - 1) ns_q + k, 0 < r < R_q,
// k < ns_q (the layout of ff::build_twiddles and, with the radix-6 pass as
// its last pass, of ff::build_twiddles6). Built on the device in double
// precision and rounded once, like the host tables of flame_init.
struct TwSpec {
  float2* out;
  int npass;
  int ns[6], radix[6], off[6];
  int count;
};
constexpr int kMaxTwTables = 4;
struct TwSpecs {
  TwSpec t[kMaxTwTables];
  int ntab;
};

__global__ void noalloc_setup_kernel(flame::FlameDev fd, flame::FlameDev* dst, TwSpecs specs) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = fd;
  for (int ti = 0; ti < specs.ntab; ++ti) {
    const TwSpec& s = specs.t[ti];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.count; i += gridDim.x * blockDim.x) {
      int q = 1;
      while (q + 1 < s.npass && i >= s.off[q + 1]) ++q;
      const int rel = i - s.off[q];
      const int ns = s.ns[q], r = s.radix[q];
      const int m = rel / ns + 1, k = rel % ns;
      const long long e = (long long)k * m % (long long)(ns * r);
      const double ang = -2.0 * M_PI * double(e) / (double(ns) * double(r));
      s.out[i] = make_float2((float)cos(ang), (float)sin(ang));
    }
  }
}

TwSpec tw_spec_pow2(float2* out, int logn, int pts) {
  const ff::PassPlan p = ff::make_pass_plan(logn, pts);
  TwSpec s{};
  s.out = out;
  s.npass = p.npass;
  for (int q = 0; q < p.npass; ++q) {
    s.ns[q] = p.ns[q];
    s.radix[q] = p.radix[q];
    s.off[q] = p.tw_off[q];
  }
  s.count = p.tw_size;
  return s;
}

// Shape6 of length 6 * 2^logp: the power-of-two passes, then the radix-6 pass.
TwSpec tw_spec_six(float2* out, int logp, int pts) {
  TwSpec s = tw_spec_pow2(out, logp, pts);
  const int q = s.npass;
  s.ns[q] = 1 << logp;
  s.radix[q] = 6;
  s.off[q] = s.count;
  s.npass = q + 1;
  s.count += 5 * (1 << logp);
  return s;
}

}  // namespace

extern "C" {

const char* flame_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------ circular flames

static int check_circle(const flame_circle_desc* d, int* logn) {
  if (!d) return fail(FLAME_ERR_INVALID_ARG, "null flame_circle_desc");
  const int l = ilog2_exact(d->n);
  if (l < 0 || l < flame::kMinLog || l > flame::kMaxLog)
    return fail(FLAME_ERR_UNSUPPORTED_SIZE, "circle of %d points: a power of two in [16, 16384]", d->n);
  if (!(std::isfinite(d->gamma) && d->gamma >= 0.0)) return fail(FLAME_ERR_INVALID_ARG, "gamma must be finite and >= 0");
  if (!(std::isfinite(d->seg) && d->seg > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "seg must be > 0");
  if (!(std::isfinite(d->t0) && d->t0 > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "t0 must be > 0");
  if (!(std::isfinite(d->dt) && d->dt > 0.0)) return fail(FLAME_ERR_INVALID_ARG, "dt must be > 0");
  if (logn) *logn = l;
  return FLAME_OK;
}

static flame::CircleDev circle_dev(const flame_circle_desc* d, int32_t n_circles, void* states) {
  flame::CircleDev cd;
  std::memset(&cd, 0, sizeof cd);
  cd.S = static_cast<float2*>(states);
  cd.n_circles = n_circles;
  cd.seg = (float)d->seg;
  cd.gamma = (float)d->gamma;
  cd.t0 = d->t0;
  cd.dt = d->dt;
  return cd;
}

int flame_circle_state_bytes(const flame_circle_desc* desc, size_t* bytes) {
  if (!bytes) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  const int rc = check_circle(desc, nullptr);
  if (rc) return rc;
  *bytes = (size_t)(desc->n / 4) * sizeof(float2);
  return FLAME_OK;
}

// Steps per launch: a launch keeps every spectrum in registers; longer runs
// are split so that no single launch runs for long.
constexpr int kCircleStepsPerLaunch = 2000;

int flame_circle_step(const flame_circle_desc* desc, int32_t n_circles, void* states, int64_t n, int32_t nsteps,
                      void* hip_stream) {
  int logn = 0;
  int rc = check_circle(desc, &logn);
  if (rc) return rc;
  if (n_circles < 0 || nsteps < 0) return fail(FLAME_ERR_INVALID_ARG, "n_circles and nsteps must be >= 0");
  if (n_circles == 0 || nsteps == 0) return FLAME_OK;
  if (!states) return fail(FLAME_ERR_INVALID_ARG, "null states pointer");
  if (reinterpret_cast<uintptr_t>(states) % 8) return fail(FLAME_ERR_INVALID_ARG, "states must be 8-byte aligned");
  const flame::CircleDev cd = circle_dev(desc, n_circles, states);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int32_t done = 0; done < nsteps;) {
    const int k = std::min(kCircleStepsPerLaunch, nsteps - done);
    if (!flame::launch_circle_step(logn, cd, n + done, k, st))
      return fail(FLAME_ERR_UNSUPPORTED_SIZE, "no circle kernel for %d points", desc->n);
    done += k;
  }
  return last_launch("circle step launch");
}

int flame_circle_diagnostics(const flame_circle_desc* desc, int32_t n_circles, const void* states, int64_t n,
                             double* out4, void* hip_stream) {
  int logn = 0;
  int rc = check_circle(desc, &logn);
  if (rc) return rc;
  if (n_circles < 0) return fail(FLAME_ERR_INVALID_ARG, "n_circles must be >= 0");
  if (n_circles == 0) return FLAME_OK;
  if (!states || !out4) return fail(FLAME_ERR_INVALID_ARG, "null states or output pointer");
  if (reinterpret_cast<uintptr_t>(states) % 8 || reinterpret_cast<uintptr_t>(out4) % 8)
    return fail(FLAME_ERR_INVALID_ARG, "states and out4 must be 8-byte aligned");
  const flame::CircleDev cd = circle_dev(desc, n_circles, const_cast<void*>(states));
  if (!flame::launch_circle_diag(logn, cd, n, out4, static_cast<hipStream_t>(hip_stream)))
    return fail(FLAME_ERR_UNSUPPORTED_SIZE, "no circle kernel for %d points", desc->n);
  return last_launch("circle diagnostics launch");
}

int flame_step_noalloc(const flame_desc* desc, void* state, int64_t n, int32_t nsteps, void* hip_stream) {
  Sizes s{};
  int rc = check_desc(desc, &s);
  if (rc) return rc;
  if (!state) return fail(FLAME_ERR_INVALID_ARG, "null state pointer");
  if (reinterpret_cast<uintptr_t>(state) % 16) return fail(FLAME_ERR_INVALID_ARG, "state must be 16-byte aligned");
  if (desc->r0_law != 0) return fail(FLAME_ERR_INVALID_ARG, "flame_step_noalloc takes r0(t) = t only (r0_law = 0)");
  if (desc->integrator != 0)
    return fail(FLAME_ERR_INVALID_ARG, "flame_step_noalloc takes integrating-factor Euler only (integrator = 0)");
  if (nsteps < 0) return fail(FLAME_ERR_INVALID_ARG, "nsteps must be >= 0");
  // the default configuration of flame_init: the product grid for n1 >= 128,
  // 16 points per thread, plain stores, direct launches
  const bool product = s.logn1 >= flame::kMinLogProduct;
  const int rows = product ? 3 * desc->n1 / 4 : desc->n1;
  const size_t cols = (size_t)std::max(s.tiles * s.tcol, (desc->n2 / 4 + s.tq - 1) / s.tq * s.tq);
  const size_t wq = cols * (size_t)rows;  // elements of Q, and of each of Wp and Wm
  TwSpecs specs{};
  size_t off = align_up(sizeof(flame::FlameDev));
  size_t tw_off[kMaxTwTables] = {};
  auto add_table = [&](const TwSpec& t) {
    tw_off[specs.ntab] = off;
    specs.t[specs.ntab++] = t;
    off = align_up(off + (size_t)std::max(t.count, 1) * sizeof(float2));
  };
  // pointers are filled in once the scratch address is known
  if (product) add_table(tw_spec_six(nullptr, s.logn1 - 3, ff::kPts));
  else add_table(tw_spec_pow2(nullptr, s.logn1, ff::kPts));
  add_table(tw_spec_pow2(nullptr, s.logn2, ff::kPts));
  const size_t off_w = off;
  off = align_up(off + 2 * wq * sizeof(float2));
  const size_t off_q = off;
  off = align_up(off + wq * sizeof(float2));
  if (off > kScratchBytes)
    return fail(FLAME_ERR_WORKSPACE_TOO_SMALL,
                "grid %d x %d needs %zu bytes of scratch; the static scratch of flame_step_noalloc holds %zu",
                desc->n1, desc->n2, off, kScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int max_lds = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  const int need_lds = flame::lds_bytes_needed(s.logn1, s.logn2);
  if (need_lds > max_lds)
    return fail(FLAME_ERR_UNSUPPORTED_SIZE, "grid %d x %d needs %d bytes of LDS per workgroup, the device has %d",
                desc->n1, desc->n2, need_lds, max_lds);
  void* base_v = nullptr;
  rc = scratch_address(dev, &base_v);
  if (rc) return rc;
  char* base = static_cast<char*>(base_v);
  for (int i = 0; i < specs.ntab; ++i) specs.t[i].out = reinterpret_cast<float2*>(base + tw_off[i]);
  flame::FlameDev fd;
  std::memset(&fd, 0, sizeof fd);
  fd.S = static_cast<float2*>(state);
  fd.Wp = reinterpret_cast<float2*>(base + off_w);
  fd.Wm = fd.Wp + wq;
  fd.Q = reinterpret_cast<float2*>(base + off_q);
  const float2* tw_col = specs.t[0].out;
  const float2* tw_row = specs.t[1].out;
  fd.tw1 = product ? nullptr : tw_col;
  fd.tw6 = product ? tw_col : nullptr;
  fd.tw2 = tw_row;
  fd.n1 = desc->n1;
  fd.n2 = desc->n2;
  fd.m = desc->n2 / 4;
  fd.h1 = desc->n1 / 2;
  fd.tshift = ilog2_exact(s.tq);
  fd.rows = rows;
  fd.cols = desc->n2;
  const bool lit = desc->axis_scale[0] == 0.0;
  fd.s1 = (float)(lit ? desc->theta_pi : desc->axis_scale[0]);
  fd.s2 = (float)(lit ? desc->theta_pi : desc->axis_scale[1]);
  fd.gamma = (float)desc->gamma;
  fd.t0 = desc->t0;
  fd.dt = desc->dt;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  flame::FlameDev* dfl = reinterpret_cast<flame::FlameDev*>(base);
  // the flame table and the twiddles; every other scratch location a kernel
  // reads for a stored result is written earlier in this call
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(32), dim3(256), 0, st, fd, dfl, specs);
  rc = last_launch("flame_step_noalloc setup launch");
  if (rc) return rc;
  // W from the state, then the steps (the kernel sequence of flame_step)
  if (product)
    flame::launch_colp(s.logn1, flame::COL_FIRST, s.tiles, 1, st, dfl, n, nullptr, ff::kPts);
  else
    flame::launch_col(s.logn1, flame::COL_FIRST, s.tiles, 1, st, dfl, n);
  const int rgroups = (rows / 2 + s.rpairs - 1) / s.rpairs;
  for (int i = 0; i < nsteps; ++i) {
    flame::launch_row(s.logn2, flame::ROW_STEP, rgroups, 1, st, dfl, n + i, nullptr, nullptr, ff::kPts);
    if (product)
      flame::launch_colp(s.logn1, flame::COL_STEP, s.tiles, 1, st, dfl, n + i, nullptr, ff::kPts);
    else
      flame::launch_col(s.logn1, flame::COL_STEP, s.tiles, 1, st, dfl, n + i, nullptr, ff::kPts);
  }
  return last_launch("flame_step_noalloc launch");
}

int flame_state_bytes(const flame_desc* desc, size_t* bytes) {
  if (!bytes) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  int rc = check_desc(desc, nullptr);
  if (rc) return rc;
  *bytes = (size_t)(desc->n2 / 4) * (size_t)(desc->n1 / 2) * sizeof(float2);
  return FLAME_OK;
}

int flame_workspace_bytes(const flame_desc* descs, int32_t n_flames, size_t* bytes) {
  if (!bytes) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  Layout L;
  int rc = plan_layout(descs, n_flames, &L);
  if (rc) return rc;
  *bytes = L.total;
  return FLAME_OK;
}

int flame_init(const flame_desc* descs, int32_t n_flames, void* const* states, void* ws, size_t ws_bytes,
               void* hip_stream, flame_plan* out) {
  if (!out) return fail(FLAME_ERR_INVALID_ARG, "null plan output pointer");
  *out = nullptr;
  if (!states) return fail(FLAME_ERR_INVALID_ARG, "null state array");
  if (!ws) return fail(FLAME_ERR_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(FLAME_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  flame_plan p = new (std::nothrow) flame_plan_s();
  if (!p) return fail(FLAME_ERR_INVALID_ARG, "out of host memory");
  int rc = plan_layout(descs, n_flames, &p->layout);
  if (rc) {
    delete p;
    return rc;
  }
  if (ws_bytes < p->layout.total) {
    const size_t need = p->layout.total;
    delete p;
    return fail(FLAME_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, need %zu", ws_bytes, need);
  }
  for (int f = 0; f < n_flames; ++f) {
    if (!states[f]) {
      delete p;
      return fail(FLAME_ERR_INVALID_ARG, "null state pointer for flame %d", f);
    }
    if (reinterpret_cast<uintptr_t>(states[f]) % 16) {
      delete p;
      return fail(FLAME_ERR_INVALID_ARG, "state of flame %d must be 16-byte aligned", f);
    }
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  // every kernel of every flame must fit the device's LDS per workgroup
  int max_lds = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  for (int f = 0; f < n_flames; ++f) {
    const Sizes& s = p->layout.sizes[f];
    const int need = flame::lds_bytes_needed(s.logn1, s.logn2);
    if (need > max_lds) {
      delete p;
      return fail(FLAME_ERR_UNSUPPORTED_SIZE, "grid %d x %d needs %d bytes of LDS per workgroup, the device has %d",
                  descs[f].n1, descs[f].n2, need, max_lds);
    }
  }
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->nfl = n_flames;
  p->descs.assign(descs, descs + n_flames);
  p->w_valid.assign(n_flames, 0);
  char* base = static_cast<char*>(ws);
  const Layout& L = p->layout;
  // twiddle tables, built in double precision and rounded once
  p->tw_host.resize(flame::kMaxLog + 1);
  p->tw_host8.resize(flame::kMaxLog + 1);
  for (int l = flame::kMinLog; l <= flame::kMaxLog; ++l) {
    bool used = false;
    for (const Sizes& s : L.sizes) used |= (s.logn1 == l || s.logn2 == l);
    if (!used) continue;
    for (int pts : {16, 8}) {
      auto& host = pts == 16 ? p->tw_host[l] : p->tw_host8[l];
      const ff::PassPlan pp = ff::make_pass_plan(l, pts);
      host.assign(pp.tw_size > 0 ? pp.tw_size : 1, make_float2(1.f, 0.f));
      ff::build_twiddles(l, host.data(), pts);
      e = hipMemcpyAsync(base + (pts == 16 ? L.off_tw[l] : L.off_tw8[l]), host.data(), host.size() * sizeof(float2),
                         hipMemcpyHostToDevice, p->stream);
      if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "twiddle upload");
      }
    }
  }
  p->tw_host6.resize(flame::kMaxLog + 1);
  p->tw_host6_8.resize(flame::kMaxLog + 1);
  for (int l = flame::kMinLogProduct; l <= flame::kMaxLog; ++l) {
    bool used = false;
    for (const Sizes& s : L.sizes) used |= s.logn1 == l;
    if (!used) continue;
    for (int pts : {16, 8}) {
      auto& host = pts == 16 ? p->tw_host6[l] : p->tw_host6_8[l];
      host.assign(ff::twiddles6_size(l - 3, pts), make_float2(1.f, 0.f));
      ff::build_twiddles6(l - 3, host.data(), pts);
      e = hipMemcpyAsync(base + (pts == 16 ? L.off_tw6[l] : L.off_tw6_8[l]), host.data(),
                         host.size() * sizeof(float2), hipMemcpyHostToDevice, p->stream);
      if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "twiddle upload");
      }
    }
  }
  p->tw_host12.resize(flame::kMaxLog + 1);
  for (int l = flame::kMinLogRow12; l <= flame::kMaxLog; ++l) {
    bool used = false;
    for (const Sizes& s : L.sizes)
      used |= (s.logn1 == l && l >= flame::kMinLogProduct) || s.logn2 == l;
    if (!used) continue;
    const ff::PassPlan pp = ff::make_plan12(l - 4);
    auto& host = p->tw_host12[l];
    host.assign(std::max(1, pp.tw_size), make_float2(1.f, 0.f));
    ff::build_twiddles_plan(pp, host.data());
    e = hipMemcpyAsync(base + L.off_tw12[l], host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice,
                       p->stream);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "twiddle upload");
    }
  }
  // device flame table, ordered so that flames of one grid size are contiguous
  p->hdev.resize(n_flames);
  for (int f = 0; f < n_flames; ++f) {
    const flame_desc& d = descs[f];
    const Sizes& s = L.sizes[f];
    flame::FlameDev& fd = p->hdev[f];
    std::memset(&fd, 0, sizeof fd);
    fd.S = static_cast<float2*>(states[f]);
    fd.Wp = reinterpret_cast<float2*>(base + L.off_w[f]);
    fd.Wm = fd.Wp + s.wq_elems;
    fd.Q = reinterpret_cast<float2*>(base + L.off_q[f]);
    fd.A1 = reinterpret_cast<float2*>(base + L.off_a1[f]);
    fd.A2 = reinterpret_cast<float2*>(base + L.off_a2[f]);
    fd.S2 = fd.A2;  // Heun's predictor: A2 is free between the calls that use it
    fd.part = reinterpret_cast<double*>(base + L.off_part[f]);
    fd.tw1 = reinterpret_cast<const float2*>(base + L.off_tw[s.logn1]);
    fd.tw2 = reinterpret_cast<const float2*>(base + L.off_tw[s.logn2]);
    fd.tw1_8 = reinterpret_cast<const float2*>(base + L.off_tw8[s.logn1]);
    fd.tw2_8 = reinterpret_cast<const float2*>(base + L.off_tw8[s.logn2]);
    const bool p6 = s.logn1 >= flame::kMinLogProduct;
    fd.tw6 = p6 ? reinterpret_cast<const float2*>(base + L.off_tw6[s.logn1]) : nullptr;
    fd.tw6_8 = p6 ? reinterpret_cast<const float2*>(base + L.off_tw6_8[s.logn1]) : nullptr;
    fd.tw12a = p6 ? reinterpret_cast<const float2*>(base + L.off_tw12[s.logn1]) : nullptr;
    fd.tw12b = s.logn2 >= flame::kMinLogRow12 ? reinterpret_cast<const float2*>(base + L.off_tw12[s.logn2]) : nullptr;
    fd.n1 = d.n1;
    fd.n2 = d.n2;
    fd.m = d.n2 / 4;
    fd.h1 = d.n1 / 2;
    fd.tshift = ilog2_exact(s.tq);
    const bool lit = d.axis_scale[0] == 0.0;
    fd.s1 = (float)(lit ? d.theta_pi : d.axis_scale[0]);
    fd.s2 = (float)(lit ? d.theta_pi : d.axis_scale[1]);
    fd.gamma = (float)d.gamma;
    fd.t0 = d.t0;
    fd.dt = d.dt;
  }
  // groups of consecutive flames with equal grids (one launch per group); the
  // step uses the product grid wherever the column kernel for it exists
  p->group_of.resize(n_flames);
  for (int f = 0; f < n_flames; ++f) {
    const Sizes& s = L.sizes[f];
    if (!p->groups.empty() && p->groups.back().logn1 == s.logn1 && p->groups.back().logn2 == s.logn2 &&
        p->groups.back().integrator == descs[f].integrator) {
      p->groups.back().count++;
    } else {
      Group gr{s.logn1, s.logn2, f, 1, s.tiles, s.rpairs};
      gr.product = s.logn1 >= flame::kMinLogProduct;
      gr.integrator = descs[f].integrator;
      p->groups.push_back(gr);
    }
    p->group_of[f] = (int)p->groups.size() - 1;
  }
  for (int f = 0; f < n_flames; ++f) {
    p->hdev[f].rows = p->groups[p->group_of[f]].rows();
    p->hdev[f].cols = p->groups[p->group_of[f]].cols();
  }
  // the physical-grid W of the diagnostics goes to the adjoint scratch A1..A2
  // (2 wq_elems, contiguous), so the step's W stays valid
  p->hdev_full = p->hdev;
  for (int f = 0; f < n_flames; ++f) {
    p->hdev_full[f].Wp = p->hdev[f].A1;
    p->hdev_full[f].Wm = p->hdev[f].A1 + p->layout.sizes[f].wq_elems;
    p->hdev_full[f].rows = p->descs[f].n1;
    p->hdev_full[f].cols = p->descs[f].n2;
  }
  p->ddev = reinterpret_cast<flame::FlameDev*>(base + L.off_dev);
  p->ddev_full = reinterpret_cast<flame::FlameDev*>(base + L.off_dev_full);
  p->counter = reinterpret_cast<long long*>(base + L.off_counter);
  p->d_items = reinterpret_cast<flame::EnsembleItem*>(base + L.off_ens_items);
  p->d_arrive = reinterpret_cast<unsigned*>(base + L.off_ens_arrive);
  p->d_err = reinterpret_cast<int*>(base + L.off_ens_err);
  e = hipMemcpyAsync(p->ddev, p->hdev.data(), sizeof(flame::FlameDev) * n_flames, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ddev_full, p->hdev_full.data(), sizeof(flame::FlameDev) * n_flames, hipMemcpyHostToDevice,
                       p->stream);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "flame table upload");
  }
  // the host copies must outlive the asynchronous uploads
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "init synchronise");
  }
  *out = p;
  return FLAME_OK;
}

int flame_set_spectrum(flame_plan p, int32_t flame, const void* half, int64_t n) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!half) return fail(FLAME_ERR_INVALID_ARG, "null spectrum pointer");
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  const int total = (p->descs[flame].n2 / 4) * (p->descs[flame].n1 / 2);
  (void)s;
  flame::launch_set_spectrum(p->stream, p->ddev, flame, total, half);
  p->n = n;
  p->w_valid[flame] = 0;
  return last_launch("set_spectrum launch");
}

int flame_get_spectrum(flame_plan p, int32_t flame, void* half) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!half) return fail(FLAME_ERR_INVALID_ARG, "null spectrum pointer");
  DeviceGuard g(p->device);
  const int total = (p->descs[flame].n1 / 2 - 1) * (p->descs[flame].n2 / 4);
  flame::launch_get_spectrum(p->stream, p->ddev, flame, total, half);
  return last_launch("get_spectrum launch");
}

int flame_set_state(flame_plan p, int32_t flame, const float* phi, int64_t n) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!phi) return fail(FLAME_ERR_INVALID_ARG, "null field pointer");
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  p->n = n;
  flame::launch_row(s.logn2, flame::ROW_FORWARD, s.rgroups, 1, p->stream, p->ddev + flame, p->n, phi, nullptr);
  flame::launch_col(s.logn1, flame::COL_PROJECT, s.tiles, 1, p->stream, p->ddev + flame, p->n);
  p->w_valid[flame] = !p->groups[p->group_of[flame]].product;  // the W just written is the physical grid's
  return last_launch("set_state launch");
}

int flame_get_state(flame_plan p, int32_t flame, float* phi) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!phi) return fail(FLAME_ERR_INVALID_ARG, "null field pointer");
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  flame::launch_col(s.logn1, flame::COL_SYNTH, s.tiles, 1, p->stream, p->ddev + flame, p->n);
  flame::launch_row(s.logn2, flame::ROW_SYNTH, s.rgroups, 1, p->stream, p->ddev + flame, p->n, nullptr, phi);
  return last_launch("get_state launch");
}

int flame_state_modified(flame_plan p, int32_t flame, int64_t n) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (flame < -1 || flame >= p->nfl)
    return fail(FLAME_ERR_INVALID_ARG, "flame index %d out of range [-1, %d)", flame, p->nfl);
  p->n = n;
  if (flame < 0)
    for (auto& v : p->w_valid) v = 0;
  else
    p->w_valid[flame] = 0;
  return FLAME_OK;
}

int flame_step_index(flame_plan p, int64_t* n) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!n) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  *n = p->n;
  return FLAME_OK;
}

}  // extern "C"

// Persistent ensemble launch: partition, graph and launches (C++ helpers of
// the entry points below).
namespace {

// Why the flames of group gr cannot run in the persistent ensemble kernel
// (null if they can).
const char* ens_reason(const Group& gr) {
  if (!flame::ensemble_supports(gr.logn1, gr.logn2)) return "the persistent kernel has bodies for n1 in [128, 1024], n2 in [128, 2048]";
  if (!gr.product || gr.col_pts != 12) return "the persistent kernel steps the product grid with 12 column points per thread";
  if (gr.row_pts != 16) return "the persistent kernel's row transforms use 16 points per thread";
  if (gr.nt != 0) return "the persistent kernel uses plain stores";
  if (gr.integrator != 0 || gr.forced) return "the persistent kernel runs unforced integrating-factor Euler";
  return nullptr;
}

int ens_check(flame_plan p) {
  for (const Group& gr : p->groups)
    if (const char* why = ens_reason(gr))
      return fail(FLAME_ERR_INVALID_ARG, "flames of grid %d x %d: %s", 1 << gr.logn1, 1 << gr.logn2, why);
  return FLAME_OK;
}

std::vector<int> ens_signature(flame_plan p, int wgs) {
  std::vector<int> sig{wgs};
  for (const Group& gr : p->groups) sig.insert(sig.end(), {gr.first, gr.count, gr.rgroups(), gr.tiles});
  return sig;
}

// Split the flames over at most `wgs` workgroups with about equal work: each
// flame has u = row-pair groups + column tiles of work per step; with a
// target of t per workgroup, a flame with u >= t is shared by ceil(u / t)
// workgroups (no more than it has tiles in a phase), and flames with u < t
// go floor(t / u) to a workgroup. t starts at the total work over wgs and
// grows until the items fit.
int ens_partition(flame_plan p, int wgs, std::vector<flame::EnsembleItem>* out) {
  long long total = 0;
  for (const Group& gr : p->groups) total += (long long)gr.count * (gr.rgroups() + gr.tiles);
  std::vector<flame::EnsembleItem> items;
  for (long long t = std::max(1LL, (total + wgs - 1) / wgs); t <= total; ++t) {
    items.clear();
    for (const Group& gr : p->groups) {
      const int rt = gr.rgroups(), ct = gr.tiles, u = rt + ct;
      if (u >= t) {
        const int parts = (int)std::min<long long>((u + t - 1) / t, std::max(rt, ct));
        for (int f = gr.first; f < gr.first + gr.count; ++f)
          for (int part = 0; part < parts; ++part)
            items.push_back(flame::EnsembleItem{f, 1, part, parts, gr.logn1, gr.logn2, rt, ct});
      } else {
        const int fpw = (int)(t / u);
        for (int f = gr.first; f < gr.first + gr.count; f += fpw)
          items.push_back(
              flame::EnsembleItem{f, std::min(fpw, gr.first + gr.count - f), 0, 1, gr.logn1, gr.logn2, rt, ct});
      }
    }
    if ((long long)items.size() <= wgs) {
      *out = std::move(items);
      return FLAME_OK;
    }
  }
  return fail(FLAME_ERR_UNSUPPORTED_SIZE, "%zu grid groups do not fit %d persistent workgroups", p->groups.size(), wgs);
}

// The partition for the current group configuration, built and uploaded
// when it changed.
int ens_prepare(flame_plan p) {
  int rc = ens_check(p);
  if (rc) return rc;
  int per_cu = flame::ensemble_blocks_per_cu(), cus = 0;
  if (per_cu <= 0) return fail(FLAME_ERR_HIP, "occupancy query of the persistent kernel failed");
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(multiprocessor count)");
  int wgs = std::min(per_cu * cus, kMaxEnsItems);
  if (p->ens_wgs > 0) wgs = std::min(wgs, p->ens_wgs);
  const std::vector<int> sig = ens_signature(p, wgs);
  if (!p->ens_items.empty() && sig == p->ens_sig) return FLAME_OK;
  // an earlier upload may still read the host table; the graph holds the old grid
  drop_ens_graph(p);
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronise");
  std::vector<flame::EnsembleItem> items;
  rc = ens_partition(p, wgs, &items);
  if (rc) return rc;
  p->ens_items = std::move(items);
  p->ens_sig = sig;
  e = hipMemcpyAsync(p->d_items, p->ens_items.data(), sizeof(flame::EnsembleItem) * p->ens_items.size(),
                     hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) {
    p->ens_items.clear();
    return hip_fail(e, "persistent item table upload");
  }
  return FLAME_OK;
}

// The persistent launch as a graph: a node that zeroes the arrival counters,
// then the ensemble kernel as a cooperative node for graph_steps steps from
// the step index the replay reads from the workspace counter.
int build_ens_graph(flame_plan p) {
  drop_ens_graph(p);
  hipError_t e = hipGraphCreate(&p->ens_graph, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphCreate (persistent)");
  const flame::KernelLaunch rk = flame::ensemble_reset_info(), ek = flame::ensemble_kernel_info();
  unsigned* arrive = p->d_arrive;
  int narrive = p->nfl * flame::kEnsArriveStride, clear = 0;
  int* err = p->d_err;
  void* rargs[] = {&arrive, &narrive, &err, &clear};
  hipKernelNodeParams rp{};
  rp.func = const_cast<void*>(rk.func);
  rp.gridDim = dim3(std::min(1024, std::max(1, (narrive + 255) / 256)));
  rp.blockDim = dim3(rk.threads);
  rp.sharedMemBytes = 0;
  rp.kernelParams = rargs;
  hipGraphNode_t rn, en;
  e = hipGraphAddKernelNode(&rn, p->ens_graph, nullptr, 0, &rp);
  if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (persistent reset)");
  const flame::FlameDev* fls = p->ddev;
  const flame::EnsembleItem* items = p->d_items;
  long long n0 = 0;
  const long long* nbase = p->counter;
  int steps = p->graph_steps;
  unsigned long long limit = p->ens_limit;
  void* eargs[] = {&fls, &items, &arrive, &err, &n0, &nbase, &steps, &limit};
  hipKernelNodeParams ep{};
  ep.func = const_cast<void*>(ek.func);
  ep.gridDim = dim3((unsigned)p->ens_items.size());
  ep.blockDim = dim3(ek.threads);
  ep.sharedMemBytes = (unsigned)ek.lds;
  ep.kernelParams = eargs;
  e = hipGraphAddKernelNode(&en, p->ens_graph, &rn, 1, &ep);
  if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (persistent)");
  hipKernelNodeAttrValue coop{};
  coop.cooperative = 1;
  e = hipGraphKernelNodeSetAttribute(en, hipKernelNodeAttributeCooperative, &coop);
  if (e != hipSuccess) return hip_fail(e, "hipGraphKernelNodeSetAttribute (cooperative)");
  e = hipGraphInstantiate(&p->ens_graph_exec, p->ens_graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate (persistent)");
  return FLAME_OK;
}

// nsteps steps of every flame: replays of the persistent graph while
// graph_steps (at most kEnsMaxSteps) steps remain, the rest as direct
// cooperative launches of at most kEnsMaxSteps steps; then waits for them
// and reports a wait that ran out.
int ens_steps(flame_plan p, int nsteps) {
  int rc = ens_prepare(p);
  if (rc) return rc;
  const int narrive = p->nfl * flame::kEnsArriveStride;
  flame::launch_ensemble_reset(p->stream, p->d_arrive, narrive, p->d_err, true);
  rc = last_launch("persistent ensemble reset");
  if (rc) return rc;
  const int gs = p->graph_steps;
  if (gs > 0 && gs <= kEnsMaxSteps && nsteps >= gs) {
    if (!p->ens_graph_exec) {
      rc = build_ens_graph(p);
      if (rc) return rc;
    }
    while (nsteps >= gs) {
      flame::launch_set_step(p->stream, p->counter, p->n);
      {
        Timed tm(p, KIND_GRAPH);
        const hipError_t e = hipGraphLaunch(p->ens_graph_exec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch (persistent)");
      }
      p->n += gs;
      nsteps -= gs;
    }
  }
  while (nsteps > 0) {
    const int k = std::min(nsteps, kEnsMaxSteps);
    {
      Timed tm(p, KIND_GRAPH);
      const hipError_t e = flame::launch_ensemble(p->stream, p->ddev, p->d_items, (int)p->ens_items.size(),
                                                  p->d_arrive, narrive, p->d_err, p->n, k, p->ens_limit);
      if (e != hipSuccess) return hip_fail(e, "persistent ensemble launch");
    }
    p->n += k;
    nsteps -= k;
  }
  break_chain(p);
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, p->d_err, sizeof flag, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "persistent ensemble status");
  if (flag)
    return fail(FLAME_ERR_TIMEOUT,
                "a wait of the persistent ensemble kernel ran out before step index %lld; the states are undefined",
                p->n);
  return FLAME_OK;
}

}  // namespace

extern "C" {

int flame_step(flame_plan p, int32_t nsteps) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (nsteps < 0) return fail(FLAME_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (nsteps > 0) {
    rc = check_r0(p, 0, p->nfl, p->n, p->n + nsteps - 1, true);
    if (rc) return rc;
  }
  DeviceGuard g(p->device);
  for (int f = 0; f < p->nfl; ++f)
    if (!p->w_valid[f]) {
      rc = rebuild_w(p, f);
      if (rc) return rc;
    }
  if (p->persistent) return nsteps > 0 ? ens_steps(p, nsteps) : FLAME_OK;
  if (p->graph_steps > 0 && nsteps >= p->graph_steps) {
    if (!p->graph_exec) {
      rc = build_graph(p);
      if (rc) return rc;
    }
    while (nsteps >= p->graph_steps) {
      flame::launch_set_step(p->stream, p->counter, p->n);
      {
        Timed tm(p, KIND_GRAPH);
        const hipError_t e = hipGraphLaunch(p->graph_exec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      }
      p->n += p->graph_steps;
      nsteps -= p->graph_steps;
      break_chain(p);
    }
  }
  break_chain(p);
  int max_passes = 1;
  for (const Group& gr : p->groups) max_passes = std::max(max_passes, gr.passes());
  for (int s = 0; s < nsteps; ++s) {
    for (int pass = 0; pass < max_passes; ++pass) {
      for (const Group& gr : p->groups) {
        if (pass >= gr.passes()) continue;
        KernelEvents ev(p, KIND_ROW);
        launch_step_row(p, gr, p->n, ev.start, ev.stop);
      }
      for (const Group& gr : p->groups) {
        if (pass >= gr.passes()) continue;
        KernelEvents ev(p, KIND_COL);
        launch_step_col(p, gr, p->n, pass, ev.start, ev.stop);
      }
    }
    p->n += 1;
  }
  return last_launch("step launch");
}

int flame_diagnostics(flame_plan p, int32_t flame, double* out4, void* dJ_dstate) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!out4) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  rc = check_r0(p, flame, flame + 1, p->n, p->n);
  if (rc) return rc;
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  // the area is a grid mean on the physical N1 x N2 grid: with the product
  // grid, its W is built into the adjoint scratch and the step's W is kept
  const bool product = p->groups[p->group_of[flame]].product;
  if (!product && !p->w_valid[flame]) {
    rc = rebuild_w(p, flame);
    if (rc) return rc;
  }
  {
    Timed tm(p, KIND_OTHER);
    flame::FlameDev* fd = product ? p->ddev_full + flame : p->ddev + flame;
    if (product) flame::launch_col(s.logn1, flame::COL_FIRST, s.tiles, 1, p->stream, fd, p->n);
    flame::launch_row(s.logn2, flame::ROW_DIAG, s.rgroups, 1, p->stream, fd, p->n, nullptr, nullptr);
    double* part = p->hdev[flame].part;
    flame::launch_diag_spectral(p->stream, p->ddev, flame, s.n_spec, part + s.rgroups);
    flame::launch_diag_final(p->stream, p->ddev, flame, p->n, s.rgroups, s.n_spec, out4);
  }
  break_chain(p);
  rc = last_launch("diagnostics launch");
  if (rc || !dJ_dstate) return rc;
  return flame_area_gradient(p, flame, p->n, p->hdev[flame].S, dJ_dstate);
}

int flame_diagnostics_host(flame_plan p, int32_t flame, double* host_out4) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!host_out4) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  double* dev = reinterpret_cast<double*>(reinterpret_cast<char*>(p->ddev) - p->layout.off_dev + p->layout.off_diag) +
                4 * (size_t)flame;
  rc = flame_diagnostics(p, flame, dev, nullptr);
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipError_t e = hipMemcpyAsync(host_out4, dev, 4 * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
  if (host_out4[3] != 1.0)
    return fail(FLAME_ERR_NONFINITE, "flame %d: the state at step index %lld holds non-finite values", flame, p->n);
  return FLAME_OK;
}

int flame_adjoint_step(flame_plan p, int32_t flame, int64_t n, const void* state_n, const void* lam_in,
                       void* lam_out) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!state_n || !lam_in || !lam_out) return fail(FLAME_ERR_INVALID_ARG, "null state or cotangent pointer");
  if (state_n == lam_out) return fail(FLAME_ERR_INVALID_ARG, "state_n must not alias lam_out");
  if (p->descs[flame].integrator != 0)
    return fail(FLAME_ERR_INVALID_ARG, "flame %d: the adjoint step is the transpose of IF-Euler (integrator 0)", flame);
  rc = check_r0(p, flame, flame + 1, n, n);
  if (rc) return rc;
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  flame::FlameDev* fd = p->ddev + flame;
  const Group& gr = p->groups[p->group_of[flame]];
  if (gr.product) {  // the transpose of the step on its product grid
    flame::launch_adjp_col(s.logn1, flame::ADJ_A, s.tiles, p->stream, fd, n, state_n, lam_in, nullptr);
    flame::launch_adj_row(s.logn2, flame::ROW_ADJ, gr.rgroups(), p->stream, fd, n);
    flame::launch_adjp_col(s.logn1, flame::ADJ_C, s.tiles, p->stream, fd, n, nullptr, lam_in, lam_out);
  } else {
    flame::launch_adj_col(s.logn1, flame::ADJ_A, s.tiles, p->stream, fd, n, state_n, lam_in, nullptr);
    flame::launch_adj_row(s.logn2, flame::ROW_ADJ, s.rgroups, p->stream, fd, n);
    flame::launch_adj_col(s.logn1, flame::ADJ_C, s.tiles, p->stream, fd, n, nullptr, lam_in, lam_out);
  }
  p->w_valid[flame] = 0;
  return last_launch("adjoint step launch");
}

int flame_area_gradient(flame_plan p, int32_t flame, int64_t n, const void* state, void* lam_out) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!state || !lam_out) return fail(FLAME_ERR_INVALID_ARG, "null state or cotangent pointer");
  if (state == lam_out) return fail(FLAME_ERR_INVALID_ARG, "state must not alias lam_out");
  rc = check_r0(p, flame, flame + 1, n, n);
  if (rc) return rc;
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  flame::FlameDev* fd = p->ddev + flame;
  flame::launch_col(s.logn1, flame::COL_FIRST, s.tiles, 1, p->stream, fd, n, state);
  flame::launch_adj_row(s.logn2, flame::ROW_SEED, s.rgroups, p->stream, fd, n);
  flame::launch_adj_col(s.logn1, flame::SEED_C, s.tiles, p->stream, fd, n, nullptr, nullptr, lam_out);
  p->w_valid[flame] = 0;
  return last_launch("area gradient launch");
}

// Rewrite the device copies of flame's two descriptors (step grid and full
// grid) from the host copies; waits, so the host copies may change again.
static int upload_dev(flame_plan p, int32_t flame, const char* what) {
  hipError_t e = hipMemcpyAsync(p->ddev + flame, &p->hdev[flame], sizeof(flame::FlameDev), hipMemcpyHostToDevice,
                                p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ddev_full + flame, &p->hdev_full[flame], sizeof(flame::FlameDev), hipMemcpyHostToDevice,
                       p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, what);
  return FLAME_OK;
}

int flame_set_r0_table(flame_plan p, int32_t flame, const double* table, int64_t n_entries) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (p->descs[flame].r0_law != 1) return fail(FLAME_ERR_INVALID_ARG, "flame %d has r0_law = 0 (r0 = t)", flame);
  if (!table || n_entries <= 0) return fail(FLAME_ERR_INVALID_ARG, "need a table of at least one entry");
  if (reinterpret_cast<uintptr_t>(table) % 8) return fail(FLAME_ERR_INVALID_ARG, "table must be 8-byte aligned");
  DeviceGuard g(p->device);
  p->hdev[flame].r0tab = table;
  p->hdev[flame].r0n = n_entries;
  p->hdev_full[flame].r0tab = table;
  p->hdev_full[flame].r0n = n_entries;
  return upload_dev(p, flame, "r0 table update");
}

int flame_set_forcing(flame_plan p, int32_t flame, const void* forcing) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(forcing) % 8) return fail(FLAME_ERR_INVALID_ARG, "forcing must be 8-byte aligned");
  DeviceGuard g(p->device);
  const float2* fp = static_cast<const float2*>(forcing);
  p->hdev[flame].F = fp;
  p->hdev_full[flame].F = fp;
  rc = upload_dev(p, flame, "forcing update");
  if (rc) return rc;
  // the group's steps use the forced column kernel while any member has a forcing
  Group& gr = p->groups[p->group_of[flame]];
  bool any = false;
  for (int f = gr.first; f < gr.first + gr.count; ++f) any = any || p->hdev[f].F != nullptr;
  if (any != gr.forced) {
    gr.forced = any;
    drop_graph(p);
  }
  return FLAME_OK;
}

int flame_synthesize(flame_plan p, int32_t flame, const void* spec, float* phi) {
  int rc = check_plan(p, flame);
  if (rc) return rc;
  if (!spec || !phi) return fail(FLAME_ERR_INVALID_ARG, "null spectrum or field pointer");
  DeviceGuard g(p->device);
  const Sizes& s = p->layout.sizes[flame];
  flame::launch_col(s.logn1, flame::COL_SYNTH, s.tiles, 1, p->stream, p->ddev + flame, p->n, spec);
  flame::launch_row(s.logn2, flame::ROW_SYNTH, s.rgroups, 1, p->stream, p->ddev + flame, p->n, nullptr, phi);
  return last_launch("synthesize launch");
}

int flame_timing_begin(flame_plan p) {
  int rc = check_plan(p);
  if (rc) return rc;
  std::vector<hipEvent_t> all;
  for (auto& v : p->ev_used) {
    all.insert(all.end(), v.begin(), v.end());
    v.clear();
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  p->ev_pool.insert(p->ev_pool.end(), all.begin(), all.end());
  p->chain = nullptr;
  p->timing = true;
  return FLAME_OK;
}

int flame_set_points_per_thread(flame_plan p, int32_t n1, int32_t n2, int32_t col_pts, int32_t row_pts) {
  int rc = check_plan(p);
  if (rc) return rc;
  auto valid = [](int v) { return v == 8 || v == 12 || v == 16; };
  if (!valid(col_pts) || !valid(row_pts)) return fail(FLAME_ERR_INVALID_ARG, "points per thread must be 8, 12 or 16");
  bool found = false;
  for (const Group& gr : p->groups) {
    if ((1 << gr.logn1) != n1 || (1 << gr.logn2) != n2) continue;
    found = true;
    if (col_pts == 12 && !gr.product)
      return fail(FLAME_ERR_INVALID_ARG, "col_pts = 12 runs on the product grid: enable it first (n1 >= %d)",
                  1 << flame::kMinLogProduct);
    if (row_pts == 12 && gr.logn2 < flame::kMinLogRow12)
      return fail(FLAME_ERR_UNSUPPORTED_SIZE, "row_pts = 12 needs n2 >= %d", 1 << flame::kMinLogRow12);
    if ((col_pts == 8 && gr.logn1 > flame::kMaxLog8) || (row_pts == 8 && gr.logn2 > flame::kMaxLog8))
      return fail(FLAME_ERR_UNSUPPORTED_SIZE, "8 points per thread needs lengths up to %d", 1 << flame::kMaxLog8);
  }
  if (!found) return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
  DeviceGuard g(p->device);
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    Group& gr = p->groups[gi];
    if ((1 << gr.logn1) != n1 || (1 << gr.logn2) != n2) continue;
    const bool cols_change = (gr.row_pts == 12) != (row_pts == 12);
    gr.col_pts = col_pts;
    gr.row_pts = row_pts;
    if (cols_change) {
      rc = apply_rows(p, (int)gi);
      if (rc) return rc;
    }
  }
  drop_graph(p);
  return FLAME_OK;
}

int flame_get_points_per_thread(flame_plan p, int32_t n1, int32_t n2, int32_t* col_pts, int32_t* row_pts) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!col_pts || !row_pts) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  for (const Group& gr : p->groups) {
    if ((1 << gr.logn1) == n1 && (1 << gr.logn2) == n2) {
      *col_pts = gr.col_pts;
      *row_pts = gr.row_pts;
      return FLAME_OK;
    }
  }
  return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
}

int flame_set_product_grid(flame_plan p, int32_t n1, int32_t n2, int32_t enable) {
  int rc = check_plan(p);
  if (rc) return rc;
  bool found = false;
  DeviceGuard g(p->device);
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    Group& gr = p->groups[gi];
    if ((1 << gr.logn1) != n1 || (1 << gr.logn2) != n2) continue;
    found = true;
    if (enable && gr.logn1 < flame::kMinLogProduct)
      return fail(FLAME_ERR_UNSUPPORTED_SIZE, "the product grid needs n1 >= %d", 1 << flame::kMinLogProduct);
    if (!enable && gr.col_pts == 12)
      return fail(FLAME_ERR_INVALID_ARG, "col_pts = 12 runs on the product grid: choose 8 or 16 points first");
    if (gr.product != (enable != 0)) {
      gr.product = enable != 0;
      rc = apply_rows(p, (int)gi);
      if (rc) return rc;
    }
  }
  if (!found) return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
  drop_graph(p);
  return FLAME_OK;
}

int flame_get_product_grid(flame_plan p, int32_t n1, int32_t n2, int32_t* enabled) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!enabled) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  for (const Group& gr : p->groups) {
    if ((1 << gr.logn1) == n1 && (1 << gr.logn2) == n2) {
      *enabled = gr.product ? 1 : 0;
      return FLAME_OK;
    }
  }
  return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
}

int flame_set_streaming_stores(flame_plan p, int32_t n1, int32_t n2, int32_t enable) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (enable < 0 || enable > 3) return fail(FLAME_ERR_INVALID_ARG, "store kind %d: 0, 1, 2 or 3", enable);
  bool found = false;
  for (Group& gr : p->groups) {
    if ((1 << gr.logn1) == n1 && (1 << gr.logn2) == n2) {
      gr.nt = enable;
      found = true;
    }
  }
  if (!found) return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
  DeviceGuard g(p->device);
  drop_graph(p);
  return FLAME_OK;
}

int flame_get_streaming_stores(flame_plan p, int32_t n1, int32_t n2, int32_t* enabled) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!enabled) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  for (const Group& gr : p->groups) {
    if ((1 << gr.logn1) == n1 && (1 << gr.logn2) == n2) {
      *enabled = gr.nt;
      return FLAME_OK;
    }
  }
  return fail(FLAME_ERR_INVALID_ARG, "no flame of grid %d x %d in this plan", n1, n2);
}

// A configuration replaces the default only if it runs in at most this
// fraction of the default's time.
constexpr float kAutotuneMargin = 0.98f;
// Rounds over all configurations (each keeps its fastest time; the first also
// runs while the GPU raises its clocks).
constexpr int kAutotuneRounds = 3;

struct TuneCfg {
  bool product;
  int c, r;
  int nt;  // store kind, as Group::nt
  bool operator==(const TuneCfg& o) const { return product == o.product && c == o.c && r == o.r && nt == o.nt; }
};

static std::vector<TuneCfg> tune_cfgs(const Group& gr) {
  std::vector<TuneCfg> cfgs;
  std::vector<int> rows = {16};
  if (gr.logn2 <= flame::kMaxLog8) rows.push_back(8);
  if (gr.logn2 >= flame::kMinLogRow12) rows.push_back(12);
  std::vector<int> cols = {16}, pcols = {16};
  if (gr.logn1 <= flame::kMaxLog8) {
    cols.push_back(8);
    pcols.push_back(8);
  }
  pcols.push_back(12);
  for (int nt : {0, 1}) {
    for (int c : cols)
      for (int r : rows) cfgs.push_back(TuneCfg{false, c, r, nt});
    if (gr.logn1 >= flame::kMinLogProduct)
      for (int c : pcols)
        for (int r : rows) cfgs.push_back(TuneCfg{true, c, r, nt});
  }
  return cfgs;
}

static int tune_select(flame_plan p, size_t gi, const TuneCfg& cf) {
  Group& gr = p->groups[gi];
  const bool grid_change = gr.product != cf.product || (gr.row_pts == 12) != (cf.r == 12);
  gr.col_pts = cf.c;
  gr.row_pts = cf.r;
  gr.nt = cf.nt;
  gr.product = cf.product;
  if (grid_change) return apply_rows(p, (int)gi);
  return FLAME_OK;
}

// Joint refinement for plans of several groups that step in graphs: in a
// replay the groups' chains run concurrently, so a group's fastest choice
// alone need not be the fastest beside the others. Each trial runs `steps`
// steps of every group at once, each group's chain on a stream of its own
// (forked from and joined back to the plan's stream, as a replay's branches
// are), and coordinate descent over the groups keeps a change only if the
// trial's time falls below kAutotuneMargin of the best so far.
static int autotune_jointly(flame_plan p, int steps, long long n0, hipEvent_t ev0, hipEvent_t ev1) {
  const size_t ng = p->groups.size();
  std::vector<hipStream_t> st(ng, nullptr);
  std::vector<hipEvent_t> done(ng, nullptr);
  hipEvent_t fork = nullptr;
  int rc = FLAME_OK;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (size_t gi = 0; e == hipSuccess && gi < ng; ++gi) {
    e = hipStreamCreateWithFlags(&st[gi], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&done[gi], hipEventDisableTiming);
  }
  if (e != hipSuccess) rc = hip_fail(e, "autotune streams");
  auto trial = [&](float* ms) -> int {
    for (int f = 0; f < p->nfl; ++f)
      if (!p->w_valid[f]) {
        const int r = rebuild_w(p, f);
        if (r) return r;
      }
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {  // the first repetition warms up
      hipError_t e2 = hipEventRecord(ev0, p->stream);
      if (e2 == hipSuccess) e2 = hipEventRecord(fork, p->stream);
      for (size_t gi = 0; e2 == hipSuccess && gi < ng; ++gi) {
        e2 = hipStreamWaitEvent(st[gi], fork, 0);
        const Group& gr = p->groups[gi];
        for (int s = 0; e2 == hipSuccess && s < steps; ++s)
          for (int pass = 0; pass < gr.passes(); ++pass) {
            launch_step_row(p, gr, n0, nullptr, nullptr, st[gi]);
            launch_step_col(p, gr, n0, pass, nullptr, nullptr, st[gi]);
          }
        if (e2 == hipSuccess) e2 = hipEventRecord(done[gi], st[gi]);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(p->stream, done[gi], 0);
      }
      if (e2 == hipSuccess) e2 = hipEventRecord(ev1, p->stream);
      if (e2 == hipSuccess) e2 = hipEventSynchronize(ev1);
      float t = 0.f;
      if (e2 == hipSuccess) e2 = hipEventElapsedTime(&t, ev0, ev1);
      if (e2 != hipSuccess) return hip_fail(e2, "autotune joint timing");
      if (rep > 0) best = std::min(best, t);
    }
    *ms = best;
    return last_launch("autotune joint launch");
  };
  float best_all = 0.f;
  if (rc == FLAME_OK) rc = trial(&best_all);
  for (int round = 0; rc == FLAME_OK && round < 2; ++round) {
    bool improved = false;
    for (size_t gi = 0; rc == FLAME_OK && gi < ng; ++gi) {
      const Group& gr = p->groups[gi];
      const TuneCfg cur{gr.product, gr.col_pts, gr.row_pts, gr.nt};
      TuneCfg keep = cur;
      for (const TuneCfg& cf : tune_cfgs(gr)) {
        if (cf == cur) continue;
        rc = tune_select(p, gi, cf);
        float t = 0.f;
        if (rc == FLAME_OK) rc = trial(&t);
        if (rc) break;
        if (t < kAutotuneMargin * best_all) {
          best_all = t;
          keep = cf;
          improved = true;
        }
      }
      if (rc == FLAME_OK) rc = tune_select(p, gi, keep);
    }
    if (!improved) break;
  }
  // every stream has drained: ev1 was synchronised after the last trial
  if (rc == FLAME_OK) {
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) rc = hip_fail(e, "autotune joint sync");
  }
  for (size_t gi = 0; gi < ng; ++gi) {
    if (st[gi]) (void)hipStreamSynchronize(st[gi]);
    if (done[gi]) (void)hipEventDestroy(done[gi]);
    if (st[gi]) (void)hipStreamDestroy(st[gi]);
  }
  if (fork) (void)hipEventDestroy(fork);
  return rc;
}

// Each group alone: time every configuration of tune_cfgs in kAutotuneRounds
// rounds (keeping each one's fastest time: in the first round the early
// configurations run on a GPU that is still raising its clocks), then select
// the fastest unless the default (16 points per thread, product grid where it
// exists, plain stores) is within kAutotuneMargin of it, so that choices
// within timing noise of each other do not flip between runs. If the choice
// has both Q and W non-temporal, the same kernels with only one of them
// non-temporal are timed too (as many rounds), and the faster of those is kept
// if it is within the margin: non-temporal pieces of half a line are written
// back unmerged, so one non-temporal buffer moves fewer bytes than two.
static int autotune_alone(flame_plan p, size_t gi, int steps, long long n0, hipEvent_t ev0, hipEvent_t ev1,
                          int* tried) {
  const Group& gr = p->groups[gi];
  auto time_cfg = [&](const TuneCfg& cf, float* out) -> int {
    int rc = tune_select(p, gi, cf);
    for (int f = gr.first; rc == FLAME_OK && f < gr.first + gr.count; ++f)
      if (!p->w_valid[f]) rc = rebuild_w(p, f);
    if (rc) return rc;
    // one untimed step, then `steps` timed steps of this group alone
    hipError_t e = hipSuccess;
    for (int s = 0; s <= steps; ++s) {
      if (s == 1) e = hipEventRecord(ev0, p->stream);
      for (int pass = 0; pass < gr.passes(); ++pass) {
        launch_step_row(p, gr, n0);
        launch_step_col(p, gr, n0, pass);
      }
    }
    if (e == hipSuccess) e = hipEventRecord(ev1, p->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    rc = last_launch("autotune launch");
    if (rc) return rc;
    *out = std::min(*out, ms);
    return FLAME_OK;
  };
  const std::vector<TuneCfg> cfgs = tune_cfgs(gr);
  const TuneCfg default_cfg{gr.logn1 >= flame::kMinLogProduct, ff::kPts, ff::kPts, 0};
  std::vector<float> t_best(cfgs.size(), 1e30f);
  for (int round = 0; round < kAutotuneRounds; ++round) {
    for (size_t ci = 0; ci < cfgs.size(); ++ci) {
      const int rc = time_cfg(cfgs[ci], &t_best[ci]);
      if (rc) return rc;
      if (round == 0) ++*tried;
    }
  }
  size_t best = 0, dflt = 0;
  for (size_t ci = 0; ci < cfgs.size(); ++ci) {
    if (t_best[ci] < t_best[best]) best = ci;
    if (cfgs[ci] == default_cfg) dflt = ci;
  }
  if (t_best[best] > kAutotuneMargin * t_best[dflt]) best = dflt;
  TuneCfg pick = cfgs[best];
  if (pick.nt == 1) {
    const TuneCfg alt[2] = {TuneCfg{pick.product, pick.c, pick.r, 2}, TuneCfg{pick.product, pick.c, pick.r, 3}};
    float t_alt[2] = {1e30f, 1e30f};
    for (int round = 0; round < kAutotuneRounds; ++round)
      for (int k = 0; k < 2; ++k) {
        const int rc = time_cfg(alt[k], &t_alt[k]);
        if (rc) return rc;
        if (round == 0) ++*tried;
      }
    const int k = t_alt[0] <= t_alt[1] ? 0 : 1;
    if (kAutotuneMargin * t_alt[k] <= t_best[best]) pick = alt[k];
  }
  return tune_select(p, gi, pick);
}

int flame_autotune(flame_plan p, int32_t steps, int32_t* n_configs_tried) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (steps <= 0) return fail(FLAME_ERR_INVALID_ARG, "steps must be > 0");
  if (p->persistent)
    return fail(FLAME_ERR_INVALID_ARG, "the persistent launch runs fixed kernels: disable it before autotuning");
  rc = check_r0(p, 0, p->nfl, p->n, p->n, true);  // every timed step runs at the current index
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e != hipSuccess) {
    if (ev0) (void)hipEventDestroy(ev0);
    return hip_fail(e, "autotune events");
  }
  // save every state in its flame's adjoint scratch (each at least 2x the state)
  auto state_bytes = [&](int f) { return (size_t)(p->descs[f].n2 / 4) * (p->descs[f].n1 / 2) * sizeof(float2); };
  for (int f = 0; e == hipSuccess && f < p->nfl; ++f)
    e = hipMemcpyAsync(p->hdev[f].A1, p->hdev[f].S, state_bytes(f), hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    return hip_fail(e, "autotune save");
  }
  const long long n0 = p->n;
  const int saved_graph = p->graph_steps;
  drop_graph(p);
  p->graph_steps = 0;
  int tried = 0;
  for (int f = 0; rc == FLAME_OK && f < p->nfl; ++f)
    if (!p->w_valid[f]) rc = rebuild_w(p, f);
  for (size_t gi = 0; rc == FLAME_OK && gi < p->groups.size(); ++gi)
    rc = autotune_alone(p, gi, steps, n0, ev0, ev1, &tried);
  if (rc == FLAME_OK && saved_graph > 0 && p->groups.size() > 1) rc = autotune_jointly(p, steps, n0, ev0, ev1);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  // restore every state and the step index, after a failed trial too
  for (int f = 0; f < p->nfl; ++f) {
    e = hipMemcpyAsync(p->hdev[f].S, p->hdev[f].A1, state_bytes(f), hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess && rc == FLAME_OK) rc = hip_fail(e, "autotune restore");
    p->w_valid[f] = 0;
  }
  p->n = n0;
  p->graph_steps = saved_graph;
  if (rc) return rc;
  if (n_configs_tried) *n_configs_tried = tried;
  return FLAME_OK;
}

int flame_set_graph_steps(flame_plan p, int32_t steps) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (steps < 0) return fail(FLAME_ERR_INVALID_ARG, "steps per graph must be >= 0");
  if (steps != p->graph_steps) {
    DeviceGuard g(p->device);
    drop_graph(p);
    drop_ens_graph(p);
    p->graph_steps = steps;
  }
  return FLAME_OK;
}

int flame_set_persistent(flame_plan p, int32_t enable, int32_t workgroups, int32_t wait_limit_us) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (enable != 0 && enable != 1) return fail(FLAME_ERR_INVALID_ARG, "enable must be 0 or 1");
  if (workgroups < 0) return fail(FLAME_ERR_INVALID_ARG, "workgroups must be >= 0");
  if (wait_limit_us < 0) return fail(FLAME_ERR_INVALID_ARG, "wait_limit_us must be >= 0");
  DeviceGuard g(p->device);
  drop_ens_graph(p);  // it bakes in the grid size and the wait limit
  if (!enable) {
    p->persistent = false;
    return FLAME_OK;
  }
  rc = ens_check(p);
  if (rc) return rc;
  int coop = 0, khz = 0;
  hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (!coop) return fail(FLAME_ERR_UNSUPPORTED_SIZE, "the device has no cooperative launches");
  if (khz <= 0) return fail(FLAME_ERR_HIP, "the device reports no wall-clock rate");
  const long long us = wait_limit_us > 0 ? wait_limit_us : kEnsDefaultWaitUs;
  p->ens_limit = (unsigned long long)us * (unsigned long long)khz / 1000ULL;
  p->ens_wgs = workgroups;
  p->persistent = true;
  return FLAME_OK;
}

int flame_get_persistent(flame_plan p, int32_t* enabled, int32_t* workgroups) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!enabled || !workgroups) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  *enabled = p->persistent ? 1 : 0;
  *workgroups = p->persistent ? (int32_t)p->ens_items.size() : 0;
  return FLAME_OK;
}

int flame_timing_end(flame_plan p, double* ms4, int64_t* counts4) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!ms4 || !counts4) return fail(FLAME_ERR_INVALID_ARG, "null output pointer");
  DeviceGuard g(p->device);
  p->timing = false;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "timing synchronise");
  for (int k = 0; k < 4; ++k) {
    double total = 0.0;
    const auto& v = p->ev_used[k];
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, v[i], v[i + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      total += ms;
    }
    ms4[k] = total;
    counts4[k] = (int64_t)(v.size() / 2);
  }
  return FLAME_OK;
}

int flame_destroy(flame_plan p) {
  if (!p) return fail(FLAME_ERR_INVALID_ARG, "null plan");
  {
    // the plan's graph and events may still be in use by queued work
    DeviceGuard g(p->device);
    (void)hipStreamSynchronize(p->stream);
  }
  delete p;
  return FLAME_OK;
}

}  // extern "C"
