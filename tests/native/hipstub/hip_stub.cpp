// Checked model of the HIP runtime calls that flame_api.hip makes, for the
// host-sanitizer build of the library's bookkeeping. Device memory is host
// memory; copies happen at once; kernels do not run, but every launch reads
// its flame table (so an offset outside the caller's workspace is an
// out-of-bounds read for the address sanitizer) and queues a reference on
// its stream. Streams keep the graph execs and events queued on them until a
// synchronisation completes them. Misuse aborts with a message:
//  * any call on a destroyed or unknown stream, event, graph or graph exec;
//  * hipGraphExecDestroy of an exec whose launch is still queued on a stream
//    (the runtime may still be using it);
//  * hipEventElapsedTime of an event that was never recorded or not completed;
//  * hipGraphAddKernelNode whose kernel-argument pointers are unreadable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "flame_kernels.hpp"

dim3 threadIdx, blockIdx, blockDim, gridDim;

struct ihipStream_t {
  int id;
};
struct ihipEvent_t {
  int id;
  bool recorded = false, done = false;
};
struct ihipGraph {
  int id;
  std::vector<std::vector<uint64_t>> nodes;  // kernel arguments copied at insertion
  std::vector<hipGraphNode*> owned;          // node handles, freed with the graph
};
struct hipGraphExec {
  int id;
  size_t nodes;
};
struct hipGraphNode {
  int id;
};

namespace {

std::set<ihipStream_t*> g_streams;
std::set<ihipEvent_t*> g_events;
std::set<ihipGraph*> g_graphs;
std::set<hipGraphExec*> g_execs;
std::vector<hipGraphNode*> g_nodes;
// work queued per stream (the null stream is key nullptr): graph execs and events
std::map<ihipStream_t*, std::vector<hipGraphExec*>> g_pending_exec;
std::map<ihipStream_t*, std::vector<ihipEvent_t*>> g_pending_event;
int g_next = 1;
long g_launches = 0, g_graph_launches = 0, g_syncs = 0;

[[noreturn]] void violation(const char* what) {
  std::fprintf(stderr, "HIP STUB VIOLATION: %s\n", what);
  std::fflush(stderr);
  std::abort();
}

void check_stream(hipStream_t s) {
  if (s && !g_streams.count(s)) violation("use of a destroyed or unknown stream");
}
void check_event(hipEvent_t e) {
  if (!e || !g_events.count(e)) violation("use of a destroyed or unknown event");
}

void complete_stream(hipStream_t s) {
  g_pending_exec[s].clear();
  for (ihipEvent_t* e : g_pending_event[s]) e->done = true;
  g_pending_event[s].clear();
  ++g_syncs;
}

}  // namespace

long hip_stub_count(int what) { return what == 0 ? g_launches : (what == 1 ? g_graph_launches : g_syncs); }

// a launch or copy on `s` completes only at the next synchronisation
void hip_stub_launch(const void* kernel, hipStream_t s) {
  if (!kernel) violation("launch of a null kernel");
  check_stream(s);
  ++g_launches;
}

hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  switch (a) {
    case hipDeviceAttributeMaxSharedMemoryPerBlock: *v = 160 * 1024; break;
    case hipDeviceAttributeMultiprocessorCount: *v = 256; break;
    case hipDeviceAttributeWallClockRate: *v = 100000; break;
    case hipDeviceAttributeCooperativeLaunch: *v = 1; break;
    default: *v = 0;
  }
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  check_stream(s);
  if (n) std::memmove(dst, src, n);  // both sides are host memory here
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  check_stream(s);
  complete_stream(s);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t{g_next++};
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!g_streams.count(s)) violation("destroy of a destroyed or unknown stream");
  complete_stream(s);  // the runtime waits for its work
  g_streams.erase(s);
  g_pending_exec.erase(s);
  g_pending_event.erase(s);
  delete s;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  check_stream(s);
  check_event(e);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t{g_next++};
  g_events.insert(*e);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  check_event(e);
  // the runtime releases a pending event once it completes; drop its queue entries
  for (auto& kv : g_pending_event) kv.second.erase(std::remove(kv.second.begin(), kv.second.end(), e), kv.second.end());
  g_events.erase(e);
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  check_event(e);
  check_stream(s);
  e->recorded = true;
  e->done = false;
  g_pending_event[s].push_back(e);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  check_event(e);
  if (!e->recorded) violation("hipEventSynchronize of an event never recorded");
  // complete the stream that holds it, up to and including it
  for (auto& kv : g_pending_event) {
    auto it = std::find(kv.second.begin(), kv.second.end(), e);
    if (it == kv.second.end()) continue;
    for (auto j = kv.second.begin(); j <= it; ++j) (*j)->done = true;
    kv.second.erase(kv.second.begin(), it + 1);
    g_pending_exec[kv.first].clear();
  }
  e->done = true;
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  check_event(a);
  check_event(b);
  if (!a->recorded || !b->recorded) violation("hipEventElapsedTime of an event never recorded");
  if (!a->done || !b->done) violation("hipEventElapsedTime of an event not completed");
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipGraphCreate(hipGraph_t* g, unsigned) {
  *g = new ihipGraph{g_next++, {}};
  g_graphs.insert(*g);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  if (!g_graphs.count(g)) violation("destroy of a destroyed or unknown graph");
  for (hipGraphNode* nd : g->owned) {
    g_nodes.erase(std::remove(g_nodes.begin(), g_nodes.end(), nd), g_nodes.end());
    delete nd;
  }
  g_graphs.erase(g);
  delete g;
  return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p) {
  if (!g_graphs.count(g)) violation("kernel node added to a destroyed or unknown graph");
  if (!p || !p->func || !p->kernelParams) violation("kernel node without a kernel or arguments");
  for (size_t i = 0; i < ndeps; ++i)
    if (!deps || std::find(g_nodes.begin(), g_nodes.end(), deps[i]) == g_nodes.end())
      violation("kernel node depends on an unknown node");
  // the runtime copies the arguments now; every kernel the library puts in a
  // graph takes a device pointer first (its sizes beyond that vary)
  std::vector<uint64_t> args;
  uint64_t v;
  std::memcpy(&v, p->kernelParams[0], sizeof v);
  args.push_back(v);
  g->nodes.push_back(args);
  *node = new hipGraphNode{g_next++};
  g->owned.push_back(*node);
  g_nodes.push_back(*node);
  return hipSuccess;
}
hipError_t hipGraphKernelNodeSetAttribute(hipGraphNode_t node, hipKernelNodeAttrID attr,
                                          const hipKernelNodeAttrValue* value) {
  if (std::find(g_nodes.begin(), g_nodes.end(), node) == g_nodes.end()) violation("attribute of an unknown node");
  if (attr != hipKernelNodeAttributeCooperative || !value) violation("unexpected kernel node attribute");
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  if (!g_graphs.count(g)) violation("instantiation of a destroyed or unknown graph");
  *x = new hipGraphExec{g_next++, g->nodes.size()};
  g_execs.insert(*x);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  if (!g_execs.count(x)) violation("destroy of a destroyed or unknown graph exec");
  for (auto& kv : g_pending_exec)
    if (std::find(kv.second.begin(), kv.second.end(), x) != kv.second.end())
      violation("graph exec destroyed while a launch of it is still queued");
  g_execs.erase(x);
  delete x;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (!g_execs.count(x)) violation("launch of a destroyed or unknown graph exec");
  check_stream(s);
  g_pending_exec[s].push_back(x);
  ++g_graph_launches;
  return hipSuccess;
}

// ------------------------------------------------------------ kernel launchers
// Each reads the flame table it is given (the device table lives in the
// caller's workspace) and checks the events it records.

namespace flame {

namespace {
const char kDummyKernel[1] = {0};

void touch(const FlameDev* fl, int nfl) {
  volatile char sink = 0;
  for (int f = 0; f < nfl; ++f) {
    FlameDev d;
    std::memcpy(&d, fl + f, sizeof d);
    sink = sink + (char)d.n1;
  }
  (void)sink;
}

void timed(hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (e0) hipEventRecord(e0, st);
  if (e1) hipEventRecord(e1, st);
}
}  // namespace

KernelLaunch col_step_kernel(int, int pts, int) { return KernelLaunch{pts == 12 ? nullptr : kDummyKernel, 256, 0}; }
KernelLaunch row_step_kernel(int, int, bool) { return KernelLaunch{kDummyKernel, 256, 0}; }
KernelLaunch colp_kernel_info(int logn1, int, int, int) {
  return KernelLaunch{logn1 >= kMinLogProduct ? kDummyKernel : nullptr, 256, 0};
}
void launch_set_step(hipStream_t st, long long* counter, long long value) {
  *counter = value;
  hip_stub_launch(kDummyKernel, st);
}
int lds_bytes_needed(int, int) { return 1024; }
void launch_col(int, int, int, int nfl, hipStream_t st, const FlameDev* fl, long long, const void*, int, hipEvent_t e0,
                hipEvent_t e1, int) {
  touch(fl, nfl);
  timed(st, e0, e1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_colp(int, int, int, int nfl, hipStream_t st, const FlameDev* fl, long long, const void*, int,
                 hipEvent_t e0, hipEvent_t e1, int) {
  touch(fl, nfl);
  timed(st, e0, e1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_row(int, int, int, int nfl, hipStream_t st, const FlameDev* fl, long long, const float*, float*, int,
                hipEvent_t e0, hipEvent_t e1, bool) {
  touch(fl, nfl);
  timed(st, e0, e1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_adj_col(int, int, int, hipStream_t st, const FlameDev* fl, long long, const void*, const void*, void*) {
  touch(fl, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_adj_row(int, int, int, hipStream_t st, const FlameDev* fl, long long) {
  touch(fl, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_adjp_col(int, int, int, hipStream_t st, const FlameDev* fl, long long, const void*, const void*, void*) {
  touch(fl, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_set_spectrum(hipStream_t st, const FlameDev* fl, int flame, int, const void*) {
  touch(fl + flame, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_get_spectrum(hipStream_t st, const FlameDev* fl, int flame, int, void*) {
  touch(fl + flame, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_diag_spectral(hipStream_t st, const FlameDev* fl, int flame, int, double*) {
  touch(fl + flame, 1);
  hip_stub_launch(kDummyKernel, st);
}
void launch_diag_final(hipStream_t st, const FlameDev* fl, int flame, long long, int, int, double*) {
  touch(fl + flame, 1);
  hip_stub_launch(kDummyKernel, st);
}
bool ensemble_supports(int logn1, int logn2) {
  return logn1 >= kEnsMinLog1 && logn1 <= kEnsMaxLog1 && logn2 >= kEnsMinLog2 && logn2 <= kEnsMaxLog2;
}
KernelLaunch ensemble_kernel_info() { return KernelLaunch{kDummyKernel, kEnsThreads, 1024}; }
KernelLaunch ensemble_reset_info() { return KernelLaunch{kDummyKernel, 256, 0}; }
void launch_ensemble_reset(hipStream_t st, unsigned* arrive, int narrive, int* err, bool clear_err) {
  std::memset(arrive, 0, sizeof(unsigned) * (size_t)narrive);
  if (clear_err) *err = 0;
  hip_stub_launch(kDummyKernel, st);
}
int ensemble_blocks_per_cu() { return 2; }
// Reads every item and the flames it names, and checks the partition: every
// flame is stepped either whole by exactly one item or by parts 0 .. parts-1,
// each exactly once, and its arrival counter lies inside the counter array.
hipError_t launch_ensemble(hipStream_t st, const FlameDev* fls, const EnsembleItem* items, int nitems,
                           unsigned* arrive, int narrive, int* err, long long, int steps, unsigned long long) {
  if (nitems <= 0 || nitems > 2 * 256) violation("persistent grid outside the co-resident capacity");
  if (steps <= 0) violation("persistent launch of no steps");
  if (narrive % kEnsArriveStride) violation("arrival counters not a whole number of flames");
  const int nfl = narrive / kEnsArriveStride;
  std::vector<std::vector<int>> seen(nfl);
  for (int i = 0; i < nitems; ++i) {
    EnsembleItem it;
    std::memcpy(&it, items + i, sizeof it);
    if (it.flame < 0 || it.nfl < 1 || it.flame + it.nfl > nfl) violation("persistent item names flames outside the plan");
    if (it.parts < 1 || it.part < 0 || it.part >= it.parts) violation("persistent item part out of range");
    if (it.parts > 1 && it.nfl != 1) violation("a shared persistent item holds several flames");
    if (it.parts > 1 && it.parts > (it.rtiles > it.ctiles ? it.rtiles : it.ctiles))
      violation("more parts than tiles in a phase");
    touch(fls + it.flame, it.nfl);
    for (int f = it.flame; f < it.flame + it.nfl; ++f) {
      FlameDev d;
      std::memcpy(&d, fls + f, sizeof d);
      if (d.n1 != 1 << it.logn1 || d.n2 != 1 << it.logn2) violation("persistent item grid differs from its flame's");
      if (seen[f].empty()) seen[f].assign(it.parts, 0);
      if ((int)seen[f].size() != it.parts) violation("flame split into differing part counts");
      ++seen[f][it.part];
    }
  }
  for (int f = 0; f < nfl; ++f) {
    if (seen[f].empty()) violation("flame left out of the persistent partition");
    for (int c : seen[f])
      if (c != 1) violation("flame part stepped other than once");
  }
  std::memset(arrive, 0, sizeof(unsigned) * (size_t)narrive);
  (void)err;
  hip_stub_launch(kDummyKernel, st);
  hip_stub_launch(kDummyKernel, st);
  return hipSuccess;
}
bool launch_circle_step(int, const CircleDev&, long long, int, hipStream_t st) {
  hip_stub_launch(kDummyKernel, st);
  return true;
}
bool launch_circle_diag(int, const CircleDev&, long long, double*, hipStream_t st) {
  hip_stub_launch(kDummyKernel, st);
  return true;
}

}  // namespace flame
