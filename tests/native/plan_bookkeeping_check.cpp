// Host-sanitizer drive of the library's plan, graph and event bookkeeping.
//
// flame_api.hip is compiled for the host against tests/native/hipstub (a
// checked model of the HIP calls it makes) with -fsanitize=address,undefined
// and driven through long sequences of the calls that build, replay, drop and
// rebuild step graphs and that take and return timing events: points per
// thread, grids, store kinds, forcing, graph lengths, timing, autotuning
// (alone and jointly, with graphs set), adjoint calls and plan teardown.
// Prints "ALL OK" when every call succeeded; the sanitizers or the stub abort
// on any heap error or misuse. With the argument "control" it instead queues
// a graph launch and destroys its exec without waiting, which the stub must
// report (a check that the model catches that pattern).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "flame.h"

long hip_stub_count(int what);

namespace {

#define CHECK(x)                                                                              \
  do {                                                                                        \
    const int rc_ = (x);                                                                      \
    if (rc_ != FLAME_OK) {                                                                    \
      std::fprintf(stderr, "%s:%d: %s returned %d: %s\n", __FILE__, __LINE__, #x, rc_,       \
                   flame_last_error());                                                       \
      std::exit(3);                                                                           \
    }                                                                                         \
  } while (0)

flame_desc desc(int n1, int n2, int integrator = 0, int r0_law = 0) {
  flame_desc d;
  std::memset(&d, 0, sizeof d);
  d.n1 = n1;
  d.n2 = n2;
  d.gamma = 0.8;
  d.theta_pi = 1.0;
  d.t0 = 200.0;
  d.dt = 0.25;
  d.r0_law = r0_law;
  d.integrator = integrator;
  return d;
}

void* aligned(size_t bytes, size_t align = 256) {
  void* p = std::aligned_alloc(align, (bytes + align - 1) / align * align);
  if (!p) std::exit(4);
  std::memset(p, 0, bytes);
  return p;
}

struct Plan {
  std::vector<flame_desc> d;
  std::vector<void*> states;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  flame_plan p = nullptr;
  std::vector<double> r0tab;
  Plan(std::vector<flame_desc> descs, hipStream_t st) : d(std::move(descs)) {
    for (const flame_desc& x : d) {
      size_t b = 0;
      CHECK(flame_state_bytes(&x, &b));
      states.push_back(aligned(b, 16));
    }
    CHECK(flame_workspace_bytes(d.data(), (int)d.size(), &ws_bytes));
    ws = aligned(ws_bytes);
    CHECK(flame_init(d.data(), (int)d.size(), states.data(), ws, ws_bytes, st, &p));
  }
  ~Plan() {
    if (p) CHECK(flame_destroy(p));
    for (void* s : states) std::free(s);
    std::free(ws);
  }
};

int control() {
  hipStream_t st = nullptr;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  hipGraph_t g = nullptr;
  hipGraphCreate(&g, 0);
  const char k = 0;
  long long n = 0;
  void* a0 = nullptr;
  void* args[] = {&a0, &n, &a0, &a0};
  hipKernelNodeParams prm{};
  prm.func = const_cast<char*>(&k);
  prm.kernelParams = args;
  hipGraphNode_t node;
  hipGraphAddKernelNode(&node, g, nullptr, 0, &prm);
  hipGraphExec_t x = nullptr;
  hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  hipGraphLaunch(x, st);
  hipGraphExecDestroy(x);  // without waiting for the stream: the stub must object
  std::printf("control: not caught\n");
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "control") == 0) return control();
  hipStream_t st = nullptr;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);

  for (int round = 0; round < 3; ++round) {
    // four groups: two equal small grids, a product grid, a Heun flame, a tabulated-radius flame
    Plan pl({desc(64, 128), desc(64, 128), desc(256, 512), desc(256, 512, 1), desc(128, 64, 0, 1)},
            round == 1 ? nullptr : st);
    flame_plan p = pl.p;
    pl.r0tab.assign(3 * 4000, 0.0);
    for (int i = 0; i < 4000; ++i) {
      const double t = 200.0 + 0.25 * i;
      pl.r0tab[3 * i] = t;
      pl.r0tab[3 * i + 1] = 0.25 / t;
      pl.r0tab[3 * i + 2] = 0.25 / (t * t);
    }
    CHECK(flame_set_r0_table(p, 4, pl.r0tab.data(), 4000));
    std::vector<float> spec(64 * 512 * 2, 0.f);
    for (int f = 0; f < 5; ++f) CHECK(flame_set_spectrum(p, f, spec.data(), 0));
    CHECK(flame_step(p, 3));
    for (int gs : {4, 1, 7, 0, 3}) {
      CHECK(flame_set_graph_steps(p, gs));
      CHECK(flame_step(p, 10));
    }
    // graph rebuilds between replays, as a tuner timing one configuration per graph would do
    for (int it = 0; it < 60; ++it) {
      const int cp = it % 3 == 0 ? 12 : (it % 3 == 1 ? 16 : 8);
      CHECK(flame_set_points_per_thread(p, 256, 512, cp, it % 2 ? 12 : 16));
      CHECK(flame_set_streaming_stores(p, 64, 128, it % 2));
      CHECK(flame_step(p, 3 + it % 5));
      if (it % 7 == 0) {
        CHECK(flame_set_points_per_thread(p, 256, 512, 16, 16));
        CHECK(flame_set_product_grid(p, 128, 64, it % 2));
      }
      if (it % 5 == 0) CHECK(flame_set_forcing(p, 0, spec.data()));
      if (it % 5 == 2) CHECK(flame_set_forcing(p, 0, nullptr));
      if (it % 11 == 0) CHECK(flame_set_graph_steps(p, 1 + it % 4));
    }
    // timing sessions, including one left open at destruction
    double ms[4];
    int64_t cnt[4];
    double out4[4 * 5];
    std::vector<float> seed(256 * 512, 0.f);  // the adjoint seed of any flame of the plan
    for (int it = 0; it < 20; ++it) {
      CHECK(flame_timing_begin(p));
      CHECK(flame_step(p, 1 + it % 4));
      CHECK(flame_diagnostics(p, it % 5, out4, it % 4 == 1 ? seed.data() : nullptr));
      if (it % 3) CHECK(flame_timing_end(p, ms, cnt));
    }
    // autotuning alone and jointly (graphs set, several groups)
    int tried = 0;
    CHECK(flame_autotune(p, 2, &tried));
    CHECK(flame_set_graph_steps(p, 0));
    CHECK(flame_autotune(p, 1, &tried));
    CHECK(flame_set_graph_steps(p, 5));
    CHECK(flame_step(p, 11));
    // adjoint, gradient, synthesis and state I/O
    std::vector<float> lam(64 * 128 * 2, 0.f), phi(256 * 512, 0.f);
    CHECK(flame_adjoint_step(p, 0, 2, pl.states[0], lam.data(), lam.data()));
    CHECK(flame_area_gradient(p, 2, 3, pl.states[2], lam.data()));
    CHECK(flame_synthesize(p, 2, pl.states[2], phi.data()));
    CHECK(flame_get_state(p, 2, phi.data()));
    CHECK(flame_set_state(p, 2, phi.data(), 5));
    CHECK(flame_state_modified(p, 2, 5));
    CHECK(flame_state_modified(p, -1, 5));
    if (flame_state_modified(p, 5, 5) != FLAME_ERR_INVALID_ARG) return 7;
    CHECK(flame_step(p, 6));
    CHECK(flame_timing_begin(p));
    CHECK(flame_step(p, 7));
  }
  // persistent launches: the bench ensemble's grids and an uneven mix, on
  // every grid size, with the configuration changed between steps
  {
    std::vector<flame_desc> ds;
    for (int i = 0; i < 128; ++i) ds.push_back(desc(128, 256));
    for (int i = 0; i < 96; ++i) ds.push_back(desc(256, 512));
    for (int i = 0; i < 32; ++i) ds.push_back(desc(512, 1024));
    Plan pl(ds, st);
    const int grids[3][2] = {{128, 256}, {256, 512}, {512, 1024}};
    for (const auto& g : grids) CHECK(flame_set_points_per_thread(pl.p, g[0], g[1], 12, 16));
    CHECK(flame_set_persistent(pl.p, 1, 0, 0));
    if (flame_autotune(pl.p, 1, nullptr) != FLAME_ERR_INVALID_ARG) return 8;
    CHECK(flame_step(pl.p, 3));
    int32_t on = 0, wgs = 0;
    CHECK(flame_get_persistent(pl.p, &on, &wgs));
    if (on != 1 || wgs != 512) {
      std::fprintf(stderr, "persistent grid %d (enabled %d), expected 512\n", wgs, on);
      return 5;
    }
    for (int w : {3, 7, 100, 300, 512, 0}) {
      CHECK(flame_set_persistent(pl.p, 1, w, 50));
      CHECK(flame_step(pl.p, 2));
    }
    // graph replays of the persistent launch, rebuilt on every setting that bakes into them
    for (int gs : {5, 3, 1000, 1001, 0, 7}) {
      CHECK(flame_set_graph_steps(pl.p, gs));
      CHECK(flame_step(pl.p, 11));
      CHECK(flame_set_persistent(pl.p, 1, gs == 7 ? 100 : 0, 0));
      CHECK(flame_step(pl.p, 7));
    }
    // a configuration the persistent kernel lacks is refused, then restored
    CHECK(flame_set_points_per_thread(pl.p, 256, 512, 16, 16));
    if (flame_step(pl.p, 1) != FLAME_ERR_INVALID_ARG) return 6;
    CHECK(flame_set_points_per_thread(pl.p, 256, 512, 12, 16));
    CHECK(flame_step(pl.p, 1001));
    CHECK(flame_set_persistent(pl.p, 0, 0, 0));
    CHECK(flame_step(pl.p, 2));
  }
  {
    std::vector<flame_desc> ds = {desc(1024, 2048), desc(128, 128), desc(128, 128), desc(128, 128),
                                  desc(512, 256),   desc(256, 2048)};
    Plan pl(ds, st);
    for (const flame_desc& d : ds) CHECK(flame_set_points_per_thread(pl.p, d.n1, d.n2, 12, 16));
    for (int w : {0, 4, 6, 40}) {
      CHECK(flame_set_persistent(pl.p, 1, w, 0));
      CHECK(flame_step(pl.p, 4));
    }
  }
  // the allocation-free step and the circles
  {
    flame_desc d = desc(256, 512);
    std::vector<float> s(256 * 512 / 4, 0.f);
    CHECK(flame_step_noalloc(&d, s.data(), 0, 4, st));
    CHECK(flame_step_noalloc(&d, s.data(), 4, 0, st));
    flame_circle_desc c{1024, 0.8, 1.0, 200.0, 0.25};
    std::vector<float> cs(7 * 256 * 2, 0.f);
    CHECK(flame_circle_step(&c, 7, cs.data(), 0, 4500, st));
    std::vector<double> co(7 * 4);
    CHECK(flame_circle_diagnostics(&c, 7, cs.data(), 4500, co.data(), st));
  }
  hipStreamSynchronize(st);
  hipStreamDestroy(st);
  std::printf("launches %ld, graph launches %ld, synchronisations %ld\n", hip_stub_count(0), hip_stub_count(1),
              hip_stub_count(2));
  std::printf("ALL OK\n");
  return 0;
}
