// Persistent ensemble kernel of the flame step (gfx950): the steps of every
// flame of a plan in one launch whose workgroups are all resident at once (a
// cooperative launch). Each workgroup runs the bodies of the step kernels
// (step_bodies.hpp) on the row-pair groups and column tiles of its
// EnsembleItem, step after step. A flame stepped by one workgroup needs only
// that workgroup's barriers between its phases; a flame shared by several
// meets at its arrival counter after each phase, because the column pass of
// step n reads Q of all its rows and the row pass of step n + 1 reads W of
// all its columns (Section 3: each transform pass needs the whole output of
// the one before it).

#include <hip/hip_runtime.h>

#include "flame_dev.hpp"
#include "flame_kernels.hpp"
#include "step_bodies.hpp"

namespace flame {

static_assert(ColCfg<kEnsMinLog1, 12>::THREADS == kEnsThreads && ColCfg<kEnsMaxLog1, 12>::THREADS == kEnsThreads,
              "column bodies of the ensemble kernel: 256 threads");
static_assert(RowCfg<kEnsMinLog2, 16>::THREADS == kEnsThreads && RowCfg<kEnsMaxLog2, 16>::THREADS == kEnsThreads,
              "row bodies of the ensemble kernel: 256 threads");

namespace {

template <int L>
constexpr int ens_col_lds() {
  if constexpr (L > kEnsMaxLog1) {
    return 0;
  } else {
    return ColCfg<L, 12>::LDS_BYTES > ens_col_lds<L + 1>() ? ColCfg<L, 12>::LDS_BYTES : ens_col_lds<L + 1>();
  }
}
template <int L>
constexpr int ens_row_lds() {
  if constexpr (L > kEnsMaxLog2) {
    return 0;
  } else {
    return RowCfg<L, 16>::LDS_BYTES > ens_row_lds<L + 1>() ? RowCfg<L, 16>::LDS_BYTES : ens_row_lds<L + 1>();
  }
}
constexpr int kEnsLds = ens_col_lds<kEnsMinLog1>() > ens_row_lds<kEnsMinLog2>() ? ens_col_lds<kEnsMinLog1>()
                                                                                 : ens_row_lds<kEnsMinLog2>();

template <int L>
__device__ __forceinline__ void ens_row(int logn2, const FlameDev& f, long long n, int group, int tid) {
  if constexpr (L <= kEnsMaxLog2) {
    if (logn2 != L) {
      ens_row<L + 1>(logn2, f, n, group, tid);
      return;
    }
    row_body<L, ROW_STEP, 16, false>(f, n, nullptr, nullptr, group, group, tid);
  }
}

template <int L>
__device__ __forceinline__ void ens_col(int logn1, const FlameDev& f, long long n, int tile, int tid) {
  if constexpr (L <= kEnsMaxLog1) {
    if (logn1 != L) {
      ens_col<L + 1>(logn1, f, n, tile, tid);
      return;
    }
    col_body<L, COL_STEP, 12, VAR_EULER>(f, n, nullptr, tile, tid);
  }
}

// The thread's index in its workgroup, as a value the compiler cannot move
// out of the loops: what the bodies derive from it is then computed per body
// instead of once per launch and kept (spilled) across all of them.
__device__ __forceinline__ int opaque_tid() {
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

// s_waitcnt immediate (GFX9 encoding) that waits for vmcnt = 0 and leaves
// expcnt (7) and lgkmcnt (15) at their maxima, i.e. not waited on.
constexpr int kWaitVmcnt0 = 0x0F70;

// This workgroup's arrival at a shared flame's counter after a phase, then a
// wait for `target` arrivals. Each wave first waits until its stores of the
// phase have completed (reached the L2); after the barrier, thread 0 releases
// them at agent scope (an L2 write-back for the other XCDs) and counts the
// workgroup in, and once the count is reached it acquires (invalidates the
// caches the next phase reads through) and the barrier passes that on. One
// agent-scope release per workgroup instead of one per wave: the write-backs
// stall the XCD's L2, and one per wave made the launch about 1.8x slower.
// The wait is bounded: it ends when another workgroup has reported a failure,
// after `limit` ticks of the constant-rate wall clock, or after limit / 16 +
// 1024 polls (each takes well over 16 ticks: a load from memory and a sleep),
// and then reports the failure in *err and returns false.
__device__ bool ens_meet(unsigned* cnt, unsigned target, int* err, unsigned long long limit) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // the write-back has completed before the count
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = (unsigned long long)wall_clock64();
    const unsigned long long polls = limit / 16 + 1024;
    int good = 1;
    for (unsigned long long i = 0; __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++i) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || i > polls ||
          (unsigned long long)wall_clock64() - t0 > limit) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // the invalidation has completed before the barrier
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

}  // namespace

// Steps n0 .. n0 + steps - 1 of every flame, one EnsembleItem per workgroup
// (graph replays add the step index *nbase to n0). A launch that finds *err
// already set (by an earlier launch of the same call) does nothing.
__global__ void __launch_bounds__(kEnsThreads) __attribute__((amdgpu_waves_per_eu(COL_WAVES_PER_EU)))
    ensemble_kernel(const FlameDev* __restrict__ fls, const EnsembleItem* __restrict__ items,
                    unsigned* __restrict__ arrive, int* __restrict__ err, long long n0,
                    const long long* __restrict__ nbase, int steps, unsigned long long limit) {
  if (nbase) n0 += *nbase;
  const EnsembleItem it = items[blockIdx.x];
  if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  unsigned* const cnt = arrive + (size_t)it.flame * kEnsArriveStride;
  for (int s = 0; s < steps; ++s) {
    const long long n = n0 + s;
    for (int fi = 0; fi < it.nfl; ++fi)
      for (int g = it.part; g < it.rtiles; g += it.parts) {
        ens_row<kEnsMinLog2>(it.logn2, fls[it.flame + fi], n, g, opaque_tid());
        __syncthreads();  // the next body reuses the LDS; Q is read by this workgroup next
      }
    if (it.parts > 1 && !ens_meet(cnt, (unsigned)(2 * s + 1) * (unsigned)it.parts, err, limit)) return;
    for (int fi = 0; fi < it.nfl; ++fi)
      for (int c = it.part; c < it.ctiles; c += it.parts) {
        ens_col<kEnsMinLog1>(it.logn1, fls[it.flame + fi], n, c, opaque_tid());
        __syncthreads();
      }
    if (it.parts > 1 && !ens_meet(cnt, (unsigned)(2 * s + 2) * (unsigned)it.parts, err, limit)) return;
  }
}

// Zeroes the arrival counters (and the failure flag if clear_err) before a launch.
__global__ void ensemble_reset_kernel(unsigned* __restrict__ arrive, int count, int* __restrict__ err,
                                      int clear_err) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) arrive[i] = 0u;
  if (clear_err && blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

bool ensemble_supports(int logn1, int logn2) {
  return logn1 >= kEnsMinLog1 && logn1 <= kEnsMaxLog1 && logn2 >= kEnsMinLog2 && logn2 <= kEnsMaxLog2;
}

KernelLaunch ensemble_kernel_info() {
  return KernelLaunch{reinterpret_cast<const void*>(&ensemble_kernel), kEnsThreads, kEnsLds};
}

int ensemble_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ensemble_kernel, kEnsThreads, kEnsLds) != hipSuccess)
    return 0;
  return nb;
}

KernelLaunch ensemble_reset_info() {
  return KernelLaunch{reinterpret_cast<const void*>(&ensemble_reset_kernel), 256, 0};
}

void launch_ensemble_reset(hipStream_t st, unsigned* arrive, int narrive, int* err, bool clear_err) {
  const int rb = (narrive + 255) / 256 < 1024 ? (narrive + 255) / 256 : 1024;
  hipLaunchKernelGGL(ensemble_reset_kernel, dim3(rb > 0 ? rb : 1), dim3(256), 0, st, arrive, narrive, err,
                     clear_err ? 1 : 0);
}

hipError_t launch_ensemble(hipStream_t st, const FlameDev* fls, const EnsembleItem* items, int nitems,
                           unsigned* arrive, int narrive, int* err, long long n0, int steps,
                           unsigned long long limit) {
  launch_ensemble_reset(st, arrive, narrive, err, false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long* nbase = nullptr;
  void* args[] = {&fls, &items, &arrive, &err, &n0, &nbase, &steps, &limit};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&ensemble_kernel), dim3(nitems),
                                    dim3(kEnsThreads), args, (unsigned)kEnsLds, st);
}

}  // namespace flame
