// Launchers of the flame kernels (defined in flame_kernels.hip).

#pragma once

#include <hip/hip_runtime.h>

#include "flame_dev.hpp"

namespace flame {

// A kernel function and its launch shape, for graph nodes.
struct KernelLaunch {
  const void* func;
  int threads;
  int lds;
};

// The step kernels for a transform length (arguments: fls, n, nbase, src / in, out).
// var (StepVar): the column kernel's integrator stage and whether it reads
// the flames' forcing spectra (flames without one are stepped unforced), or-ed
// with VAR_NT for non-temporal W stores; nt: non-temporal Q stores.
KernelLaunch col_step_kernel(int logn1, int pts, int var = VAR_EULER);
KernelLaunch row_step_kernel(int logn2, int pts, bool nt = false);
void launch_set_step(hipStream_t st, long long* counter, long long value);
// Largest dynamic LDS (bytes per workgroup) any kernel of an N1 x N2 flame
// asks for (row, column, product-grid and adjoint kernels, every variant).
int lds_bytes_needed(int logn1, int logn2);

// Column kernel over `tiles` tiles of T columns for `nfl` flames of one size
// (fl points at their consecutive FlameDev entries in device memory). src,
// if not null, replaces the state read by COL_FIRST and COL_SYNTH.
// With ev_start/ev_stop (step mode only) the events mark the kernel's start and end;
// var selects the step variant (StepVar).
void launch_col(int logn1, int mode, int tiles, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                const void* src = nullptr, int pts = ff::kPts, hipEvent_t ev_start = nullptr,
                hipEvent_t ev_stop = nullptr, int var = VAR_EULER);

// Column kernel of the step on the product grid (3 N1/4 rows; N1 >= 128),
// mode COL_STEP or COL_FIRST; colp_kernel_info gives its function and shape
// (func null for an unsupported size).
KernelLaunch colp_kernel_info(int logn1, int mode, int pts, int var = VAR_EULER);
void launch_colp(int logn1, int mode, int tiles, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                 const void* src = nullptr, int pts = ff::kPts, hipEvent_t ev_start = nullptr,
                 hipEvent_t ev_stop = nullptr, int var = VAR_EULER);

// Adjoint kernels (adjoint_kernels.hip); see the modes in flame_dev.hpp.
void launch_adj_col(int logn1, int mode, int tiles, hipStream_t st, const FlameDev* fl, long long n,
                    const void* state, const void* lam_in, void* lam_out);
void launch_adj_row(int logn2, int mode, int groups, hipStream_t st, const FlameDev* fl, long long n);
// ADJ_A / ADJ_C on the product grid (3 N1/4 rows; N1 >= 128), with ROW_ADJ reading the step's row count.
void launch_adjp_col(int logn1, int mode, int tiles, hipStream_t st, const FlameDev* fl, long long n,
                     const void* state, const void* lam_in, void* lam_out);

// Row kernel over `groups` groups of B row pairs for `nfl` flames of one size.
void launch_row(int logn2, int mode, int groups, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                const float* in, float* out, int pts = ff::kPts, hipEvent_t ev_start = nullptr,
                hipEvent_t ev_stop = nullptr, bool nt = false);

// Circular flames (circle_kernels.hip): nsteps steps of every circle of the
// batch in one launch, or their diagnostics (4 doubles per circle); false if
// the length 2^logn has no kernel.
bool launch_circle_step(int logn, const CircleDev& d, long long n, int nsteps, hipStream_t st);
bool launch_circle_diag(int logn, const CircleDev& d, long long n, double* out, hipStream_t st);

// Persistent ensemble kernel (EnsembleItem): whether it has the bodies for an
// N1 x N2 flame, its function and shape (arguments: fls, items, arrive, err,
// n0, nbase, steps, limit), and how many of its workgroups fit on one
// compute unit (0 if the query fails). launch_ensemble_reset zeroes the
// narrive arrival counters (and *err if clear_err; function and shape from
// ensemble_reset_info, arguments arrive, narrive, err, clear_err as int).
// launch_ensemble zeroes the counters, then launches nitems workgroups
// cooperatively for steps n0 .. n0 + steps - 1; a bounded wait that runs out
// (limit: wall-clock ticks) sets *err. It returns the launch's error code.
bool ensemble_supports(int logn1, int logn2);
KernelLaunch ensemble_kernel_info();
KernelLaunch ensemble_reset_info();
int ensemble_blocks_per_cu();
void launch_ensemble_reset(hipStream_t st, unsigned* arrive, int narrive, int* err, bool clear_err);
hipError_t launch_ensemble(hipStream_t st, const FlameDev* fls, const EnsembleItem* items, int nitems,
                           unsigned* arrive, int narrive, int* err, long long n0, int steps,
                           unsigned long long limit);

void launch_set_spectrum(hipStream_t st, const FlameDev* fl, int flame, int total, const void* half);
void launch_get_spectrum(hipStream_t st, const FlameDev* fl, int flame, int total, void* half);
void launch_diag_spectral(hipStream_t st, const FlameDev* fl, int flame, int blocks, double* part);
void launch_diag_final(hipStream_t st, const FlameDev* fl, int flame, long long n, int n_area, int n_spec,
                       double* out);

}  // namespace flame
