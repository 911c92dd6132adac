// Device-side description of one flame and the kernel configuration shared
// by the kernels and the host runtime.

#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_engine.hpp"

namespace flame {

// Minimum waves per SIMD the row and column kernels are compiled for (a
// register budget of 512 / waves VGPRs).
#ifndef ROW_WAVES_PER_EU
#define ROW_WAVES_PER_EU 3
#endif
#ifndef COL_WAVES_PER_EU
#define COL_WAVES_PER_EU 2
#endif
#ifndef ADJ_ROW_WAVES_PER_EU
#define ADJ_ROW_WAVES_PER_EU 2
#endif

// Per-flame pointers and constants read by every kernel (one entry per flame
// in a device array; blockIdx.y selects the flame inside a launch).
struct FlameDev {
  float2* S;           // state, [M][H1]
  float2* Wp;          // column transforms of (i kappa1 - kappa2) Phi~ and ...
  float2* Wm;          // ... the conj of those of (i kappa1 + kappa2) Phi~, interleaved
                       // [j1/4][m][j1%4], Wp and Wm in the two halves of W (index with w_index)
  float2* Q;           // row transforms of |grad Phi|^2 (and scratch), tiled [m/TQ][j1][m%TQ]
  float2* A1;          // adjoint scratch, same layout: row transform of w1 = m g1
  float2* A2;          // adjoint scratch, same layout: i kappa2 x row transform of w2 = m g2
  const float2* tw1;   // twiddles of the length-N1 transform, 16 points per thread
  const float2* tw2;   // twiddles of the length-N2 transform, 16 points per thread
  const float2* tw1_8; // the same for 8 points per thread
  const float2* tw2_8;
  const float2* tw6;   // twiddles of the length-3N1/4 transform (product grid), or null
  const float2* tw6_8; // the same for 8 points per thread
  const float2* tw12a; // twiddles of the length-3N1/4 transform, 12 points per thread (Shape12), or null
  const float2* tw12b; // the same for the length-3N2/4 transform
  double* part;        // per-workgroup partial sums of the diagnostics
  const double* r0tab; // reference-radius table {r0(t_n), I1_n, I2_n} (r0_law = 1), or null for r0 = t
  long long r0n;       // its entries
  const float2* F;     // forcing f~ of Eq. (1) in the state layout [M][H1], or null (f~ = 0)
  float2* S2;          // Heun's predictor Phi* in the state layout (workspace; the A2 scratch)
  int n1, n2;
  int m;               // stored k2 columns, N2/4
  int h1;              // stored k1 slots, N1/2
  int tshift;          // log2 of the tile width TQ of Q, A1, A2
  int rows;            // theta rows of the step's product grid: 3 N1/4, or N1
  float s1, s2;        // axis scales of kappa
  float gamma;
  int cols;            // phi points of the step's product grid: 3 N2/4, or N2
  double t0, dt;
};

// A batch of circular flames (the one-dimensional form of Eq. (1)) of one
// grid: spectra S[c][k], k = 0 .. N/4 - 1, complex64, caller-owned.
struct CircleDev {
  float2* S;
  int n_circles;
  float seg;     // segment integer: kappa_k = seg k
  float gamma;
  int pad_;
  double t0, dt;
};

// Register shape of a length-N transform with PTS points per thread: the
// power-of-two plans (8 or 16 points), or, for PTS = 12, the length-3N/4
// transform of a product grid in the 12-point plan (ff::Shape12), which also
// uses N/16 threads. LOW, HIGH: registers i < LOW hold the spectral positions
// k = t + G i >= 0 of the retained box, i >= HIGH the negative ones (k - L,
// L the transform length); the registers between hold padding.
template <int LOGN, int PTS>
struct TfShape {
  using S = ff::Shape<LOGN, PTS>;
  static constexpr int LOW = PTS / 4, HIGH = 3 * PTS / 4;
};
template <int LOGN>
struct TfShape<LOGN, 12> {
  using S = ff::Shape12<LOGN - 4>;
  static constexpr int LOW = 4, HIGH = 8;
};
template <int LOGN, int PTS>
using TShape = typename TfShape<LOGN, PTS>::S;

// Column kernel: T = max(1, 16*256/N1) columns per workgroup, interleaved
// (thread tid works on column tid % T, FFT lane tid / T); the transform of
// each column uses G = N1/PTS threads. T does not depend on PTS.
//
// Q is tiled [m/TQ][j1][m%TQ] with TQ = 2T for N1 >= 2048 (else TQ = T): a
// row-kernel workgroup at N2 = 4096 holds one row pair, so with TQ = T its
// pieces of Q (2 rows x TQ columns of 8 bytes) would be 32 or 16 bytes, and
// HBM writes in pieces under 64 bytes run at about half the bandwidth of
// longer ones. The column kernel then reads half of each 2-row piece and the
// neighbouring workgroup (same XCD) the other half.
constexpr int col_tile_for(int g16) { return g16 >= 256 ? 1 : 256 / g16; }
constexpr int q_tile_for(int g16) { return g16 >= 128 ? 2 * col_tile_for(g16) : col_tile_for(g16); }

template <int LOGN1, int PTS = ff::kPts>
struct ColCfg {
  static constexpr int G16 = ff::Shape<LOGN1>::G;
  static constexpr int G = TShape<LOGN1, PTS>::G;
  static constexpr int T = col_tile_for(G16);
  static constexpr int TQ = q_tile_for(G16);
  static constexpr int QS = ff::ilog2c(TQ);
  static constexpr int THREADS = T * G;
  static constexpr int LDS_BYTES = TShape<LOGN1, PTS>::LDS * T * 8;
};

// Product grid of the step: |grad Phi|^2 is formed on M1 = 3 N1/4 theta rows
// instead of N1. The product of two fields with |k1| <= K1 = N1/4 - 1 has
// |k1| <= 2 K1, and on M1 >= 3 K1 + 1 rows no alias of it lands in
// |k1| <= K1, so the truncated quadratic term is the same as on N1 rows up to
// rounding. The column transforms have length M1 = 6 * N1/8 (Shape6:
// radix-PTS passes, then radix 6), with G = M1/PTS threads per column. Used
// for N1 >= 128.
constexpr int kMinLogProduct = 7;
// The phi product grid (3 N2/4 points, 12 points per thread) needs N2 >= 64.
constexpr int kMinLogRow12 = 6;

template <int LOGN1, int PTS = 16>
struct ColCfgP {
  using S = ff::Shape6<LOGN1 - 3, PTS>;
  static constexpr int M1 = S::N;
  static constexpr int G = S::G;
  static constexpr int G16 = ff::Shape<LOGN1>::G;
  static constexpr int T = col_tile_for(G16);
  static constexpr int TQ = q_tile_for(G16);
  static constexpr int QS = ff::ilog2c(TQ);
  static constexpr int THREADS = T * G;
  static constexpr int LDS_BYTES = S::LDS * T * 8;
  static_assert(THREADS % 64 == 0, "whole waves");
};

// Split variant of the product-grid column kernel: per column 2G threads
// (G = M1/16) run the forward transform with 8 points each (Shape6 with
// PTS 8), then split into two groups of G threads that run the Wp and the Wm
// inverse transforms side by side with 16 points each, each group in its own
// LDS buffer. Twice the waves of ColCfgP<., 16> for the same columns.
template <int LOGN1>
struct ColCfgQ {
  using SF = ff::Shape6<LOGN1 - 3, 8>;   // forward
  using SI = ff::Shape6<LOGN1 - 3, 16>;  // inverse
  static constexpr int M1 = SF::N;
  static constexpr int G8 = SF::G, G16 = SI::G;
  static constexpr int T = ColCfgP<LOGN1, 16>::T;
  static constexpr int TQ = ColCfgP<LOGN1, 16>::TQ;
  static constexpr int QS = ColCfgP<LOGN1, 16>::QS;
  static constexpr int SLOTS = SF::LDS;  // padded slots of one buffer
  static constexpr int THREADS = T * G8;
  static constexpr int LDS_BYTES = 2 * SLOTS * T * 8;
  static_assert(G8 == 2 * G16, "two inverse groups");
  static_assert(THREADS % 64 == 0, "whole waves");
};

// The row kernel's 12-point plan keeps the twiddles of the passes with
// Ns >= this in registers and reads the others from a copy in LDS (SplitTw).
constexpr int kRow12MinNs = 192;
// Table entries of the passes p >= 1 with Ns < min_ns (they come first in the table).
constexpr int lds_twiddles(const ff::PassPlan& p, int min_ns) {
  int q = 1;
  while (q < p.npass && p.ns[q] < min_ns) ++q;
  return p.tw_off[q] > 0 ? p.tw_off[q] : 1;
}

// Row kernel: B = max(1, 16*256/N2) row pairs per workgroup, interleaved.
// WPE: the minimum waves per SIMD it is compiled for; at N2 = 8192 with 16
// points per thread a workgroup is 8 waves (2 per SIMD), which may then use
// the whole register budget instead of spilling.
template <int LOGN2, int PTS = ff::kPts>
struct RowCfg {
  static constexpr int G16 = ff::Shape<LOGN2>::G;
  static constexpr int G = TShape<LOGN2, PTS>::G;
  static constexpr int B = G16 >= 256 ? 1 : 256 / G16;
  static constexpr int THREADS = B * G;
  static constexpr int DATA_SLOTS = TShape<LOGN2, PTS>::LDS * B;  // transform exchange area
  // with 12 points per thread, the small-Ns passes' twiddles follow in LDS (SplitTw)
  static constexpr int TW_SLOTS = PTS == 12 ? lds_twiddles(TShape<LOGN2, PTS>::plan, kRow12MinNs) : 0;
  static constexpr int LDS_BYTES = (DATA_SLOTS + TW_SLOTS) * 8;
  static constexpr int WPE = THREADS >= 512 && PTS >= 12 ? 2 : ROW_WAVES_PER_EU;
};

constexpr int col_tile(int logn1) { return col_tile_for((1 << logn1) / ff::kPts); }
constexpr int q_tile(int logn1) { return q_tile_for((1 << logn1) / ff::kPts); }
constexpr int row_pairs(int logn2) { return (1 << logn2) / ff::kPts >= 256 ? 1 : 256 / ((1 << logn2) / ff::kPts); }

enum ColMode : int { COL_STEP = 0, COL_FIRST = 1, COL_PROJECT = 2, COL_SYNTH = 3 };
// Variants of the step's column kernel (COL_STEP): integrating-factor Euler
// without the forcing term (compiled out) or with it, and the two stages of
// integrating-factor Heun, which read the forcing when one is bound:
//   VAR_HEUN_P: predictor Phi* = E (Phi~^n + dt (f~ - c_n N(Phi~^n))) -> S2;
//   VAR_HEUN_C: corrector Phi~^{n+1} = (Phi* + E Phi~^n + dt (f~ - c_{n+1} N(Phi*))) / 2 -> S.
enum StepVar : int { VAR_EULER = 0, VAR_EULER_F = 1, VAR_HEUN_P = 2, VAR_HEUN_C = 3 };
// Or-ed into a StepVar: the column kernel writes W with non-temporal stores
// (the row kernel's Q stores take the same choice through its NT argument).
constexpr int VAR_NT = 4;
enum RowMode : int { ROW_STEP = 0, ROW_FORWARD = 1, ROW_SYNTH = 2, ROW_DIAG = 3 };
// Adjoint column kernel: ADJ_A forms mu = E lambda and the column transforms
// of mu and of the state's packed gradient; ADJ_C / SEED_C form the
// divergence from the row transforms in A1, A2 and write the cotangent.
enum AdjColMode : int { ADJ_A = 0, ADJ_C = 1, SEED_C = 2 };
// Adjoint row kernel: ROW_ADJ forms w = m grad Phi, ROW_SEED forms
// w = grad Phi / (r0^2 sqrt(1 + |grad Phi|^2 / r0^2)); both write the row
// transforms of w1 and i kappa2 w2 to A1, A2.
enum AdjRowMode : int { ROW_ADJ = 0, ROW_SEED = 1 };

// Keep each thread's twiddles in registers for a kernel's lifetime (the
// alternative reads the table in every pass).
#ifndef FLAME_CACHE_TWIDDLES
#define FLAME_CACHE_TWIDDLES 1
#endif
constexpr bool kCacheTwiddles = FLAME_CACHE_TWIDDLES != 0;
// Passes with Ns >= this keep their twiddles in registers (2: every pass).
#ifndef FLAME_TW_CACHE_MIN_NS
#define FLAME_TW_CACHE_MIN_NS 2
#endif
constexpr int kTwCacheMinNs = FLAME_TW_CACHE_MIN_NS;
// Prune the first butterfly of inverse transforms whose input is zero in the
// middle half of the padded spectrum.
#ifndef FLAME_PRUNE
#define FLAME_PRUNE 1
#endif
constexpr bool kPrune = FLAME_PRUNE != 0;


constexpr int kMinLog = 4;
constexpr int kMaxLog = 14;
// Lengths up to 2^kMaxLog8 have the 8-points-per-thread kernels (beyond it
// they would need more than 1024 threads per workgroup), and so does the
// split product-grid column kernel.
constexpr int kMaxLog8 = 13;
constexpr int kDiagThreads = 256;

// Persistent ensemble kernel: one co-resident grid of workgroups steps every
// flame of a plan for all steps of a launch. A workgroup's share is either
// `nfl` whole flames from `flame` on, which it steps alone (parts == 1), or
// part `part` of the `parts` workgroups that share flame `flame`: it takes
// the row-pair groups and column tiles part, part + parts, ... of each step
// and meets the others at that flame's arrival counter after each phase.
struct EnsembleItem {
  int flame, nfl, part, parts;
  int logn1, logn2;    // the grid of its flames
  int rtiles, ctiles;  // row-pair groups and column tiles of one flame
};
// Its step kernels' bodies: the product-grid column transforms with 12
// points per thread (N1 = 2^7 .. 2^10) and the row transforms with 16 (N2 =
// 2^7 .. 2^11), all of them 256 threads per workgroup.
constexpr int kEnsThreads = 256;
constexpr int kEnsMinLog1 = 7, kEnsMaxLog1 = 10;
constexpr int kEnsMinLog2 = 7, kEnsMaxLog2 = 11;
constexpr int kEnsArriveStride = 32;  // 128 bytes between two flames' arrival counters

}  // namespace flame
