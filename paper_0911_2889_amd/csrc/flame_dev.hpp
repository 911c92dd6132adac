// Device-side description of one flame and the kernel configuration shared
// by the kernels and the host runtime.

#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_engine.hpp"

namespace flame {

// Per-flame pointers and constants read by every kernel (one entry per flame
// in a device array; blockIdx.y selects the flame inside a launch).
struct FlameDev {
  float2* S;           // state, [M][H1]
  float2* Wp;          // column transforms of (i kappa1 - kappa2) Phi~, tiled [m/T][j1][m%T]
  float2* Wm;          // conj of column transforms of (i kappa1 + kappa2) Phi~, same layout
  float2* Q;           // row transforms of |grad Phi|^2 (and scratch), same layout
  const float2* tw1;   // twiddles of the length-N1 transform
  const float2* tw2;   // twiddles of the length-N2 transform
  double* part;        // per-workgroup partial sums of the diagnostics
  int n1, n2;
  int m;               // stored k2 columns, N2/4
  int h1;              // stored k1 slots, N1/2
  int tshift;          // log2 of the tile width T of Wp/Wm/Q
  int pad_;
  float s1, s2;        // axis scales of kappa
  float gamma;
  float pad2_;
  double t0, dt;
};

// Column kernel: T = max(1, 256/G) columns per workgroup, interleaved
// (thread tid works on column tid % T, FFT lane tid / T).
template <int LOGN1>
struct ColCfg {
  static constexpr int G = ff::Shape<LOGN1>::G;
  static constexpr int T = G >= 256 ? 1 : 256 / G;
  static constexpr int THREADS = T * G;
  static constexpr int LDS_BYTES = ff::Shape<LOGN1>::LDS * T * 8;
};

// Row kernel: B = max(1, 256/G) row pairs per workgroup, interleaved.
template <int LOGN2>
struct RowCfg {
  static constexpr int G = ff::Shape<LOGN2>::G;
  static constexpr int B = G >= 256 ? 1 : 256 / G;
  static constexpr int THREADS = B * G;
  static constexpr int LDS_BYTES = ff::Shape<LOGN2>::LDS * B * 8;
};

constexpr int col_tile(int logn1) { return (1 << logn1) / ff::kPts >= 256 ? 1 : 256 / ((1 << logn1) / ff::kPts); }
constexpr int row_pairs(int logn2) { return (1 << logn2) / ff::kPts >= 256 ? 1 : 256 / ((1 << logn2) / ff::kPts); }

enum ColMode : int { COL_STEP = 0, COL_FIRST = 1, COL_PROJECT = 2, COL_SYNTH = 3 };
enum RowMode : int { ROW_STEP = 0, ROW_FORWARD = 1, ROW_SYNTH = 2, ROW_DIAG = 3 };

// Keep each thread's twiddles in registers for a kernel's lifetime (the
// alternative reads the table in every pass).
#ifndef FLAME_CACHE_TWIDDLES
#define FLAME_CACHE_TWIDDLES 1
#endif
constexpr bool kCacheTwiddles = FLAME_CACHE_TWIDDLES != 0;

constexpr int kMinLog = 4;
constexpr int kMaxLog = 12;
constexpr int kDiagThreads = 256;

}  // namespace flame
