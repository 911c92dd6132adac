// Bodies of the step's column and row kernels: one workgroup's work on one
// column tile or one group of row pairs of a flame. The kernels of
// flame_kernels.hip run one body per workgroup; the persistent ensemble kernel
// (ensemble_kernel.hip) runs many, one after another.

#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_engine.hpp"
#include "flame_dev.hpp"
#include "kernel_common.hpp"

namespace flame {

// PTS 16 or 8: the column transforms have length N1 (the grid's theta rows).
// PTS 12: they have length L = 3 N1/4 (the product grid, N1 >= 128) in the
// 12-point plan (ff::Shape12), on the same N1/16 threads per column as
// PTS 16 on N1 rows; the kept modes sit in the first and last third of the
// registers instead of the first and last quarter (TfShape). COL_STEP and
// COL_FIRST only for PTS 12.
//
// col_body is the work of thread tid of a workgroup on column tile `tile` of
// flame f at step index n: col_kernel runs it on tile xcd_swizzle(blockIdx.x),
// the persistent ensemble kernel on the tiles of its part of a flame.
template <int LOGN1, int MODE, int PTS = ff::kPts, int SV = VAR_EULER>
__device__ __forceinline__ void col_body(const FlameDev& f, long long n, const float2* src, int tile, int tid) {
  constexpr int VAR = SV & ~VAR_NT;
  constexpr bool NT = MODE == COL_STEP && (SV & VAR_NT) != 0;
  static_assert(PTS != 12 || MODE == COL_STEP || MODE == COL_FIRST, "12 points per thread: step modes only");
  using TS = TfShape<LOGN1, PTS>;
  using S = typename TS::S;
  constexpr int G = S::G, T = ColCfg<LOGN1, PTS>::T, N1 = 1 << LOGN1, L = S::N;
  constexpr int LOW = TS::LOW, HIGH = TS::HIGH, KEEP = LOW + PTS - HIGH;
  extern __shared__ float2 lds[];
  const int c = tid % T, t = tid / T;
  const int m = tile * T + c;
  const bool live = m < f.m;
  float2* my = lds + c;
  constexpr int TQ = ColCfg<LOGN1, PTS>::TQ, QS = ColCfg<LOGN1, PTS>::QS;
  gf2* const Qc = glob(f.Q) + ((((size_t)m >> QS) * L) << QS) + (m & (TQ - 1));  // column m: Qc[j1 * TQ]
  gf2* const Wpc = glob(f.Wp);  // element (j1, m) at w_index(j1, m, M)
  gf2* const Wmc = glob(f.Wm);
  // column m of the state: Sc[k1]; COL_FIRST and COL_SYNTH may read another
  // spectrum in the same layout (src), the other modes update the state
  gf2* const Sc = glob((MODE == COL_FIRST || MODE == COL_SYNTH) && src ? const_cast<float2*>(src) : f.S) +
                  (size_t)m * f.h1 + N1 / 4;
  gf2* const Pc = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)m * f.h1 + N1 / 4;  // Heun's predictor
  const auto tw1 = AxisTw<LOGN1, PTS>::make(f.tw1, f.tw1_8, f.tw12a, t);

  float2 v[PTS];
  float2 sv[KEEP];

  if constexpr (MODE == COL_STEP || MODE == COL_PROJECT) {
    // The loads carry no condition, so that no branch between them makes one
    // wait for another: a column past the grid reads its padded slots of Q and
    // column 0 of the state (its results are never stored).
    const int ms = live ? m : 0;
    gf2* const Sl = glob(f.S) + (size_t)ms * f.h1 + N1 / 4;
    gf2* const Pl = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)ms * f.h1 + N1 / 4;
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = ld(Qc + (t + G * i) * TQ);
    // the old state is loaded before the transform so its latency is hidden
    // frc: the forcing (not in VAR_EULER); prd: Heun's predictor (VAR_HEUN_C)
    constexpr bool FORCED = MODE == COL_STEP && VAR != VAR_EULER;
    float2 old[KEEP], frc[KEEP], prd[KEEP];
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) {
      const int i = kept_reg<LOGN1, PTS>(kk);
      const int k1 = t + G * i - (i >= HIGH ? L : 0);
      old[kk] = MODE == COL_STEP ? ld(Sl + k1) : make_float2(0.f, 0.f);
      frc[kk] = FORCED ? forcing_at(f, ms, k1) : make_float2(0.f, 0.f);
      prd[kk] = MODE == COL_STEP && VAR == VAR_HEUN_C ? ld(Pl + k1) : make_float2(0.f, 0.f);
    }
    fft_s<S, false>(v, t, my, T, tw1);
    StepScalars sc{};
    float ac = 0.f;  // the corrector's dt c_{n+1} / P
    if constexpr (MODE == COL_STEP) sc = step_scalars(f, n, L, f.cols);
    if constexpr (MODE == COL_STEP && VAR == VAR_HEUN_C) ac = step_scalars(f, n + 1, L, f.cols).a;
    const float inv_p = 1.0f / ((float)f.n1 * (float)f.n2);
    const float kap2c = f.s2 * (float)m;
    const float dtf = (float)f.dt;
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) {
      const int i = kept_reg<LOGN1, PTS>(kk);
      const int k1 = t + G * i - (i >= HIGH ? L : 0);
      const int s = k1 + N1 / 4;
      float2 val;
      if constexpr (MODE == COL_STEP) {
        const float kap1 = f.s1 * (float)k1;
        const float kk2 = kap1 * kap1 + kap2c * kap2c;
        const float e = growth_factor(kk2, sc, f.gamma);
        if constexpr (VAR == VAR_HEUN_C)
          val = make_float2(0.5f * (prd[kk].x + e * old[kk].x + ac * v[i].x + dtf * frc[kk].x),
                            0.5f * (prd[kk].y + e * old[kk].y + ac * v[i].y + dtf * frc[kk].y));
        else
          val = make_float2(e * (old[kk].x + sc.a * v[i].x + dtf * frc[kk].x),
                            e * (old[kk].y + sc.a * v[i].y + dtf * frc[kk].y));
      } else {
        val = ff::cscale(v[i], inv_p);
      }
      if (s == 0) val = make_float2(0.f, 0.f);
      sv[kk] = val;
    }
    if (tile == 0) {
      // symmetrise column k2 = 0 (group c == 0): copy k1 > 0 conjugated onto -k1
      if (c == 0) {
#pragma unroll
        for (int kk = 0; kk < LOW; ++kk) {
          const int k1 = t + G * kk;
          lds[k1] = sv[kk];
        }
      }
      __syncthreads();
      if (c == 0) {
#pragma unroll
        for (int kk = LOW; kk < KEEP; ++kk) {
          const int k1 = t + G * kept_reg<LOGN1, PTS>(kk) - L;
          if (k1 > -N1 / 4) sv[kk] = ff::cconj(lds[-k1]);
        }
        if (t == 0) sv[0].y = 0.f;
      }
      __syncthreads();
    }
    if (live) {
      gf2* const Dc = VAR == VAR_HEUN_P ? Pc : Sc;  // the predictor goes to S2
#pragma unroll
      for (int kk = 0; kk < KEEP; ++kk) {
        const int i = kept_reg<LOGN1, PTS>(kk);
        const int k1 = t + G * i - (i >= HIGH ? L : 0);
        st(Dc + k1, sv[kk]);
      }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) {
      const int i = kept_reg<LOGN1, PTS>(kk);
      const int k1 = t + G * i - (i >= HIGH ? L : 0);
      sv[kk] = live ? ld(Sc + k1) : make_float2(0.f, 0.f);
    }
  }

  if constexpr (MODE == COL_SYNTH) {
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) v[kept_reg<LOGN1, PTS>(kk)] = sv[kk];
    fft_s<S, true, kPrune>(v, t, my, T, tw1);
    if (live) {
#pragma unroll
      for (int i = 0; i < PTS; ++i) st(Qc + (t + G * i) * TQ, v[i]);
    }
  } else {
    const float kap2 = f.s2 * (float)m;
    // Z+ = IFFT_k1((i kappa1 - kappa2) Phi~), stored as is
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) {
      const int i = kept_reg<LOGN1, PTS>(kk);
      const float kap1 = f.s1 * (float)(t + G * i - (i >= HIGH ? L : 0));
      v[i] = make_float2(-kap1 * sv[kk].y - kap2 * sv[kk].x, kap1 * sv[kk].x - kap2 * sv[kk].y);
    }
    fft_s<S, true, kPrune>(v, t, my, T, tw1);
    if (live) {
#pragma unroll
      for (int i = 0; i < PTS; ++i) st_nt<NT>(Wpc + w_index(t + G * i, m, f.m), v[i]);
    }
    // Z- column for k2 = -m: conj(IFFT_k1((i kappa1 + kappa2) Phi~))
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < KEEP; ++kk) {
      const int i = kept_reg<LOGN1, PTS>(kk);
      const float kap1 = f.s1 * (float)(t + G * i - (i >= HIGH ? L : 0));
      v[i] = make_float2(-kap1 * sv[kk].y + kap2 * sv[kk].x, kap1 * sv[kk].x + kap2 * sv[kk].y);
    }
    fft_s<S, true, kPrune>(v, t, my, T, tw1);
    if (live) {
#pragma unroll
      for (int i = 0; i < PTS; ++i) st_nt<NT>(Wmc + w_index(t + G * i, m, f.m), ff::cconj(v[i]));
    }
  }
}

// PTS 16 or 8: the row transforms have length N2. PTS 12 (ROW_STEP only):
// the quadratic term is formed on L2 = 3 N2/4 phi points (the product grid
// along phi, N2 >= 64), with the 12-point plan on N2/16 threads per row pair.
// row_body is the work of thread tid of a workgroup on row-pair group `group`
// of flame f (ROW_DIAG writes its partial sum to f.part[slot]).
template <int LOGN2, int MODE, int PTS = ff::kPts, bool NT = false>
__device__ __forceinline__ void row_body(const FlameDev& f, long long n, const float* __restrict__ phys_in,
                                         float* __restrict__ phys_out, int group, int slot, int tid) {
  static_assert(PTS != 12 || MODE == ROW_STEP, "12 points per thread: the step only");
  using TS = TfShape<LOGN2, PTS>;
  using S = typename TS::S;
  constexpr int G = S::G, B = RowCfg<LOGN2, PTS>::B, N2 = 1 << LOGN2, L2 = S::N;
  constexpr int LOW = TS::LOW, HIGH = TS::HIGH;
  extern __shared__ float2 lds[];
  const int p = tid % B, t = tid / B;
  const int pair = group * B + p;
  // the step runs on the product grid's rows; the other modes on the grid's
  const int n1 = MODE == ROW_STEP ? f.rows : f.n1, ts = f.tshift, mcols = f.m;
  const bool live = pair < n1 / 2;
  const int ja = 2 * pair, jb = 2 * pair + 1;
  float2* my = lds + p;
  // 12 points per thread: the small-Ns passes read their twiddles from LDS
  using Tw12 = SplitTw<S, kRow12MinNs>;
  float2* const lds_tw = lds + RowCfg<LOGN2, PTS>::DATA_SLOTS;
  if constexpr (PTS == 12) Tw12::stage(lds_tw, f.tw12b, tid, RowCfg<LOGN2, PTS>::THREADS);
  const auto tw2 = [&] {
    if constexpr (PTS == 12) {
      static_assert(Tw12::LDS_ENTRIES <= RowCfg<LOGN2, PTS>::TW_SLOTS, "LDS twiddle area");
      return Tw12(f.tw12b, lds_tw, t);
    } else {
      return AxisTw<LOGN2, PTS>::make(f.tw2, f.tw2_8, f.tw12b, t);
    }
  }();
  gf2* const Wp = glob(f.Wp);
  gf2* const Wm = glob(f.Wm);
  gf2* const Q = glob(f.Q);

  float2 y[PTS];

  if constexpr (MODE == ROW_STEP || MODE == ROW_DIAG) {
    float qa[PTS];
    double area = 0.0;
    const float inv_r2 = [&] {
      const double r = r0_at(f, n);
      return (float)(1.0 / (r * r));
    }();
    // both rows' inputs come in one 16-byte load per register (w_index layout).
    // The loads carry no condition, so that no branch between them makes one
    // wait for another: a pair past the grid reads pair 0 (its results are
    // never stored), and the one position past the box (k2 = -N2/4, at t = 0)
    // is read in bounds and zeroed.
    float2 vr[2][PTS];
    const int pl = live ? pair : 0;
    const int pbase4 = (pl >> 1) * mcols, poff = (pl & 1) << 1;
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const int idx = t + G * i;
      float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
      if (i < LOW) {
        ld_pair(Wp + (((pbase4 + idx) << 2) + poff), a, b);
      } else if (i >= HIGH) {
        const int mm = L2 - idx;  // < mcols except at i = HIGH, t = 0
        ld_pair(Wm + (((pbase4 + (i > HIGH || t > 0 ? mm : 0)) << 2) + poff), a, b);
      }
      vr[0][i] = a;
      vr[1][i] = b;
    }
    // zeroed once every load is issued (a select, not a branch that would wait on the load)
    vr[0][HIGH] = t > 0 ? vr[0][HIGH] : make_float2(0.f, 0.f);
    vr[1][HIGH] = t > 0 ? vr[1][HIGH] : make_float2(0.f, 0.f);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      fft_s<S, true, kPrune>(vr[half], t, my, B, tw2);
#pragma unroll
      for (int i = 0; i < PTS; ++i) {
        const float q = vr[half][i].x * vr[half][i].x + vr[half][i].y * vr[half][i].y;
        if constexpr (MODE == ROW_DIAG) {
          const double x = (double)q * (double)inv_r2;
          area += x / (1.0 + sqrt(1.0 + x));
        } else {
          if (half == 0)
            qa[i] = q;
          else
            y[i] = make_float2(qa[i], q);
        }
      }
    }
    if constexpr (MODE == ROW_DIAG) {
      // deterministic workgroup reduction of the area sums
      __syncthreads();
      double* red = reinterpret_cast<double*>(lds);
      red[tid] = live ? area : 0.0;
      __syncthreads();
      for (int w = RowCfg<LOGN2, PTS>::THREADS / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) f.part[slot] = red[0];
      return;
    }
  } else if constexpr (MODE == ROW_FORWARD) {
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const int idx = t + G * i;
      y[i] = live ? make_float2(glob(phys_in)[(size_t)ja * N2 + idx], glob(phys_in)[(size_t)jb * N2 + idx])
                  : make_float2(0.f, 0.f);
    }
  } else {  // ROW_SYNTH: Y = X_a + i X_b with X(k2) = A(m) for k2 = m >= 0, conj(A(m)) for k2 = -m
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const int idx = t + G * i;
      float2 val = make_float2(0.f, 0.f);
      if (live) {
        if (i < LOW) {
          const float2 a = ld(Q + tiled(ja, idx, n1, ts)), b = ld(Q + tiled(jb, idx, n1, ts));
          val = make_float2(a.x - b.y, a.y + b.x);
        } else if (i >= HIGH) {
          const int mm = N2 - idx;
          if (mm < mcols) {
            const float2 a = ld(Q + tiled(ja, mm, n1, ts)), b = ld(Q + tiled(jb, mm, n1, ts));
            // conj(a) + i conj(b)
            val = make_float2(a.x + b.y, -a.y + b.x);
          }
        }
      }
      y[i] = val;
    }
    fft_s<S, true, kPrune>(y, t, my, B, tw2);
    if (live) {
#pragma unroll
      for (int i = 0; i < PTS; ++i) {
        const int idx = t + G * i;
        glob(phys_out)[(size_t)ja * N2 + idx] = y[i].x;
        glob(phys_out)[(size_t)jb * N2 + idx] = y[i].y;
      }
    }
    return;
  }

  // forward transform of the two packed real rows, then split:
  // Q_a(k) = (Y(k) + conj(Y(-k)))/2, Q_b(k) = (Y(k) - conj(Y(-k)))/(2i), k in [0, K2]
  fft_s<S, false>(y, t, my, B, tw2);
  __syncthreads();
  ff::FftS<S, false>::scatter(y, t, my, B);
  __syncthreads();
  if (live) {
#pragma unroll
    for (int i = 0; i < LOW; ++i) {
      const int k = t + G * i;
      const float2 yk = my[S::nat(k) * B];
      const float2 ym = my[S::nat(k == 0 ? 0 : L2 - k) * B];
      const float2 qa = make_float2(0.5f * (yk.x + ym.x), 0.5f * (yk.y - ym.y));
      const float2 qb = make_float2(0.5f * (yk.y + ym.y), 0.5f * (ym.x - yk.x));
      st_nt<NT>(Q + tiled(ja, k, n1, ts), qa);
      st_nt<NT>(Q + tiled(jb, k, n1, ts), qb);
    }
  }
}

}  // namespace flame
