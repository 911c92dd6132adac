// HIP kernels of the spectral flame step (gfx950).
//
// One step of Eq. (1) is two kernels:
//  * row_kernel<ROW_STEP>: for each pair of grid rows j1, load the column-
//    transformed gradient spectrum Z(j1, k2) (k2 in [-K2, K2]), inverse
//    transform along phi to z = g1 + i g2 (the two gradient components packed
//    into one complex field), form q = |z|^2 = |grad Phi|^2, and transform the
//    two real rows back with one complex forward transform, keeping
//    k2 in [0, K2] -> Q. (Section 3: row transform, pointwise product, row
//    inverse transform.)
//  * col_kernel<COL_STEP>: for each stored column k2 = m, forward transform Q
//    along theta, keep |k1| <= K1, apply the integrating-factor Euler update
//    with the exact linear propagator, symmetrise the k2 = 0 column (Section 3),
//    store the state, then immediately form the next step's column transforms
//    of (i kappa1 -+ kappa2) Phi~ -> Wp, Wm. (Section 3: column transforms of
//    k1 Psi and k2 Psi; the inverse column transform of the product.)
// The global transposes of Section 3 are the layouts of Wp/Wm and Q in HBM:
// each kernel reads long contiguous runs and writes pieces of at least 64
// bytes (2 rows x 4 columns of Q; 4 rows x 2 columns of Wp, and of Wm).

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_engine.hpp"
#include "flame_dev.hpp"
#include "flame_kernels.hpp"
#include "kernel_common.hpp"
#include "step_bodies.hpp"

namespace flame {

template <int LOGN1, int MODE, int PTS = ff::kPts, int SV = VAR_EULER>
__global__ void __launch_bounds__((ColCfg<LOGN1, PTS>::THREADS)) __attribute__((amdgpu_waves_per_eu(COL_WAVES_PER_EU)))
    col_kernel(const FlameDev* __restrict__ fls, long long n, const long long* nbase, const float2* src) {
  if (nbase) n += *nbase;  // graph replays read the step index from device memory
  col_body<LOGN1, MODE, PTS, SV>(fls[blockIdx.y], n, src, xcd_swizzle(blockIdx.x, gridDim.x), threadIdx.x);
}

template <int LOGN2, int MODE, int PTS = ff::kPts, bool NT = false>
__global__ void __launch_bounds__((RowCfg<LOGN2, PTS>::THREADS)) __attribute__((amdgpu_waves_per_eu(RowCfg<LOGN2, PTS>::WPE)))
    row_kernel(const FlameDev* __restrict__ fls, long long n, const long long* nbase,
               const float* __restrict__ phys_in, float* __restrict__ phys_out) {
  if (nbase) n += *nbase;
  row_body<LOGN2, MODE, PTS, NT>(fls[blockIdx.y], n, phys_in, phys_out, xcd_swizzle(blockIdx.x, gridDim.x),
                                 blockIdx.x, threadIdx.x);
}

// Column kernel of the step on the product grid (M1 = 3 N1/4 theta rows, see
// ColCfgP): the same work as col_kernel<COL_STEP> (or <COL_FIRST>), with the
// length-M1 transforms of ff::Shape6. The forward transform leaves the
// spectrum in the radix-6 output map (position j + r*N6, j = t + G*it); the
// update is applied there, the kept modes (|k1| <= K1: r in {0, 1}, r in
// {4, 5} except position 4*N6, which is k1 = -(K1 + 1)) go through LDS back
// to the natural map t + G*i (the k2 = 0 column symmetrised on the way), the
// state is stored from that map, and the two inverse transforms start there.
template <int LOGN1, int MODE, int PTS = 16, int SV = VAR_EULER>
__global__ void __launch_bounds__((ColCfgP<LOGN1, PTS>::THREADS))
    __attribute__((amdgpu_waves_per_eu(COL_WAVES_PER_EU)))
    colp_kernel(const FlameDev* __restrict__ fls, long long n, const long long* nbase, const float2* src) {
  constexpr int VAR = SV & ~VAR_NT;
  constexpr bool NT = MODE == COL_STEP && (SV & VAR_NT) != 0;
  static_assert(MODE == COL_STEP || MODE == COL_FIRST, "step modes only");
  if (nbase) n += *nbase;
  using Cfg = ColCfgP<LOGN1, PTS>;
  using S6 = typename Cfg::S;
  constexpr int LOGP = LOGN1 - 3;
  constexpr int G = S6::G, T = Cfg::T, M1 = S6::N, N6 = S6::N6, IT = S6::IT6, N1 = 1 << LOGN1;
  constexpr int TQ = Cfg::TQ, QS = Cfg::QS;
  constexpr int K1 = N1 / 4 - 1;
  extern __shared__ float2 lds[];
  const FlameDev f = fls[blockIdx.y];
  const int tid = threadIdx.x;
  const int c = tid % T, t = tid / T;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int m = tile * T + c;
  const bool live = m < f.m;
  float2* my = lds + c;
  gf2* const Qc = glob(f.Q) + ((((size_t)m >> QS) * M1) << QS) + (m & (TQ - 1));  // column m: Qc[j1 * TQ]
  gf2* const Sc = glob(MODE == COL_FIRST && src ? const_cast<float2*>(src) : f.S) + (size_t)m * f.h1 + N1 / 4;
  gf2* const Pc = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)m * f.h1 + N1 / 4;  // Heun's predictor
  const auto tw = KernelTw6<LOGP, PTS>::make(PTS == 8 ? f.tw6_8 : f.tw6, t);
  // k1 of natural position p, and whether it is kept (|k1| <= K1)
  auto k1_of = [](int p) { return p < M1 / 2 ? p : p - M1; };
  auto kept_at = [](int p) { return p < 2 * N6 || p > 4 * N6; };

  float2 sv[PTS];  // spectrum at natural positions t + G*i, zero outside the box
  if constexpr (MODE == COL_STEP) {
    // The loads carry no condition, so that no branch between them makes one
    // wait for another. A column past the grid reads its padded slots of Q
    // and column 0 of the state (its results are never stored); a slot that
    // holds no kept mode reads k1 = 0, and its value is not used.
    const int ms = live ? m : 0;
    gf2* const Sl = glob(f.S) + (size_t)ms * f.h1 + N1 / 4;
    gf2* const Pl = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)ms * f.h1 + N1 / 4;
    float2 v[PTS];
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = ld(Qc + (t + G * i) * TQ);
    // the old state in the radix-6 output map, loaded before the transform
    constexpr int KR[4] = {0, 1, 4, 5};
    // frc: the forcing (not in VAR_EULER); prd: Heun's predictor (VAR_HEUN_C)
    constexpr bool FORCED = VAR != VAR_EULER;
    float2 old[IT][4], frc[IT][4], prd[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + G * it;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pos = j + KR[q] * N6;
        const int k1 = j < N6 && kept_at(pos) ? k1_of(pos) : 0;
        old[it][q] = ld(Sl + k1);
        frc[it][q] = FORCED ? forcing_at(f, ms, k1) : make_float2(0.f, 0.f);
        prd[it][q] = VAR == VAR_HEUN_C ? ld(Pl + k1) : make_float2(0.f, 0.f);
      }
    }
    float2 o[IT * 6];
    fft6<LOGP, false, PTS>(v, o, t, my, T, tw);
    const StepScalars sc = step_scalars(f, n, M1, f.cols);
    const float ac = VAR == VAR_HEUN_C ? step_scalars(f, n + 1, M1, f.cols).a : 0.f;  // the corrector's dt c_{n+1} / P
    const float kap2c = f.s2 * (float)m;
    const float dtf = (float)f.dt;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + G * it;
      if (j < N6) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          const int pos = j + r * N6;
          float2 val = make_float2(0.f, 0.f);
          if (r != 2 && r != 3 && kept_at(pos)) {
            const int q = r < 2 ? r : r - 2;
            const float kap1 = f.s1 * (float)k1_of(pos);
            const float kk2 = kap1 * kap1 + kap2c * kap2c;
            const float e = growth_factor(kk2, sc, f.gamma);
            if constexpr (VAR == VAR_HEUN_C)
              val = make_float2(
                  0.5f * (prd[it][q].x + e * old[it][q].x + ac * o[it * 6 + r].x + dtf * frc[it][q].x),
                  0.5f * (prd[it][q].y + e * old[it][q].y + ac * o[it * 6 + r].y + dtf * frc[it][q].y));
            else
              val = make_float2(e * (old[it][q].x + sc.a * o[it * 6 + r].x + dtf * frc[it][q].x),
                                e * (old[it][q].y + sc.a * o[it * 6 + r].y + dtf * frc[it][q].y));
          }
          my[ff::lds_pad(pos) * T] = val;
        }
      }
    }
    __syncthreads();
    if (tile == 0) {
      // symmetrise column k2 = 0 (c == 0): k1 > 0 conjugated onto -k1, Im at k1 = 0 zeroed
      if (c == 0) {
#pragma unroll
        for (int i = 0; i < PTS; ++i) {
          const int k1 = t + G * i;
          if (k1 >= 1 && k1 <= K1) my[ff::lds_pad(M1 - k1) * T] = ff::cconj(my[ff::lds_pad(k1) * T]);
        }
        if (t == 0) my[0].y = 0.f;
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PTS; ++i) sv[i] = my[ff::lds_pad(t + G * i) * T];
    __syncthreads();  // the LDS is reused by the inverse transforms
    if (live) {
      gf2* const Dc = VAR == VAR_HEUN_P ? Pc : Sc;  // the predictor goes to S2
#pragma unroll
      for (int i = 0; i < PTS; ++i) {
        const int pos = t + G * i;
        if (kept_at(pos)) st(Dc + k1_of(pos), sv[i]);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const int pos = t + G * i;
      sv[i] = live && kept_at(pos) ? ld(Sc + k1_of(pos)) : make_float2(0.f, 0.f);
    }
  }

  const float kap2 = f.s2 * (float)m;
  gf2* const Wpc = glob(f.Wp);
  gf2* const Wmc = glob(f.Wm);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    // pass 0: Z+ = IFFT_k1((i kappa1 - kappa2) Phi~) -> Wp; pass 1: conj(IFFT_k1((i kappa1 + kappa2) Phi~)) -> Wm
    const float sg = pass == 0 ? -1.f : 1.f;
    float2 v[PTS];
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
      const float kap1 = f.s1 * (float)k1_of(t + G * i);
      v[i] = make_float2(-kap1 * sv[i].y + sg * kap2 * sv[i].x, kap1 * sv[i].x + sg * kap2 * sv[i].y);
    }
    float2 o[IT * 6];
    fft6<LOGP, true, PTS>(v, o, t, my, T, tw);
    if (live) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int j = t + G * it;
        if (j < N6) {
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            const int j1 = j + r * N6;
            if (pass == 0)
              st_nt<NT>(Wpc + w_index(j1, m, f.m), o[it * 6 + r]);
            else
              st_nt<NT>(Wmc + w_index(j1, m, f.m), ff::cconj(o[it * 6 + r]));
          }
        }
      }
    }
  }
}

// Split variant of colp_kernel (ColCfgQ): the forward transform with 8 points
// per thread over 2G threads, then the Wp and Wm inverse transforms side by
// side, 16 points per thread, G threads each. Same results as colp_kernel up
// to rounding. Every barrier is reached by every thread.
template <int LOGN1, int MODE, int SV = VAR_EULER>
__global__ void __launch_bounds__((ColCfgQ<LOGN1>::THREADS)) __attribute__((amdgpu_waves_per_eu(3)))
    colq_kernel(const FlameDev* __restrict__ fls, long long n, const long long* nbase, const float2* src) {
  constexpr int VAR = SV & ~VAR_NT;
  constexpr bool NT = MODE == COL_STEP && (SV & VAR_NT) != 0;
  static_assert(MODE == COL_STEP || MODE == COL_FIRST, "step modes only");
  if (nbase) n += *nbase;
  using Cfg = ColCfgQ<LOGN1>;
  using SF = typename Cfg::SF;
  constexpr int LOGP = LOGN1 - 3;
  constexpr int G8 = Cfg::G8, G16 = Cfg::G16, T = Cfg::T, M1 = Cfg::M1, N6 = SF::N6, N1 = 1 << LOGN1;
  constexpr int ITF = SF::IT6, ITI = ff::Shape6<LOGP, 16>::IT6;
  constexpr int TQ = Cfg::TQ, QS = Cfg::QS, K1 = N1 / 4 - 1;
  extern __shared__ float2 lds[];
  const FlameDev f = fls[blockIdx.y];
  const int tid = threadIdx.x;
  const int c = tid % T, t8 = tid / T;           // forward: lane t8 of 2G
  const int grp = t8 / G16, t16 = t8 % G16;       // inverse: group (0: Wp, 1: Wm), lane t16 of G
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int m = tile * T + c;
  const bool live = m < f.m;
  float2* const buf0 = lds + c;                          // forward exchange, then the updated spectrum
  float2* const bufg = lds + grp * (Cfg::SLOTS * T) + c;  // this group's inverse exchange
  gf2* const Qc = glob(f.Q) + ((((size_t)m >> QS) * M1) << QS) + (m & (TQ - 1));
  gf2* const Sc = glob(MODE == COL_FIRST && src ? const_cast<float2*>(src) : f.S) + (size_t)m * f.h1 + N1 / 4;
  gf2* const Pc = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)m * f.h1 + N1 / 4;  // Heun's predictor
  auto k1_of = [](int p) { return p < M1 / 2 ? p : p - M1; };
  auto kept_at = [](int p) { return p < 2 * N6 || p > 4 * N6; };

  float2 sv[16];  // spectrum at natural positions t16 + G16*i
  if constexpr (MODE == COL_STEP) {
    {
      // unconditional loads, as in colp_kernel: a column past the grid reads
      // its padded slots of Q and column 0 of the state; a slot that holds no
      // kept mode reads k1 = 0, and its value is not used
      const int ms = live ? m : 0;
      gf2* const Sl = glob(f.S) + (size_t)ms * f.h1 + N1 / 4;
      gf2* const Pl = glob(VAR >= VAR_HEUN_P ? f.S2 : f.S) + (size_t)ms * f.h1 + N1 / 4;
      const auto twf = KernelTw6<LOGP, 8>::make(f.tw6_8, t8);
      float2 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = ld(Qc + (t8 + G8 * i) * TQ);
      constexpr int KR[4] = {0, 1, 4, 5};
      // frc: the forcing (not in VAR_EULER); prd: Heun's predictor (VAR_HEUN_C)
      constexpr bool FORCED = VAR != VAR_EULER;
      float2 old[ITF][4], frc[ITF][4], prd[ITF][4];
#pragma unroll
      for (int it = 0; it < ITF; ++it) {
        const int j = t8 + G8 * it;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pos = j + KR[q] * N6;
          const int k1 = j < N6 && kept_at(pos) ? k1_of(pos) : 0;
          old[it][q] = ld(Sl + k1);
          frc[it][q] = FORCED ? forcing_at(f, ms, k1) : make_float2(0.f, 0.f);
          prd[it][q] = VAR == VAR_HEUN_C ? ld(Pl + k1) : make_float2(0.f, 0.f);
        }
      }
      float2 o[ITF * 6];
      fft6<LOGP, false, 8>(v, o, t8, buf0, T, twf);
      const StepScalars sc = step_scalars(f, n, M1, f.cols);
      const float ac = VAR == VAR_HEUN_C ? step_scalars(f, n + 1, M1, f.cols).a : 0.f;  // the corrector's dt c_{n+1} / P
      const float kap2c = f.s2 * (float)m;
      const float dtf = (float)f.dt;
#pragma unroll
      for (int it = 0; it < ITF; ++it) {
        const int j = t8 + G8 * it;
        if (j < N6) {
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            const int pos = j + r * N6;
            float2 val = make_float2(0.f, 0.f);
            if (r != 2 && r != 3 && kept_at(pos)) {
              const int q = r < 2 ? r : r - 2;
              const float kap1 = f.s1 * (float)k1_of(pos);
              const float e = growth_factor(kap1 * kap1 + kap2c * kap2c, sc, f.gamma);
              if constexpr (VAR == VAR_HEUN_C)
                val = make_float2(
                    0.5f * (prd[it][q].x + e * old[it][q].x + ac * o[it * 6 + r].x + dtf * frc[it][q].x),
                    0.5f * (prd[it][q].y + e * old[it][q].y + ac * o[it * 6 + r].y + dtf * frc[it][q].y));
              else
                val = make_float2(e * (old[it][q].x + sc.a * o[it * 6 + r].x + dtf * frc[it][q].x),
                                  e * (old[it][q].y + sc.a * o[it * 6 + r].y + dtf * frc[it][q].y));
            }
            buf0[ff::lds_pad(pos) * T] = val;
          }
        }
      }
    }
    __syncthreads();
    if (tile == 0) {
      // symmetrise column k2 = 0: k1 > 0 conjugated onto -k1, Im at k1 = 0 zeroed
      if (c == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k1 = t8 + G8 * i;
          if (k1 >= 1 && k1 <= K1) buf0[ff::lds_pad(M1 - k1) * T] = ff::cconj(buf0[ff::lds_pad(k1) * T]);
        }
        if (t8 == 0) buf0[0].y = 0.f;
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) sv[i] = buf0[ff::lds_pad(t16 + G16 * i) * T];
    __syncthreads();  // both groups have read the spectrum before buffer 0 is reused
    if (live && grp == 0) {
      gf2* const Dc = VAR == VAR_HEUN_P ? Pc : Sc;  // the predictor goes to S2
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int pos = t16 + G16 * i;
        if (kept_at(pos)) st(Dc + k1_of(pos), sv[i]);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int pos = t16 + G16 * i;
      sv[i] = live && kept_at(pos) ? ld(Sc + k1_of(pos)) : make_float2(0.f, 0.f);
    }
  }

  // group 0: Z+ = IFFT_k1((i kappa1 - kappa2) Phi~) -> Wp; group 1: conj(IFFT_k1((i kappa1 + kappa2) Phi~)) -> Wm
  const auto twi = KernelTw6<LOGP, 16>::make(f.tw6, t16);
  const float kap2 = f.s2 * (float)m * (grp == 0 ? -1.f : 1.f);
  float2 v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float kap1 = f.s1 * (float)k1_of(t16 + G16 * i);
    v[i] = make_float2(-kap1 * sv[i].y + kap2 * sv[i].x, kap1 * sv[i].x + kap2 * sv[i].y);
  }
  float2 o[ITI * 6];
  fft6<LOGP, true, 16>(v, o, t16, bufg, T, twi);
  if (live) {
    gf2* const dst = glob(grp == 0 ? f.Wp : f.Wm);
    const float cs = grp == 0 ? 1.f : -1.f;  // Wm holds the conjugate
#pragma unroll
    for (int it = 0; it < ITI; ++it) {
      const int j = t16 + G16 * it;
      if (j < N6) {
#pragma unroll
        for (int r = 0; r < 6; ++r)
          st_nt<NT>(dst + w_index(j + r * N6, m, f.m), make_float2(o[it * 6 + r].x, cs * o[it * 6 + r].y));
      }
    }
  }
}

// Canonical half spectrum -> state, with the k2 = 0 symmetrisation.
__global__ void set_spectrum_kernel(const FlameDev* __restrict__ fls, int flame, const float2* __restrict__ half) {
  const FlameDev f = fls[flame];
  const int total = f.m * f.h1;
  const int k1max = f.n1 / 4 - 1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int m = e / f.h1, s = e % f.h1;
    const int k1 = s - f.n1 / 4;
    float2 val = make_float2(0.f, 0.f);
    if (s > 0) {
      if (m == 0 && k1 < 0) {
        val = ff::cconj(half[(size_t)(-k1 + k1max) * f.m]);
      } else {
        val = half[(size_t)(k1 + k1max) * f.m + m];
        if (m == 0 && k1 == 0) val.y = 0.f;
      }
    }
    f.S[e] = val;
  }
}

__global__ void get_spectrum_kernel(const FlameDev* __restrict__ fls, int flame, float2* __restrict__ half) {
  const FlameDev f = fls[flame];
  const int rows = f.n1 / 2 - 1;
  const int total = rows * f.m;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int r = e / f.m, m = e % f.m;
    half[e] = f.S[(size_t)m * f.h1 + r + 1];
  }
}

// Spectral sums: per workgroup partial of sum_k w_k |kappa|^2 |Phi~_k|^2 (w = 1 on
// k2 = 0, 2 elsewhere) and a count of non-finite entries.
__global__ void __launch_bounds__(kDiagThreads)
    diag_spectral_kernel(const FlameDev* __restrict__ fls, int flame, double* __restrict__ part) {
  const FlameDev f = fls[flame];
  __shared__ double red[kDiagThreads];
  __shared__ double bad[kDiagThreads];
  const int total = f.m * f.h1;
  double acc = 0.0, nb = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int m = e / f.h1, s = e % f.h1;
    const float2 v = f.S[e];
    if (!isfinite(v.x) || !isfinite(v.y)) {
      nb += 1.0;
      continue;
    }
    const double k1 = (double)f.s1 * (double)(s - f.n1 / 4), k2 = (double)f.s2 * (double)m;
    const double w = m == 0 ? 1.0 : 2.0;
    acc += w * (k1 * k1 + k2 * k2) * ((double)v.x * v.x + (double)v.y * v.y);
  }
  red[threadIdx.x] = acc;
  bad[threadIdx.x] = nb;
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      bad[threadIdx.x] += bad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0];
    part[2 * blockIdx.x + 1] = bad[0];
  }
}

__global__ void __launch_bounds__(kDiagThreads)
    diag_final_kernel(const FlameDev* __restrict__ fls, int flame, long long n, int n_area, int n_spec,
                      double* __restrict__ out) {
  const FlameDev f = fls[flame];
  __shared__ double ra[kDiagThreads], rs[kDiagThreads], rb[kDiagThreads];
  double a = 0.0, s = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_area; i += blockDim.x) a += f.part[i];
  const double* sp = f.part + n_area;
  for (int i = threadIdx.x; i < n_spec; i += blockDim.x) {
    s += sp[2 * i];
    b += sp[2 * i + 1];
  }
  ra[threadIdx.x] = a;
  rs[threadIdx.x] = s;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = r0_at(f, n);
    const float2 s00 = f.S[f.n1 / 4];
    out[0] = r + (double)s00.x;
    out[1] = rs[0] / (2.0 * r * r);
    out[2] = ra[0] / ((double)f.n1 * (double)f.n2);
    out[3] = (rb[0] == 0.0 && isfinite(out[2])) ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------------------ dispatch

namespace {

template <int LOGN>
struct ColTable {
  static void launch(int mode, dim3 grid, hipStream_t st, const FlameDev* fl, long long n, const float2* src) {
    constexpr int th = ColCfg<LOGN>::THREADS, lds = ColCfg<LOGN>::LDS_BYTES;
    const long long* nb = nullptr;
    switch (mode) {
      case COL_STEP: hipLaunchKernelGGL((col_kernel<LOGN, COL_STEP>), grid, dim3(th), lds, st, fl, n, nb, src); break;
      case COL_FIRST:
        hipLaunchKernelGGL((col_kernel<LOGN, COL_FIRST>), grid, dim3(th), lds, st, fl, n, nb, src);
        break;
      case COL_PROJECT:
        hipLaunchKernelGGL((col_kernel<LOGN, COL_PROJECT>), grid, dim3(th), lds, st, fl, n, nb, src);
        break;
      default: hipLaunchKernelGGL((col_kernel<LOGN, COL_SYNTH>), grid, dim3(th), lds, st, fl, n, nb, src); break;
    }
  }
  template <int VAR>
  static KernelLaunch step_kernel_v(int pts) {
    if (pts == 12) return KernelLaunch{nullptr, 0, 0};  // product grid only (ColPTable)
    if (pts == 8) {
      if constexpr (LOGN <= kMaxLog8)
        return KernelLaunch{reinterpret_cast<const void*>(&col_kernel<LOGN, COL_STEP, 8, VAR>),
                            ColCfg<LOGN, 8>::THREADS, ColCfg<LOGN, 8>::LDS_BYTES};
      else
        return KernelLaunch{nullptr, 0, 0};
    }
    return KernelLaunch{reinterpret_cast<const void*>(&col_kernel<LOGN, COL_STEP, ff::kPts, VAR>),
                        ColCfg<LOGN>::THREADS, ColCfg<LOGN>::LDS_BYTES};
  }
  static KernelLaunch step_kernel(int pts, int var) {
    switch (var) {
      case VAR_EULER_F: return step_kernel_v<VAR_EULER_F>(pts);
      case VAR_HEUN_P: return step_kernel_v<VAR_HEUN_P>(pts);
      case VAR_HEUN_C: return step_kernel_v<VAR_HEUN_C>(pts);
      case VAR_NT | VAR_EULER: return step_kernel_v<VAR_NT | VAR_EULER>(pts);
      case VAR_NT | VAR_EULER_F: return step_kernel_v<VAR_NT | VAR_EULER_F>(pts);
      case VAR_NT | VAR_HEUN_P: return step_kernel_v<VAR_NT | VAR_HEUN_P>(pts);
      case VAR_NT | VAR_HEUN_C: return step_kernel_v<VAR_NT | VAR_HEUN_C>(pts);
      default: return step_kernel_v<VAR_EULER>(pts);
    }
  }
};

template <int LOGN>
struct RowTable {
  static void launch(int mode, dim3 grid, hipStream_t st, const FlameDev* fl, long long n, const float* in,
                     float* out) {
    constexpr int th = RowCfg<LOGN>::THREADS, lds = RowCfg<LOGN>::LDS_BYTES;
    const long long* nb = nullptr;
    switch (mode) {
      case ROW_STEP:
        hipLaunchKernelGGL((row_kernel<LOGN, ROW_STEP>), grid, dim3(th), lds, st, fl, n, nb, in, out);
        break;
      case ROW_FORWARD:
        hipLaunchKernelGGL((row_kernel<LOGN, ROW_FORWARD>), grid, dim3(th), lds, st, fl, n, nb, in, out);
        break;
      case ROW_SYNTH:
        hipLaunchKernelGGL((row_kernel<LOGN, ROW_SYNTH>), grid, dim3(th), lds, st, fl, n, nb, in, out);
        break;
      default: hipLaunchKernelGGL((row_kernel<LOGN, ROW_DIAG>), grid, dim3(th), lds, st, fl, n, nb, in, out); break;
    }
  }
  template <bool NT>
  static KernelLaunch step_kernel_nt(int pts) {
    if (pts == 12) {
      if constexpr (LOGN >= kMinLogRow12)
        return KernelLaunch{reinterpret_cast<const void*>(&row_kernel<LOGN, ROW_STEP, 12, NT>),
                            RowCfg<LOGN, 12>::THREADS, RowCfg<LOGN, 12>::LDS_BYTES};
      else
        return KernelLaunch{nullptr, 0, 0};
    }
    if (pts == 8) {
      if constexpr (LOGN <= kMaxLog8)
        return KernelLaunch{reinterpret_cast<const void*>(&row_kernel<LOGN, ROW_STEP, 8, NT>),
                            RowCfg<LOGN, 8>::THREADS, RowCfg<LOGN, 8>::LDS_BYTES};
      else
        return KernelLaunch{nullptr, 0, 0};
    }
    return KernelLaunch{reinterpret_cast<const void*>(&row_kernel<LOGN, ROW_STEP, ff::kPts, NT>),
                        RowCfg<LOGN>::THREADS, RowCfg<LOGN>::LDS_BYTES};
  }
  static KernelLaunch step_kernel(int pts, bool nt) { return nt ? step_kernel_nt<true>(pts) : step_kernel_nt<false>(pts); }
};

template <int LOGN>
struct ColPTable {
  template <int VAR>
  static KernelLaunch info(int mode) {
    if (mode == COL_FIRST)
      return KernelLaunch{reinterpret_cast<const void*>(&colp_kernel<LOGN, COL_FIRST, 16>),
                          ColCfgP<LOGN, 16>::THREADS, ColCfgP<LOGN, 16>::LDS_BYTES};
    return KernelLaunch{reinterpret_cast<const void*>(&colp_kernel<LOGN, COL_STEP, 16, VAR>),
                        ColCfgP<LOGN, 16>::THREADS, ColCfgP<LOGN, 16>::LDS_BYTES};
  }
  template <int VAR>
  static KernelLaunch split(int mode) {
    if constexpr (LOGN > kMaxLog8) {
      return KernelLaunch{nullptr, 0, 0};
    } else {
      if (mode == COL_FIRST)
        return KernelLaunch{reinterpret_cast<const void*>(&colq_kernel<LOGN, COL_FIRST>), ColCfgQ<LOGN>::THREADS,
                            ColCfgQ<LOGN>::LDS_BYTES};
      return KernelLaunch{reinterpret_cast<const void*>(&colq_kernel<LOGN, COL_STEP, VAR>), ColCfgQ<LOGN>::THREADS,
                          ColCfgQ<LOGN>::LDS_BYTES};
    }
  }
  template <int VAR>
  static KernelLaunch twelve(int mode) {
    if (mode == COL_FIRST)
      return KernelLaunch{reinterpret_cast<const void*>(&col_kernel<LOGN, COL_FIRST, 12>),
                          ColCfg<LOGN, 12>::THREADS, ColCfg<LOGN, 12>::LDS_BYTES};
    return KernelLaunch{reinterpret_cast<const void*>(&col_kernel<LOGN, COL_STEP, 12, VAR>),
                        ColCfg<LOGN, 12>::THREADS, ColCfg<LOGN, 12>::LDS_BYTES};
  }
  template <int VAR>
  static KernelLaunch pick(int mode, int pts) {
    return pts == 8 ? split<VAR>(mode) : (pts == 12 ? twelve<VAR>(mode) : info<VAR>(mode));
  }
  // pts 16: colp_kernel<., 16> (radix-16 passes, then radix 6); pts 8: the split
  // kernel (8 points per thread in the forward transform); pts 12: col_kernel
  // in the 12-point plan (ff::Shape12)
  static KernelLaunch step_kernel(int mode, int pts, int var) {
    switch (var) {
      case VAR_EULER_F: return pick<VAR_EULER_F>(mode, pts);
      case VAR_HEUN_P: return pick<VAR_HEUN_P>(mode, pts);
      case VAR_HEUN_C: return pick<VAR_HEUN_C>(mode, pts);
      case VAR_NT | VAR_EULER: return pick<VAR_NT | VAR_EULER>(mode, pts);
      case VAR_NT | VAR_EULER_F: return pick<VAR_NT | VAR_EULER_F>(mode, pts);
      case VAR_NT | VAR_HEUN_P: return pick<VAR_NT | VAR_HEUN_P>(mode, pts);
      case VAR_NT | VAR_HEUN_C: return pick<VAR_NT | VAR_HEUN_C>(mode, pts);
      default: return pick<VAR_EULER>(mode, pts);
    }
  }
};

template <int L>
void dispatch_colp(int logn, int mode, int pts, int var, KernelLaunch* out) {
  if constexpr (L <= kMaxLog) {
    if (logn == L)
      *out = ColPTable<L>::step_kernel(mode, pts, var);
    else
      dispatch_colp<L + 1>(logn, mode, pts, var, out);
  }
}

template <template <int> class Tab, int L, class... A>
void dispatch_log(int logn, A... args) {
  if constexpr (L <= kMaxLog) {
    if (logn == L)
      Tab<L>::launch(args...);
    else
      dispatch_log<Tab, L + 1>(logn, args...);
  }
}

template <template <int> class Tab, int L, class... A>
void dispatch_info(int logn, KernelLaunch* out, A... args) {
  if constexpr (L <= kMaxLog) {
    if (logn == L)
      *out = Tab<L>::step_kernel(args...);
    else
      dispatch_info<Tab, L + 1>(logn, out, args...);
  }
}

}  // namespace

// Step-mode launches go through the kernel tables; with timing events they
// use hipExtLaunchKernel, which records the events in the kernel's own
// dispatch (kernel start and end, no extra queue packets).
void launch_col(int logn1, int mode, int tiles, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                const void* src, int pts, hipEvent_t ev_start, hipEvent_t ev_stop, int var) {
  if (mode == COL_STEP && (var != VAR_EULER || pts != ff::kPts || ev_start || ev_stop)) {
    const KernelLaunch kl = col_step_kernel(logn1, pts, var);
    if (!kl.func) return;
    const long long* nb = nullptr;
    const float2* s = static_cast<const float2*>(src);
    void* args[] = {&fl, &n, &nb, &s};
    if (ev_start || ev_stop)
      (void)hipExtLaunchKernel(kl.func, dim3(tiles, nfl), dim3(kl.threads), args, kl.lds, st, ev_start, ev_stop, 0);
    else
      (void)hipLaunchKernel(kl.func, dim3(tiles, nfl), dim3(kl.threads), args, kl.lds, st);
    return;
  }
  dispatch_log<ColTable, kMinLog>(logn1, mode, dim3(tiles, nfl), st, fl, n, static_cast<const float2*>(src));
}

void launch_row(int logn2, int mode, int groups, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                const float* in, float* out, int pts, hipEvent_t ev_start, hipEvent_t ev_stop, bool nt) {
  if (mode == ROW_STEP && (pts != ff::kPts || nt || ev_start || ev_stop)) {
    const KernelLaunch kl = row_step_kernel(logn2, pts, nt);
    if (!kl.func) return;
    const long long* nb = nullptr;
    void* args[] = {&fl, &n, &nb, &in, &out};
    if (ev_start || ev_stop)
      (void)hipExtLaunchKernel(kl.func, dim3(groups, nfl), dim3(kl.threads), args, kl.lds, st, ev_start, ev_stop, 0);
    else
      (void)hipLaunchKernel(kl.func, dim3(groups, nfl), dim3(kl.threads), args, kl.lds, st);
    return;
  }
  dispatch_log<RowTable, kMinLog>(logn2, mode, dim3(groups, nfl), st, fl, n, in, out);
}

KernelLaunch colp_kernel_info(int logn1, int mode, int pts, int var) {
  KernelLaunch out{nullptr, 0, 0};
  if (logn1 >= kMinLogProduct) dispatch_colp<kMinLogProduct>(logn1, mode, pts, var, &out);
  return out;
}

void launch_colp(int logn1, int mode, int tiles, int nfl, hipStream_t st, const FlameDev* fl, long long n,
                 const void* src, int pts, hipEvent_t ev_start, hipEvent_t ev_stop, int var) {
  const KernelLaunch kl = colp_kernel_info(logn1, mode, pts, var);
  if (!kl.func) return;
  const long long* nb = nullptr;
  const float2* s = static_cast<const float2*>(src);
  void* args[] = {&fl, &n, &nb, &s};
  if (ev_start || ev_stop)
    (void)hipExtLaunchKernel(kl.func, dim3(tiles, nfl), dim3(kl.threads), args, kl.lds, st, ev_start, ev_stop, 0);
  else
    (void)hipLaunchKernel(kl.func, dim3(tiles, nfl), dim3(kl.threads), args, kl.lds, st);
}

namespace {

template <int L>
int col_lds(int logn1) {
  if constexpr (L <= kMaxLog) {
    if (logn1 != L) return col_lds<L + 1>(logn1);
    int b = ColCfg<L, 16>::LDS_BYTES > ColCfg<L, 8>::LDS_BYTES ? ColCfg<L, 16>::LDS_BYTES : ColCfg<L, 8>::LDS_BYTES;
    if constexpr (L >= kMinLogProduct) {
      if (ColCfgP<L, 16>::LDS_BYTES > b) b = ColCfgP<L, 16>::LDS_BYTES;
      if constexpr (L <= kMaxLog8)
        if (ColCfgQ<L>::LDS_BYTES > b) b = ColCfgQ<L>::LDS_BYTES;
      if (ColCfg<L, 12>::LDS_BYTES > b) b = ColCfg<L, 12>::LDS_BYTES;
    }
    return b;
  }
  return 0;
}

template <int L>
int row_lds(int logn2) {
  if constexpr (L <= kMaxLog) {
    if (logn2 != L) return row_lds<L + 1>(logn2);
    int b = RowCfg<L, 16>::LDS_BYTES > RowCfg<L, 8>::LDS_BYTES ? RowCfg<L, 16>::LDS_BYTES : RowCfg<L, 8>::LDS_BYTES;
    if constexpr (L >= kMinLogRow12) {
      if (RowCfg<L, 12>::LDS_BYTES > b) b = RowCfg<L, 12>::LDS_BYTES;
    }
    return b;
  }
  return 0;
}

}  // namespace

int lds_bytes_needed(int logn1, int logn2) {
  const int c = col_lds<kMinLog>(logn1), r = row_lds<kMinLog>(logn2);
  return c > r ? c : r;
}

KernelLaunch col_step_kernel(int logn1, int pts, int var) {
  KernelLaunch out{nullptr, 0, 0};
  dispatch_info<ColTable, kMinLog>(logn1, &out, pts, var);
  return out;
}

KernelLaunch row_step_kernel(int logn2, int pts, bool nt) {
  KernelLaunch out{nullptr, 0, 0};
  dispatch_info<RowTable, kMinLog>(logn2, &out, pts, nt);
  return out;
}

// One thread stores the step index that graph replays read (a vector store).
__global__ void set_step_kernel(long long* __restrict__ counter, long long value) {
  if (threadIdx.x == 0) {
    volatile long long* p = counter;
    *p = value;
  }
}

void launch_set_step(hipStream_t st, long long* counter, long long value) {
  hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, counter, value);
}

void launch_set_spectrum(hipStream_t st, const FlameDev* fl, int flame, int total, const void* half) {
  const int blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  hipLaunchKernelGGL(set_spectrum_kernel, dim3(blocks), dim3(256), 0, st, fl, flame,
                     static_cast<const float2*>(half));
}

void launch_get_spectrum(hipStream_t st, const FlameDev* fl, int flame, int total, void* half) {
  const int blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  hipLaunchKernelGGL(get_spectrum_kernel, dim3(blocks), dim3(256), 0, st, fl, flame, static_cast<float2*>(half));
}

void launch_diag_spectral(hipStream_t st, const FlameDev* fl, int flame, int blocks, double* part) {
  hipLaunchKernelGGL(diag_spectral_kernel, dim3(blocks), dim3(kDiagThreads), 0, st, fl, flame, part);
}

void launch_diag_final(hipStream_t st, const FlameDev* fl, int flame, long long n, int n_area, int n_spec,
                       double* out) {
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kDiagThreads), 0, st, fl, flame, n, n_area, n_spec, out);
}


}  // namespace flame
