// Adjoint of the flame step and of the area functional (gfx950).
//
// Cotangents hold the Fourier coefficients of a real band-limited grid field
// (the gradient with respect to the grid values of Phi), in the state layout.
// For the step n -> n+1 (integrating-factor Euler)
//     Phi^{n+1} = E^n (Phi^n + dt c_n Pi |grad Phi^n|^2),
// the transpose of its Jacobian is
//     lambda^n = mu - 2 dt c_n Pi div(m grad Phi^n),   mu = E^n lambda^{n+1},
// with m the grid field of mu; E^n is a real even multiplier (self-adjoint),
// the projection Pi is self-adjoint, and the adjoint of the spectral gradient
// restricted to the box is -Pi div with div taken by the grid transform.
// The area excess J = (1/P) sum sqrt(1 + |grad Phi|^2/r0^2) - 1 has
//     dJ/dPhi = -Pi div( grad Phi / (P r0^2 sqrt(1 + |grad Phi|^2/r0^2)) ).
//
// One adjoint step is three kernels (on the step's grid: N1 rows, or the
// 3 N1/4-row product grid with adjp_col in place of adj_col):
//  * adj_col<ADJ_A>: mu = E lambda per column; column inverse transforms of mu
//    (-> Q) and of (i kappa1 -+ kappa2) Phi~^n (-> Wp, Wm, as the forward step);
//  * adj_row<ROW_ADJ>: per row pair, m (one packed real synthesis for two
//    rows), z = g1 + i g2, zeta = m z = w1 + i w2, forward row transform of
//    zeta split by Hermitian symmetry into the row transforms of w1 (-> A1)
//    and i kappa2 w2 (-> A2);
//  * adj_col<ADJ_C>: column forward transforms of A1 and A2, divergence
//    i kappa1 A1 + A2 on the box, lambda^n = mu - 2 dt c_n div / P.
// The seed uses adj_row<ROW_SEED> (zeta = z / (r0^2 sqrt(1 + x))) and
// adj_col<SEED_C> (lambda = -div / P^2) after the column transforms of the
// state.

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"
#include "flame_dev.hpp"
#include "flame_kernels.hpp"
#include "kernel_common.hpp"

namespace flame {

namespace {

__device__ __forceinline__ float efactor(const FlameDev& f, const StepScalars& sc, int k1, float kap2) {
  const float kap1 = f.s1 * (float)k1;
  const float kk2 = kap1 * kap1 + kap2 * kap2;
  return growth_factor(kk2, sc, f.gamma);
}

}  // namespace

template <int LOGN1, int MODE>
__global__ void __launch_bounds__(ColCfg<LOGN1>::THREADS) __attribute__((amdgpu_waves_per_eu(COL_WAVES_PER_EU)))
    adj_col_kernel(const FlameDev* __restrict__ fls, long long n, const float2* state, const float2* lam_in,
                   float2* lam_out) {
  using S = ff::Shape<LOGN1>;
  constexpr int G = S::G, T = ColCfg<LOGN1>::T, N1 = S::N;
  extern __shared__ float2 lds[];
  const FlameDev f = fls[blockIdx.y];
  const int tid = threadIdx.x;
  const int c = tid % T, t = tid / T;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int m = tile * T + c;
  const bool live = m < f.m;
  float2* my = lds + c;
  constexpr int TQ = ColCfg<LOGN1>::TQ, QS = ColCfg<LOGN1>::QS;
  const size_t tile_base = ((((size_t)m >> QS) * N1) << QS) + (m & (TQ - 1));  // column m of Q, A1, A2
  const size_t col = (size_t)m * f.h1 + N1 / 4;  // element k1 of column m at col + k1
  // loads carry no condition (a branch around a load makes the compiler wait
  // for every load issued before it): a column past the grid reads column 0
  // of the spectra and its padded slots of A1 and A2, and is never stored
  const size_t coll = (size_t)(live ? m : 0) * f.h1 + N1 / 4;
  const auto tw1 = KernelTw<LOGN1>::make(f.tw1, t);
  const float kap2 = f.s2 * (float)m;

  float2 v[ff::kPts];
  float2 lam[8];
  if constexpr (MODE != SEED_C) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int i = kept_reg<LOGN1, ff::kPts>(kk);
      const int k1 = t + G * i - (i >= 12 ? N1 : 0);
      lam[kk] = ld(glob(const_cast<float2*>(lam_in)) + coll + k1);
    }
  }

  if constexpr (MODE == ADJ_A) {
    const StepScalars sc = step_scalars(f, n, f.n1, f.n2);
    float2 sv[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int i = kept_reg<LOGN1, ff::kPts>(kk);
      const int k1 = t + G * i - (i >= 12 ? N1 : 0);
      sv[kk] = ld(glob(const_cast<float2*>(state)) + coll + k1);
    }
    // M = column synthesis of mu = E lambda  -> Q
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) v[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int i = kept_reg<LOGN1, ff::kPts>(kk);
      const int k1 = t + G * i - (i >= 12 ? N1 : 0);
      v[i] = ff::cscale(lam[kk], efactor(f, sc, k1, kap2));
    }
    fft<LOGN1, true, kPrune>(v, t, my, T, tw1);
    if (live) {
#pragma unroll
      for (int i = 0; i < ff::kPts; ++i) st(glob(f.Q) + tile_base + (t + G * i) * TQ, v[i]);
    }
    // Z+ and Z- of the state, exactly as the forward column kernel
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const float sgn = pass == 0 ? -1.f : 1.f;
#pragma unroll
      for (int i = 0; i < ff::kPts; ++i) v[i] = make_float2(0.f, 0.f);
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int i = kept_reg<LOGN1, ff::kPts>(kk);
        const float kap1 = f.s1 * (float)(t + G * i - (i >= 12 ? N1 : 0));
        v[i] = make_float2(-kap1 * sv[kk].y + sgn * kap2 * sv[kk].x, kap1 * sv[kk].x + sgn * kap2 * sv[kk].y);
      }
      fft<LOGN1, true, kPrune>(v, t, my, T, tw1);
      if (live) {
        gf2* dst = glob(pass == 0 ? f.Wp : f.Wm);
#pragma unroll
        for (int i = 0; i < ff::kPts; ++i)
          st(dst + w_index(t + G * i, m, f.m), pass == 0 ? v[i] : ff::cconj(v[i]));
      }
    }
  } else {
    // forward column transforms of the row transforms of w1 and i kappa2 w2
    float2 u[8], w[8];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      gf2* srcp = glob(pass == 0 ? f.A1 : f.A2) + tile_base;
#pragma unroll
      for (int i = 0; i < ff::kPts; ++i) v[i] = ld(srcp + (t + G * i) * TQ);
      fft<LOGN1, false>(v, t, my, T, tw1);
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) (pass == 0 ? u : w)[kk] = v[kept_reg<LOGN1, ff::kPts>(kk)];
    }
    float2 out[8];
    const float inv_p = 1.0f / ((float)f.n1 * (float)f.n2);
    StepScalars sc{};
    if constexpr (MODE == ADJ_C) sc = step_scalars(f, n, f.n1, f.n2);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int i = kept_reg<LOGN1, ff::kPts>(kk);
      const int k1 = t + G * i - (i >= 12 ? N1 : 0);
      const float kap1 = f.s1 * (float)k1;
      // raw divergence i kappa1 U1 + V2 (sums without the 1/P factors)
      const float2 div = make_float2(-kap1 * u[kk].y + w[kk].x, kap1 * u[kk].x + w[kk].y);
      float2 val;
      if constexpr (MODE == ADJ_C) {
        const float e = efactor(f, sc, k1, kap2);
        val = make_float2(e * lam[kk].x - 2.f * sc.a * div.x, e * lam[kk].y - 2.f * sc.a * div.y);
      } else {
        val = ff::cscale(div, -inv_p * inv_p);
      }
      if (k1 == -N1 / 4) val = make_float2(0.f, 0.f);
      out[kk] = val;
    }
    if (tile == 0) {  // symmetrise column k2 = 0: copy k1 > 0 conjugated onto -k1
      if (c == 0) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) lds[t + G * kk] = out[kk];
      }
      __syncthreads();
      if (c == 0) {
#pragma unroll
        for (int kk = 4; kk < 8; ++kk) {
          const int k1 = t + G * kept_reg<LOGN1, ff::kPts>(kk) - N1;
          if (k1 > -N1 / 4) out[kk] = ff::cconj(lds[-k1]);
        }
        if (t == 0) out[0].y = 0.f;
      }
      __syncthreads();
    }
    if (live) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int i = kept_reg<LOGN1, ff::kPts>(kk);
        const int k1 = t + G * i - (i >= 12 ? N1 : 0);
        st(glob(lam_out) + col + k1, out[kk]);
      }
    }
  }
}

// adj_col on the product grid (ColCfgP, M1 = 3 N1/4 rows; see colp_kernel):
// ADJ_A and ADJ_C with the length-M1 transforms. ADJ_A's inputs are in the
// natural map, so its three inverse transforms need no remap; ADJ_C's forward
// transforms leave A1 and A2 in the radix-6 output map, where the update is
// formed; the kept modes go through LDS to the natural map (column k2 = 0
// symmetrised on the way) and are stored from there.
template <int LOGN1, int MODE>
__global__ void __launch_bounds__((ColCfgP<LOGN1, 16>::THREADS))
    __attribute__((amdgpu_waves_per_eu(COL_WAVES_PER_EU)))
    adjp_col_kernel(const FlameDev* __restrict__ fls, long long n, const float2* state, const float2* lam_in,
                    float2* lam_out) {
  static_assert(MODE == ADJ_A || MODE == ADJ_C, "product-grid adjoint modes");
  using Cfg = ColCfgP<LOGN1, 16>;
  using S6 = typename Cfg::S;
  constexpr int LOGP = LOGN1 - 3;
  constexpr int G = S6::G, T = Cfg::T, M1 = S6::N, N6 = S6::N6, IT = S6::IT6, N1 = 1 << LOGN1;
  constexpr int TQ = Cfg::TQ, QS = Cfg::QS, K1 = N1 / 4 - 1;
  extern __shared__ float2 lds[];
  const FlameDev f = fls[blockIdx.y];
  const int tid = threadIdx.x;
  const int c = tid % T, t = tid / T;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int m = tile * T + c;
  const bool live = m < f.m;
  float2* my = lds + c;
  const size_t tile_base = ((((size_t)m >> QS) * M1) << QS) + (m & (TQ - 1));  // column m of Q, A1, A2
  const size_t col = (size_t)m * f.h1 + N1 / 4;  // element k1 of column m at col + k1
  // loads carry no condition, as in adj_col_kernel; a slot that holds no kept
  // mode reads k1 = 0 and its value is replaced or unused
  const size_t coll = (size_t)(live ? m : 0) * f.h1 + N1 / 4;
  const auto tw = KernelTw6<LOGP, 16>::make(f.tw6, t);
  const float kap2 = f.s2 * (float)m;
  const StepScalars sc = step_scalars(f, n, M1, f.n2);
  auto k1_of = [](int p) { return p < M1 / 2 ? p : p - M1; };
  auto kept_at = [](int p) { return p < 2 * N6 || p > 4 * N6; };
  gf2* const lin = glob(const_cast<float2*>(lam_in));

  if constexpr (MODE == ADJ_A) {
    float2 sv[16], v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int pos = t + G * i;
      const int k1 = kept_at(pos) ? k1_of(pos) : 0;
      v[i] = ld(lin + coll + k1);
      sv[i] = ld(glob(const_cast<float2*>(state)) + coll + k1);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {  // mu = E lambda, zero outside the box (selects, after every load)
      const int pos = t + G * i;
      const bool kept = kept_at(pos);
      const float e = efactor(f, sc, kept ? k1_of(pos) : 0, kap2);
      v[i] = kept ? ff::cscale(v[i], e) : make_float2(0.f, 0.f);
      sv[i] = kept ? sv[i] : make_float2(0.f, 0.f);
    }
    float2 o[IT * 6];
    fft6<LOGP, true, 16>(v, o, t, my, T, tw);  // M = column synthesis of mu -> Q
    if (live) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int j = t + G * it;
        if (j < N6) {
#pragma unroll
          for (int r = 0; r < 6; ++r) st(glob(f.Q) + tile_base + (size_t)(j + r * N6) * TQ, o[it * 6 + r]);
        }
      }
    }
    // Z+ and Z- of the state, as the forward column kernel
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const float sgn = pass == 0 ? -1.f : 1.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float kap1 = f.s1 * (float)k1_of(t + G * i);
        v[i] = make_float2(-kap1 * sv[i].y + sgn * kap2 * sv[i].x, kap1 * sv[i].x + sgn * kap2 * sv[i].y);
      }
      fft6<LOGP, true, 16>(v, o, t, my, T, tw);
      if (live) {
        gf2* dst = glob(pass == 0 ? f.Wp : f.Wm);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          const int j = t + G * it;
          if (j < N6) {
#pragma unroll
            for (int r = 0; r < 6; ++r)
              st(dst + w_index(j + r * N6, m, f.m), pass == 0 ? o[it * 6 + r] : ff::cconj(o[it * 6 + r]));
          }
        }
      }
    }
  } else {
    // lambda^{n+1} at the kept modes, in the radix-6 output map
    constexpr int KR[4] = {0, 1, 4, 5};
    float2 lam[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = t + G * it;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pos = j + KR[q] * N6;
        lam[it][q] = ld(lin + coll + (j < N6 && kept_at(pos) ? k1_of(pos) : 0));
      }
    }
    // forward column transforms of the row transforms of w1 and i kappa2 w2
    float2 ou[IT * 6], ow[IT * 6];
    {
      float2 v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = ld(glob(f.A1) + tile_base + (size_t)(t + G * i) * TQ);
      fft6<LOGP, false, 16>(v, ou, t, my, T, tw);
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = ld(glob(f.A2) + tile_base + (size_t)(t + G * i) * TQ);
      fft6<LOGP, false, 16>(v, ow, t, my, T, tw);
    }
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
            const int k1 = k1_of(pos);
            const float kap1 = f.s1 * (float)k1;
            const float2 u = ou[it * 6 + r], w = ow[it * 6 + r];
            // raw divergence i kappa1 U1 + V2 (sums without the 1/P factors)
            const float2 div = make_float2(-kap1 * u.y + w.x, kap1 * u.x + w.y);
            const float e = efactor(f, sc, k1, kap2);
            val = make_float2(e * lam[it][q].x - 2.f * sc.a * div.x, e * lam[it][q].y - 2.f * sc.a * div.y);
          }
          my[ff::lds_pad(pos) * T] = val;
        }
      }
    }
    __syncthreads();
    if (tile == 0) {  // symmetrise column k2 = 0: k1 > 0 conjugated onto -k1, Im at k1 = 0 zeroed
      if (c == 0) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int k1 = t + G * i;
          if (k1 >= 1 && k1 <= K1) my[ff::lds_pad(M1 - k1) * T] = ff::cconj(my[ff::lds_pad(k1) * T]);
        }
        if (t == 0) my[0].y = 0.f;
      }
      __syncthreads();
    }
    if (live) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int pos = t + G * i;
        if (kept_at(pos)) st(glob(lam_out) + col + k1_of(pos), my[ff::lds_pad(pos) * T]);
      }
    }
  }
}

template <int LOGN2, int MODE>
__global__ void __launch_bounds__(RowCfg<LOGN2>::THREADS) __attribute__((amdgpu_waves_per_eu(ADJ_ROW_WAVES_PER_EU)))
    adj_row_kernel(const FlameDev* __restrict__ fls, long long n) {
  using S = ff::Shape<LOGN2>;
  constexpr int G = S::G, B = RowCfg<LOGN2>::B, N2 = S::N;
  extern __shared__ float2 lds[];
  const FlameDev f = fls[blockIdx.y];
  const int tid = threadIdx.x;
  const int p = tid % B, t = tid / B;
  const int pair = xcd_swizzle(blockIdx.x, gridDim.x) * B + p;
  // the adjoint step runs on the step's product grid; the seed on the grid's rows
  const int n1 = MODE == ROW_ADJ ? f.rows : f.n1, ts = f.tshift, mcols = f.m;
  const bool live = pair < n1 / 2;
  const int ja = 2 * pair, jb = 2 * pair + 1;
  // rows the loads read: a pair past the grid reads pair 0 (never stored), so
  // that no load sits behind a branch
  const int jal = live ? ja : 0, jbl = live ? jb : 1;
  float2* my = lds + p;
  const auto tw2 = KernelTw<LOGN2>::make(f.tw2, t);
  gf2* const Wp = glob(f.Wp);
  gf2* const Wm = glob(f.Wm);
  gf2* const Q = glob(f.Q);
  gf2* const A1 = glob(f.A1);
  gf2* const A2 = glob(f.A2);
  const float inv_r2 = [&] {
    const double r = r0_at(f, n);
    return (float)(1.0 / (r * r));
  }();

  // both rows' packed-gradient spectra, loaded before m's transform so that
  // their latency is hidden behind it
  float2 wv[2][ff::kPts];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int row = half ? jbl : jal;
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) {
      const int idx = t + G * i;
      float2 val = make_float2(0.f, 0.f);
      if (i < 4) {
        val = ld(Wp + w_index(row, idx, mcols));
      } else if (i >= 12) {
        const int mm = N2 - idx;  // < mcols except at i = 12, t = 0
        val = ld(Wm + w_index(row, i > 12 || t > 0 ? mm : 0, mcols));
      }
      wv[half][i] = val;
    }
  }

  float ma[ff::kPts], mb[ff::kPts];
  if constexpr (MODE == ROW_ADJ) {
    // m for both rows: Y = X_a + i X_b, X(k2) = M(k2), X(-k2) = conj(M(k2))
    float2 y[ff::kPts];
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) {
      const int idx = t + G * i;
      float2 val = make_float2(0.f, 0.f);
      if (i < 4) {
        const float2 a = ld(Q + tiled(jal, idx, n1, ts)), b = ld(Q + tiled(jbl, idx, n1, ts));
        val = make_float2(a.x - b.y, a.y + b.x);
      } else if (i >= 12) {
        const int mm = N2 - idx;  // < mcols except at i = 12, t = 0
        const int mc = i > 12 || t > 0 ? mm : 0;
        const float2 a = ld(Q + tiled(jal, mc, n1, ts)), b = ld(Q + tiled(jbl, mc, n1, ts));
        val = make_float2(a.x + b.y, -a.y + b.x);
      }
      y[i] = val;
    }
    y[12] = t > 0 ? y[12] : make_float2(0.f, 0.f);  // a select once every load is issued
    fft<LOGN2, true, kPrune>(y, t, my, B, tw2);
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) {
      ma[i] = y[i].x;
      mb[i] = y[i].y;
    }
  }

#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int row = half ? jb : ja;  // the row this half stores (live pairs only)
    float2 v[ff::kPts];
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) v[i] = wv[half][i];
    v[12] = t > 0 ? v[12] : make_float2(0.f, 0.f);  // the position past the box
    fft<LOGN2, true, kPrune>(v, t, my, B, tw2);  // z = g1 + i g2 on the row
#pragma unroll
    for (int i = 0; i < ff::kPts; ++i) {
      float s;
      if constexpr (MODE == ROW_ADJ) {
        s = half ? mb[i] : ma[i];
      } else {
        const float x = (v[i].x * v[i].x + v[i].y * v[i].y) * inv_r2;
        s = inv_r2 / sqrtf(1.f + x);
      }
      v[i] = ff::cscale(v[i], s);  // zeta = w1 + i w2
    }
    fft<LOGN2, false>(v, t, my, B, tw2);
    __syncthreads();
    ff::Fft<LOGN2, false>::scatter(v, t, my, B);
    __syncthreads();
    if (live) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = t + G * i;
        const float2 xk = my[ff::Shape<LOGN2>::nat(k) * B];
        const float2 xm = my[ff::Shape<LOGN2>::nat((N2 - k) & (N2 - 1)) * B];
        // row transform of w1: (Xi(k) + conj(Xi(-k)))/2; of i kappa2 w2: kappa2 (Xi(k) - conj(Xi(-k)))/2
        const float2 u1 = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
        const float h = 0.5f * f.s2 * (float)k;
        const float2 v2 = make_float2(h * (xk.x - xm.x), h * (xk.y + xm.y));
        st(A1 + tiled(row, k, n1, ts), u1);
        st(A2 + tiled(row, k, n1, ts), v2);
      }
    }
    __syncthreads();
  }
}

namespace {

template <int LOGN>
struct AdjColTable {
  static void launch(int mode, dim3 grid, hipStream_t st, const FlameDev* fl, long long n, const float2* s,
                     const float2* li, float2* lo) {
    constexpr int th = ColCfg<LOGN>::THREADS, lds = ColCfg<LOGN>::LDS_BYTES;
    switch (mode) {
      case ADJ_A: hipLaunchKernelGGL((adj_col_kernel<LOGN, ADJ_A>), grid, dim3(th), lds, st, fl, n, s, li, lo); break;
      case ADJ_C: hipLaunchKernelGGL((adj_col_kernel<LOGN, ADJ_C>), grid, dim3(th), lds, st, fl, n, s, li, lo); break;
      default: hipLaunchKernelGGL((adj_col_kernel<LOGN, SEED_C>), grid, dim3(th), lds, st, fl, n, s, li, lo); break;
    }
  }
};

template <int LOGN>
struct AdjRowTable {
  static void launch(int mode, dim3 grid, hipStream_t st, const FlameDev* fl, long long n) {
    constexpr int th = RowCfg<LOGN>::THREADS, lds = RowCfg<LOGN>::LDS_BYTES;
    if (mode == ROW_ADJ)
      hipLaunchKernelGGL((adj_row_kernel<LOGN, ROW_ADJ>), grid, dim3(th), lds, st, fl, n);
    else
      hipLaunchKernelGGL((adj_row_kernel<LOGN, ROW_SEED>), grid, dim3(th), lds, st, fl, n);
  }
};

template <template <int> class Tab, int L, class... A>
void dispatch_adj(int logn, A... args) {
  if constexpr (L <= kMaxLog) {
    if (logn == L)
      Tab<L>::launch(args...);
    else
      dispatch_adj<Tab, L + 1>(logn, args...);
  }
}

}  // namespace

template <int L>
void dispatch_adjp(int logn, int mode, dim3 grid, hipStream_t st, const FlameDev* fl, long long n, const float2* s,
                   const float2* li, float2* lo) {
  if constexpr (L <= kMaxLog) {
    if (logn != L) return dispatch_adjp<L + 1>(logn, mode, grid, st, fl, n, s, li, lo);
    constexpr int th = ColCfgP<L, 16>::THREADS, lds = ColCfgP<L, 16>::LDS_BYTES;
    if (mode == ADJ_A)
      hipLaunchKernelGGL((adjp_col_kernel<L, ADJ_A>), grid, dim3(th), lds, st, fl, n, s, li, lo);
    else
      hipLaunchKernelGGL((adjp_col_kernel<L, ADJ_C>), grid, dim3(th), lds, st, fl, n, s, li, lo);
  }
}

void launch_adjp_col(int logn1, int mode, int tiles, hipStream_t st, const FlameDev* fl, long long n,
                     const void* state, const void* lam_in, void* lam_out) {
  if (logn1 < kMinLogProduct || (mode != ADJ_A && mode != ADJ_C)) return;
  dispatch_adjp<kMinLogProduct>(logn1, mode, dim3(tiles, 1), st, fl, n, static_cast<const float2*>(state),
                                static_cast<const float2*>(lam_in), static_cast<float2*>(lam_out));
}

void launch_adj_col(int logn1, int mode, int tiles, hipStream_t st, const FlameDev* fl, long long n,
                    const void* state, const void* lam_in, void* lam_out) {
  dispatch_adj<AdjColTable, kMinLog>(logn1, mode, dim3(tiles, 1), st, fl, n, static_cast<const float2*>(state),
                                     static_cast<const float2*>(lam_in), static_cast<float2*>(lam_out));
}

void launch_adj_row(int logn2, int mode, int groups, hipStream_t st, const FlameDev* fl, long long n) {
  dispatch_adj<AdjRowTable, kMinLog>(logn2, mode, dim3(groups, 1), st, fl, n);
}

}  // namespace flame
