// Device helpers shared by the forward and adjoint kernels.

#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_engine.hpp"
#include "flame_dev.hpp"

namespace flame {

template <int LOGN, bool INV, bool OUTER, int PTS, int P = 0, class TW>
__device__ __forceinline__ void fft_passes(float2 (&v)[PTS], int t, float2* lds, int stride, const TW& tw) {
  using S = ff::Shape<LOGN, PTS>;
  if constexpr (P < S::NPASS) {
    ff::Fft<LOGN, INV, PTS>::template butterflies<P, TW, OUTER>(v, t, lds, stride, tw);
    if constexpr (P + 1 < S::NPASS) {
      __syncthreads();
      ff::Fft<LOGN, INV, PTS>::template gather<P>(v, t, lds, stride);
      __syncthreads();
    }
    fft_passes<LOGN, INV, OUTER, PTS, P + 1>(v, t, lds, stride, tw);
  }
}

// Transform the PTS registers of every group of the workgroup (all threads
// must call it: it contains workgroup barriers). On entry v[i] holds the
// input at position t + G*i, on exit the output at the same position.
// OUTER: the input is known to vanish in the middle half of the registers
// (the retained box fills only the first and last quarter of a padded
// spectrum).
template <int LOGN, bool INV, bool OUTER = false, class TW, int PTS>
__device__ __forceinline__ void fft(float2 (&v)[PTS], int t, float2* lds, int stride, const TW& tw) {
  fft_passes<LOGN, INV, OUTER, PTS, 0>(v, t, lds, stride, tw);
}

// The same for any register shape S (ff::Shape, ff::Shape12); with
// ff::Shape12, OUTER means the middle third of the registers vanishes.
template <class S, bool INV, bool OUTER = false, int P = 0, class TW>
__device__ __forceinline__ void fft_s(float2 (&v)[S::PTS], int t, float2* lds, int stride, const TW& tw) {
  if constexpr (P < S::NPASS) {
    ff::FftS<S, INV>::template butterflies<P, TW, OUTER>(v, t, lds, stride, tw);
    if constexpr (P + 1 < S::NPASS) {
      __syncthreads();
      ff::FftS<S, INV>::template gather<P>(v, t, lds, stride);
      __syncthreads();
    }
    fft_s<S, INV, OUTER, P + 1>(v, t, lds, stride, tw);
  }
}

// Global-memory views: loads and stores through these pointers compile to
// global_* instructions (flat ones would also wait on LDS counters).
using v2f = float __attribute__((ext_vector_type(2)));
using gf2 = __attribute__((address_space(1))) v2f;
using gf1 = __attribute__((address_space(1))) float;
__device__ __forceinline__ gf2* glob(float2* p) { return (gf2*)p; }
__device__ __forceinline__ const gf1* glob(const float* p) { return (const gf1*)p; }
__device__ __forceinline__ gf1* glob(float* p) { return (gf1*)p; }
__device__ __forceinline__ float2 ld(const gf2* p) {
  const v2f v = *p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st(gf2* p, float2 a) {
  v2f v;
  v.x = a.x;
  v.y = a.y;
  *p = v;
}
// Store that is non-temporal if NT (the line is not kept in L2 for reuse).
template <bool NT>
__device__ __forceinline__ void st_nt(gf2* p, float2 a) {
  v2f v;
  v.x = a.x;
  v.y = a.y;
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Twiddle source of a kernel: cached in registers for the kernel's lifetime
// (each kernel runs two or three transforms of one length), or read from the
// table in every pass.
struct GlobalFetch {
  const gf2* tw;
  __device__ __forceinline__ float2 operator()(int i) const { return ld(tw + i); }
};

// 16384-point transforms take 1024 threads per workgroup, i.e. at most 128
// registers per thread: there they read the twiddles from the table (cached
// in L1/L2) at each use instead of holding 42 of them in registers.
template <int LOGN>
constexpr bool cache_twiddles() { return kCacheTwiddles && LOGN <= 13; }

template <int LOGN, int PTS = ff::kPts>
struct KernelTw {
  using Type = typename std::conditional<cache_twiddles<LOGN>(), ff::RegTw<LOGN, GlobalFetch, kTwCacheMinNs, PTS>,
                                         ff::GlobalTw<LOGN, PTS>>::type;
  static __device__ __forceinline__ Type make(const float2* tw, int t) {
    if constexpr (cache_twiddles<LOGN>()) {
      return Type(GlobalFetch{(const gf2*)tw}, t);
    } else {
      return Type{tw, t};
    }
  }
};

// Twiddles of a step kernel's transform along an axis of 2^LOGN points with
// PTS points per thread: the power-of-two plans (tables p16, p8), or, for
// PTS = 12, the length-3*2^LOGN/4 transform of the 12-point plan (table p12),
// cached in registers.
template <int LOGN, int PTS>
struct AxisTw {
  using Type = typename std::conditional<PTS == 12, ff::RegTwS<TShape<LOGN, PTS>, GlobalFetch, kTwCacheMinNs>,
                                         typename KernelTw<LOGN, PTS == 12 ? 16 : PTS>::Type>::type;
  static __device__ __forceinline__ Type make(const float2* p16, const float2* p8, const float2* p12, int t) {
    if constexpr (PTS == 12) {
      return Type(GlobalFetch{(const gf2*)p12}, t);
    } else {
      return KernelTw<LOGN, PTS>::make(PTS == 8 ? p8 : p16, t);
    }
  }
};

// Twiddle source for kernels short of registers: the passes with
// Ns >= MIN_NS keep their twiddles in registers for the kernel's lifetime
// (loaded from the global table), the passes with smaller Ns read theirs at
// each use from a copy of the first LDS_ENTRIES entries of the table in LDS
// (those passes' part), which the kernel writes before its first transform's
// second pass. The passes with small Ns have few distinct twiddles, so the
// lanes of a wave read few LDS addresses.
template <class S, int MIN_NS>
struct SplitTw {
  using Reg = ff::RegTwS<S, GlobalFetch, MIN_NS>;
  static constexpr int first_cached() {
    int p = 1;
    while (p < S::NBF && !Reg::cached(p)) ++p;
    return p;
  }
  static constexpr int LDS_ENTRIES = S::tw_off(first_cached()) > 0 ? S::tw_off(first_cached()) : 1;
  Reg reg;
  const float2* tab;
  int t;
  __device__ __forceinline__ SplitTw(const float2* global_tab, const float2* lds_tab, int t_)
      : reg(GlobalFetch{(const gf2*)global_tab}, t_), tab(lds_tab), t(t_) {}
  // copy the table's first LDS_ENTRIES entries into LDS (every thread of the workgroup calls it)
  static __device__ __forceinline__ void stage(float2* lds_tab, const float2* global_tab, int tid, int threads) {
    for (int i = tid; i < LDS_ENTRIES; i += threads) lds_tab[i] = ld((const gf2*)global_tab + i);
  }
  template <int P>
  __device__ __forceinline__ float2 get(int b, int r) const {
    if constexpr (Reg::cached(P)) {
      return reg.template get<P>(b, r);
    } else {
      constexpr int NS = S::ns(P);
      return tab[S::tw_off(P) + (r - 1) * NS + ff::mod_ns<NS>(t + b * S::G)];
    }
  }
};

// Twiddles of a length 6*2^LOGP transform, cached in registers.
template <int LOGP, int PTS>
struct KernelTw6 {
  using Type = ff::RegTwS<ff::Shape6<LOGP, PTS>, GlobalFetch, kTwCacheMinNs>;
  static __device__ __forceinline__ Type make(const float2* tw, int t) { return Type(GlobalFetch{(const gf2*)tw}, t); }
};

// Transform of length 6*2^LOGP (ff::Shape6): on entry v[i] holds the input at
// position t + G*i; on exit o[it*6 + r] holds the output at position
// j + r*N6, j = t + G*it (zero where j >= N6). Contains workgroup barriers
// (all threads must call it), the last one after the radix-6 pass has read
// LDS, so the caller may write LDS at once.
template <int LOGP, int PTS>
using Out6 = float2[ff::Shape6<LOGP, PTS>::IT6 * 6];
template <int PTS>
using Regs = float2[PTS];

template <int LOGP, bool INV, int PTS, class TW, int P = 0>
__device__ __forceinline__ void fft6(Regs<PTS>& v, Out6<LOGP, PTS>& o, int t, float2* lds, int stride, const TW& tw) {
  using S = ff::Shape6<LOGP, PTS>;
  using F = ff::FftS<S, INV>;
  if constexpr (P < S::NBF) {
    F::template butterflies<P, TW, false>(v, t, lds, stride, tw);
    __syncthreads();
    if constexpr (P + 1 < S::NBF) {
      F::template gather<P>(v, t, lds, stride);
      __syncthreads();
    }
    fft6<LOGP, INV, PTS, TW, P + 1>(v, o, t, lds, stride, tw);
  } else {
    F::last6(o, t, lds, stride, tw);
    __syncthreads();
  }
}

struct StepScalars {
  float a;    // dt * c_n / P, multiplies the raw transform of |grad Phi|^2
  float i1;   // int_{t_n}^{t_{n+1}} dt / r0
  float i2;   // int_{t_n}^{t_{n+1}} dt / r0^2
};

// Entry of the reference-radius table for step index n (clamped to the
// table; the host checks the range before every launch).
__device__ __forceinline__ const double* r0_entry(const FlameDev& f, long long n) {
  const long long i = n < 0 ? 0 : (n >= f.r0n ? f.r0n - 1 : n);
  return f.r0tab + 3 * i;
}

// r0(t_n): the table's, or t_n for the paper's law r0(t) = t (Section 2).
__device__ __forceinline__ double r0_at(const FlameDev& f, long long n) {
  return f.r0tab ? r0_entry(f, n)[0] : f.t0 + (double)n * f.dt;
}

// Scalars of step n: c_n = 1/(2 r0(t_n)^2), I1 = int r0^-1, I2 = int r0^-2
// over [t_n, t_{n+1}]: for r0(t) = t in closed form, I1 = ln(t_{n+1}/t_n),
// I2 = 1/t_n - 1/t_{n+1} (the time formed in double); else from the table.
// `rows` x `cols` is the grid the quadratic term was formed on (N1 or
// 3 N1/4 theta rows, N2 or 3 N2/4 phi points): the forward transforms are
// unnormalised, so a = dt c_n / (rows cols).
__device__ __forceinline__ StepScalars step_scalars(const FlameDev& f, long long n, int rows, int cols) {
  StepScalars s;
  if (f.r0tab) {
    const double* e = r0_entry(f, n);
    s.a = (float)(f.dt / (2.0 * e[0] * e[0] * (double)rows * (double)cols));
    s.i1 = (float)e[1];
    s.i2 = (float)e[2];
    return s;
  }
  const float t = (float)(f.t0 + (double)n * f.dt);
  const float dt = (float)f.dt;
  const float x = dt / t;
  s.a = 0.5f * x / (t * (float)rows * (float)cols);
  s.i1 = log1pf(x);
  s.i2 = x / (t + dt);
  return s;
}

// Exact linear propagator of one step for |kappa|^2 = kk2 (Eq. (1) linear part
// integrated over [t_n, t_n+1]): exp(-|kappa|^2 I2 + gamma |kappa| I1 / 2).
// The hardware exp2 and square root: the exponent's rounding costs a relative
// error of about |x| 2^-24 in E, which matters only where E << 1.
__device__ __forceinline__ float growth_factor(float kk2, const StepScalars& sc, float gamma) {
  return __expf(-kk2 * sc.i2 + 0.5f * gamma * __builtin_amdgcn_sqrtf(kk2) * sc.i1);
}

// f~_k of Eq. (1) for stored column m and wavenumber k1, read from the bound
// forcing spectrum (state layout), or zero when none is bound. The update
// takes dt f~ inside the propagator, like the quadratic term:
// E (Phi~ + dt (f~ - c N)). m must be a stored column. The load is issued
// either way (from the state, which has the same layout, when no forcing is
// bound) and the value selected afterwards: a branch around it would make
// the compiler wait for every load issued before it.
__device__ __forceinline__ float2 forcing_at(const FlameDev& f, int m, int k1) {
  const float2* base = f.F ? f.F : f.S;
  const float2 v = ld((const gf2*)base + (size_t)m * f.h1 + (f.n1 >> 2) + k1);
  return f.F ? v : make_float2(0.f, 0.f);
}

// Offset of element (j1, m) of Wp from f.Wp, and of Wm from f.Wm (Wp and Wm
// fill the two halves of the W buffer): [j1/4][m][j1%4], so that the two rows
// of a row pair are adjacent (the row kernel reads both with one 16-byte load
// per lane) and a column workgroup of T columns writes four rows of them as
// one 32 T-byte piece of Wp (64 bytes at T = 2), and one of Wm, each complete
// when it is stored.
__device__ __forceinline__ int w_index(int j1, int m, int mcols) {
  return (((j1 >> 2) * mcols + m) << 2) + (j1 & 3);
}

using v4f = float __attribute__((ext_vector_type(4)));
using gf4 = __attribute__((address_space(1))) v4f;
// Elements (2 q, m) and (2 q + 1, m) of Wp (or Wm) at p = f.Wp + w_index(2 q, m, M) (or f.Wm + ...).
__device__ __forceinline__ void ld_pair(const gf2* p, float2& a, float2& b) {
  const v4f v = *(const gf4*)p;
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}

// Offset of element (j1, m) in the tiled [m/TQ][j1][m%TQ] layout of Q (and of
// the adjoint scratch A1, A2); n1 is the number of rows j1 of the grid the
// array holds (N1, or 3 N1/4 on the product grid), tshift = log2(TQ).
__device__ __forceinline__ int tiled(int j1, int m, int n1, int tshift) {
  return (((m >> tshift) * n1 + j1) << tshift) + (m & ((1 << tshift) - 1));
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give every XCD a contiguous range of work items so that neighbouring
// rows, which share cache lines of the tiled arrays, meet in one L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Register slot kk (0..7) of the kept spectral positions: registers
// 0..LOW-1 hold k = t + G*i >= 0, registers HIGH..PTS-1 hold k = t + G*i - L < 0
// (the first and last quarter of a padded length L = N, or the first and
// last third of a product-grid length L = 3N/4; TfShape).
template <int LOGN, int PTS>
__device__ __forceinline__ constexpr int kept_reg(int kk) {
  return kk < TfShape<LOGN, PTS>::LOW ? kk : kk + (TfShape<LOGN, PTS>::HIGH - TfShape<LOGN, PTS>::LOW);
}


}  // namespace flame
