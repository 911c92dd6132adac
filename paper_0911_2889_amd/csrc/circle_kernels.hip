// HIP kernels of the circular (two-dimensional) flames: the one-dimensional
// form of Eq. (1) (Section 2 compares such flames with the spherical ones),
//
//   dPhi~_k/dt = (-kappa_k^2/r0^2 + gamma |kappa_k|/(2 r0)) Phi~_k
//                - 1/(2 r0^2) sum_l kappa_l kappa_{k-l} Phi~_l Phi~_{k-l},
//
// kappa_k = s k, r0(t) = t, truncated to |k| <= K = N/4 - 1 and evaluated on
// the N-point augmented grid of Section 3 with integrating-factor Euler, as
// the spherical step is.
//
// One workgroup column of G = N/16 threads steps a pair of circles: their
// gradients g_a, g_b travel as one complex field z = g_a + i g_b (one inverse
// transform), and q_a = g_a^2, q_b = g_b^2 as one complex field q_a + i q_b
// (one forward transform, split by Hermitian symmetry). The spectra stay in
// registers for all the steps of a launch (thread t holds k = t + G i,
// i < 4), so HBM is touched only to load them at the start and store them
// at the end. The twiddles are computed in double precision at the start
// and rounded once, so the kernels need no table or workspace.

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"
#include "flame_dev.hpp"
#include "flame_kernels.hpp"
#include "kernel_common.hpp"

namespace flame {

namespace {

// Table entry i of the power-of-two plan of S (the layout of
// ff::build_twiddles), computed from its definition in double precision.
template <class S>
struct ComputedTw {
  __device__ __forceinline__ float2 operator()(int i) const {
    int q = 1;
    while (q + 1 < S::NBF && i >= S::tw_off(q + 1)) ++q;
    const int ns = S::ns(q), r = S::radix(q);
    const int rel = i - S::tw_off(q);
    const int m = rel / ns + 1, k = rel % ns;
    const long long e = (long long)k * m % (long long)(ns * r);
    double sn, cs;
    sincos(-2.0 * M_PI * double(e) / (double(ns) * double(r)), &sn, &cs);
    return make_float2((float)cs, (float)sn);
  }
};

template <int LOGN>
struct CircleCfg {
  using S = ff::Shape<LOGN, 16>;
  static constexpr int G = S::G;
  static constexpr int B = G >= 256 ? 1 : 256 / G;  // circle pairs per workgroup, interleaved
  static constexpr int THREADS = B * G;
  static constexpr int LDS_BYTES = S::LDS * B * 8;
};

struct CircleScalars {
  float a;   // dt c_n / N: multiplies the unnormalised transform of the squared gradient
  float i1;  // int_{t_n}^{t_{n+1}} ds / r0
  float i2;  // int ds / r0^2
};

__device__ __forceinline__ CircleScalars circle_scalars(const CircleDev& d, long long n, int npts) {
  const float t = (float)(d.t0 + (double)n * d.dt);
  const float dt = (float)d.dt;
  const float x = dt / t;
  CircleScalars s;
  s.a = 0.5f * x / (t * (float)npts);
  s.i1 = log1pf(x);
  s.i2 = x / (t + dt);
  return s;
}

// The packed gradient spectrum of the pair (i kappa (Phi~_a + i Phi~_b) at
// k >= 0, and its mirror image at -k) through LDS into the registers of the
// inverse transform (natural order t + G i, zero in the middle half).
template <class S>
__device__ __forceinline__ void gradient_spectrum(const float2 (&sa)[4], const float2 (&sb)[4], const float (&kap)[4],
                                                  int t, float2* my, int stride, float2 (&v)[16]) {
  constexpr int G = S::G, N = S::N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = t + G * i;
    const float2 pa = sa[i], pb = sb[i];
    // u = Pa + i Pb at +k; w = conj(Pa) + i conj(Pb) at -k
    const float2 u = make_float2(pa.x - pb.y, pa.y + pb.x);
    const float2 w = make_float2(pa.x + pb.y, pb.x - pa.y);
    my[ff::lds_pad(k) * stride] = make_float2(-kap[i] * u.y, kap[i] * u.x);
    if (k > 0) my[ff::lds_pad(N - k) * stride] = make_float2(kap[i] * w.y, -kap[i] * w.x);
  }
  if (t == 0) my[ff::lds_pad(3 * N / 4) * stride] = make_float2(0.f, 0.f);  // k = -N/4 lies outside the box
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i)
    v[i] = (i < 4 || i >= 12) ? my[ff::lds_pad(t + G * i) * stride] : make_float2(0.f, 0.f);
  __syncthreads();  // the transform reuses the LDS
}

template <int LOGN>
__global__ void __launch_bounds__(CircleCfg<LOGN>::THREADS)
    circle_step_kernel(CircleDev d, long long n0, int nsteps) {
  using Cfg = CircleCfg<LOGN>;
  using S = typename Cfg::S;
  constexpr int G = S::G, B = Cfg::B, N = S::N, H = N / 4;  // H = K + 1 stored modes per circle
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int p = tid % B, t = tid / B;
  const int pair = blockIdx.x * B + p;
  const int ca = 2 * pair, cb = 2 * pair + 1;
  const bool live_a = ca < d.n_circles, live_b = cb < d.n_circles;
  float2* my = lds + p;
  const ff::RegTwS<S, ComputedTw<S>, 2> tw(ComputedTw<S>{}, t);
  gf2* const sg = glob(d.S);
  // loads without conditions: a circle past the batch reads circle 0 (never stored)
  const size_t oa = (size_t)(live_a ? ca : 0) * H, ob = (size_t)(live_b ? cb : 0) * H;
  float2 sa[4], sb[4];
  float kap[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = t + G * i;
    sa[i] = ld(sg + oa + k);
    sb[i] = ld(sg + ob + k);
    kap[i] = d.seg * (float)k;
  }
  for (int s = 0; s < nsteps; ++s) {
    const CircleScalars sc = circle_scalars(d, n0 + s, N);
    float2 v[16];
    gradient_spectrum<S>(sa, sb, kap, t, my, B, v);
    fft_s<S, true, kPrune>(v, t, my, B, tw);
    // q_a + i q_b: the squared gradients of the two circles
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_float2(v[i].x * v[i].x, v[i].y * v[i].y);
    fft_s<S, false>(v, t, my, B, tw);
    __syncthreads();
    ff::FftS<S, false>::scatter(v, t, my, B);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = t + G * i;
      const float2 yk = my[S::nat(k) * B];
      const float2 ym = my[S::nat(k == 0 ? 0 : N - k) * B];
      const float2 na = make_float2(0.5f * (yk.x + ym.x), 0.5f * (yk.y - ym.y));
      const float2 nb = make_float2(0.5f * (yk.y + ym.y), 0.5f * (ym.x - yk.x));
      const float kk = kap[i] * kap[i];
      const float e = __expf(-kk * sc.i2 + 0.5f * d.gamma * fabsf(kap[i]) * sc.i1);
      sa[i] = make_float2(e * (sa[i].x + sc.a * na.x), e * (sa[i].y + sc.a * na.y));
      sb[i] = make_float2(e * (sb[i].x + sc.a * nb.x), e * (sb[i].y + sc.a * nb.y));
    }
    if (t == 0) {  // Im Phi~_0 = 0 (symmetrisation)
      sa[0].y = 0.f;
      sb[0].y = 0.f;
    }
    __syncthreads();  // the next step writes the LDS
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = t + G * i;
    if (live_a) st(sg + oa + k, sa[i]);
    if (live_b) st(sg + ob + k, sb[i]);
  }
}

// Per circle: out[4 c + 0] = r0 + Re Phi~_0, [1] = <Phi_t> = sum_k w_k kappa_k^2
// |Phi~_k|^2 / (2 r0^2) (w = 1 at k = 0, 2 elsewhere), [2] = length excess
// (1/N) sum_j x/(1 + sqrt(1 + x)), x = g^2/r0^2, [3] = 1 if every stored
// coefficient is finite, else 0; sums in double.
template <int LOGN>
__global__ void __launch_bounds__(CircleCfg<LOGN>::THREADS)
    circle_diag_kernel(CircleDev d, long long n, double* __restrict__ out) {
  using Cfg = CircleCfg<LOGN>;
  using S = typename Cfg::S;
  constexpr int G = S::G, B = Cfg::B, N = S::N, H = N / 4;
  extern __shared__ float2 lds[];
  static_assert(3 * Cfg::THREADS * 8 <= Cfg::LDS_BYTES, "reduction area in the transform's LDS");
  double(*red)[Cfg::THREADS] = reinterpret_cast<double(*)[Cfg::THREADS]>(lds);  // after the transform
  const int tid = threadIdx.x;
  const int p = tid % B, t = tid / B;
  const int pair = blockIdx.x * B + p;
  const int ca = 2 * pair, cb = 2 * pair + 1;
  const bool live_a = ca < d.n_circles, live_b = cb < d.n_circles;
  float2* my = lds + p;
  const ff::RegTwS<S, ComputedTw<S>, 2> tw(ComputedTw<S>{}, t);
  gf2* const sg = glob(d.S);
  const size_t oa = (size_t)(live_a ? ca : 0) * H, ob = (size_t)(live_b ? cb : 0) * H;
  float2 sa[4], sb[4];
  float kap[4];
  double va = 0.0, vb = 0.0, bad_a = 0.0, bad_b = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = t + G * i;
    sa[i] = ld(sg + oa + k);
    sb[i] = ld(sg + ob + k);
    kap[i] = d.seg * (float)k;
    const double w = k == 0 ? 1.0 : 2.0, kk = (double)kap[i] * (double)kap[i];
    va += w * kk * ((double)sa[i].x * sa[i].x + (double)sa[i].y * sa[i].y);
    vb += w * kk * ((double)sb[i].x * sb[i].x + (double)sb[i].y * sb[i].y);
    const bool fa = isfinite(sa[i].x) && isfinite(sa[i].y), fb = isfinite(sb[i].x) && isfinite(sb[i].y);
    bad_a += fa ? 0.0 : 1.0;
    bad_b += fb ? 0.0 : 1.0;
    // the pair shares one transform: a non-finite coefficient of one circle
    // enters it as zero, so that the other circle's length excess stays its own
    if (!fa) sa[i] = make_float2(0.f, 0.f);
    if (!fb) sb[i] = make_float2(0.f, 0.f);
  }
  const double r = d.t0 + (double)n * d.dt;
  float2 v[16];
  gradient_spectrum<S>(sa, sb, kap, t, my, B, v);
  fft_s<S, true, kPrune>(v, t, my, B, tw);
  double ja = 0.0, jb = 0.0;
  const double inv_r2 = 1.0 / (r * r);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double xa = (double)v[i].x * v[i].x * inv_r2, xb = (double)v[i].y * v[i].y * inv_r2;
    ja += xa / (1.0 + sqrt(1.0 + xa));
    jb += xb / (1.0 + sqrt(1.0 + xb));
  }
  // per pair: tree sums over the G threads of column p (stride B); the
  // transform's last pass left the LDS free
  __syncthreads();
  for (int half = 0; half < 2; ++half) {
    red[0][tid] = half ? vb : va;
    red[1][tid] = half ? jb : ja;
    red[2][tid] = half ? bad_b : bad_a;
    __syncthreads();
    for (int w = G / 2; w > 0; w >>= 1) {
      if (t < w)
        for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + w * B];
      __syncthreads();
    }
    const int c = half ? cb : ca;
    if (t == 0 && c < d.n_circles) {
      const float2 s0 = half ? sb[0] : sa[0];
      out[4 * (size_t)c + 0] = r + (double)s0.x;
      out[4 * (size_t)c + 1] = red[0][tid] / (2.0 * r * r);
      out[4 * (size_t)c + 2] = red[1][tid] / (double)N;
      out[4 * (size_t)c + 3] = (red[2][tid] == 0.0 && isfinite(red[1][tid])) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
}

template <int L>
bool circle_dispatch(int logn, bool diag, const CircleDev& d, long long n, int nsteps, double* out, hipStream_t st) {
  if constexpr (L > kMaxLog) {
    return false;
  } else {
    if (logn != L) return circle_dispatch<L + 1>(logn, diag, d, n, nsteps, out, st);
    using Cfg = CircleCfg<L>;
    const int pairs = (d.n_circles + 1) / 2;
    const int blocks = (pairs + Cfg::B - 1) / Cfg::B;
    if (diag)
      hipLaunchKernelGGL(circle_diag_kernel<L>, dim3(blocks), dim3(Cfg::THREADS), Cfg::LDS_BYTES, st, d, n, out);
    else
      hipLaunchKernelGGL(circle_step_kernel<L>, dim3(blocks), dim3(Cfg::THREADS), Cfg::LDS_BYTES, st, d, n, nsteps);
    return true;
  }
}

}  // namespace

bool launch_circle_step(int logn, const CircleDev& d, long long n, int nsteps, hipStream_t st) {
  return circle_dispatch<kMinLog>(logn, false, d, n, nsteps, nullptr, st);
}

bool launch_circle_diag(int logn, const CircleDev& d, long long n, double* out, hipStream_t st) {
  return circle_dispatch<kMinLog>(logn, true, d, n, 0, out, st);
}

}  // namespace flame
