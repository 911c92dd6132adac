// Register/LDS Stockham FFT engine for gfx950 (wave64).
//
// One length-N transform (N = 2^LOGN, 16 <= N <= 16384) is owned by a group
// of G = N/PTS threads (PTS = 16 or 8 points per thread). Thread t holds the
// points x[t + G*i], i = 0..PTS-1, in registers. A pass of radix R (PTS, or
// the smaller power-of-two remainder in the last pass) lets each thread run
// PTS/R butterflies on its own registers; between
// passes the group exchanges data through LDS (Stockham autosort ordering,
// so input and output both come out in natural order with the same
// "t + G*i" register map). Global loads and stores therefore stay coalesced:
// consecutive threads touch consecutive positions.
//
// Several groups share a workgroup by interleaving: group g of B stores
// element idx at lds[slot(idx) * B + g], where the slot map of each exchange
// inserts spare slots to break the power-of-two bank strides (lds_pad,
// lds_pad32 and lds_pad32_256 below; a Shape chooses them per exchange).
//
// Twiddles come from a table built on the host in double precision and
// rounded once to float: pass p >= 1 with Ns = 16^p and radix R stores
// w(k, r) = exp(-2 pi i r k / (Ns R)) at [(r - 1) * Ns + k], 0 < r < R,
// k < Ns, so that the lanes of a wave (consecutive k) read consecutive
// addresses for each r.
//
// The pass functions are __host__ __device__ so the same code can be
// driven thread by thread on the CPU to check the index maps.

#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ff {

constexpr int kPts = 16;  // default points per thread

constexpr int kMaxPass = 8;

struct PassPlan {
  int logn, n, g, npass;
  int radix[kMaxPass];
  int ns[kMaxPass];
  int tw_off[kMaxPass];
  int tw_size;
};

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// Radix-PTS passes, the remainder radix last.
constexpr PassPlan make_pass_plan(int logn, int pts = kPts) {
  PassPlan p{};
  const int lp = ilog2c(pts);
  p.logn = logn;
  p.n = 1 << logn;
  p.g = p.n / pts;
  const int full = logn / lp, rem = logn % lp;
  p.npass = full + (rem ? 1 : 0);
  int ns = 1, off = 0;
  for (int q = 0; q < p.npass; ++q) {
    p.radix[q] = q < full ? pts : (1 << rem);
    p.ns[q] = ns;
    p.tw_off[q] = off;
    if (q > 0) off += ns * (p.radix[q] - 1);
    ns *= p.radix[q];
  }
  for (int q = p.npass; q < kMaxPass; ++q) {
    p.radix[q] = 1;
    p.ns[q] = ns;
    p.tw_off[q] = off;
  }
  p.tw_size = off;
  return p;
}

// Length 12 * 2^e with 12 points per thread: a radix-12 pass, then radix-4
// passes, and a radix-2 pass last when e is odd (every radix divides 12, so
// each thread runs 12/R butterflies of a pass on its own registers).
constexpr PassPlan make_plan12(int e) {
  PassPlan p{};
  p.logn = -1;  // not a power of two
  p.n = 12 << e;
  p.g = 1 << e;
  p.npass = 1 + e / 2 + (e & 1);
  int ns = 1, off = 0;
  for (int q = 0; q < kMaxPass; ++q) {
    const int r = q == 0 ? 12 : (q < p.npass ? (q <= e / 2 ? 4 : 2) : 1);
    p.radix[q] = r;
    p.ns[q] = ns;
    p.tw_off[q] = off;
    if (q > 0 && q < p.npass) off += ns * (r - 1);
    ns *= r;
  }
  p.tw_size = off;
  return p;
}

// LDS layouts of a transform's exchange areas (slots of 8 bytes; the LDS has
// 64 banks of 4 bytes, and a wave's 8-byte accesses go 32 lanes at a time, so
// an access is free of bank conflicts when its 32 lanes hit 32 distinct slots
// modulo 32).
// lds_pad: a spare slot after every 16 elements (N + N/16 slots). With
// several transforms interleaved in one area (stride > 1) it keeps both the
// strided writes of the butterflies and the unit-stride reads free of
// conflicts; with one transform per area (stride 1) the unit-stride reads
// take two passes over the banks.
__host__ __device__ __forceinline__ constexpr int lds_pad(int idx) { return idx + (idx >> 4); }
// For one transform per area: a spare slot after every 32 elements keeps the
// unit-stride reads and the stride-16 writes of a first radix-16 pass (Ns = 1)
// free of conflicts; the second pass (Ns = 16) writes two runs of 16 elements
// 256 apart, which 8 more slots after every 256 elements put into the other
// half of the banks. Both fit in N + N/16 slots.
__host__ __device__ __forceinline__ constexpr int lds_pad32(int idx) { return idx + (idx >> 5); }
__host__ __device__ __forceinline__ constexpr int lds_pad32_256(int idx) { return idx + (idx >> 5) + 8 * (idx >> 8); }

template <int LOGN, int PTS_ = kPts>
struct Shape {
  static constexpr int PTS = PTS_;
  static constexpr PassPlan plan = make_pass_plan(LOGN, PTS);
  static constexpr int N = 1 << LOGN;
  static constexpr int G = N / PTS;
  static constexpr int NPASS = plan.npass;
  static constexpr int NBF = NPASS;  // passes run by Fft::butterflies (all of them)
  static constexpr int LDS = N + N / 16;  // padded slots per transform
  static constexpr int radix(int p) { return plan.radix[p]; }
  static constexpr int ns(int p) { return plan.ns[p]; }
  static constexpr int tw_off(int p) { return plan.tw_off[p]; }
  // The kernels give transforms of N >= 4096 an exchange area of their own
  // (stride 1); those use the layouts for one transform per area.
  static constexpr bool SOLO = LOGN >= 12 && PTS == 16;
  // slot of element i in the exchange after pass P, and in a natural-order exchange (scatter)
  template <int P>
  static __host__ __device__ __forceinline__ constexpr int slot(int i) {
    if constexpr (SOLO) return ns(P) == 16 ? lds_pad32_256(i) : lds_pad32(i);
    return lds_pad(i);
  }
  static __host__ __device__ __forceinline__ constexpr int nat(int i) { return SOLO ? lds_pad32(i) : lds_pad(i); }
  static_assert(LOGN >= 4 && LOGN <= 14, "transform length must be 16..16384");
  static_assert(PTS == 8 || PTS == 16, "8 or 16 points per thread");
};

// Transform of N = 6 * 2^LOGP points: the radix-PTS passes of the length-2^LOGP
// plan run over the whole array (G = N/PTS threads, PTS points each), then a
// last radix-6 pass with Ns = N6 = 2^LOGP. Its N6 butterflies are spread over
// the G threads as j = t + G*it, it < IT6 (the last round partly idle); it
// reads its inputs x[j + r*N6] from LDS and leaves output r of butterfly j,
// the transform at position j + r*N6, in register it*6 + r. The twiddles of
// the power-of-two passes are those of the length-2^LOGP table (they depend
// on Ns*R only); the radix-6 pass adds exp(-2 pi i r k / N) at
// [TW6 + (r - 1)*N6 + k], 0 < r < 6, k < N6.
template <int LOGP, int PTS_ = kPts>
struct Shape6 {
  static constexpr int PTS = PTS_;
  static constexpr PassPlan plan = make_pass_plan(LOGP, PTS);
  static constexpr int N6 = 1 << LOGP;
  static constexpr int N = 6 * N6;
  static constexpr int G = N / PTS;
  static constexpr int NBF = plan.npass;  // power-of-two passes (Fft::butterflies)
  static constexpr int NPASS = NBF + 1;
  static constexpr int IT6 = (N6 + G - 1) / G;
  static constexpr int TW6 = plan.tw_size;
  static constexpr int TW_SIZE = TW6 + 5 * N6;
  static constexpr int LDS = N + N / 16;
  static constexpr int radix(int p) { return p < NBF ? plan.radix[p] : 6; }
  static constexpr int ns(int p) { return p < NBF ? plan.ns[p] : N6; }
  static constexpr int tw_off(int p) { return p < NBF ? plan.tw_off[p] : TW6; }
  template <int P>
  static __host__ __device__ __forceinline__ constexpr int slot(int i) { return lds_pad(i); }
  static __host__ __device__ __forceinline__ constexpr int nat(int i) { return lds_pad(i); }
  static_assert(LOGP >= 4 && LOGP <= 11, "power-of-two part must be 16..2048");
  static_assert(PTS == 8 || PTS == 16, "8 or 16 points per thread");
};

// Transform of N = 12 * 2^E points with 12 points per thread (make_plan12):
// G = 2^E threads, thread t holding x[t + G*i], i < 12, like Shape. With
// N = 3 * 2^q the length-N transform of a product grid (3/4 of a power of
// two) runs on G = N/12 threads, which makes waves per CU a multiple of four
// where 16 points per thread would not.
template <int E>
struct Shape12 {
  static constexpr int PTS = 12;
  static constexpr PassPlan plan = make_plan12(E);
  static constexpr int N = 12 << E;
  static constexpr int G = 1 << E;
  static constexpr int NPASS = plan.npass;
  static constexpr int NBF = NPASS;
  static constexpr int LDS = N + N / 16;
  static constexpr int radix(int p) { return plan.radix[p]; }
  static constexpr int ns(int p) { return plan.ns[p]; }
  static constexpr int tw_off(int p) { return plan.tw_off[p]; }
  template <int P>
  static __host__ __device__ __forceinline__ constexpr int slot(int i) { return lds_pad(i); }
  static __host__ __device__ __forceinline__ constexpr int nat(int i) { return lds_pad(i); }
  static_assert(E >= 2 && E <= 10, "length 48..12288");
};

// k mod ns for k >= 0 (ns a compile-time constant, not always a power of two)
template <int NS>
__host__ __device__ __forceinline__ constexpr int mod_ns(int k) {
  if constexpr ((NS & (NS - 1)) == 0) {
    return k & (NS - 1);
  } else {
    return (int)((unsigned)k % (unsigned)NS);
  }
}

// ---------------------------------------------------------------- complex

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by the quarter-turn root: -i for the forward transform, +i for the inverse
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_q(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// multiply by exp(-+ i pi/4) (the eighth root of the transform's direction)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_e1(float2 a) {
  constexpr float c = 0.70710678118654752440f;
  return INV ? make_float2(c * (a.x - a.y), c * (a.x + a.y)) : make_float2(c * (a.x + a.y), c * (a.y - a.x));
}

// multiply by exp(-+ 3 i pi/4)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_e3(float2 a) {
  constexpr float c = 0.70710678118654752440f;
  return INV ? make_float2(-c * (a.x + a.y), c * (a.x - a.y)) : make_float2(c * (a.y - a.x), -c * (a.x + a.y));
}

// multiply by exp(s * i * theta) with (cos, sin) given for the forward sign convention
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_root(float2 a, float c, float s) {
  // forward root: c - i s ; inverse: c + i s
  return INV ? make_float2(a.x * c - a.y * s, a.x * s + a.y * c) : make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
}

// ------------------------------------------------------- small DFTs in registers
// X[m] = sum_r x[r] w^(r m), w = exp(-2 pi i / R) (forward) or exp(+2 pi i / R) (inverse)

template <bool INV>
__host__ __device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

template <bool INV>
__host__ __device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = mul_q<INV>(csub(x1, x3));
  x0 = cadd(a0, a2);
  x2 = csub(a0, a2);
  x1 = cadd(a1, a3);
  x3 = csub(a1, a3);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft8(float2* x) {
  float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = mul_e1<INV>(o1);
  o2 = mul_q<INV>(o2);
  o3 = mul_e3<INV>(o3);
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft16(float2* x) {
  // r = 4 r1 + r2, m = m1 + 4 m2: length-4 transforms over r1, inner roots, length-4 over r2
  constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
  float2 y[16];
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) {
    float2 a = x[r2], b = x[r2 + 4], c = x[r2 + 8], d = x[r2 + 12];
    dft4<INV>(a, b, c, d);
    y[4 * r2 + 0] = a;
    y[4 * r2 + 1] = b;
    y[4 * r2 + 2] = c;
    y[4 * r2 + 3] = d;
  }
  // y[4 r2 + m1] *= w16^(r2 m1)
  y[5] = mul_root<INV>(y[5], c1, s1);    // w^1
  y[6] = mul_e1<INV>(y[6]);              // w^2
  y[7] = mul_root<INV>(y[7], s1, c1);    // w^3: cos(3pi/8) = sin(pi/8)
  y[9] = mul_e1<INV>(y[9]);              // w^2
  y[10] = mul_q<INV>(y[10]);             // w^4
  y[11] = mul_e3<INV>(y[11]);            // w^6
  y[13] = mul_root<INV>(y[13], s1, c1);  // w^3
  y[14] = mul_e3<INV>(y[14]);            // w^6
  y[15] = mul_root<INV>(y[15], -c1, -s1);  // w^9: cos(9pi/8) = -cos(pi/8), sin(9pi/8) = -sin(pi/8)
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) {
    float2 a = y[m1], b = y[4 + m1], c = y[8 + m1], d = y[12 + m1];
    dft4<INV>(a, b, c, d);
    x[m1] = a;
    x[m1 + 4] = b;
    x[m1 + 8] = c;
    x[m1 + 12] = d;
  }
}

// dft16 for inputs x[4..11] == 0 (only the first and last quarter set).
template <bool INV>
__host__ __device__ __forceinline__ void dft16_outer(float2* x) {
  constexpr float c1 = 0.92387953251128675613f;
  constexpr float s1 = 0.38268343236508977173f;
  float2 y[16];
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) {
    // length-4 transform of (x[r2], 0, 0, x[r2 + 12])
    const float2 a = x[r2], d = x[r2 + 12], qd = mul_q<INV>(d);
    y[4 * r2 + 0] = cadd(a, d);
    y[4 * r2 + 1] = csub(a, qd);
    y[4 * r2 + 2] = csub(a, d);
    y[4 * r2 + 3] = cadd(a, qd);
  }
  y[5] = mul_root<INV>(y[5], c1, s1);
  y[6] = mul_e1<INV>(y[6]);
  y[7] = mul_root<INV>(y[7], s1, c1);
  y[9] = mul_e1<INV>(y[9]);
  y[10] = mul_q<INV>(y[10]);
  y[11] = mul_e3<INV>(y[11]);
  y[13] = mul_root<INV>(y[13], s1, c1);
  y[14] = mul_e3<INV>(y[14]);
  y[15] = mul_root<INV>(y[15], -c1, -s1);
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) {
    float2 a = y[m1], b = y[4 + m1], c = y[8 + m1], d = y[12 + m1];
    dft4<INV>(a, b, c, d);
    x[m1] = a;
    x[m1 + 4] = b;
    x[m1 + 8] = c;
    x[m1 + 12] = d;
  }
}

// dft8 for inputs x[2..5] == 0.
template <bool INV>
__host__ __device__ __forceinline__ void dft8_outer(float2* x) {
  // even part: length-4 transform of (x0, 0, 0, x6); odd part of (x1, 0, 0, x7)
  const float2 qe = mul_q<INV>(x[6]), qo = mul_q<INV>(x[7]);
  const float2 e0 = cadd(x[0], x[6]), e1 = csub(x[0], qe), e2 = csub(x[0], x[6]), e3 = cadd(x[0], qe);
  float2 o0 = cadd(x[1], x[7]), o1 = csub(x[1], qo), o2 = csub(x[1], x[7]), o3 = cadd(x[1], qo);
  o1 = mul_e1<INV>(o1);
  o2 = mul_q<INV>(o2);
  o3 = mul_e3<INV>(o3);
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

// length-3 DFT: w3 = exp(-+ 2 pi i / 3) = -1/2 -+ i sqrt(3)/2
template <bool INV>
__host__ __device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  constexpr float h = 0.86602540378443864676f;  // sqrt(3)/2
  const float2 s = cadd(b, c), d = csub(b, c);
  const float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
  // forward: X1 = m - i h d, X2 = m + i h d (inverse swaps them)
  const float2 ihd = make_float2(-h * d.y, h * d.x);
  a = cadd(a, s);
  b = INV ? cadd(m, ihd) : csub(m, ihd);
  c = INV ? csub(m, ihd) : cadd(m, ihd);
}

// length-6 DFT as 3 x 2: r = 3 r1 + r2, m = m1 + 2 m2; radix-2 over r1, the
// inner roots w6^(r2 m1), radix-3 over r2
template <bool INV>
__host__ __device__ __forceinline__ void dft6(float2* x) {
  constexpr float h = 0.86602540378443864676f;
  float2 a0 = cadd(x[0], x[3]), b0 = csub(x[0], x[3]);
  float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
  float2 a2 = cadd(x[2], x[5]), b2 = csub(x[2], x[5]);
  // b1 *= w6 = 1/2 -+ i h, b2 *= w6^2 = -1/2 -+ i h
  b1 = INV ? make_float2(0.5f * b1.x - h * b1.y, 0.5f * b1.y + h * b1.x)
           : make_float2(0.5f * b1.x + h * b1.y, 0.5f * b1.y - h * b1.x);
  b2 = INV ? make_float2(-0.5f * b2.x - h * b2.y, -0.5f * b2.y + h * b2.x)
           : make_float2(-0.5f * b2.x + h * b2.y, -0.5f * b2.y - h * b2.x);
  dft3<INV>(a0, a1, a2);
  dft3<INV>(b0, b1, b2);
  x[0] = a0;
  x[2] = a1;
  x[4] = a2;
  x[1] = b0;
  x[3] = b1;
  x[5] = b2;
}

// length-12 DFT as 4 x 3: r = 3 a + b, m = c + 4 d. Length-4 transforms over
// a for each b, the inner roots w12^(b c), then length-3 transforms over b:
// X[c + 4 d] = sum_b w3^(b d) w12^(b c) sum_a x[3 a + b] w4^(a c).
// ZMID: the caller guarantees x[4..7] == 0 (a spectrum kept in the first and
// last third), which drops the terms that vanish.
template <bool INV, bool ZMID = false>
__host__ __device__ __forceinline__ void dft12(float2* x) {
  constexpr float h = 0.86602540378443864676f;  // sqrt(3)/2 = cos(pi/6)
  float2 y[3][4];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    float2 a0 = x[b], a1 = x[3 + b], a2 = x[6 + b], a3 = x[9 + b];
    if constexpr (ZMID) {
      // zero inputs: x[4] (a=1,b=1), x[5] (a=1,b=2), x[6] (a=2,b=0), x[7] (a=2,b=1)
      if (b == 0) {  // a2 == 0
        const float2 s13 = cadd(a1, a3), d13 = mul_q<INV>(csub(a1, a3));
        y[b][0] = cadd(a0, s13);
        y[b][2] = csub(a0, s13);
        y[b][1] = cadd(a0, d13);
        y[b][3] = csub(a0, d13);
      } else if (b == 1) {  // a1 == a2 == 0
        const float2 qa3 = mul_q<INV>(a3);
        y[b][0] = cadd(a0, a3);
        y[b][1] = csub(a0, qa3);
        y[b][2] = csub(a0, a3);
        y[b][3] = cadd(a0, qa3);
      } else {  // a1 == 0
        const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2), qa3 = mul_q<INV>(a3);
        y[b][0] = cadd(s02, a3);
        y[b][2] = csub(s02, a3);
        y[b][1] = csub(d02, qa3);
        y[b][3] = cadd(d02, qa3);
      }
    } else {
      dft4<INV>(a0, a1, a2, a3);
      y[b][0] = a0;
      y[b][1] = a1;
      y[b][2] = a2;
      y[b][3] = a3;
    }
  }
  // inner roots: w12^1 = (h, -+1/2), w12^2 = (1/2, -+h), w12^3 = -+i, w12^4 = (-1/2, -+h), w12^6 = -1
  y[1][1] = mul_root<INV>(y[1][1], h, 0.5f);
  y[1][2] = mul_root<INV>(y[1][2], 0.5f, h);
  y[1][3] = mul_q<INV>(y[1][3]);
  y[2][1] = mul_root<INV>(y[2][1], 0.5f, h);
  y[2][2] = mul_root<INV>(y[2][2], -0.5f, h);
  y[2][3] = make_float2(-y[2][3].x, -y[2][3].y);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float2 p = y[0][c], q = y[1][c], r = y[2][c];
    dft3<INV>(p, q, r);
    x[c] = p;
    x[c + 4] = q;
    x[c + 8] = r;
  }
}

template <int R, bool INV>
__host__ __device__ __forceinline__ void dft(float2* x) {
  if constexpr (R == 2) {
    dft2<INV>(x[0], x[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 8) {
    dft8<INV>(x);
  } else if constexpr (R == 12) {
    dft12<INV>(x);
  } else {
    static_assert(R == 16, "radix");
    dft16<INV>(x);
  }
}

// ------------------------------------------------------------ Stockham passes

// Twiddle source reading the table in global memory on every use.
template <class S>
struct GlobalTwS {
  const float2* tw;
  int t;
  template <int P>
  __host__ __device__ __forceinline__ float2 get(int b, int r) const {
    constexpr int NS = S::ns(P);
    const int k = mod_ns<NS>(t + b * S::G);
    return tw[S::tw_off(P) + (r - 1) * NS + k];
  }
  // radix-6 pass of a Shape6 transform: round `it`, butterfly j = t + G*it
  __host__ __device__ __forceinline__ float2 get6(int it, int r) const {
    const int j = t + it * S::G;
    return tw[S::TW6 + (r - 1) * S::N6 + (j < S::N6 ? j : 0)];
  }
};
template <int LOGN, int PTS = kPts>
using GlobalTw = GlobalTwS<Shape<LOGN, PTS>>;

template <class S>
constexpr int six_twiddles() {
  if constexpr (S::NPASS > S::NBF) {
    return S::IT6 * 5;
  } else {
    return 0;
  }
}

// Twiddle source holding in registers the twiddles thread t needs in the
// passes with Ns >= MIN_NS (others are read from the table at each use; a pass
// with Ns <= 16 has at most 16 distinct twiddles per radix index, one cache
// line per wave), and those of a radix-6 last pass. Loaded once and reused by
// every transform of one length in a kernel. `fetch(i)` returns table entry i.
template <class S, class F, int MIN_NS = 2>
struct RegTwS {
  static constexpr int PTS = S::PTS;
  static constexpr bool cached(int p) { return p > 0 && p < S::NBF && S::ns(p) >= MIN_NS; }
  static constexpr int per_pass(int p) { return cached(p) ? PTS - PTS / S::radix(p) : 0; }
  static constexpr int offset(int p) {
    int o = 0;
    for (int q = 1; q < p; ++q) o += per_pass(q);
    return o;
  }
  static constexpr int C6 = six_twiddles<S>();
  static constexpr int COUNT = offset(S::NBF) + C6 > 0 ? offset(S::NBF) + C6 : 1;
  float2 w[COUNT];
  F fetch;
  int t;

  __host__ __device__ __forceinline__ RegTwS(const F& f, int t_) : fetch(f), t(t_) {
    load_pass<1>();
    if constexpr (C6 > 0) {
#pragma unroll
      for (int it = 0; it < S::IT6; ++it) {
        const int j = t + it * S::G;
#pragma unroll
        for (int r = 1; r < 6; ++r)
          w[offset(S::NBF) + it * 5 + (r - 1)] = fetch(S::TW6 + (r - 1) * S::N6 + (j < S::N6 ? j : 0));
      }
    }
  }

  template <int P>
  __host__ __device__ __forceinline__ void load_pass() {
    if constexpr (P < S::NBF) {
      if constexpr (cached(P)) {
        constexpr int R = S::radix(P), NS = S::ns(P), NB = PTS / R;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int k = mod_ns<NS>(t + b * S::G);
#pragma unroll
          for (int r = 1; r < R; ++r) w[offset(P) + b * (R - 1) + (r - 1)] = fetch(S::tw_off(P) + (r - 1) * NS + k);
        }
      }
      load_pass<P + 1>();
    }
  }

  template <int P>
  __host__ __device__ __forceinline__ float2 get(int b, int r) const {
    if constexpr (cached(P)) {
      return w[offset(P) + b * (S::radix(P) - 1) + (r - 1)];
    } else {
      constexpr int NS = S::ns(P);
      return fetch(S::tw_off(P) + (r - 1) * NS + mod_ns<NS>(t + b * S::G));
    }
  }

  __host__ __device__ __forceinline__ float2 get6(int it, int r) const { return w[offset(S::NBF) + it * 5 + (r - 1)]; }
};
template <int LOGN, class F, int MIN_NS = 2, int PTS = kPts>
using RegTw = RegTwS<Shape<LOGN, PTS>, F, MIN_NS>;

template <class S, bool INV>
struct FftS {
  static constexpr int PTS = S::PTS;

  // Pass P < S::NBF: thread t runs PTS/R butterflies on its registers.
  // Butterfly b has global index j = t + b*G and inputs x[j + r*N/R] =
  // v[b + r*PTS/R]; it applies the twiddles w(j mod Ns, r), the radix-R DFT,
  // and sends output r to position (j / Ns) * Ns * R + (j mod Ns) + r * Ns:
  // into LDS, or, in the last pass (Ns * R = N), back into the same registers.
  // OUTER: the caller guarantees v[PTS/4 .. 3PTS/4 - 1] == 0 on entry to
  // pass 0 (inputs confined to the first and last quarter), which prunes the
  // first butterfly; with 12 points per thread, v[4 .. 7] == 0 (inputs
  // confined to the first and last third).
  template <int P, class TW, bool OUTER = false>
  static __host__ __device__ __forceinline__ void butterflies(float2 (&v)[PTS], int t, float2* lds, int stride,
                                                              const TW& tw) {
    constexpr int R = S::radix(P), NS = S::ns(P), NB = PTS / R;
    constexpr bool LAST = (P + 1 == S::NPASS);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float2 x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[b + r * NB];
      const int j = t + b * S::G;
      const int k = mod_ns<NS>(j);
      if constexpr (P > 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 wr = tw.template get<P>(b, r);
          if (INV) wr.y = -wr.y;
          x[r] = cmul(x[r], wr);
        }
      }
      if constexpr (OUTER && P == 0 && R == 16 && PTS == 16) {
        dft16_outer<INV>(x);
      } else if constexpr (OUTER && P == 0 && R == 8 && PTS == 8) {
        dft8_outer<INV>(x);
      } else if constexpr (OUTER && P == 0 && R == 12 && PTS == 12) {
        dft12<INV, true>(x);
      } else {
        dft<R, INV>(x);
      }
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b + r * NB] = x[r];
      } else {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[S::template slot<P>(base + r * NS) * stride] = x[r];
      }
    }
  }

  // Radix-6 last pass of a Shape6 transform (after the power-of-two passes
  // have written LDS and the group has synchronised): round it, butterfly
  // j = t + G*it < N6 reads x[j + r*N6], applies exp(-+2 pi i r j / N) and the
  // length-6 DFT, and leaves output r (position j + r*N6) in o[it*6 + r].
  // Rounds past N6 leave zeros.
  template <class TW, class SS = S>
  static __host__ __device__ __forceinline__ void last6(float2 (&o)[SS::IT6 * 6], int t, const float2* lds, int stride,
                                                       const TW& tw) {
#pragma unroll
    for (int it = 0; it < S::IT6; ++it) {
      const int j = t + it * S::G;
      float2 x[6];
      if (it + 1 < S::IT6 || j < S::N6) {
#pragma unroll
        for (int r = 0; r < 6; ++r) x[r] = lds[S::template slot<S::NBF - 1>(j + r * S::N6) * stride];
#pragma unroll
        for (int r = 1; r < 6; ++r) {
          float2 wr = tw.get6(it, r);
          if (INV) wr.y = -wr.y;
          x[r] = cmul(x[r], wr);
        }
        dft6<INV>(x);
      } else {
#pragma unroll
        for (int r = 0; r < 6; ++r) x[r] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) o[it * 6 + r] = x[r];
    }
  }

  // Natural-order read of the exchange after pass P (the next pass's inputs).
  template <int P>
  static __host__ __device__ __forceinline__ void gather(float2 (&v)[PTS], int t, const float2* lds, int stride) {
#pragma unroll
    for (int i = 0; i < PTS; ++i) v[i] = lds[S::template slot<P>(t + S::G * i) * stride];
  }

  // Natural-order write of the registers (position t + G*i at slot S::nat).
  static __host__ __device__ __forceinline__ void scatter(const float2 (&v)[PTS], int t, float2* lds, int stride) {
#pragma unroll
    for (int i = 0; i < PTS; ++i) lds[S::nat(t + S::G * i) * stride] = v[i];
  }
};
template <int LOGN, bool INV, int PTS = kPts>
using Fft = FftS<Shape<LOGN, PTS>, INV>;

// Host: fill the twiddle table of a pass plan (tw_size entries).
inline void build_twiddles_plan(const PassPlan& p, float2* out) {
  for (int q = 1; q < p.npass; ++q) {
    const int ns = p.ns[q], r = p.radix[q];
    const double span = double(ns) * double(r);
    for (int m = 1; m < r; ++m)
      for (int k = 0; k < ns; ++k) {
        const long long e = (long long)k * m % (long long)(ns * r);
        const double ang = -2.0 * M_PI * double(e) / span;
        out[p.tw_off[q] + (m - 1) * ns + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
}

// Host: fill the twiddle table of a length 2^logn transform with pts points
// per thread (tw_size entries of that pass plan).
inline void build_twiddles(int logn, float2* out, int pts = kPts) {
  const PassPlan p = make_pass_plan(logn, pts);
  for (int q = 1; q < p.npass; ++q) {
    const int ns = p.ns[q], r = p.radix[q];
    const double span = double(ns) * double(r);
    for (int m = 1; m < r; ++m)
      for (int k = 0; k < ns; ++k) {
        // reduce m*k modulo span exactly in integers before the angle
        const long long e = (long long)k * m % (long long)(ns * r);
        const double ang = -2.0 * M_PI * double(e) / span;
        out[p.tw_off[q] + (m - 1) * ns + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
}

// Host: the twiddle table of a length 6*2^logp transform (Shape6 layout): the
// power-of-two passes' table, then exp(-2 pi i r k / N) at TW6 + (r-1)*N6 + k.
inline void build_twiddles6(int logp, float2* out, int pts = kPts) {
  build_twiddles(logp, out, pts);
  const PassPlan p = make_pass_plan(logp, pts);
  const int n6 = 1 << logp;
  const long long n = 6LL * n6;
  for (int r = 1; r < 6; ++r)
    for (int k = 0; k < n6; ++k) {
      const long long e = (long long)k * r % n;
      const double ang = -2.0 * M_PI * double(e) / double(n);
      out[p.tw_size + (r - 1) * n6 + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
}

inline int twiddles6_size(int logp, int pts = kPts) { return make_pass_plan(logp, pts).tw_size + 5 * (1 << logp); }

}  // namespace ff
