// Host-side drive of the device FFT engine, thread by thread, for CPU tests.
//
// Reads "logn inv stride" then 2^logn complex64 values from stdin (binary),
// runs the Stockham passes of ff::Fft with every thread of one group emulated
// in turn (all threads finish a pass before any gathers), and writes the
// 2^logn transformed values to stdout. The LDS array is shared by `stride`
// interleaved groups; this group uses slot offset stride - 1. Odd strides
// take the twiddles from the register cache, even strides from the table.

#include <cstdio>
#include <vector>

#include "fft_engine.hpp"

namespace {

struct Regs {
  float2 a[ff::kPts];
};

template <int LOGN, bool INV, int P>
void passes(std::vector<Regs>& v, float2* lds, int stride, const float2* tw, bool cached) {
  using S = ff::Shape<LOGN>;
  using F = ff::Fft<LOGN, INV>;
  if constexpr (P < S::NPASS) {
    for (int t = 0; t < S::G; ++t) {
      if (cached) {
        ff::RegTw<LOGN> rt;
        rt.load([tw](int i) { return tw[i]; }, t);
        F::template butterflies<P>(v[t].a, t, lds, stride, rt);
      } else {
        F::template butterflies<P>(v[t].a, t, lds, stride, ff::GlobalTw<LOGN>{tw, t});
      }
    }
    if constexpr (P + 1 < S::NPASS) {
      for (int t = 0; t < S::G; ++t) F::gather(v[t].a, t, lds, stride);
    }
    passes<LOGN, INV, P + 1>(v, lds, stride, tw, cached);
  }
}

template <int LOGN, bool INV>
void run(std::vector<float2>& x, int stride) {
  using S = ff::Shape<LOGN>;
  std::vector<float2> tw(S::plan.tw_size + 1);
  ff::build_twiddles(LOGN, tw.data());
  std::vector<Regs> v(S::G);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < ff::kPts; ++i) v[t].a[i] = x[t + S::G * i];
  std::vector<float2> lds(size_t(S::LDS) * stride, make_float2(1e30f, 1e30f));
  // odd strides use the twiddles cached in registers, even strides the table
  passes<LOGN, INV, 0>(v, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < ff::kPts; ++i) x[t + S::G * i] = v[t].a[i];
}

template <int LOGN>
bool dispatch(int logn, int inv, std::vector<float2>& x, int stride) {
  if constexpr (LOGN > 13) {
    return false;
  } else {
    if (logn != LOGN) return dispatch<LOGN + 1>(logn, inv, x, stride);
    if (inv)
      run<LOGN, true>(x, stride);
    else
      run<LOGN, false>(x, stride);
    return true;
  }
}

}  // namespace

int main() {
  int hdr[3];
  if (fread(hdr, sizeof(int), 3, stdin) != 3) return 2;
  const int logn = hdr[0], inv = hdr[1], stride = hdr[2];
  if (logn < 4 || logn > 13 || stride < 1) return 3;
  std::vector<float2> x(size_t(1) << logn);
  if (fread(x.data(), sizeof(float2), x.size(), stdin) != x.size()) return 4;
  if (!dispatch<4>(logn, inv, x, stride)) return 5;
  fwrite(x.data(), sizeof(float2), x.size(), stdout);
  return 0;
}
