// Host-side drive of the device FFT engine, thread by thread, for CPU tests.
//
// Reads "logn inv stride outer pts" then 2^logn complex64 values from stdin (binary),
// runs the Stockham passes of ff::Fft with every thread of one group emulated
// in turn (all threads finish a pass before any gathers), and writes the
// 2^logn transformed values to stdout. The LDS array is shared by `stride`
// interleaved groups; this group uses slot offset stride - 1. Odd strides
// take the twiddles from the register cache, even strides from the table.
// With outer != 0 the middle half of the input is zeroed and the pruned first
// pass is used.

#include <cstdio>
#include <vector>

#include "fft_engine.hpp"

namespace {

template <int PTS>
struct Regs {
  float2 a[PTS];
};

struct TableFetch {
  const float2* tw;
  float2 operator()(int i) const { return tw[i]; }
};

template <int LOGN, bool INV, int P, bool OUTER, int PTS>
void passes(std::vector<Regs<PTS>>& v, float2* lds, int stride, const float2* tw, bool cached) {
  using S = ff::Shape<LOGN, PTS>;
  using F = ff::Fft<LOGN, INV, PTS>;
  if constexpr (P < S::NPASS) {
    for (int t = 0; t < S::G; ++t) {
      if (cached) {
        ff::RegTw<LOGN, TableFetch, 2, PTS> rt(TableFetch{tw}, t);
        F::template butterflies<P, decltype(rt), OUTER>(v[t].a, t, lds, stride, rt);
      } else {
        F::template butterflies<P, ff::GlobalTw<LOGN, PTS>, OUTER>(v[t].a, t, lds, stride,
                                                                  ff::GlobalTw<LOGN, PTS>{tw, t});
      }
    }
    if constexpr (P + 1 < S::NPASS) {
      for (int t = 0; t < S::G; ++t) F::gather(v[t].a, t, lds, stride);
    }
    passes<LOGN, INV, P + 1, OUTER, PTS>(v, lds, stride, tw, cached);
  }
}

template <int LOGN, bool INV, int PTS>
void run(std::vector<float2>& x, int stride, bool outer) {
  using S = ff::Shape<LOGN, PTS>;
  std::vector<float2> tw(S::plan.tw_size + 1);
  ff::build_twiddles(LOGN, tw.data(), PTS);
  std::vector<Regs<PTS>> v(S::G);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < PTS; ++i) v[t].a[i] = x[t + S::G * i];
  std::vector<float2> lds(size_t(S::LDS) * stride, make_float2(1e30f, 1e30f));
  // odd strides use the twiddles cached in registers, even strides the table
  if (outer)
    passes<LOGN, INV, 0, true, PTS>(v, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  else
    passes<LOGN, INV, 0, false, PTS>(v, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < PTS; ++i) x[t + S::G * i] = v[t].a[i];
}

template <int LOGN>
bool dispatch(int logn, int inv, std::vector<float2>& x, int stride, bool outer, int pts) {
  if constexpr (LOGN > 13) {
    return false;
  } else {
    if (logn != LOGN) return dispatch<LOGN + 1>(logn, inv, x, stride, outer, pts);
    if (pts == 8) {
      if (inv)
        run<LOGN, true, 8>(x, stride, outer);
      else
        run<LOGN, false, 8>(x, stride, outer);
    } else {
      if (inv)
        run<LOGN, true, 16>(x, stride, outer);
      else
        run<LOGN, false, 16>(x, stride, outer);
    }
    return true;
  }
}

}  // namespace

int main() {
  int hdr[5];
  if (fread(hdr, sizeof(int), 5, stdin) != 5) return 2;
  const int logn = hdr[0], inv = hdr[1], stride = hdr[2], outer = hdr[3], pts = hdr[4];
  if (pts != 8 && pts != 16) return 3;
  if (logn < 4 || logn > 13 || stride < 1) return 3;
  std::vector<float2> x(size_t(1) << logn);
  if (fread(x.data(), sizeof(float2), x.size(), stdin) != x.size()) return 4;
  if (outer)  // the pruned first pass assumes the middle half of the input is zero
    for (size_t i = x.size() / 4; i < 3 * x.size() / 4; ++i) x[i] = make_float2(0.f, 0.f);
  if (!dispatch<4>(logn, inv, x, stride, outer != 0, pts)) return 5;
  fwrite(x.data(), sizeof(float2), x.size(), stdout);
  return 0;
}
