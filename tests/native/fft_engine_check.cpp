// Host-side drive of the device FFT engine, thread by thread, for CPU tests.
//
// Reads "logn inv stride outer pts six" then the complex64 values from stdin (binary),
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
      for (int t = 0; t < S::G; ++t) F::template gather<P>(v[t].a, t, lds, stride);
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

// Shape6 (N = 6 * 2^LOGP): the power-of-two passes, then the radix-6 pass
// read from LDS; output r of round it lands at position j + r*N6.
template <int LOGP, bool INV, int PTS, int P>
void passes6(std::vector<Regs<PTS>>& v, std::vector<std::vector<float2>>& o, float2* lds, int stride,
             const float2* tw, bool cached) {
  using S = ff::Shape6<LOGP, PTS>;
  using F = ff::FftS<S, INV>;
  if constexpr (P < S::NBF) {
    for (int t = 0; t < S::G; ++t) {
      if (cached) {
        ff::RegTwS<S, TableFetch, 2> rt(TableFetch{tw}, t);
        F::template butterflies<P, decltype(rt), false>(v[t].a, t, lds, stride, rt);
      } else {
        F::template butterflies<P, ff::GlobalTwS<S>, false>(v[t].a, t, lds, stride, ff::GlobalTwS<S>{tw, t});
      }
    }
    if constexpr (P + 1 < S::NBF) {
      for (int t = 0; t < S::G; ++t) F::template gather<P>(v[t].a, t, lds, stride);
    }
    passes6<LOGP, INV, PTS, P + 1>(v, o, lds, stride, tw, cached);
  } else {
    for (int t = 0; t < S::G; ++t) {
      float2 out[S::IT6 * 6];
      if (cached) {
        ff::RegTwS<S, TableFetch, 2> rt(TableFetch{tw}, t);
        F::last6(out, t, lds, stride, rt);
      } else {
        F::last6(out, t, lds, stride, ff::GlobalTwS<S>{tw, t});
      }
      o[t].assign(out, out + S::IT6 * 6);
    }
  }
}

template <int LOGP, bool INV, int PTS>
void run6(std::vector<float2>& x, int stride) {
  using S = ff::Shape6<LOGP, PTS>;
  std::vector<float2> tw(S::TW_SIZE + 1);
  ff::build_twiddles6(LOGP, tw.data(), PTS);
  std::vector<Regs<PTS>> v(S::G);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < PTS; ++i) v[t].a[i] = x[t + S::G * i];
  std::vector<float2> lds(size_t(S::LDS) * stride, make_float2(1e30f, 1e30f));
  std::vector<std::vector<float2>> o(S::G);
  passes6<LOGP, INV, PTS, 0>(v, o, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  std::vector<int> seen(S::N, 0);
  for (int t = 0; t < S::G; ++t)
    for (int it = 0; it < S::IT6; ++it) {
      const int j = t + S::G * it;
      if (j >= S::N6) continue;
      for (int r = 0; r < 6; ++r) {
        x[j + r * S::N6] = o[t][it * 6 + r];
        ++seen[j + r * S::N6];
      }
    }
  for (int i = 0; i < S::N; ++i)
    if (seen[i] != 1) x[i] = make_float2(1e30f, 1e30f);  // every position exactly once
}

// Shape12 (N = 12 * 2^E, 12 points per thread): the mixed-radix passes in
// natural order, like Shape.
template <int E, bool INV, int P, bool OUTER>
void passes12(std::vector<Regs<12>>& v, float2* lds, int stride, const float2* tw, bool cached) {
  using S = ff::Shape12<E>;
  using F = ff::FftS<S, INV>;
  if constexpr (P < S::NPASS) {
    for (int t = 0; t < S::G; ++t) {
      if (cached) {
        ff::RegTwS<S, TableFetch, 2> rt(TableFetch{tw}, t);
        F::template butterflies<P, decltype(rt), OUTER>(v[t].a, t, lds, stride, rt);
      } else {
        F::template butterflies<P, ff::GlobalTwS<S>, OUTER>(v[t].a, t, lds, stride, ff::GlobalTwS<S>{tw, t});
      }
    }
    if constexpr (P + 1 < S::NPASS) {
      for (int t = 0; t < S::G; ++t) F::template gather<P>(v[t].a, t, lds, stride);
    }
    passes12<E, INV, P + 1, OUTER>(v, lds, stride, tw, cached);
  }
}

template <int E, bool INV>
void run12(std::vector<float2>& x, int stride, bool outer) {
  using S = ff::Shape12<E>;
  std::vector<float2> tw(S::plan.tw_size + 1);
  ff::build_twiddles_plan(S::plan, tw.data());
  std::vector<Regs<12>> v(S::G);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < 12; ++i) v[t].a[i] = x[t + S::G * i];
  std::vector<float2> lds(size_t(S::LDS) * stride, make_float2(1e30f, 1e30f));
  if (outer)
    passes12<E, INV, 0, true>(v, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  else
    passes12<E, INV, 0, false>(v, lds.data() + (stride - 1), stride, tw.data(), stride % 2 == 1);
  for (int t = 0; t < S::G; ++t)
    for (int i = 0; i < 12; ++i) x[t + S::G * i] = v[t].a[i];
}

template <int E>
bool dispatch12(int e, int inv, std::vector<float2>& x, int stride, bool outer) {
  if constexpr (E > 10) {
    return false;
  } else {
    if (e != E) return dispatch12<E + 1>(e, inv, x, stride, outer);
    if (inv)
      run12<E, true>(x, stride, outer);
    else
      run12<E, false>(x, stride, outer);
    return true;
  }
}

template <int LOGN>
bool dispatch(int logn, int inv, std::vector<float2>& x, int stride, bool outer, int pts) {
  if constexpr (LOGN > 14) {
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

template <int LOGP>
bool dispatch6(int logp, int inv, std::vector<float2>& x, int stride, int pts) {
  if constexpr (LOGP > 11) {
    return false;
  } else {
    if (logp != LOGP) return dispatch6<LOGP + 1>(logp, inv, x, stride, pts);
    if (pts == 8) {
      if (inv)
        run6<LOGP, true, 8>(x, stride);
      else
        run6<LOGP, false, 8>(x, stride);
    } else {
      if (inv)
        run6<LOGP, true, 16>(x, stride);
      else
        run6<LOGP, false, 16>(x, stride);
    }
    return true;
  }
}

}  // namespace

// Header: logn inv stride outer pts six. With six = 1 the length is
// 6 * 2^logn (Shape6, outer unused); with six = 2 it is 12 * 2^logn
// (Shape12, pts unused; outer zeroes the middle third of the input).
int main() {
  int hdr[6];
  if (fread(hdr, sizeof(int), 6, stdin) != 6) return 2;
  const int logn = hdr[0], inv = hdr[1], stride = hdr[2], outer = hdr[3], pts = hdr[4], six = hdr[5];
  if (stride < 1) return 3;
  if (six == 2) {  // Shape12 with E = logn: length 12 * 2^E
    if (logn < 2 || logn > 10) return 3;
    std::vector<float2> x(size_t(12) << logn);
    if (fread(x.data(), sizeof(float2), x.size(), stdin) != x.size()) return 4;
    if (outer)  // the pruned first pass assumes the middle third of the input is zero
      for (size_t i = x.size() / 3; i < 2 * x.size() / 3; ++i) x[i] = make_float2(0.f, 0.f);
    if (!dispatch12<2>(logn, inv, x, stride, outer != 0)) return 5;
    fwrite(x.data(), sizeof(float2), x.size(), stdout);
    return 0;
  }
  if (pts != 8 && pts != 16) return 3;
  if (six) {
    if (logn < 4 || logn > 11) return 3;
    std::vector<float2> x(size_t(6) << logn);
    if (fread(x.data(), sizeof(float2), x.size(), stdin) != x.size()) return 4;
    if (!dispatch6<4>(logn, inv, x, stride, pts)) return 5;
    fwrite(x.data(), sizeof(float2), x.size(), stdout);
    return 0;
  }
  if (logn < 4 || logn > 14) return 3;
  std::vector<float2> x(size_t(1) << logn);
  if (fread(x.data(), sizeof(float2), x.size(), stdin) != x.size()) return 4;
  if (outer)  // the pruned first pass assumes the middle half of the input is zero
    for (size_t i = x.size() / 4; i < 3 * x.size() / 4; ++i) x[i] = make_float2(0.f, 0.f);
  if (!dispatch<4>(logn, inv, x, stride, outer != 0, pts)) return 5;
  fwrite(x.data(), sizeof(float2), x.size(), stdout);
  return 0;
}
