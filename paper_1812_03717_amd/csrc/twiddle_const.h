// Compile-time twiddle factors: cos(2 pi k / N) for 0 <= k <= N / 4, evaluated
// by the compiler in double-double arithmetic (error-free sums and products)
// with a Taylor series on [0, pi / 4], then rounded once to double.  The other
// angles follow by exact quarter-turn symmetry (twiddle_c in fft_reg.h), so
// equal magnitudes are equal constants and in fully unrolled code every
// twiddle is an immediate.  Plain C++17, no device code: host tests compile it.
#pragma once

namespace sgw {
namespace ctw {
struct DD {
  double hi, lo;
};
constexpr DD quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
constexpr DD two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
constexpr DD split(double a) {  // Veltkamp split into two 26-bit halves
  const double t = 134217729.0 * a, hi = t - (t - a);
  return {hi, a - hi};
}
constexpr DD two_prod(double a, double b) {  // Dekker's exact product
  const double p = a * b;
  const DD x = split(a), y = split(b);
  return {p, ((x.hi * y.hi - p) + x.hi * y.lo + x.lo * y.hi) + x.lo * y.lo};
}
constexpr DD add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const DD t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
constexpr DD mul(DD a, DD b) {
  DD p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
constexpr DD div(DD a, double n) {  // n a small integer; two correction steps
  const DD p1 = two_prod(a.hi / n, n);
  const DD r = add(a, DD{-p1.hi, -p1.lo});
  const DD p2 = two_prod(r.hi / n, n);
  const DD r2 = add(r, DD{-p2.hi, -p2.lo});
  return add(quick_two_sum(a.hi / n, r.hi / n), DD{r2.hi / n, 0.0});
}
constexpr double trig(DD x, bool sine) {  // cos or sin of x in [0, pi / 4]
  const DD x2 = mul(x, x);
  DD term = sine ? x : DD{1.0, 0.0};
  DD sum = term;
  for (int j = 1; j < 16; ++j) {
    const int a = sine ? 2 * j : 2 * j - 1;
    term = div(div(mul(term, x2), a), a + 1);
    term = DD{-term.hi, -term.lo};  // the series alternates
    sum = add(sum, term);
  }
  return sum.hi + sum.lo;
}
// cos(2 pi k / n) for 0 <= k <= n / 4 (n divisible by 4)
constexpr double quarter_cos(int k, int n) {
  constexpr DD pi = {3.141592653589793116, 1.2246467991473532072e-16};
  return 8 * k <= n ? trig(div(mul(pi, DD{2.0 * k, 0.0}), n), false)
                    : trig(div(mul(pi, DD{2.0 * (n / 4 - k), 0.0}), n), true);
}
template <int N> struct QuarterCos {
  static_assert(N % 4 == 0, "quarter-wave table needs N divisible by 4");
  double v[N / 4 + 1];
  constexpr QuarterCos() : v() {
    for (int k = 0; k <= N / 4; ++k) v[k] = quarter_cos(k, N);
  }
};
template <int N> constexpr QuarterCos<N> kQuarterCos{};
}  // namespace ctw

}  // namespace sgw
