// Small DFTs held entirely in registers, and the two-stage split used by the
// plane and stick kernels.
//
// RegDft<N, SIGN>::run(v) replaces v[0..N) by X[k] = sum_n v[n] exp(SIGN 2 pi i n k / N).
// Sizes 2, 3, 4, 8 are written out (fft_lds.h); 6 and 12 use the prime-factor
// (Good-Thomas) mapping, which needs no twiddles for coprime factors; 9 is
// 3 x 3 Cooley-Tukey with the ninth roots of unity as constants.
//
// A length-N transform with N = A * B is done in two register stages:
//   stage 1: for each b < B, an A-point DFT over x[B a + b]   (a < A),
//            then multiply element ka by w_N^(SIGN b ka)
//   stage 2: for each ka < A, a B-point DFT over the stage-1 results (b < B),
//            giving X[ka + A kb]
// with one exchange of values between threads in between.
#pragma once

#include "fft_lds.h"
#include "twiddle_const.h"

namespace sgw {

template <int N> struct Split;
template <> struct Split<16> { static constexpr int a = 4, b = 4; };
template <> struct Split<24> { static constexpr int a = 8, b = 3; };
template <> struct Split<32> { static constexpr int a = 8, b = 4; };
template <> struct Split<48> { static constexpr int a = 8, b = 6; };
template <> struct Split<64> { static constexpr int a = 8, b = 8; };
template <> struct Split<72> { static constexpr int a = 8, b = 9; };

template <int N, int SIGN> struct RegDft;
template <int SIGN> struct RegDft<2, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { Dft<2, SIGN>::run(v); }
};
template <int SIGN> struct RegDft<3, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { Dft<3, SIGN>::run(v); }
};
template <int SIGN> struct RegDft<4, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { Dft<4, SIGN>::run(v); }
};
template <int SIGN> struct RegDft<8, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { Dft<8, SIGN>::run(v); }
};

constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

// prime-factor DFT of length P*Q, gcd(P, Q) = 1
template <int P, int Q, int SIGN, class C2>
__device__ __forceinline__ void pfa_dft(C2 *v) {
  constexpr int N = P * Q;
  constexpr int U = inv_mod(Q % P, P);
  constexpr int V = inv_mod(P % Q, Q);
  C2 y[P][Q];
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    C2 t[P];
#pragma unroll
    for (int n1 = 0; n1 < P; ++n1) t[n1] = v[(Q * n1 + P * n2) % N];
    RegDft<P, SIGN>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) y[k1][n2] = t[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    C2 t[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) t[n2] = y[k1][n2];
    RegDft<Q, SIGN>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) v[(Q * U * k1 + P * V * k2) % N] = t[k2];
  }
}

template <int SIGN> struct RegDft<6, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { pfa_dft<2, 3, SIGN>(v); }
};
template <int SIGN> struct RegDft<12, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) { pfa_dft<4, 3, SIGN>(v); }
};

// exp(2 pi i m / 9) for m = 1, 2, 4
template <class C2>
__device__ __forceinline__ C2 root9(int m) {
  using R = typename CT<C2>::R;
  return m == 1 ? CT<C2>::make(R(0.7660444431189780352024), R(0.6427876096865393263226))
       : m == 2 ? CT<C2>::make(R(0.1736481776669303488517), R(0.9848077530122080593667))
                : CT<C2>::make(R(-0.9396926207859083840541), R(0.3420201433256687330441));
}

template <int SIGN> struct RegDft<9, SIGN> {
  template <class C2>
  __device__ __forceinline__ static void run(C2 *v) {
    C2 y[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      C2 t[3] = {v[b], v[3 + b], v[6 + b]};
      Dft<3, SIGN>::run(t);
#pragma unroll
      for (int ka = 0; ka < 3; ++ka) {
        if (b * ka != 0) {
          C2 w = root9<C2>(b * ka);
          if (SIGN < 0) w.y = -w.y;
          t[ka] = c_mul(t[ka], w);
        }
        y[b][ka] = t[ka];
      }
    }
#pragma unroll
    for (int ka = 0; ka < 3; ++ka) {
      C2 t[3] = {y[0][ka], y[1][ka], y[2][ka]};
      Dft<3, SIGN>::run(t);
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) v[ka + 3 * kb] = t[kb];
    }
  }
};

// multiply v by w_N^(SIGN * m) read from a table tw[t] = exp(-2 pi i t / N)
template <int SIGN, class C2>
__device__ __forceinline__ C2 twiddle(C2 v, const C2 *tw, int m) {
  C2 w = tw[m];
  if (SIGN > 0) w.y = -w.y;
  return c_mul(v, w);
}



// v * exp(SIGN 2 pi i m / N) with m known at compile time after unrolling
template <int N, int SIGN, class C2>
__device__ __forceinline__ C2 twiddle_c(C2 v, int m) {
  using R = typename CT<C2>::R;
  m %= N;
  const int q = (4 * m) / N, r = m - q * (N / 4);
  if (r == 0) {  // a power of i: exact
    const int e = (SIGN > 0 ? q : 4 - q) % 4;
    return e == 0 ? v : e == 1 ? CT<C2>::make(-v.y, v.x) : e == 2 ? CT<C2>::make(-v.x, -v.y) : CT<C2>::make(v.y, -v.x);
  }
  const double c = ctw::kQuarterCos<N>.v[r], s = ctw::kQuarterCos<N>.v[N / 4 - r];
  // exp(i 2 pi m / N) = i^q (c + i s)
  const double wr = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
  const double wi = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
  return c_mul(v, CT<C2>::make(R(wr), R(SIGN > 0 ? wi : -wi)));
}


// DFT of length A (4 or 8) whose inputs vanish for a in [A/4, 3A/4): only v[0..A/4) and
// v[3A/4..A) are read.  Same operations as RegDft<A> on those inputs, without the zero terms
// (lines whose support is the central half of a grid: |m| < N/4, as a sphere that the grid can hold
// twice over has).
template <int A, int SIGN> struct HalfDft;
template <int SIGN> struct HalfDft<4, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) {
    // inputs v0, v3:  X = (v0 + v3, v0 - s i v3, v0 - v3, v0 + s i v3), s = SIGN
    const C2 a = v[0], d = c_mul_si<SIGN>(v[3]);
    const C2 b = v[3];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, d);
    v[2] = c_sub(a, b);
    v[3] = c_add(a, d);
  }
};
template <int SIGN> struct HalfDft<8, SIGN> {
  template <class C2> __device__ __forceinline__ static void run(C2 *v) {
    using R = typename CT<C2>::R;
    constexpr R c = R(0.70710678118654752440);  // cos(pi/4)
    constexpr R sg = R(SIGN);
    C2 e[4], o[4];
    e[0] = v[0];
    e[3] = v[6];
    o[0] = v[1];
    o[3] = v[7];
    HalfDft<4, SIGN>::run(e);
    HalfDft<4, SIGN>::run(o);
    // w^k o[k], w = exp(SIGN i pi / 4), as in Dft<8>
    const C2 o1 = CT<C2>::make(c * (o[1].x - sg * o[1].y), c * (o[1].y + sg * o[1].x));
    const C2 o2 = c_mul_si<SIGN>(o[2]);
    const C2 o3 = CT<C2>::make(c * (-o[3].x - sg * o[3].y), c * (-o[3].y + sg * o[3].x));
    v[0] = c_add(e[0], o[0]);
    v[4] = c_sub(e[0], o[0]);
    v[1] = c_add(e[1], o1);
    v[5] = c_sub(e[1], o1);
    v[2] = c_add(e[2], o2);
    v[6] = c_sub(e[2], o2);
    v[3] = c_add(e[3], o3);
    v[7] = c_sub(e[3], o3);
  }
};

}  // namespace sgw
