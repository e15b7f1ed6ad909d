// Batched 1D FFTs held in LDS, executed cooperatively by a workgroup, in FP64
// (double2) or FP32 (float2).
//
// Self-sorting (Stockham) mixed-radix passes: a pass of radix R over a length-N
// transform takes the R inputs j + r*N/R (j < N/R), multiplies input r by the
// twiddle w^(r*(j mod Ns)*N/(Ns*R)), applies an R-point DFT and writes output r
// to (j div Ns)*Ns*R + (j mod Ns) + r*Ns, where Ns is the product of the radices
// of the earlier passes.  After the last pass the result is in natural order:
//   X[k] = sum_n x[n] exp(SIGN * 2*pi*i * n*k / N)   (unnormalised).
//
// Each pass is done in place: every thread first loads all butterflies it owns
// into registers, the workgroup synchronises, then every thread writes its
// outputs.  Transforms are processed in rounds small enough for the register
// budget, so any number of transforms is handled.
#pragma once

#include <hip/hip_runtime.h>

namespace sgw {

// complex types: double2 (FP64) and float2 (FP32); CT<C2>::R is the real type
template <class C2> struct CT;
template <> struct CT<double2> {
  using R = double;
  __host__ __device__ static __forceinline__ double2 make(double a, double b) { return make_double2(a, b); }
};
template <> struct CT<float2> {
  using R = float;
  __host__ __device__ static __forceinline__ float2 make(float a, float b) { return make_float2(a, b); }
};

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by SIGN * i
template <int SIGN, class C2>
__device__ __forceinline__ C2 c_mul_si(C2 a) {
  return SIGN > 0 ? CT<C2>::make(-a.y, a.x) : CT<C2>::make(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// radix plans (product of the radices = N)
// ---------------------------------------------------------------------------
template <int N> struct FftPlan;
template <> struct FftPlan<8>  { static constexpr int np = 1; static constexpr int r[1] = {8}; };
template <> struct FftPlan<12> { static constexpr int np = 2; static constexpr int r[2] = {4, 3}; };
template <> struct FftPlan<16> { static constexpr int np = 2; static constexpr int r[2] = {4, 4}; };
template <> struct FftPlan<24> { static constexpr int np = 2; static constexpr int r[2] = {8, 3}; };
template <> struct FftPlan<32> { static constexpr int np = 2; static constexpr int r[2] = {8, 4}; };
template <> struct FftPlan<48> { static constexpr int np = 3; static constexpr int r[3] = {4, 4, 3}; };
template <> struct FftPlan<64> { static constexpr int np = 2; static constexpr int r[2] = {8, 8}; };
template <> struct FftPlan<72> { static constexpr int np = 3; static constexpr int r[3] = {8, 3, 3}; };
template <> struct FftPlan<96> { static constexpr int np = 3; static constexpr int r[3] = {8, 4, 3}; };

template <int N>
constexpr int fft_min_radix() {
  int m = 64;
  for (int p = 0; p < FftPlan<N>::np; ++p) m = FftPlan<N>::r[p] < m ? FftPlan<N>::r[p] : m;
  return m;
}

// ---------------------------------------------------------------------------
// R-point DFTs in registers, y_k = sum_r v_r exp(SIGN 2 pi i r k / R)
// ---------------------------------------------------------------------------
template <int R, int SIGN> struct Dft;

template <int SIGN> struct Dft<2, SIGN> {
  template <class C2>
  __device__ __forceinline__ static void run(C2 *v) {
    C2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <int SIGN> struct Dft<3, SIGN> {
  template <class C2>
  __device__ __forceinline__ static void run(C2 *v) {
    using R = typename CT<C2>::R;
    constexpr R h = R(0.86602540378443864676);  // sin(2 pi / 3)
    C2 s = c_add(v[1], v[2]);
    C2 d = c_sub(v[1], v[2]);
    C2 t = CT<C2>::make(v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y);
    C2 u = c_mul_si<SIGN>(c_scale(d, h));
    v[0] = c_add(v[0], s);
    v[1] = c_add(t, u);
    v[2] = c_sub(t, u);
  }
};

template <int SIGN> struct Dft<4, SIGN> {
  template <class C2>
  __device__ __forceinline__ static void run(C2 *v) {
    C2 s0 = c_add(v[0], v[2]), d0 = c_sub(v[0], v[2]);
    C2 s1 = c_add(v[1], v[3]), d1 = c_mul_si<SIGN>(c_sub(v[1], v[3]));
    v[0] = c_add(s0, s1);
    v[2] = c_sub(s0, s1);
    v[1] = c_add(d0, d1);
    v[3] = c_sub(d0, d1);
  }
};

template <int SIGN> struct Dft<8, SIGN> {
  template <class C2>
  __device__ __forceinline__ static void run(C2 *v) {
    using R = typename CT<C2>::R;
    constexpr R c = R(0.70710678118654752440);  // cos(pi/4)
    constexpr R sg = R(SIGN);
    C2 e[4] = {v[0], v[2], v[4], v[6]};
    C2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, SIGN>::run(e);
    Dft<4, SIGN>::run(o);
    // w^k, w = exp(SIGN i pi / 4)
    C2 o1 = CT<C2>::make(c * (o[1].x - sg * o[1].y), c * (o[1].y + sg * o[1].x));
    C2 o2 = c_mul_si<SIGN>(o[2]);
    C2 o3 = CT<C2>::make(c * (-o[3].x - sg * o[3].y), c * (-o[3].y + sg * o[3].x));
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

// ---------------------------------------------------------------------------
// one Stockham pass over `count` transforms
//   element e of transform t lives at buf[base(t) + e * es]
//   TMAJOR: consecutive threads take consecutive transforms (use when es > 1,
//           so a wavefront touches consecutive LDS addresses)
//   tw: N entries, tw[t] = exp(-2 pi i t / N)
// ---------------------------------------------------------------------------
template <int N, int R, int NS, int SIGN, int MAXB, bool TMAJOR, class Base, class C2>
__device__ __forceinline__ void fft_pass(C2 *buf, int count, Base base, int es, const C2 *tw, int tid, int nthr) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  const int tpr = (MAXB * nthr) / NB;  // transforms per round (>= 1: MAXB*nthr >= NB)
  for (int t0 = 0; t0 < count; t0 += tpr) {
    const int tc = min(tpr, count - t0);
    const int nbf = tc * NB;
    C2 v[MAXB][R];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int bf = tid + b * nthr;
      if (bf < nbf) {
        int t, j;
        if (TMAJOR) { j = bf / tc; t = t0 + (bf - j * tc); }
        else        { t = t0 + bf / NB; j = bf % NB; }
        const C2 *p = buf + base(t);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = p[(j + r * NB) * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int bf = tid + b * nthr;
      if (bf < nbf) {
        int t, j;
        if (TMAJOR) { j = bf / tc; t = t0 + (bf - j * tc); }
        else        { t = t0 + bf / NB; j = bf % NB; }
        const int k0 = j % NS;
        if (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            C2 w = tw[k0 * r * TWS];
            if (SIGN > 0) w = c_conj(w);
            v[b][r] = c_mul(v[b][r], w);
          }
        }
        Dft<R, SIGN>::run(v[b]);
        C2 *p = buf + base(t);
        const int o = (j / NS) * NS * R + k0;
#pragma unroll
        for (int r = 0; r < R; ++r) p[(o + r * NS) * es] = v[b][r];
      }
    }
    __syncthreads();
  }
}

template <int N, int R, int CMAX, int NT>
constexpr int fft_maxb() {
  // butterflies a thread must hold for CMAX transforms in one round, capped by a
  // register budget of ~24 complex values per thread
  int need = (CMAX * (N / R) + NT - 1) / NT;
  int cap = 24 / R;
  if (cap < 1) cap = 1;
  int m = need < cap ? need : cap;
  // at least one transform per round
  int one = (N / R + NT - 1) / NT;
  return m > one ? m : (one > 0 ? one : 1);
}

template <int N, int SIGN, int CMAX, int NT, bool TMAJOR, int P = 0, int NS = 1, class Base, class C2>
__device__ __forceinline__ void lds_fft(C2 *buf, int count, Base base, int es, const C2 *tw, int tid) {
  if constexpr (P < FftPlan<N>::np) {
    constexpr int R = FftPlan<N>::r[P];
    constexpr int MAXB = fft_maxb<N, R, CMAX, NT>();
    fft_pass<N, R, NS, SIGN, MAXB, TMAJOR>(buf, count, base, es, tw, tid, NT);
    lds_fft<N, SIGN, CMAX, NT, TMAJOR, P + 1, NS * R>(buf, count, base, es, tw, tid);
  }
}

}  // namespace sgw
