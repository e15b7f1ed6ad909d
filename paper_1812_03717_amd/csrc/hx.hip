// H.x in plane waves (Sec. 2.1): kinetic diagonal plus the local potential
// applied on the real-space grid through a pruned 3D FFT, batched over vectors.
//
// The plane-wave sphere occupies, along grid axis 2, a set of "sticks" (one per
// (m0, m1) column).  The transform runs in three kernels:
//   sticks_inv : per stick, scatter the coefficients into a length-N2 column and
//                inverse-FFT along axis 2; write T[vec][i2][stick]
//   planes     : per (vec, i2) plane, place the stick values, inverse-FFT along
//                axis 1 (only the rows that hold sticks) and axis 0, multiply by
//                V(r), forward-FFT along axis 0 and axis 1, gather the sticks
//   sticks_fwd : per stick, forward-FFT along axis 2, gather the sphere, scale by
//                1/N, add the kinetic term
// Only the stick data (N2 * n_stick values per vector) travels through HBM; a
// full plane lives in LDS.
#include "fft_lds.h"
#include "fft_reg.h"
#include "sgw_internal.h"

namespace sgw {
namespace {

struct StrideBase {
  int ld;
  __device__ __forceinline__ int operator()(int t) const { return t * ld; }
};
struct UnitBase {
  __device__ __forceinline__ int operator()(int t) const { return t; }
};
// rows of a plane that hold sticks: row t -> i0 = (m0_lo + t) mod N0
struct RowBase {
  int m0_lo, n0, ld;
  __device__ __forceinline__ int operator()(int t) const {
    int i0 = m0_lo + t;
    i0 += (i0 < 0) ? n0 : 0;
    return i0 * ld;
  }
};

template <int N2> constexpr int sticks_per_block() { return N2 <= 32 ? 64 : 32; }
constexpr int kStickThreads = 256;

template <int N2>
__global__ __launch_bounds__(kStickThreads) void k_sticks_inv(VecSrc x, double2 *__restrict__ T, int n_stick,
                                                              const int32_t *__restrict__ stick_off,
                                                              const int32_t *__restrict__ pw_stick,
                                                              const int32_t *__restrict__ pw_z,
                                                              const double2 *__restrict__ twg, int groups) {
  constexpr int SG = sticks_per_block<N2>();
  constexpr int LDC = N2 + 1;
  __shared__ double2 col[SG * LDC];
  __shared__ double2 tw[N2];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const double2 *xv = x.ptr(vec);
  for (int i = tid; i < SG * LDC; i += kStickThreads) col[i] = make_double2(0.0, 0.0);
  for (int i = tid; i < N2; i += kStickThreads) tw[i] = twg[i];
  __syncthreads();
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int g = g0 + tid; g < g1; g += kStickThreads) col[(pw_stick[g] - s0) * LDC + pw_z[g]] = xv[g];
  __syncthreads();
  lds_fft<N2, +1, SG, kStickThreads, false>(col, ns, StrideBase{LDC}, 1, tw, tid);
  double2 *Tv = T + (long)vec * N2 * n_stick + s0;
  for (int i = tid; i < ns * N2; i += kStickThreads) {
    const int z = i / ns, s = i - z * ns;
    Tv[(long)z * n_stick + s] = col[s * LDC + z];
  }
}

template <int N2>
__global__ __launch_bounds__(kStickThreads) void k_sticks_fwd(const double2 *__restrict__ T, int n_stick,
                                                              const int32_t *__restrict__ stick_off,
                                                              const int32_t *__restrict__ pw_stick,
                                                              const int32_t *__restrict__ pw_z,
                                                              const double2 *__restrict__ twg, int groups,
                                                              VecSrc x, const double *__restrict__ kin,
                                                              double2 *__restrict__ y, long ldy, double scale) {
  constexpr int SG = sticks_per_block<N2>();
  constexpr int LDC = N2 + 1;
  __shared__ double2 col[SG * LDC];
  __shared__ double2 tw[N2];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  for (int i = tid; i < N2; i += kStickThreads) tw[i] = twg[i];
  const double2 *Tv = T + (long)vec * N2 * n_stick + s0;
  for (int i = tid; i < ns * N2; i += kStickThreads) {
    const int z = i / ns, s = i - z * ns;
    col[s * LDC + z] = Tv[(long)z * n_stick + s];
  }
  __syncthreads();
  lds_fft<N2, -1, SG, kStickThreads, false>(col, ns, StrideBase{LDC}, 1, tw, tid);
  const double2 *xv = x.ptr(vec);
  double2 *yv = y + (long)vec * ldy;
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int g = g0 + tid; g < g1; g += kStickThreads) {
    const double2 c = col[(pw_stick[g] - s0) * LDC + pw_z[g]];
    const double2 xg = xv[g];
    const double t = kin[g];
    yv[g] = make_double2(fma(c.x, scale, t * xg.x), fma(c.y, scale, t * xg.y));
  }
}

template <int N0, int N1> constexpr int plane_threads() { return N0 * N1 <= 48 * 48 ? 256 : 512; }

// One (vector, i2) plane: 2D inverse FFT of the stick values, multiplication by
// V(r), 2D forward FFT, back to the stick values.  Every 1D transform is split
// N = A * B into two register stages (fft_reg.h) with one LDS exchange; along
// axis 0 the inverse's second stage, the potential and the forward's first
// stage run on the same registers.  Rows (fixed i0) that hold no stick are
// zero before the axis-0 transform and not needed after it, so they are never
// stored.  LD = N1 + 1 keeps row-strided and column-strided accesses free of
// LDS bank conflicts.
template <int N0, int N1>
__global__ __launch_bounds__((plane_threads<N0, N1>())) void k_planes(double2 *__restrict__ T, int n2,
                                                                   int n_stick,
                                                                   const int32_t *__restrict__ stick_at,
                                                                   int m0_lo, int n_row,
                                                                   const double *__restrict__ vt,
                                                                   const double2 *__restrict__ tw0g,
                                                                   const double2 *__restrict__ tw1g) {
  constexpr int NT = plane_threads<N0, N1>();
  constexpr int LD = N1 + 1;
  constexpr int A0 = Split<N0>::a, B0 = Split<N0>::b;
  constexpr int A1 = Split<N1>::a, B1 = Split<N1>::b;
  constexpr int MT = (N1 * B0 + NT - 1) / NT;  // column tasks held per thread
  __shared__ double2 plane[N0 * LD];
  __shared__ double2 tw0[N0];
  __shared__ double2 tw1[N1];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / n2;
  const int z = blockIdx.x - vec * n2;
  double2 *Tz = T + ((long)vec * n2 + z) * n_stick;
  for (int i = tid; i < N0; i += NT) tw0[i] = tw0g[i];
  for (int i = tid; i < N1; i += NT) tw1[i] = tw1g[i];
  __syncthreads();
  auto row_i0 = [&](int t) {
    int i0 = m0_lo + t;
    return i0 < 0 ? i0 + N0 : i0;
  };
  auto has_sticks = [&](int i0) {
    int t = i0 - m0_lo;
    t = t < 0 ? t + N0 : (t >= N0 ? t - N0 : t);
    return t < n_row;
  };

  // ---- axis 1, inverse, rows holding sticks (thread-consecutive rows) ----
  for (int task = tid; task < n_row * B1; task += NT) {
    const int t = task % n_row, b = task / n_row;
    const int i0 = row_i0(t);
    double2 v[A1];
#pragma unroll
    for (int a = 0; a < A1; ++a) {
      const int s = stick_at[i0 * N1 + B1 * a + b];
      v[a] = s >= 0 ? Tz[s] : make_double2(0.0, 0.0);
    }
    RegDft<A1, +1>::run(v);
#pragma unroll
    for (int ka = 0; ka < A1; ++ka) plane[i0 * LD + b * A1 + ka] = (b * ka) ? twiddle<+1>(v[ka], tw1, b * ka) : v[ka];
  }
  __syncthreads();
  for (int task = tid; task < n_row * A1; task += NT) {
    const int t = task % n_row, ka = task / n_row;
    const int i0 = row_i0(t);
    double2 v[B1];
#pragma unroll
    for (int b = 0; b < B1; ++b) v[b] = plane[i0 * LD + b * A1 + ka];
    RegDft<B1, +1>::run(v);
#pragma unroll
    for (int kb = 0; kb < B1; ++kb) plane[i0 * LD + ka + A1 * kb] = v[kb];
  }
  __syncthreads();

  // ---- axis 0, inverse stage 1 (thread-consecutive columns) ----
  double2 h[MT][A0];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, b = task / N1;
#pragma unroll
      for (int a = 0; a < A0; ++a) {
        const int i0 = B0 * a + b;
        h[m][a] = has_sticks(i0) ? plane[i0 * LD + i1] : make_double2(0.0, 0.0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, b = task / N1;
      RegDft<A0, +1>::run(h[m]);
#pragma unroll
      for (int ka = 0; ka < A0; ++ka)
        plane[(b * A0 + ka) * LD + i1] = (b * ka) ? twiddle<+1>(h[m][ka], tw0, b * ka) : h[m][ka];
    }
  }
  __syncthreads();
  // ---- axis 0: inverse stage 2, times V(r), forward stage 1 ----
  const double *vz = vt + (long)z * N0 * N1;
  for (int task = tid; task < N1 * A0; task += NT) {
    const int i1 = task % N1, ka = task / N1;
    double2 v[B0];
#pragma unroll
    for (int b = 0; b < B0; ++b) v[b] = plane[(b * A0 + ka) * LD + i1];
    RegDft<B0, +1>::run(v);
#pragma unroll
    for (int kb = 0; kb < B0; ++kb) v[kb] = c_scale(v[kb], vz[(ka + A0 * kb) * N1 + i1]);
    RegDft<B0, -1>::run(v);
#pragma unroll
    for (int e = 0; e < B0; ++e) plane[(e * A0 + ka) * LD + i1] = (ka * e) ? twiddle<-1>(v[e], tw0, ka * e) : v[e];
  }
  __syncthreads();
  // ---- axis 0, forward stage 2; only rows holding sticks are kept ----
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, e = task / N1;
#pragma unroll
      for (int c = 0; c < A0; ++c) h[m][c] = plane[(e * A0 + c) * LD + i1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, e = task / N1;
      RegDft<A0, -1>::run(h[m]);
#pragma unroll
      for (int f = 0; f < A0; ++f) {
        const int i0 = e + B0 * f;
        if (has_sticks(i0)) plane[i0 * LD + i1] = h[m][f];
      }
    }
  }
  __syncthreads();

  // ---- axis 1, forward, rows holding sticks; gather the sticks ----
  for (int task = tid; task < n_row * A1; task += NT) {
    const int t = task % n_row, c = task / n_row;
    const int i0 = row_i0(t);
    double2 v[B1];
#pragma unroll
    for (int d = 0; d < B1; ++d) v[d] = plane[i0 * LD + c + A1 * d];
    RegDft<B1, -1>::run(v);
#pragma unroll
    for (int e = 0; e < B1; ++e) plane[i0 * LD + e * A1 + c] = (c * e) ? twiddle<-1>(v[e], tw1, c * e) : v[e];
  }
  __syncthreads();
  for (int task = tid; task < n_row * B1; task += NT) {
    const int t = task % n_row, e = task / n_row;
    const int i0 = row_i0(t);
    double2 v[A1];
#pragma unroll
    for (int c = 0; c < A1; ++c) v[c] = plane[i0 * LD + e * A1 + c];
    RegDft<A1, -1>::run(v);
#pragma unroll
    for (int f = 0; f < A1; ++f) {
      const int s = stick_at[i0 * N1 + e + B1 * f];
      if (s >= 0) Tz[s] = v[f];
    }
  }
}

template <int N2>
sgw_status launch_sticks(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy,
                         double2 *tbuf, bool inverse) {
  constexpr int SG = sticks_per_block<N2>();
  const int groups = (h->n_stick + SG - 1) / SG;
  const long blocks = (long)groups * n_vec;
  const double2 *tw = h->d_tw + h->tw_off[2];
  const double n2 = N2, nst = h->n_stick, npw = h->n_pw;
  PendingTiming tm;
  if (inverse) {
    timing_begin(ctx, K_STICKS_INV, n_vec * (npw * 16.0 + n2 * nst * 16.0), 0.0, &tm);
    hipLaunchKernelGGL(k_sticks_inv<N2>, dim3(blocks), dim3(kStickThreads), 0, ctx->stream, x, tbuf,
                       h->n_stick, h->d_stick_off, h->d_pw_stick, h->d_pw_z, tw, groups);
    timing_end(ctx, &tm);
  } else {
    const double scale = 1.0 / ((double)h->n[0] * h->n[1] * h->n[2]);
    timing_begin(ctx, K_STICKS_FWD, n_vec * (npw * 32.0 + n2 * nst * 16.0), 0.0, &tm);
    hipLaunchKernelGGL(k_sticks_fwd<N2>, dim3(blocks), dim3(kStickThreads), 0, ctx->stream, tbuf, h->n_stick,
                       h->d_stick_off, h->d_pw_stick, h->d_pw_z, tw, groups, x, h->d_kin, y, ldy, scale);
    timing_end(ctx, &tm);
  }
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

template <int N0, int N1>
sgw_status launch_planes(sgw_ctx *ctx, const sgw_ham *h, int n_vec, double2 *tbuf) {
  const long blocks = (long)n_vec * h->n[2];
  PendingTiming tm;
  // algorithmic bytes: stick values in and out; the potential is read once per launch
  const double bytes = (double)n_vec * h->n[2] * h->n_stick * 32.0 + (double)N0 * N1 * h->n[2] * 8.0;
  timing_begin(ctx, K_PLANES, bytes, 0.0, &tm);
  hipLaunchKernelGGL((k_planes<N0, N1>), dim3(blocks), dim3(plane_threads<N0, N1>()), 0, ctx->stream, tbuf,
                     h->n[2], h->n_stick, h->d_stick_at, h->m0_lo, h->n_row, h->d_vt, h->d_tw + h->tw_off[0],
                     h->d_tw + h->tw_off[1]);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

#define SGW_GRID_LIST(X) X(16) X(24) X(32) X(48) X(64) X(72)

sgw_status dispatch_sticks(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy,
                           double2 *tbuf, bool inverse) {
  switch (h->n[2]) {
#define SGW_CASE(N) \
  case N:           \
    return launch_sticks<N>(ctx, h, n_vec, x, y, ldy, tbuf, inverse);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 2 not supported");
}

template <int N0>
sgw_status dispatch_planes_n1(sgw_ctx *ctx, const sgw_ham *h, int n_vec, double2 *tbuf) {
  switch (h->n[1]) {
#define SGW_CASE(N) \
  case N:           \
    return launch_planes<N0, N>(ctx, h, n_vec, tbuf);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 1 not supported");
}

sgw_status dispatch_planes(sgw_ctx *ctx, const sgw_ham *h, int n_vec, double2 *tbuf) {
  switch (h->n[0]) {
#define SGW_CASE(N) \
  case N:           \
    return dispatch_planes_n1<N>(ctx, h, n_vec, tbuf);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 0 not supported");
}

}  // namespace

bool hx_grid_supported(int n) {
  switch (n) {
#define SGW_CASE(N) \
  case N:           \
    return true;
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return false;
}

sgw_status hx_batch(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, double2 *tbuf) {
  if (n_vec <= 0) return SGW_OK;
  sgw_status st = dispatch_sticks(ctx, h, n_vec, x, nullptr, 0, tbuf, true);
  if (st != SGW_OK) return st;
  st = dispatch_planes(ctx, h, n_vec, tbuf);
  if (st != SGW_OK) return st;
  return dispatch_sticks(ctx, h, n_vec, x, y, ldy, tbuf, false);
}

}  // namespace sgw
