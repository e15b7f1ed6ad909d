// Plane pass of the pruned 3D FFT H.x (Sec. 2.1): for one (vector, i2) plane,
// 2D inverse FFT of the stick values, multiplication by V(r), 2D forward FFT,
// back to the stick values.
//
// Every 1D transform is split N = A * B into two register stages (fft_reg.h)
// with one LDS exchange in between; along axis 0 the inverse's second stage,
// the potential and the forward's first stage run on the same registers, so a
// column makes three LDS round trips for inverse + V + forward.  Rows (fixed
// i0) outside the sticks' m0 range are zero on input and not needed on output:
// the axis-0 stages skip their LDS reads (using 0) and their final writes.
//
// Stick lookup: within a row the sticks are one contiguous run of m1 values
// (the basis is a sphere, so its (m0, m1) projection is convex); rows[t] =
// {index of the first stick, m1_lo, m1_hi} for row m0 = m0_lo + t.
//
// LD = N1 + 1 keeps row-strided and column-strided LDS accesses free of bank
// conflicts.
#pragma once

#include "fft_lds.h"
#include "fft_reg.h"
#include "sgw_internal.h"

namespace sgw {

// Threads per plane workgroup.  Planes up to 48 x 48 fit four workgroups of 256 per CU.  Larger
// planes fill most of the LDS with one workgroup per CU, so it takes one thread per axis-0 column
// task (whole wavefronts): more waves to hide LDS latency and one task's registers per thread.
template <int N0, int N1> constexpr int plane_threads() {
  constexpr int tasks = N1 * (Split<N0>::a > Split<N0>::b ? Split<N0>::a : Split<N0>::b);
  constexpr int nt = (tasks + 63) / 64 * 64;
  return N0 * N1 <= 48 * 48 ? 256 : (nt > 1024 ? 1024 : nt);
}
template <class C2, int N0, int N1>
__global__ __launch_bounds__((plane_threads<N0, N1>())) void k_planes(C2 *__restrict__ T, int n2, int n_stick,
                                                                   const int4 *__restrict__ rows, int m0_lo,
                                                                   int n_row,
                                                                   const typename CT<C2>::R *__restrict__ vt,
                                                                   const C2 *__restrict__ tw0g,
                                                                   const C2 *__restrict__ tw1g) {
  using R = typename CT<C2>::R;
  constexpr int NT = plane_threads<N0, N1>();
  constexpr int LD = N1 + 1;
  constexpr int A0 = Split<N0>::a, B0 = Split<N0>::b;
  constexpr int A1 = Split<N1>::a, B1 = Split<N1>::b;
  constexpr int MTC = (N1 * B0 + NT - 1) / NT;  // axis-0 stage-1/3 tasks per thread
  constexpr int MTB = (N1 * A0 + NT - 1) / NT;  // axis-0 stage-2 tasks per thread
  __shared__ C2 plane[N0 * LD];
  __shared__ C2 tw0[N0];
  __shared__ C2 tw1[N1];
  __shared__ int4 rinfo[N0];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / n2;
  const int z = blockIdx.x - vec * n2;
  C2 *Tz = T + ((long)vec * n2 + z) * n_stick;
  const R *vz = vt + (long)z * N0 * N1;

  // Planes up to 48 x 48 prefetch this thread's potential values for the axis-0 middle stage (the
  // registers do not lower their occupancy, which the LDS sets); larger planes load them there.
  constexpr bool kPrefetchV = N0 * N1 <= 48 * 48;
  R vpre[kPrefetchV ? MTB : 1][B0];
  if constexpr (kPrefetchV) {
#pragma unroll
    for (int m = 0; m < MTB; ++m) {
      const int task = tid + m * NT;
      if (task < N1 * A0) {
        const int i1 = task % N1, ka = task / N1;
#pragma unroll
        for (int kb = 0; kb < B0; ++kb) vpre[m][kb] = vz[(ka + A0 * kb) * N1 + i1];
      }
    }
  }
  for (int i = tid; i < N0; i += NT) tw0[i] = tw0g[i];
  for (int i = tid; i < N1; i += NT) tw1[i] = tw1g[i];
  for (int i = tid; i < n_row; i += NT) rinfo[i] = rows[i];
  __syncthreads();
  // Rows outside the stick range are zero after the axis-1 inverse and unused by the axis-1
  // forward: the axis-0 stages neither read them (they use 0) nor write them back.
  auto stick_row = [&](int i0) {
    int t = i0 - m0_lo;
    t += t < 0 ? N0 : (t >= N0 ? -N0 : 0);
    return t < n_row;
  };
  auto row_i0 = [&](int t) {
    const int i0 = m0_lo + t;
    return i0 < 0 ? i0 + N0 : i0;
  };
  // stick index at (row t, i1), or -1
  auto stick = [&](const int4 &ri, int i1) {
    const int m1 = i1 <= (N1 - 1) / 2 ? i1 : i1 - N1;
    return (m1 >= ri.y && m1 <= ri.z) ? ri.x + (m1 - ri.y) : -1;
  };

  // ---- axis 1, inverse, rows holding sticks (thread-consecutive rows) ----
  for (int task = tid; task < n_row * B1; task += NT) {
    const int b = task / n_row, t = task - b * n_row;
    const int i0 = row_i0(t);
    const int4 ri = rinfo[t];
    C2 v[A1];
#pragma unroll
    for (int a = 0; a < A1; ++a) {
      const int s = stick(ri, B1 * a + b);
      v[a] = s >= 0 ? Tz[s] : CT<C2>::make(R(0), R(0));
    }
    RegDft<A1, +1>::run(v);
    C2 *row = plane + i0 * LD + b * A1;
    row[0] = v[0];
#pragma unroll
    for (int ka = 1; ka < A1; ++ka) row[ka] = twiddle<+1>(v[ka], tw1, b * ka);
  }
  __syncthreads();
  for (int task = tid; task < n_row * A1; task += NT) {
    const int ka = task / n_row, t = task - ka * n_row;
    C2 *row = plane + row_i0(t) * LD;
    C2 v[B1];
#pragma unroll
    for (int b = 0; b < B1; ++b) v[b] = row[b * A1 + ka];
    RegDft<B1, +1>::run(v);
#pragma unroll
    for (int kb = 0; kb < B1; ++kb) row[ka + A1 * kb] = v[kb];
  }
  __syncthreads();

  // ---- axis 0, inverse stage 1 (thread-consecutive columns) ----
  C2 h[MTC][A0];
#pragma unroll
  for (int m = 0; m < MTC; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, b = task / N1;
#pragma unroll
      for (int a = 0; a < A0; ++a)
        h[m][a] = stick_row(B0 * a + b) ? plane[(B0 * a + b) * LD + i1] : CT<C2>::make(R(0), R(0));
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MTC; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, b = task / N1;
      RegDft<A0, +1>::run(h[m]);
      plane[(b * A0) * LD + i1] = h[m][0];
#pragma unroll
      for (int ka = 1; ka < A0; ++ka) plane[(b * A0 + ka) * LD + i1] = twiddle<+1>(h[m][ka], tw0, b * ka);
    }
  }
  __syncthreads();
  // ---- axis 0: inverse stage 2, times V(r), forward stage 1 ----
#pragma unroll
  for (int m = 0; m < MTB; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * A0) {
      const int i1 = task % N1, ka = task / N1;
      C2 v[B0];
#pragma unroll
      for (int b = 0; b < B0; ++b) v[b] = plane[(b * A0 + ka) * LD + i1];
      R vr[B0];
#pragma unroll
      for (int kb = 0; kb < B0; ++kb) vr[kb] = kPrefetchV ? vpre[kPrefetchV ? m : 0][kb] : vz[(ka + A0 * kb) * N1 + i1];
      RegDft<B0, +1>::run(v);
#pragma unroll
      for (int kb = 0; kb < B0; ++kb) v[kb] = c_scale(v[kb], vr[kb]);
      RegDft<B0, -1>::run(v);
      plane[ka * LD + i1] = v[0];
#pragma unroll
      for (int e = 1; e < B0; ++e) plane[(e * A0 + ka) * LD + i1] = twiddle<-1>(v[e], tw0, ka * e);
    }
  }
  __syncthreads();
  // ---- axis 0, forward stage 2 ----
#pragma unroll
  for (int m = 0; m < MTC; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, e = task / N1;
#pragma unroll
      for (int c = 0; c < A0; ++c) h[m][c] = plane[(e * A0 + c) * LD + i1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MTC; ++m) {
    const int task = tid + m * NT;
    if (task < N1 * B0) {
      const int i1 = task % N1, e = task / N1;
      RegDft<A0, -1>::run(h[m]);
#pragma unroll
      for (int f = 0; f < A0; ++f)
        if (stick_row(e + B0 * f)) plane[(e + B0 * f) * LD + i1] = h[m][f];
    }
  }
  __syncthreads();

  // ---- axis 1, forward, rows holding sticks; gather the sticks ----
  for (int task = tid; task < n_row * A1; task += NT) {
    const int c = task / n_row, t = task - c * n_row;
    C2 *row = plane + row_i0(t) * LD;
    C2 v[B1];
#pragma unroll
    for (int d = 0; d < B1; ++d) v[d] = row[c + A1 * d];
    RegDft<B1, -1>::run(v);
    row[c] = v[0];
#pragma unroll
    for (int e = 1; e < B1; ++e) row[e * A1 + c] = twiddle<-1>(v[e], tw1, c * e);
  }
  __syncthreads();
  for (int task = tid; task < n_row * B1; task += NT) {
    const int e = task / n_row, t = task - e * n_row;
    const C2 *row = plane + row_i0(t) * LD;
    const int4 ri = rinfo[t];
    C2 v[A1];
#pragma unroll
    for (int c = 0; c < A1; ++c) v[c] = row[e * A1 + c];
    RegDft<A1, -1>::run(v);
#pragma unroll
    for (int f = 0; f < A1; ++f) {
      const int s = stick(ri, e + B1 * f);
      if (s >= 0) Tz[s] = v[f];
    }
  }
}

}  // namespace sgw
