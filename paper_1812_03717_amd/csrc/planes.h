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

// Whole-line variant for planes whose rows and columns fit one thread's registers: a thread holds
// a complete row (axis-1 passes) or column (axis-0 pass) and runs both stages of the split in
// registers (the exchange between them is register renaming).  Its arithmetic is that of k_planes
// value for value, without the terms that are zero by construction.
//
// Window: the kernel requires every stick to satisfy -N0/4 <= m0 < N0/4 and -N1/4 <= m1 < N1/4
// (a sphere that the grid holds twice over, as it must for the density, does).  Then along either
// axis a line's inverse input and its needed forward output live on the window i < N/4 or
// i >= 3N/4: the inverse's first stage is a HalfDft and the forward computes only window outputs.
// Window row i0 is kept in LDS slot i0 (i0 < N0/4) or i0 - N0/2 (i0 >= 3N0/4), every column access
// has a compile-time offset, and window rows without sticks are zero-filled once.  Only the window
// rows pass through LDS, once after the axis-1 inverse and once before the axis-1 forward; sticks go
// back to HBM one per thread (coalesced) through a per-stick (i0, i1) table.  The potential is
// loaded one group of the inverse's second stage ahead.  P planes per workgroup.
// split N = A * B of a whole line (A = 4 or 8 for the half-input first stage)
template <int N> struct LineSplit {
  static constexpr int a = Split<N>::a, b = Split<N>::b;
};

template <int N, int SIGN, bool IN_HALF, class C2, class Post>
__device__ __forceinline__ void reg_dft_line(C2 *x, Post &post) {
  constexpr int A = LineSplit<N>::a, B = LineSplit<N>::b;
  C2 y[A][B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    C2 t[A];
    if constexpr (IN_HALF) {
#pragma unroll
      for (int a = 0; a < A; ++a)
        if (4 * a < A || 4 * a >= 3 * A) t[a] = x[B * a + b];
      HalfDft<A, SIGN>::run(t);
    } else {
#pragma unroll
      for (int a = 0; a < A; ++a) t[a] = x[B * a + b];
      RegDft<A, SIGN>::run(t);
    }
#pragma unroll
    for (int ka = 0; ka < A; ++ka) y[ka][b] = twiddle_c<N, SIGN>(t[ka], b * ka);
  }
#pragma unroll
  for (int ka = 0; ka < A; ++ka) {
    post.prefetch(ka + 1);
    RegDft<B, SIGN>::run(y[ka]);
#pragma unroll
    for (int kb = 0; kb < B; ++kb) x[ka + A * kb] = post.apply(ka, kb, y[ka][kb]);
  }
}

struct NoPost {
  __device__ __forceinline__ void prefetch(int) {}
  template <class C2> __device__ __forceinline__ C2 apply(int, int, C2 v) { return v; }
};

// x[ka + A kb] *= V(r) at that i0, for one column; V of group ka + 1 is loaded while group ka is
// transformed
template <class C2, int N0, int N1>
struct PotentialPost {
  using R = typename CT<C2>::R;
  static constexpr int A = LineSplit<N0>::a, B = LineSplit<N0>::b;
  const R *vz;  // V at (i0 = 0, this column), stride N1 along i0
  R cur[B], nxt[B];
  __device__ __forceinline__ explicit PotentialPost(const R *v) : vz(v) {
#pragma unroll
    for (int kb = 0; kb < B; ++kb) cur[kb] = vz[(A * kb) * N1];
  }
  __device__ __forceinline__ void prefetch(int ka) {
    if (ka < A) {
#pragma unroll
      for (int kb = 0; kb < B; ++kb) nxt[kb] = vz[(ka + A * kb) * N1];
    }
  }
  template <class T> __device__ __forceinline__ T apply(int ka, int kb, T v) {
    const T r = c_scale(v, cur[kb]);
    if (kb == B - 1) {
#pragma unroll
      for (int k = 0; k < B; ++k) cur[k] = nxt[k];
    }
    return r;
  }
};

// The line kernel holds max(N0, N1) values per thread: up to 48 in FP64 (192 of 256 VGPRs at 48)
// and up to 72 in FP32 (144 VGPRs at 72).  Planes per workgroup: about 96 (FP64) or 192 (FP32)
// column threads, which measured best at 48 x 48 (LDS and registers then allow 8 resp. 12 waves per
// CU).
template <class C2, int N0, int N1> constexpr bool line_planes_fit() {
  constexpr int nmax = sizeof(C2) == 16 ? 48 : 72;
  return N0 % 4 == 0 && N1 % 4 == 0 && N0 <= nmax && N1 <= nmax && LineSplit<N0>::a % 4 == 0 &&
         LineSplit<N1>::a % 4 == 0;
}
template <class C2, int N1> constexpr int line_plane_count() {
  return (sizeof(C2) == 16 ? 96 : 192) / N1 > 0 ? (sizeof(C2) == 16 ? 96 : 192) / N1 : 1;
}
template <int P, int N1> constexpr int line_plane_threads() { return (P * N1 + 63) / 64 * 64; }
template <class C2, int N0, int N1> constexpr int line_waves_per_eu() {
  constexpr int n = N0 > N1 ? N0 : N1;
  return sizeof(C2) == 16 ? (n <= 16 ? 4 : n <= 24 ? 3 : 2) : (n <= 24 ? 4 : n <= 48 ? 3 : 2);
}
// true when every stick lies in the window the line kernel requires
inline bool line_window_ok(const int n[3], int m0_lo, int n_row, int m1_lo, int m1_hi) {
  return m0_lo >= -n[0] / 4 && m0_lo + n_row - 1 < n[0] / 4 && m1_lo >= -n[1] / 4 && m1_hi < n[1] / 4;
}

template <class C2, int N0, int N1, int P>
__global__ __launch_bounds__((line_plane_threads<P, N1>())) __attribute__((amdgpu_waves_per_eu(line_waves_per_eu<C2, N0, N1>())))
void k_planes_line(C2 *__restrict__ T, long n_planes, int n2, int n_stick, const int4 *__restrict__ rows,
                   const int *__restrict__ stick_ij, int m0_lo, int n_row, const typename CT<C2>::R *__restrict__ vt) {
  using R = typename CT<C2>::R;
  constexpr int NT = line_plane_threads<P, N1>();
  constexpr int LD = N1 + 1;
  constexpr int H0 = N0 / 2, Q0 = N0 / 4, Q1 = N1 / 4;
  __shared__ C2 buf[P][H0][LD];
  const long q0 = (long)blockIdx.x * P;
  const int tid = threadIdx.x;
  const C2 zero = CT<C2>::make(R(0), R(0));
  // window row m0 (-N0/4 <= m0 < N0/4) -> LDS slot
  auto slot_of = [](int m0) { return m0 >= 0 ? m0 : m0 + H0; };
  auto in_window1 = [](int i1) { return i1 < Q1 || i1 >= 3 * Q1; };

  // window rows without sticks read as zero in the axis-0 pass
  const int n_below = m0_lo + Q0, n_empty = H0 - n_row;
  for (int e = tid; e < P * n_empty * LD; e += NT) {
    const int p = e / (n_empty * LD), r = e - p * (n_empty * LD);
    const int k = r / LD, c = r - k * LD;
    const int m0 = k < n_below ? -Q0 + k : m0_lo + n_row + (k - n_below);
    buf[p][slot_of(m0)][c] = zero;
  }

  // ---- axis 1, inverse: one stick row per thread ----
  NoPost none;
  for (int task = tid; task < P * n_row; task += NT) {
    const int p = task / n_row, t = task - p * n_row;
    if (q0 + p >= n_planes) continue;
    const int4 ri = rows[t];
    const C2 *run = T + (q0 + p) * n_stick + (ri.x - ri.y);  // run[m1]: the row's stick at m1
    C2 x[N1];
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) {
      if (!in_window1(i1)) continue;
      // the row's sticks are one run of m1 values; outside it the row is zero
      const int m1 = i1 < Q1 ? i1 : i1 - N1;
      x[i1] = zero;
      if (m1 >= ri.y && m1 <= ri.z) x[i1] = run[m1];
    }
    reg_dft_line<N1, +1, true>(x, none);
    C2 *row = buf[p][slot_of(m0_lo + t)];
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) row[i1] = x[i1];
  }
  __syncthreads();

  // ---- axis 0: inverse, times V(r), forward; one column per thread ----
  for (int task = tid; task < P * N1; task += NT) {
    const int p = task / N1, i1 = task - p * N1;
    const long q = q0 + p;
    if (q >= n_planes) continue;
    const int z = (int)(q % n2);
    C2 x[N0];
#pragma unroll
    for (int j = 0; j < Q0; ++j) {
      x[j] = buf[p][j][i1];                   // rows i0 = j
      x[N0 - Q0 + j] = buf[p][Q0 + j][i1];    // rows i0 = 3 N0 / 4 + j
    }
    PotentialPost<C2, N0, N1> vpost(vt + (long)z * N0 * N1 + i1);
    reg_dft_line<N0, +1, true>(x, vpost);
    reg_dft_line<N0, -1, false>(x, none);
#pragma unroll
    for (int j = 0; j < Q0; ++j) {
      buf[p][j][i1] = x[j];
      buf[p][Q0 + j][i1] = x[N0 - Q0 + j];
    }
  }
  __syncthreads();

  // ---- axis 1, forward: one stick row per thread, window columns back into its slot ----
  for (int task = tid; task < P * n_row; task += NT) {
    const int p = task / n_row, t = task - p * n_row;
    if (q0 + p >= n_planes) continue;
    C2 *row = buf[p][slot_of(m0_lo + t)];
    C2 x[N1];
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) x[i1] = row[i1];
    reg_dft_line<N1, -1, false>(x, none);
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1)
      if (in_window1(i1)) row[i1] = x[i1];
  }
  __syncthreads();

  // ---- gather the sticks, one per thread ----
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (q0 + p >= n_planes) break;
    C2 *Tz = T + (q0 + p) * n_stick;
    for (int s = tid; s < n_stick; s += NT) {
      const int ij = stick_ij[s];
      const int i0 = ij >> 16;
      Tz[s] = buf[p][i0 < Q0 ? i0 : i0 - H0][ij & 0xffff];
    }
  }
}

// Pair-of-threads variant for FP64 planes, built for lines that do not fit one thread's registers
// (64 and 72 points) and usable at every size, under the same central-half window.  With window input X[k] (k < N/4 or k >= 3N/4, i.e.
// one k for each residue j = k mod N/2), the inverse line splits by the parity r of the real-space
// index n = 2m + r into two half-length transforms:
//   x[2m + r] = sum_j X[k_j] w_N^(r k_j) w_{N/2}^(m j),        k_j = j (j < N/4), j + N/2 (else)
// and the forward's window outputs are the sum of the two parities' half-length transforms:
//   X'[k_j] = sum_r w_N^(-r k_j) sum_m x'[2m + r] w_{N/2}^(-m j).
// So a row or column is handled by two threads (r = 0, 1), each holding N/2 values; the parity-1
// thread twiddles its inputs and outputs, and the two forward halves are added through LDS (parity 1
// writes, parity 0 adds its own).  The arithmetic is that of the full-length transforms
// reassociated, not the same operations: results agree with the other plane kernels to rounding.
template <int N, int SIGN, class C2>
__device__ __forceinline__ void half_line_dft(C2 *x) {
  if constexpr (N == 36) {
    pfa_dft<4, 9, SIGN>(x);
  } else if constexpr (N == 24) {
    pfa_dft<8, 3, SIGN>(x);
  } else if constexpr (N == 8 || N == 12) {
    RegDft<N, SIGN>::run(x);
  } else {
    NoPost none;
    reg_dft_line<N, SIGN, false>(x, none);
  }
}
template <class C2, int N0, int N1> constexpr bool pair_planes_fit() {
  return sizeof(C2) == 16 && N0 % 4 == 0 && N1 % 4 == 0 && N0 <= 72 && N1 <= 72;
}
// threads: one per (parity, column) and at least one per (parity, window row)
template <int N0, int N1> constexpr int pair_plane_threads() {
  return ((2 * N1 > N0 ? 2 * N1 : N0) + 63) / 64 * 64;
}

template <int N0, int N1>
__global__ __launch_bounds__((pair_plane_threads<N0, N1>())) __attribute__((amdgpu_waves_per_eu(2)))
void k_planes_pair(double2 *__restrict__ T, int n2, int n_stick, const int4 *__restrict__ rows,
                   const int *__restrict__ stick_ij, int m0_lo, int n_row, const double *__restrict__ vt) {
  constexpr int NT = pair_plane_threads<N0, N1>();
  constexpr int LD = N1 + 1;
  constexpr int H0 = N0 / 2, Q0 = N0 / 4, H1 = N1 / 2, Q1 = N1 / 4;
  __shared__ double2 buf[H0][LD];
  const long q = blockIdx.x;
  const int tid = threadIdx.x;
  const int z = (int)(q % n2);
  double2 *Tq = T + q * n_stick;
  const double *vz = vt + (long)z * N0 * N1;
  const double2 zero = make_double2(0.0, 0.0);
  auto slot_of = [](int m0) { return m0 >= 0 ? m0 : m0 + H0; };

  // window rows without sticks read as zero in the axis-0 pass
  const int n_below = m0_lo + Q0, n_empty = H0 - n_row;
  for (int e = tid; e < n_empty * LD; e += NT) {
    const int k = e / LD, c = e - k * LD;
    const int m0 = k < n_below ? -Q0 + k : m0_lo + n_row + (k - n_below);
    buf[slot_of(m0)][c] = zero;
  }

  // ---- axis 1, inverse: (parity, stick row) per thread; parity r writes the columns 2m + r ----
  const bool row_act = tid < 2 * n_row;
  const int rr = tid >= n_row;
  const int t = tid - rr * n_row;
  const int srow = slot_of(m0_lo + t);
  if (row_act) {
    const int4 ri = rows[t];
    const double2 *run = Tq + (ri.x - ri.y);  // run[m1]: the row's stick at m1
    double2 x[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j) {
      const int m1 = j < Q1 ? j : j - H1;
      x[j] = zero;
      if (m1 >= ri.y && m1 <= ri.z) x[j] = run[m1];
    }
    if (rr) {
#pragma unroll
      for (int j = 0; j < H1; ++j) x[j] = twiddle_c<N1, +1>(x[j], j < Q1 ? j : j + H1);
    }
    half_line_dft<H1, +1>(x);
#pragma unroll
    for (int m = 0; m < H1; ++m) buf[srow][2 * m + rr] = x[m];
  }
  __syncthreads();

  // ---- axis 0: inverse, times V(r), forward; (parity, column) per thread ----
  {
    const bool act = tid < 2 * N1;
    const int r = tid >= N1;
    const int i1 = tid - r * N1;
    double2 x[H0];
    if (act) {
#pragma unroll
      for (int j = 0; j < H0; ++j) x[j] = buf[j][i1];  // slot j holds window row k_j
      if (r) {
#pragma unroll
        for (int j = 0; j < H0; ++j) x[j] = twiddle_c<N0, +1>(x[j], j < Q0 ? j : j + H0);
      }
      half_line_dft<H0, +1>(x);
      const double *vc = vz + r * N1 + i1;  // V at i0 = 2m + r
#pragma unroll
      for (int m = 0; m < H0; ++m) x[m] = c_scale(x[m], vc[2 * m * N1]);
      half_line_dft<H0, -1>(x);
      if (r) {
#pragma unroll
        for (int j = 0; j < H0; ++j) x[j] = twiddle_c<N0, -1>(x[j], j < Q0 ? j : j + H0);
      }
    }
    __syncthreads();
    if (act && r) {
#pragma unroll
      for (int j = 0; j < H0; ++j) buf[j][i1] = x[j];
    }
    __syncthreads();
    if (act && !r) {
#pragma unroll
      for (int j = 0; j < H0; ++j) buf[j][i1] = c_add(x[j], buf[j][i1]);
    }
    __syncthreads();
  }

  // ---- axis 1, forward: (parity, stick row) per thread; window column k_j <- sum of parities ----
  {
    double2 x[H1];
    if (row_act) {
#pragma unroll
      for (int m = 0; m < H1; ++m) x[m] = buf[srow][2 * m + rr];
      half_line_dft<H1, -1>(x);
      if (rr) {
#pragma unroll
        for (int j = 0; j < H1; ++j) x[j] = twiddle_c<N1, -1>(x[j], j < Q1 ? j : j + H1);
      }
    }
    __syncthreads();
    if (row_act && rr) {
#pragma unroll
      for (int j = 0; j < H1; ++j) buf[srow][j < Q1 ? j : j + H1] = x[j];
    }
    __syncthreads();
    if (row_act && !rr) {
#pragma unroll
      for (int j = 0; j < H1; ++j) {
        const int c = j < Q1 ? j : j + H1;
        buf[srow][c] = c_add(x[j], buf[srow][c]);
      }
    }
    __syncthreads();
  }

  // ---- gather the sticks, one per thread ----
  for (int s = tid; s < n_stick; s += NT) {
    const int ij = stick_ij[s];
    const int i0 = ij >> 16;
    Tq[s] = buf[i0 < Q0 ? i0 : i0 - H0][ij & 0xffff];
  }
}


// Three-thread variant for FP64 planes: the real-space index of a line splits by its residue r mod 3,
// n = 3m + r (N = 3L), so each of three threads holds L = N/3 values (24 at 72 points: ~100 fewer
// VGPRs than the two-thread split, three waves per SIMD instead of two).  Under the central-half
// window (k < N/4 or k >= 3N/4), k mod L takes every residue rho once or twice: rho < N/4 from the
// lower half (k = rho), rho >= N/12 from the upper half (k = rho + 2L).  Then
//   x[3m + r] = sum_rho Y_r[rho] w_L^(m rho),  Y_r[rho] = sum_{k in window, k = rho mod L} X[k] w_N^(r k)
// and the forward's window outputs are
//   X'[k] = sum_r w_N^(-r k) Z_r[k mod L],      Z_r = forward L-point transform of x'[3m + r].
// The three residues' forward contributions are added through LDS: along axis 0 (columns) in three
// rounds (r = 2 writes, r = 1 and r = 0 add in turn); along axis 1 (rows) each residue stores its Z_r
// in the row (3L = N columns), and then one thread per (row, third of the window slots) sums the
// three residues of its slots in the same order and writes them back.  Window slot s of a line holds
// k = s (s < N/4) or k = s + N/2 (s >= N/4).
template <int N0, int N1> constexpr bool tri_planes_fit() {
  return N0 % 12 == 0 && N1 % 12 == 0 && N0 >= 24 && N1 >= 24 && N0 <= 72 && N1 <= 72;
}
template <int N0, int N1> constexpr int tri_plane_threads() {
  return ((3 * N1 > 3 * (N0 / 2) ? 3 * N1 : 3 * (N0 / 2)) + 63) / 64 * 64;
}

// y[rho] = Y_R[rho] from the window slots src[s * stride] (inverse: SIGN = +1)
template <int N, int R>
__device__ __forceinline__ void tri_fold(const double2 *src, int stride, double2 *y) {
  constexpr int L = N / 3, Q = N / 4, H = N / 2, LO = N / 12;
#pragma unroll
  for (int rho = 0; rho < L; ++rho) {
    double2 v = make_double2(0.0, 0.0);
    if (rho < Q) v = twiddle_c<N, +1>(src[rho * stride], R * rho);
    if (rho >= LO) v = c_add(v, twiddle_c<N, +1>(src[(rho + 2 * L - H) * stride], R * (rho + 2 * L)));
    y[rho] = v;
  }
}
// the window slots' forward contributions w_N^(-R k) Z[k mod L]: dst[s * stride] = (ADD ? dst + : ) c_s
template <int N, int R, bool ADD>
__device__ __forceinline__ void tri_unfold(const double2 *z, double2 *dst, int stride) {
  constexpr int L = N / 3, Q = N / 4, H = N / 2;
#pragma unroll
  for (int s = 0; s < H; ++s) {
    const int k = s < Q ? s : s + H;
    const double2 c = twiddle_c<N, -1>(z[k % L], R * k);
    dst[s * stride] = ADD ? c_add(dst[s * stride], c) : c;
  }
}
template <int N, bool ADD>
__device__ __forceinline__ void tri_unfold_r(int r, const double2 *z, double2 *dst, int stride) {
  if (r == 0) tri_unfold<N, 0, ADD>(z, dst, stride);
  else if (r == 1) tri_unfold<N, 1, ADD>(z, dst, stride);
  else tri_unfold<N, 2, ADD>(z, dst, stride);
}

// window slots s of block G (s in [G H/3, (G + 1) H/3), column k = s or s + N/2) of a line whose
// residue transforms Z_r sit at line[r * L + m]: o[j] = (w^(-2k) Z_2 + w^(-k) Z_1) + Z_0 at k mod L
template <int N, int G>
__device__ __forceinline__ void tri_gather(const double2 *line, double2 *o) {
  constexpr int L = N / 3, Q = N / 4, H = N / 2, HB = H / 3;
#pragma unroll
  for (int j = 0; j < HB; ++j) {
    const int s = G * HB + j;
    const int k = s < Q ? s : s + H;
    const double2 c2 = twiddle_c<N, -1>(line[2 * L + k % L], 2 * k);
    o[j] = c_add(c_add(c2, twiddle_c<N, -1>(line[L + k % L], k)), line[k % L]);
  }
}
template <int N, int G>
__device__ __forceinline__ void tri_scatter(const double2 *o, double2 *line) {
  constexpr int Q = N / 4, H = N / 2, HB = H / 3;
#pragma unroll
  for (int j = 0; j < HB; ++j) {
    const int s = G * HB + j;
    line[s < Q ? s : s + H] = o[j];
  }
}

template <int N0, int N1>
__global__ __launch_bounds__((tri_plane_threads<N0, N1>())) __attribute__((amdgpu_waves_per_eu(3)))
void k_planes_tri(double2 *__restrict__ T, int n2, int n_stick, const int4 *__restrict__ rows,
                  const int *__restrict__ stick_ij, int m0_lo, int n_row, const double *__restrict__ vt) {
  constexpr int NT = tri_plane_threads<N0, N1>();
  constexpr int LD = N1 + 1;
  constexpr int H0 = N0 / 2, Q0 = N0 / 4, H1 = N1 / 2, Q1 = N1 / 4, L0 = N0 / 3, L1 = N1 / 3;
  __shared__ double2 buf[H0][LD];
  const long q = blockIdx.x;
  const int tid = threadIdx.x;
  const int z = (int)(q % n2);
  double2 *Tq = T + q * n_stick;
  const double *vz = vt + (long)z * N0 * N1;
  const double2 zero = make_double2(0.0, 0.0);
  auto slot_of = [](int m0) { return m0 >= 0 ? m0 : m0 + H0; };

  // window rows without sticks read as zero in the axis-0 pass
  const int n_below = m0_lo + Q0, n_empty = H0 - n_row;
  for (int e = tid; e < n_empty * LD; e += NT) {
    const int k = e / LD, c = e - k * LD;
    const int m0 = k < n_below ? -Q0 + k : m0_lo + n_row + (k - n_below);
    buf[slot_of(m0)][c] = zero;
  }

  // ---- axis 1, inverse: (residue, stick row) per thread; residue r writes the columns 3m + r ----
  const bool row_act = tid < 3 * n_row;
  const int rr = row_act ? tid / n_row : 0;
  const int t = tid - rr * n_row;
  const int srow = slot_of(m0_lo + t);
  // the row's window values go to its LDS row by slot first (each of the three threads loads a third)
  if (row_act) {
    const int4 ri = rows[t];
    const double2 *run = Tq + (ri.x - ri.y);  // run[m1]: the row's stick at m1
    double2 w[H1 / 3];
#pragma unroll
    for (int u = 0; u < H1 / 3; ++u) {
      const int j = 3 * u + rr;
      const int m1 = j < Q1 ? j : j - H1;
      w[u] = zero;
      if (m1 >= ri.y && m1 <= ri.z) w[u] = run[m1];
    }
#pragma unroll
    for (int u = 0; u < H1 / 3; ++u) buf[srow][3 * u + rr] = w[u];
  }
  __syncthreads();
  double2 xr[L1];
  if (row_act) {
    if (rr == 0) tri_fold<N1, 0>(&buf[srow][0], 1, xr);
    else if (rr == 1) tri_fold<N1, 1>(&buf[srow][0], 1, xr);
    else tri_fold<N1, 2>(&buf[srow][0], 1, xr);
    half_line_dft<L1, +1>(xr);
  }
  __syncthreads();  // the row's window slots have been read
  if (row_act) {
#pragma unroll
    for (int m = 0; m < L1; ++m) buf[srow][3 * m + rr] = xr[m];
  }
  __syncthreads();

  // ---- axis 0: inverse, times V(r), forward; (residue, column) per thread ----
  {
    const bool act = tid < 3 * N1;
    const int r = act ? tid / N1 : 0;
    const int i1 = tid - r * N1;
    double2 x[L0];
    if (act) {
      const double2 *col = &buf[0][i1];
      if (r == 0) tri_fold<N0, 0>(col, LD, x);
      else if (r == 1) tri_fold<N0, 1>(col, LD, x);
      else tri_fold<N0, 2>(col, LD, x);
      half_line_dft<L0, +1>(x);
      const double *vc = vz + r * N1 + i1;  // V at i0 = 3m + r
#pragma unroll
      for (int m = 0; m < L0; ++m) x[m] = c_scale(x[m], vc[3 * m * N1]);
      half_line_dft<L0, -1>(x);
    }
    __syncthreads();  // every column's window slots have been read
    if (act && r == 2) tri_unfold_r<N0, false>(2, x, &buf[0][i1], LD);
    __syncthreads();
    if (act && r == 1) tri_unfold_r<N0, true>(1, x, &buf[0][i1], LD);
    __syncthreads();
    if (act && r == 0) tri_unfold_r<N0, true>(0, x, &buf[0][i1], LD);
    __syncthreads();
  }

  // ---- axis 1, forward: (residue, stick row) per thread for the transforms; then the window
  //      columns of a row are summed over the residues by (slot block, stick row) threads ----
  {
    double2 x[L1];
    if (row_act) {
#pragma unroll
      for (int m = 0; m < L1; ++m) x[m] = buf[srow][3 * m + rr];
      half_line_dft<L1, -1>(x);
    }
    __syncthreads();  // the row's real-space values have been read
    if (row_act) {  // Z_rr at columns rr * L1 + m of the row
#pragma unroll
      for (int m = 0; m < L1; ++m) buf[srow][rr * L1 + m] = x[m];
    }
    __syncthreads();
    // block g of the window slots (H1 / 3 of them) of row tg; with at least three waves, block g is
    // wave g (the compile-time slots then do not diverge within a wave)
    constexpr int HB = H1 / 3;
    const int g = NT >= 192 ? tid >> 6 : (n_row > 0 ? tid / n_row : 3);
    const int tg = NT >= 192 ? (tid & 63) : tid - g * n_row;
    const bool gact = g < 3 && tg < n_row;
    const int grow = slot_of(m0_lo + (gact ? tg : 0));
    double2 o[HB];
    if (gact) {
      if (g == 0) tri_gather<N1, 0>(&buf[grow][0], o);
      else if (g == 1) tri_gather<N1, 1>(&buf[grow][0], o);
      else tri_gather<N1, 2>(&buf[grow][0], o);
    }
    __syncthreads();  // every row's residue transforms have been read
    if (gact) {
      if (g == 0) tri_scatter<N1, 0>(o, &buf[grow][0]);
      else if (g == 1) tri_scatter<N1, 1>(o, &buf[grow][0]);
      else tri_scatter<N1, 2>(o, &buf[grow][0]);
    }
    __syncthreads();
  }

  // ---- gather the sticks, one per thread ----
  for (int s = tid; s < n_stick; s += NT) {
    const int ij = stick_ij[s];
    const int i0 = ij >> 16;
    Tq[s] = buf[i0 < Q0 ? i0 : i0 - H0][ij & 0xffff];
  }
}

}  // namespace sgw
