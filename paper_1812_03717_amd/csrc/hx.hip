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
#include "planes.h"
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
constexpr int kStickBatch = 4;

template <class C2>
__device__ __forceinline__ C2 to_c(double2 v) {
  using R = typename CT<C2>::R;
  return CT<C2>::make((R)v.x, (R)v.y);
}

template <class C2, int N2>
__global__ __launch_bounds__(kStickThreads) void k_sticks_inv(VecSrc x, C2 *__restrict__ T, int n_stick,
                                                              const int32_t *__restrict__ stick_off,
                                                              const int32_t *__restrict__ pw_stick,
                                                              const int32_t *__restrict__ pw_z,
                                                              const C2 *__restrict__ twg, int groups) {
  using R = typename CT<C2>::R;
  constexpr int SG = sticks_per_block<N2>();
  constexpr int LDC = N2 + 1;
  __shared__ C2 col[SG * LDC];
  __shared__ C2 tw[N2];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const double2 *xv = x.ptr(vec);
  for (int i = tid; i < SG * LDC; i += kStickThreads) col[i] = CT<C2>::make(R(0), R(0));
  for (int i = tid; i < N2; i += kStickThreads) tw[i] = twg[i];
  __syncthreads();
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  // kStickBatch plane waves per thread at a time: their loads are all issued before any is used
  for (int gb = g0 + tid; gb < g1; gb += kStickBatch * kStickThreads) {
    int pos[kStickBatch];
    double2 xg[kStickBatch];
#pragma unroll
    for (int u = 0; u < kStickBatch; ++u) {
      const int g = gb + u * kStickThreads;
      const bool ok = g < g1;
      pos[u] = ok ? (pw_stick[g] - s0) * LDC + pw_z[g] : 0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kStickBatch; ++u)
      if (gb + u * kStickThreads < g1) col[pos[u]] = to_c<C2>(xg[u]);
  }
  __syncthreads();
  lds_fft<N2, +1, SG, kStickThreads, false>(col, ns, StrideBase{LDC}, 1, tw, tid);
  C2 *Tv = T + (long)vec * N2 * n_stick + s0;
  for (int i = tid; i < ns * N2; i += kStickThreads) {
    const int z = i / ns, s = i - z * ns;
    Tv[(long)z * n_stick + s] = col[s * LDC + z];
  }
}

template <class C2, int N2>
__global__ __launch_bounds__(kStickThreads) void k_sticks_fwd(const C2 *__restrict__ T, int n_stick,
                                                              const int32_t *__restrict__ stick_off,
                                                              const int32_t *__restrict__ pw_stick,
                                                              const int32_t *__restrict__ pw_z,
                                                              const C2 *__restrict__ twg, int groups,
                                                              VecSrc x, const double *__restrict__ kin,
                                                              double2 *__restrict__ y, long ldy, double scale) {
  constexpr int SG = sticks_per_block<N2>();
  constexpr int LDC = N2 + 1;
  __shared__ C2 col[SG * LDC];
  __shared__ C2 tw[N2];
  const int tid = threadIdx.x;
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  for (int i = tid; i < N2; i += kStickThreads) tw[i] = twg[i];
  const C2 *Tv = T + (long)vec * N2 * n_stick + s0;
  for (int i = tid; i < ns * N2; i += kStickThreads) {
    const int z = i / ns, s = i - z * ns;
    col[s * LDC + z] = Tv[(long)z * n_stick + s];
  }
  __syncthreads();
  lds_fft<N2, -1, SG, kStickThreads, false>(col, ns, StrideBase{LDC}, 1, tw, tid);
  const double2 *xv = x.ptr(vec);
  double2 *yv = y + (long)vec * ldy;
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int gb = g0 + tid; gb < g1; gb += kStickBatch * kStickThreads) {
    int pos[kStickBatch];
    double2 xg[kStickBatch];
    double t[kStickBatch];
#pragma unroll
    for (int u = 0; u < kStickBatch; ++u) {
      const int g = gb + u * kStickThreads;
      const bool ok = g < g1;
      pos[u] = ok ? (pw_stick[g] - s0) * LDC + pw_z[g] : 0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
      t[u] = ok ? kin[g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStickBatch; ++u) {
      const int g = gb + u * kStickThreads;
      if (g < g1) {
        const C2 c = col[pos[u]];
        yv[g] = make_double2(fma((double)c.x, scale, t[u] * xg[u].x), fma((double)c.y, scale, t[u] * xg[u].y));
      }
    }
  }
}

// Whole-line stick kernels: a workgroup takes 64 consecutive sticks of one vector, one thread per
// stick transforms it in registers (planes.h: reg_dft_line).  They require the window
// -N2/4 <= m2 < N2/4 of the plane kernel's, so the inverse's first stage reads only the window
// and the forward computes only window outputs.  The window values pass through LDS
// ([window row][stick]; window row w holds m2 = w for w < N2/4, m2 = w - N2/2 otherwise) between
// the coalesced plane-wave accesses and the per-stick transforms; the T accesses of consecutive
// threads are consecutive.
constexpr int kStickLineSticks = 64;
constexpr int kGatherBatch = 8;
template <class C2, int N2>
__global__ __launch_bounds__(kStickLineSticks) __attribute__((amdgpu_waves_per_eu(line_waves_per_eu<C2, N2, N2>())))
void k_sticks_inv_line(VecSrc x, C2 *__restrict__ T, int n_stick, int groups, const int32_t *__restrict__ stick_off,
                       const int32_t *__restrict__ pw_stick, const int32_t *__restrict__ pw_z) {
  using R = typename CT<C2>::R;
  constexpr int Q = N2 / 4;
  constexpr int SG = kStickLineSticks;
  __shared__ C2 win[2 * Q][SG];
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const int tid = threadIdx.x;
  const C2 zero = CT<C2>::make(R(0), R(0));
#pragma unroll
  for (int w = 0; w < 2 * Q; ++w) win[w][tid] = zero;
  __syncthreads();
  const double2 *xv = x.ptr(vec);
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int gb = g0 + tid; gb < g1; gb += kGatherBatch * SG) {
    int z[kGatherBatch], st[kGatherBatch];
    double2 xg[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * SG;
      const bool ok = g < g1;
      z[u] = ok ? pw_z[g] : 0;
      st[u] = ok ? pw_stick[g] : s0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u)
      if (gb + u * SG < g1) win[z[u] < Q ? z[u] : z[u] - 2 * Q][st[u] - s0] = to_c<C2>(xg[u]);
  }
  __syncthreads();
  if (tid >= ns) return;
  C2 v[N2];
#pragma unroll
  for (int w = 0; w < Q; ++w) {
    v[w] = win[w][tid];
    v[N2 - Q + w] = win[Q + w][tid];
  }
  NoPost none;
  reg_dft_line<N2, +1, true>(v, none);
  C2 *Tv = T + (long)vec * N2 * n_stick + s0 + tid;
#pragma unroll
  for (int z = 0; z < N2; ++z) Tv[(long)z * n_stick] = v[z];
}

// inverse with direct loads: one thread per (vector, stick) reads its run of plane waves itself
// (one base pointer, compile-time offsets), 256 threads per workgroup and no LDS; measured faster
// than the LDS-staged kernel in FP64 (more waves resident), slower in FP32
template <class C2, int N2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(line_waves_per_eu<C2, N2, N2>())))
void k_sticks_inv_direct(VecSrc x, C2 *__restrict__ T, int n_stick, long n_items,
                         const int32_t *__restrict__ stick_off, const int32_t *__restrict__ pw_z) {
  using R = typename CT<C2>::R;
  constexpr int Q = N2 / 4;
  const long item = (long)blockIdx.x * 256 + threadIdx.x;
  if (item >= n_items) return;
  const int vec = (int)(item / n_stick), s = (int)(item - (long)vec * n_stick);
  const int g0 = stick_off[s], g1 = stick_off[s + 1];
  const int z0 = pw_z[g0];
  const int m2lo = z0 <= (N2 - 1) / 2 ? z0 : z0 - N2, m2hi = m2lo + (g1 - g0) - 1;
  const double2 *run = x.ptr(vec) + (g0 - m2lo);  // run[m2]: the coefficient at m2
  const C2 zero = CT<C2>::make(R(0), R(0));
  C2 v[N2];
#pragma unroll
  for (int i2 = 0; i2 < N2; ++i2) {
    if (i2 >= Q && i2 < 3 * Q) continue;
    const int m2 = i2 < Q ? i2 : i2 - N2;
    v[i2] = zero;
    if (m2 >= m2lo && m2 <= m2hi) v[i2] = to_c<C2>(run[m2]);
  }
  NoPost none;
  reg_dft_line<N2, +1, true>(v, none);
  C2 *Tv = T + (long)vec * N2 * n_stick + s;
#pragma unroll
  for (int z = 0; z < N2; ++z) Tv[(long)z * n_stick] = v[z];
}

// y[g] = scale * (window value of plane wave g) + kin[g] x[g] for the plane waves of sticks
// [s0, s0 + ns), read from win[window row][stick - s0] (window row w: m2 = w for w < Q, w - 2Q
// otherwise); NT threads, kGatherBatch plane waves per thread at a time, all loads issued before use
// (the gather of k_sticks_fwd_line, for other thread counts)
template <class C2, int Q, int SG, int NT>
__device__ __forceinline__ void fwd_window_gather(const C2 (*win)[SG], int s0, int ns,
                                                  const int32_t *__restrict__ stick_off,
                                                  const int32_t *__restrict__ pw_stick,
                                                  const int32_t *__restrict__ pw_z,
                                                  const double2 *__restrict__ xv, const double *__restrict__ kin,
                                                  double2 *__restrict__ yv, double scale) {
  const int tid = threadIdx.x;
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int gb = g0 + tid; gb < g1; gb += kGatherBatch * NT) {
    int z[kGatherBatch], st[kGatherBatch];
    double2 xg[kGatherBatch];
    double t[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * NT;
      const bool ok = g < g1;
      z[u] = ok ? pw_z[g] : 0;
      st[u] = ok ? pw_stick[g] : s0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
      t[u] = ok ? kin[g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * NT;
      if (g < g1) {
        const C2 c = win[z[u] < Q ? z[u] : z[u] - 2 * Q][st[u] - s0];
        yv[g] = make_double2(fma((double)c.x, scale, t[u] * xg[u].x), fma((double)c.y, scale, t[u] * xg[u].y));
      }
    }
  }
}

template <class C2, int N2>
__global__ __launch_bounds__(kStickLineSticks) __attribute__((amdgpu_waves_per_eu(line_waves_per_eu<C2, N2, N2>())))
void k_sticks_fwd_line(const C2 *__restrict__ T, int n_stick, int groups, const int32_t *__restrict__ stick_off,
                       const int32_t *__restrict__ pw_stick, const int32_t *__restrict__ pw_z, VecSrc x,
                       const double *__restrict__ kin, double2 *__restrict__ y, long ldy, double scale) {
  constexpr int Q = N2 / 4;
  constexpr int SG = kStickLineSticks;
  __shared__ C2 win[2 * Q][SG];  // window row w: m2 = w (w < Q) or w - 2Q
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const int tid = threadIdx.x;
  if (tid < ns) {
    const C2 *Tv = T + (long)vec * N2 * n_stick + s0 + tid;
    C2 v[N2];
#pragma unroll
    for (int z = 0; z < N2; ++z) v[z] = Tv[(long)z * n_stick];
    NoPost none;
    reg_dft_line<N2, -1, false>(v, none);
#pragma unroll
    for (int w = 0; w < Q; ++w) {
      win[w][tid] = v[w];
      win[Q + w][tid] = v[N2 - Q + w];
    }
  }
  __syncthreads();
  const double2 *xv = x.ptr(vec);
  double2 *yv = y + (long)vec * ldy;
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  // kGatherBatch plane waves per thread at a time: their loads are all issued before any is used
  for (int gb = g0 + tid; gb < g1; gb += kGatherBatch * SG) {
    int z[kGatherBatch], st[kGatherBatch];
    double2 xg[kGatherBatch];
    double t[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * SG;
      const bool ok = g < g1;
      z[u] = ok ? pw_z[g] : 0;
      st[u] = ok ? pw_stick[g] : s0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
      t[u] = ok ? kin[g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * SG;
      if (g < g1) {
        const C2 c = win[z[u] < Q ? z[u] : z[u] - 2 * Q][st[u] - s0];
        yv[g] = make_double2(fma((double)c.x, scale, t[u] * xg[u].x), fma((double)c.y, scale, t[u] * xg[u].y));
      }
    }
  }
}

// Stick kernels for FP64 lines too long for one thread (64 and 72 points), under the same window:
// two threads per stick split the transform by the parity r of i2 (planes.h: k_planes_pair).  The
// inverse writes T at i2 = 2m + r; the forward's two halves meet in the LDS window (parity 1 writes,
// parity 0 adds) before the coalesced gather.
// Inverse: a workgroup gathers the plane waves of 64 sticks into the LDS window once (coalesced;
// measured a third faster than each thread of a pair loading its stick's run itself), then each
// (parity, stick) thread transforms its column of the window.
template <int N2>
__global__ __launch_bounds__(2 * kStickLineSticks) __attribute__((amdgpu_waves_per_eu(2)))
void k_sticks_inv_pair(VecSrc x, double2 *__restrict__ T, int n_stick, int groups, const int32_t *__restrict__ stick_off,
                       const int32_t *__restrict__ pw_stick, const int32_t *__restrict__ pw_z) {
  constexpr int Q = N2 / 4, H = N2 / 2;
  constexpr int SG = kStickLineSticks, NT = 2 * SG;
  __shared__ double2 win[2 * Q][SG];  // window row w: m2 = w (w < Q) or w - 2Q
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * Q * SG; e += NT) win[e / SG][e % SG] = make_double2(0.0, 0.0);
  __syncthreads();
  const double2 *xv = x.ptr(vec);
  const int g0 = stick_off[s0], g1 = stick_off[s0 + ns];
  for (int gb = g0 + tid; gb < g1; gb += kGatherBatch * NT) {
    int z[kGatherBatch], st[kGatherBatch];
    double2 xg[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int g = gb + u * NT;
      const bool ok = g < g1;
      z[u] = ok ? pw_z[g] : 0;
      st[u] = ok ? pw_stick[g] : s0;
      xg[u] = ok ? xv[g] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u)
      if (gb + u * NT < g1) win[z[u] < Q ? z[u] : z[u] - 2 * Q][st[u] - s0] = xg[u];
  }
  __syncthreads();
  const int r = tid / SG, t = tid - r * SG;  // parity per wavefront
  if (t >= ns) return;
  double2 v[H];
#pragma unroll
  for (int j = 0; j < H; ++j) v[j] = win[j][t];
  if (r) {
#pragma unroll
    for (int j = 0; j < H; ++j) v[j] = twiddle_c<N2, +1>(v[j], j < Q ? j : j + H);
  }
  half_line_dft<H, +1>(v);
  double2 *Tv = T + ((long)vec * N2 + r) * n_stick + s0 + t;
#pragma unroll
  for (int m = 0; m < H; ++m) Tv[(long)(2 * m) * n_stick] = v[m];
}

template <int N2>
__global__ __launch_bounds__(2 * kStickLineSticks) __attribute__((amdgpu_waves_per_eu(2)))
void k_sticks_fwd_pair(const double2 *__restrict__ T, int n_stick, int groups, const int32_t *__restrict__ stick_off,
                       const int32_t *__restrict__ pw_stick, const int32_t *__restrict__ pw_z, VecSrc x,
                       const double *__restrict__ kin, double2 *__restrict__ y, long ldy, double scale) {
  constexpr int Q = N2 / 4, H = N2 / 2;
  constexpr int SG = kStickLineSticks;
  __shared__ double2 win[2 * Q][SG];  // window row w: m2 = w (w < Q) or w - 2Q
  const int vec = blockIdx.x / groups;
  const int s0 = (blockIdx.x - vec * groups) * SG;
  const int ns = min(SG, n_stick - s0);
  const int tid = threadIdx.x;
  const int r = tid / SG, t = tid - r * SG;  // parity per wavefront
  double2 v[H];
  if (t < ns) {
    const double2 *Tv = T + ((long)vec * N2 + r) * n_stick + s0 + t;
#pragma unroll
    for (int m = 0; m < H; ++m) v[m] = Tv[(long)(2 * m) * n_stick];
    half_line_dft<H, -1>(v);
    if (r) {
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = twiddle_c<N2, -1>(v[j], j < Q ? j : j + H);
#pragma unroll
      for (int j = 0; j < H; ++j) win[j][t] = v[j];
    }
  }
  __syncthreads();
  if (t < ns && !r) {
#pragma unroll
    for (int j = 0; j < H; ++j) win[j][t] = c_add(v[j], win[j][t]);
  }
  __syncthreads();
  fwd_window_gather<double2, Q, SG, 2 * SG>(win, s0, ns, stick_off, pw_stick, pw_z, x.ptr(vec), kin,
                                            y + (long)vec * ldy, scale);
}

template <class C2> const C2 *twiddles(const sgw_ham *h, int axis);
template <> const double2 *twiddles<double2>(const sgw_ham *h, int axis) { return h->d_tw + h->tw_off[axis]; }
template <> const float2 *twiddles<float2>(const sgw_ham *h, int axis) { return h->d_tw32 + h->tw_off[axis]; }
template <class C2> const typename CT<C2>::R *potential(const sgw_ham *h);
template <> const double *potential<double2>(const sgw_ham *h) { return h->d_vt; }
template <> const float *potential<float2>(const sgw_ham *h) { return h->d_vt32; }

template <class C2, int N2>
sgw_status launch_sticks(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, C2 *tbuf,
                         bool inverse) {
  constexpr int SG = sticks_per_block<N2>();
  const int groups = (h->n_stick + SG - 1) / SG;
  const long blocks = (long)groups * n_vec;
  const C2 *tw = twiddles<C2>(h, 2);
  const double n2 = N2, nst = h->n_stick, npw = h->n_pw, cb = sizeof(C2);
  PendingTiming tm;
  if constexpr (line_planes_fit<C2, N2, N2>()) {
    if (h->m2_lo >= -N2 / 4 && h->m2_hi < N2 / 4) {
      const int lg = (h->n_stick + kStickLineSticks - 1) / kStickLineSticks;
      if (inverse) {
        timing_begin(ctx, K_STICKS_INV, n_vec * (npw * 16.0 + n2 * nst * cb), 0.0, &tm);
        if (sizeof(C2) == 16) {
          const long items = (long)n_vec * h->n_stick;
          hipLaunchKernelGGL((k_sticks_inv_direct<C2, N2>), dim3((items + 255) / 256), dim3(256), 0, ctx->stream, x,
                             tbuf, h->n_stick, items, h->d_stick_off, h->d_pw_z);
        } else {
          hipLaunchKernelGGL((k_sticks_inv_line<C2, N2>), dim3((long)lg * n_vec), dim3(kStickLineSticks), 0,
                             ctx->stream, x, tbuf, h->n_stick, lg, h->d_stick_off, h->d_pw_stick, h->d_pw_z);
        }
      } else {
        const double scale = 1.0 / ((double)h->n[0] * h->n[1] * h->n[2]);
        timing_begin(ctx, K_STICKS_FWD, n_vec * (npw * 32.0 + n2 * nst * cb), 0.0, &tm);
        hipLaunchKernelGGL((k_sticks_fwd_line<C2, N2>), dim3((long)lg * n_vec), dim3(kStickLineSticks), 0, ctx->stream,
                           tbuf, h->n_stick, lg, h->d_stick_off, h->d_pw_stick, h->d_pw_z, x, h->d_kin, y, ldy,
                           scale);
      }
      timing_end(ctx, &tm);
      SGW_HIP(hipGetLastError());
      return SGW_OK;
    }
  }
  if constexpr (pair_planes_fit<C2, N2, N2>() && !line_planes_fit<C2, N2, N2>()) {
    if (h->m2_lo >= -N2 / 4 && h->m2_hi < N2 / 4) {
      const int lg = (h->n_stick + kStickLineSticks - 1) / kStickLineSticks;
      if (inverse) {
        timing_begin(ctx, K_STICKS_INV, n_vec * (npw * 16.0 + n2 * nst * cb), 0.0, &tm);
        hipLaunchKernelGGL((k_sticks_inv_pair<N2>), dim3((long)lg * n_vec), dim3(2 * kStickLineSticks), 0,
                           ctx->stream, x, (double2 *)tbuf, h->n_stick, lg, h->d_stick_off, h->d_pw_stick,
                           h->d_pw_z);
      } else {
        const double scale = 1.0 / ((double)h->n[0] * h->n[1] * h->n[2]);
        timing_begin(ctx, K_STICKS_FWD, n_vec * (npw * 32.0 + n2 * nst * cb), 0.0, &tm);
        hipLaunchKernelGGL((k_sticks_fwd_pair<N2>), dim3((long)lg * n_vec), dim3(2 * kStickLineSticks), 0,
                           ctx->stream, (const double2 *)tbuf, h->n_stick, lg, h->d_stick_off, h->d_pw_stick,
                           h->d_pw_z, x, h->d_kin, y, ldy, scale);
      }
      timing_end(ctx, &tm);
      SGW_HIP(hipGetLastError());
      return SGW_OK;
    }
  }
  if (inverse) {
    timing_begin(ctx, K_STICKS_INV, n_vec * (npw * 16.0 + n2 * nst * cb), 0.0, &tm);
    hipLaunchKernelGGL((k_sticks_inv<C2, N2>), dim3(blocks), dim3(kStickThreads), 0, ctx->stream, x, tbuf,
                       h->n_stick, h->d_stick_off, h->d_pw_stick, h->d_pw_z, tw, groups);
    timing_end(ctx, &tm);
  } else {
    const double scale = 1.0 / ((double)h->n[0] * h->n[1] * h->n[2]);
    timing_begin(ctx, K_STICKS_FWD, n_vec * (npw * 32.0 + n2 * nst * cb), 0.0, &tm);
    hipLaunchKernelGGL((k_sticks_fwd<C2, N2>), dim3(blocks), dim3(kStickThreads), 0, ctx->stream, tbuf,
                       h->n_stick, h->d_stick_off, h->d_pw_stick, h->d_pw_z, tw, groups, x, h->d_kin, y, ldy,
                       scale);
    timing_end(ctx, &tm);
  }
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

// The plane kernel of H.x for this grid and precision: the one the context asks for if it applies,
// else whole lines in registers, else two threads per line (FP64), else the whole plane in LDS.
// Lines in registers need every stick in the central half of the plane (a sphere that the grid
// holds twice over has them there).
template <class C2, int N0, int N1>
int plane_kernel(const sgw_ctx *ctx, const sgw_ham *h) {
  const bool win = line_window_ok(h->n, h->m0_lo, h->n_row, h->m1_lo, h->m1_hi);
  const bool line = win && line_planes_fit<C2, N0, N1>(), pair = win && pair_planes_fit<C2, N0, N1>();
  const bool tri = win && sizeof(C2) == 16 && tri_planes_fit<N0, N1>();
  const int want = ctx->fft_active ? ctx->fft_active : ctx->fft_planes;
  if (want == SGW_FFT_LINE && line) return SGW_FFT_LINE;
  if (want == SGW_FFT_PAIR && pair) return SGW_FFT_PAIR;
  if (want == SGW_FFT_TRI && tri) return SGW_FFT_TRI;
  if (want == SGW_FFT_LDS) return SGW_FFT_LDS;
  // built-in choice: the whole-line kernel where a line fits one thread, else the three-thread split
  // (24, 48, 72 points), else the two-thread one (64), else the whole plane in LDS
  return line ? SGW_FFT_LINE : tri ? SGW_FFT_TRI : pair ? SGW_FFT_PAIR : SGW_FFT_LDS;
}

template <class C2, int N0, int N1>
sgw_status launch_planes(sgw_ctx *ctx, const sgw_ham *h, int n_vec, C2 *tbuf) {
  const long blocks = (long)n_vec * h->n[2];
  PendingTiming tm;
  // algorithmic bytes: stick values in and out; the potential is read once per launch
  const double bytes = (double)n_vec * h->n[2] * h->n_stick * 2.0 * sizeof(C2) +
                       (double)N0 * N1 * h->n[2] * sizeof(typename CT<C2>::R);
  // algorithmic flops: 5 N log2 N per complex N-point transform (n_row rows and N1 columns, inverse
  // and forward) plus 2 per potential multiply, per plane
  const double per_plane = 2.0 * (h->n_row * 5.0 * N1 * std::log2((double)N1) + N1 * 5.0 * N0 * std::log2((double)N0)) +
                           2.0 * N0 * N1;
  timing_begin(ctx, K_PLANES, bytes, per_plane * h->n[2] * n_vec, &tm);
  const int use = plane_kernel<C2, N0, N1>(ctx, h);
  if constexpr (line_planes_fit<C2, N0, N1>()) {
    if (use == SGW_FFT_LINE) {
      constexpr int P = line_plane_count<C2, N1>();
      const long n_planes = (long)n_vec * h->n[2];
      hipLaunchKernelGGL((k_planes_line<C2, N0, N1, P>), dim3((n_planes + P - 1) / P),
                         dim3(line_plane_threads<P, N1>()), 0, ctx->stream, tbuf, n_planes, h->n[2], h->n_stick,
                         h->d_rows, h->d_stick_ij, h->m0_lo, h->n_row, potential<C2>(h));
    }
  }
  if constexpr (pair_planes_fit<C2, N0, N1>()) {
    if (use == SGW_FFT_PAIR)
      hipLaunchKernelGGL((k_planes_pair<N0, N1>), dim3(blocks), dim3(pair_plane_threads<N0, N1>()), 0, ctx->stream,
                         (double2 *)tbuf, h->n[2], h->n_stick, h->d_rows, h->d_stick_ij, h->m0_lo, h->n_row,
                         h->d_vt);
  }
  if constexpr (sizeof(C2) == 16 && tri_planes_fit<N0, N1>()) {
    if (use == SGW_FFT_TRI)
      hipLaunchKernelGGL((k_planes_tri<N0, N1>), dim3(blocks), dim3(tri_plane_threads<N0, N1>()), 0, ctx->stream,
                         (double2 *)tbuf, h->n[2], h->n_stick, h->d_rows, h->d_stick_ij, h->m0_lo, h->n_row,
                         h->d_vt);
  }
  if (use == SGW_FFT_LDS)
    hipLaunchKernelGGL((k_planes<C2, N0, N1>), dim3(blocks), dim3(plane_threads<N0, N1>()), 0, ctx->stream, tbuf,
                       h->n[2], h->n_stick, h->d_rows, h->m0_lo, h->n_row, potential<C2>(h), twiddles<C2>(h, 0),
                       twiddles<C2>(h, 1));
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

#define SGW_GRID_LIST(X) X(16) X(24) X(32) X(48) X(64) X(72)

template <class C2>
sgw_status dispatch_sticks(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, C2 *tbuf,
                           bool inverse) {
  switch (h->n[2]) {
#define SGW_CASE(N) \
  case N:           \
    return launch_sticks<C2, N>(ctx, h, n_vec, x, y, ldy, tbuf, inverse);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 2 not supported");
}

template <class C2, int N0>
sgw_status dispatch_planes_n1(sgw_ctx *ctx, const sgw_ham *h, int n_vec, C2 *tbuf) {
  switch (h->n[1]) {
#define SGW_CASE(N) \
  case N:           \
    return launch_planes<C2, N0, N>(ctx, h, n_vec, tbuf);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 1 not supported");
}

template <class C2>
sgw_status dispatch_planes(sgw_ctx *ctx, const sgw_ham *h, int n_vec, C2 *tbuf) {
  switch (h->n[0]) {
#define SGW_CASE(N) \
  case N:           \
    return dispatch_planes_n1<C2, N>(ctx, h, n_vec, tbuf);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return fail(SGW_ERR_UNSUPPORTED, "grid size along axis 0 not supported");
}

}  // namespace

template <class C2, int N0>
int plane_kernel_n1(const sgw_ctx *ctx, const sgw_ham *h) {
  switch (h->n[1]) {
#define SGW_CASE(N) \
  case N:           \
    return plane_kernel<C2, N0, N>(ctx, h);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return SGW_FFT_LDS;
}

int hx_plane_kernel(const sgw_ctx *ctx, const sgw_ham *h, bool fp32) {
  switch (h->n[0]) {
#define SGW_CASE(N) \
  case N:           \
    return fp32 ? plane_kernel_n1<float2, N>(ctx, h) : plane_kernel_n1<double2, N>(ctx, h);
    SGW_GRID_LIST(SGW_CASE)
#undef SGW_CASE
  }
  return SGW_FFT_LDS;
}

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

template <class C2>
sgw_status hx_run(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, C2 *tbuf) {
  sgw_status st = dispatch_sticks<C2>(ctx, h, n_vec, x, nullptr, 0, tbuf, true);
  if (st != SGW_OK) return st;
  st = dispatch_planes<C2>(ctx, h, n_vec, tbuf);
  if (st != SGW_OK) return st;
  return dispatch_sticks<C2>(ctx, h, n_vec, x, y, ldy, tbuf, false);
}

sgw_status hx_batch(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, void *tbuf,
                    bool fp32) {
  if (n_vec <= 0) return SGW_OK;
  const sgw_status st = fp32 ? hx_run<float2>(ctx, h, n_vec, x, y, ldy, (float2 *)tbuf)
                             : hx_run<double2>(ctx, h, n_vec, x, y, ldy, (double2 *)tbuf);
  if (st != SGW_OK || h->n_proj == 0) return st;
  // separable non-local term (Sec. 2.1, in reciprocal space): y += beta^T (E . (beta^H x)) on the
  // FP64 matrix cores; the stick buffer is free once the forward stick pass has run and takes the
  // overlaps
  double2 *cp = (double2 *)tbuf;
  const sgw_status s2 = proj_dot(ctx, h->n_pw, h->n_proj, h->d_beta, n_vec, x, cp, n_vec, K_NL_DOT);
  if (s2 != SGW_OK) return s2;
  return proj_apply(ctx, h->n_pw, h->n_proj, h->d_beta, n_vec, x, cp, n_vec, y, ldy, 1.0, 1, h->d_ekb, K_NL_APPLY);
}

}  // namespace sgw
