// Kernels of the multishift Sternheimer solver (Sec. 2.2-2.3).
//
// One (band v, perturbation p) pair owns a "slot": its right-hand side b, its
// Lanczos basis v_0..v_K of the seed operator A0 = H - eps_v + alpha P_occ,
// the tridiagonal coefficients, and per-shift recurrence state.  Every shift
// z_j = omega_j + i eta shares the basis: the FOM solution of the shifted
// system is x_j = V_K (T_K - z_j)^-1 ||b|| e_0, and its residual norm is
// ||b|| prod_i beta_{i+1} / |rho_i(z_j)|, where rho_i are the pivots of the
// LU factorisation of T_K - z_j.  The basis is kept in HBM, so no per-shift
// vector is updated during the iteration; x_j is formed once at the end.
#include "fft_lds.h"
#include "sgw_internal.h"
#include "solver_state.h"

namespace sgw {
namespace {

// deterministic block sum: wave butterfly (shuffle-xor) then a fixed-order
// sum over waves.  Every thread returns the total.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

// M simultaneous block sums; results in out[0..M) for every thread
template <int NT, int M>
__device__ __forceinline__ void block_sum_n(double *v, double *sh, double *out) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[m] += __shfl_xor(v[m], off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) sh[wid * M + m] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += sh[w * M + m];
    out[m] = r;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// permutation between the caller's order and the internal order
// ---------------------------------------------------------------------------
__global__ void k_permute(int npw, int n_vec, const double2 *__restrict__ in, long ldin, double2 *__restrict__ out,
                          long ldout, const int32_t *__restrict__ perm, int scatter, double scale, int tiles) {
  const int a = blockIdx.x / tiles;
  const int g = (blockIdx.x - a * tiles) * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  if (scatter) out[(long)a * ldout + perm[g]] = c_scale(in[(long)a * ldin + g], scale);
  else out[(long)a * ldout + g] = c_scale(in[(long)a * ldin + perm[g]], scale);
}

// y_a = x_a
__global__ void k_copy(int npw, VecSrc x, double2 *__restrict__ y, long ldy, int tiles) {
  const int a = blockIdx.x / tiles;
  const int g = (blockIdx.x - a * tiles) * blockDim.x + threadIdx.x;
  if (g < npw) y[(long)a * ldy + g] = x.ptr(a)[g];
}

// ---------------------------------------------------------------------------
// right-hand side source (Eq. 8): s(G'') = psi_v(G'' - G_p), zero outside the k sphere
// ---------------------------------------------------------------------------
__global__ void k_rhs_source(int npw, const int32_t *__restrict__ miller_int, const int32_t *__restrict__ box,
                             int3 box_lo, int3 box_dim, const int32_t *__restrict__ pairs, int n_pert,
                             const int32_t *__restrict__ dvm, const double2 *__restrict__ psi_v, long ld_psi,
                             double2 *__restrict__ s, long lds, int tiles) {
  const int a = blockIdx.x / tiles;
  const int g = (blockIdx.x - a * tiles) * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int pair = pairs[a];
  const int v = pair / n_pert, p = pair - v * n_pert;
  const int m0 = miller_int[3 * g] - dvm[3 * p] - box_lo.x;
  const int m1 = miller_int[3 * g + 1] - dvm[3 * p + 1] - box_lo.y;
  const int m2 = miller_int[3 * g + 2] - dvm[3 * p + 2] - box_lo.z;
  double2 val = make_double2(0.0, 0.0);
  if (m0 >= 0 && m0 < box_dim.x && m1 >= 0 && m1 < box_dim.y && m2 >= 0 && m2 < box_dim.z) {
    const int idx = box[(m0 * box_dim.y + m1) * box_dim.z + m2];
    if (idx >= 0) val = psi_v[(long)v * ld_psi + idx];
  }
  s[(long)a * lds + g] = val;
}

// ---------------------------------------------------------------------------
// slot initialisation: b = -(1 - P_occ) s, v_0 = b / ||b||
// ---------------------------------------------------------------------------
constexpr int kRowThreads = 256;

__global__ __launch_bounds__(kRowThreads) void k_init(SolverState S, const double2 *__restrict__ src,
                                                      const double2 *__restrict__ proj,
                                                      const int32_t *__restrict__ fill_slots,
                                                      const int32_t *__restrict__ fill_pairs) {
  __shared__ double sh[kRowThreads / 64];
  const int a = blockIdx.x;
  const int slot = fill_slots[a], pair = fill_pairs[a];
  const double2 *sv = src + (long)a * S.npw;   // s
  const double2 *pv = proj + (long)a * S.npw;  // (1 - P_occ) s
  double2 *bv = S.bvec + (long)slot * S.npw;
  double acc = 0.0, accs = 0.0;
  for (int g = threadIdx.x; g < S.npw; g += kRowThreads) {
    const double2 sg = sv[g];
    const double2 pg = pv[g];
    const double2 b = make_double2(-pg.x, -pg.y);
    bv[g] = b;
    acc += b.x * b.x + b.y * b.y;
    accs += sg.x * sg.x + sg.y * sg.y;
  }
  double nb = sqrt(block_sum<kRowThreads>(acc, sh));
  const double ns = sqrt(block_sum<kRowThreads>(accs, sh));
  // a source inside the occupied space leaves only cancellation noise: the
  // right-hand side is zero to working precision
  const bool zero = !(nb > kZeroRhsRel * ns);
  if (zero && isfinite(nb)) nb = 0.0;
  double2 *v0 = basis_vec(S, slot, 0);
  const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
  for (int g = threadIdx.x; g < S.npw; g += kRowThreads) {
    if (nb == 0.0) bv[g] = make_double2(0.0, 0.0);
    v0[g] = c_scale(bv[g], inv);
  }
  for (int j = threadIdx.x; j < S.n_omega; j += kRowThreads) {
    S.res[(long)slot * S.n_omega + j] = 1.0;
    S.conv[(long)slot * S.n_omega + j] = -1;
    S.rho[(long)slot * S.n_omega + j] = make_double2(1.0, 0.0);
  }
  if (threadIdx.x == 0) {
    const int v = pair / S.n_pert;
    S.pair[slot] = pair;
    S.kcur[slot] = 0;
    S.maxres[slot] = 1.0;
    S.eps[slot] = S.eps_band[v];
    S.beta[(long)slot * (S.kmax + 1)] = nb;
    int st = SLOT_RUNNING;
    if (!isfinite(nb)) st = SLOT_NONFINITE;
    else if (nb == 0.0) st = SLOT_ZERO_RHS;
    S.status[slot] = st;
  }
}

// ---------------------------------------------------------------------------
// one Lanczos step of the seed operator plus the shift recurrences
//   w = A0 v_k - beta_k v_{k-1};  a_k = <v_k, w>;  w -= a_k v_k;  beta_{k+1} = ||w||
//   A0 v_k = Y - eps_v v_k, where Y = H v_k + alpha P_occ v_k has been formed
//   by the H.x and projector kernels
// ---------------------------------------------------------------------------
// threads per vector: 256 up to 4096 plane waves (one round of workgroups for ~1000 vectors on
// 256 CUs at 16 values per thread), 512 up to 8192, 1024 up to 16384 (large bases run with fewer
// vectors per step than there are CUs, so each CU gets more waves in flight: 16 values per thread)
constexpr int kLzSmall = 256, kLzLarge = 512, kLzHuge = 1024;

template <int EPT, int kLzThreads>
__global__ __launch_bounds__(kLzThreads) void k_lanczos(SolverState S, const int32_t *__restrict__ list,
                                                        const double2 *__restrict__ Y) {
  __shared__ double sh[kLzThreads / 64];
  __shared__ int all_conv;
  const int a = blockIdx.x;
  const int slot = list[a];
  if (S.status[slot] != SLOT_RUNNING) return;
  const int k = S.kcur[slot];
  const int npw = S.npw;
  const double2 *v = basis_vec(S, slot, k);
  const double2 *vp = k > 0 ? basis_vec(S, slot, k - 1) : v;
  double2 *vn = basis_vec(S, slot, k + 1);
  const double2 *y = Y + (long)a * npw;
  const double eps = S.eps[slot];
  const double bk = k > 0 ? S.beta[(long)slot * (S.kmax + 1) + k] : 0.0;
  if (threadIdx.x == 0) all_conv = 1;
  __syncthreads();
  double2 w[EPT];
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int g = threadIdx.x + e * kLzThreads;
    if (g < npw) {
      const double2 vg = v[g];
      double2 t = y[g];
      t.x = fma(-eps, vg.x, t.x);
      t.y = fma(-eps, vg.y, t.y);
      if (k > 0) {
        const double2 pg = vp[g];
        t.x = fma(-bk, pg.x, t.x);
        t.y = fma(-bk, pg.y, t.y);
      }
      w[e] = t;
      acc = fma(vg.x, t.x, fma(vg.y, t.y, acc));
    }
  }
  const double ak = block_sum<kLzThreads>(acc, sh);
  double acc2 = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int g = threadIdx.x + e * kLzThreads;
    if (g < npw) {
      const double2 vg = v[g];
      w[e].x = fma(-ak, vg.x, w[e].x);
      w[e].y = fma(-ak, vg.y, w[e].y);
      acc2 = fma(w[e].x, w[e].x, fma(w[e].y, w[e].y, acc2));
    }
  }
  const double bn = sqrt(block_sum<kLzThreads>(acc2, sh));
  const double inv = bn > 0.0 ? 1.0 / bn : 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int g = threadIdx.x + e * kLzThreads;
    if (g < npw) vn[g] = c_scale(w[e], inv);
  }
  // shift recurrences: rho_k(z) = a_k - z - beta_k^2 / rho_{k-1}(z); res *= beta_{k+1} / |rho_k|
  double rmax = 0.0;
  for (int j = threadIdx.x; j < S.n_omega; j += kLzThreads) {
    const long idx = (long)slot * S.n_omega + j;
    double2 rho = make_double2(ak - S.omega[j], -(S.eta_j ? S.eta_j[j] : S.eta));
    if (k > 0) {
      const double2 rp = S.rho[idx];
      const double d = bk * bk / (rp.x * rp.x + rp.y * rp.y);
      rho.x -= d * rp.x;
      rho.y += d * rp.y;
    }
    S.rho[idx] = rho;
    const double r = S.res[idx] * bn / sqrt(rho.x * rho.x + rho.y * rho.y);
    S.res[idx] = r;
    rmax = fmax(rmax, isfinite(r) ? r : 1e300);
    if (!(r <= S.tol_int)) all_conv = 0;
    else if (S.conv[idx] < 0) S.conv[idx] = k + 1;
  }
  const double slot_max = block_max<kLzThreads>(rmax, sh);
  if (threadIdx.x == 0) {
    S.maxres[slot] = slot_max;
    S.alpha_t[(long)slot * S.kmax + k] = ak;
    S.beta[(long)slot * (S.kmax + 1) + k + 1] = bn;
    S.kcur[slot] = k + 1;
    int st = SLOT_RUNNING;
    if (!isfinite(ak) || !isfinite(bn)) st = SLOT_NONFINITE;
    else if (bn <= 1e-14 * (fabs(ak) + bk)) st = SLOT_BREAKDOWN;
    else if (all_conv) st = SLOT_CONVERGED;
    else if (k + 1 >= S.kmax) st = SLOT_MAXITER;
    S.status[slot] = st;
  }
}

// ---------------------------------------------------------------------------
// FOM coefficients per shift: (T_Kj - z_j) y = ||b|| e_0 (Thomas algorithm; the
// matrix is complex symmetric with a definite imaginary part, so elimination
// without pivoting is stable).  K_j is the Krylov dimension at which shift j's
// residual estimate met the stopping threshold (the pair's full dimension if it
// never did): the FOM iterate there is that shift's solution, and the larger
// spaces the pair's slower shifts needed are not used for it.  The kernel also
// ranks the pair's shifts by (K_j, j), so that the combination can group shifts
// of similar dimension.
// ---------------------------------------------------------------------------
constexpr int kTriBatch = 8;

// Krylov dimension of shift j's solution in slot `slot`
__device__ __forceinline__ int shift_dim(const SolverState &S, int slot, int j) {
  const int K = S.kcur[slot];
  const int c = S.conv[(long)slot * S.n_omega + j];
  return c >= 1 && c < K ? c : K;
}

__global__ void k_tridiag(SolverState S, const int32_t *__restrict__ flist, int nf, double2 *__restrict__ ycoef,
                          double2 *__restrict__ cp, int32_t *__restrict__ order) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf * S.n_omega) return;
  const int f = t / S.n_omega, j = t - f * S.n_omega;
  const int slot = flist[f];
  const int nw = S.n_omega;
  const int K = shift_dim(S, slot, j);
  {  // rank of shift j among the pair's shifts by (K_j, j)
    int rank = 0;
    for (int q = 0; q < nw; ++q) {
      const int kq = shift_dim(S, slot, q);
      rank += (kq < K || (kq == K && q < j)) ? 1 : 0;
    }
    order[(long)f * nw + rank] = j;
  }
  const long base = (long)f * S.kmax * nw + j;
  const double *al = S.alpha_t + (long)slot * S.kmax;
  const double *be = S.beta + (long)slot * (S.kmax + 1);
  const double zr = S.omega[j], zi = S.eta_j ? S.eta_j[j] : S.eta;
  double2 dprev = make_double2(0.0, 0.0), cprev = make_double2(0.0, 0.0);
  // the recurrence's inputs (alpha, beta) and, going back, its stored pivots are loaded kTriBatch
  // steps at a time, ahead of the dependent arithmetic
  for (int i0 = 0; i0 < K; i0 += kTriBatch) {
    double a_[kTriBatch], b_[kTriBatch], bn_[kTriBatch];
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u) {
      const int i = i0 + u;
      a_[u] = i < K ? al[i] : 0.0;
      b_[u] = i < K ? be[i] : 0.0;
      bn_[u] = i + 1 < K ? be[i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u) {
      const int i = i0 + u;
      if (i >= K) break;
      // den = (a_i - z) - beta_i * cp_{i-1}
      double2 den = make_double2(a_[u] - zr, -zi);
      double2 rhs = make_double2(i == 0 ? b_[u] : 0.0, 0.0);
      if (i > 0) {
        den.x -= b_[u] * cprev.x;
        den.y -= b_[u] * cprev.y;
        rhs.x -= b_[u] * dprev.x;
        rhs.y -= b_[u] * dprev.y;
      }
      const double dn = 1.0 / (den.x * den.x + den.y * den.y);
      const double2 iden = make_double2(den.x * dn, -den.y * dn);
      cprev = c_scale(iden, bn_[u]);
      dprev = c_mul(rhs, iden);
      cp[base + (long)i * nw] = cprev;
      ycoef[base + (long)i * nw] = dprev;
    }
  }
  double2 ynext = make_double2(0.0, 0.0);
  for (int i1 = K - 1; i1 >= 0; i1 -= kTriBatch) {
    double2 d_[kTriBatch], c_[kTriBatch];
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u) {
      const int i = i1 - u;
      d_[u] = i >= 0 ? ycoef[base + (long)i * nw] : make_double2(0.0, 0.0);
      c_[u] = i >= 0 ? cp[base + (long)i * nw] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u) {
      const int i = i1 - u;
      if (i < 0) break;
      const double2 yi = c_sub(d_[u], c_mul(c_[u], ynext));
      ycoef[base + (long)i * nw] = yi;
      ynext = yi;
    }
  }
}

// ---------------------------------------------------------------------------
// x_j = sum_k ycoef[k][j] v_k  for every shift j of a slot
// ---------------------------------------------------------------------------
constexpr int kCmbThreads = 256;
constexpr int kCmbK = 32;
constexpr int kCmbU = 8;  // basis values loaded ahead (divides kCmbK)
// workgroups are dealt round-robin to the GPU's 8 XCDs (each with its own L2)
constexpr int kXcds = 8;

// One workgroup per (slot, tile of 256 plane waves, chunk of kCmbJ shifts; kCmbJ is 16 or 20,
// whichever pads the shift count less, so 64 and 100 shifts split without a ragged chunk).  A
// chunk holds kCmbJ consecutive shifts of the pair's order by Krylov dimension (k_tridiag), so it
// runs only to the largest dimension among its own shifts.  The chunks of a tile read the same
// basis vectors; workgroup ids are arranged so that they run on one XCD (ids spaced by kXcds,
// dispatched close together) and share that XCD's L2 copy of the tile.
template <int kCmbJ>
__global__ __launch_bounds__(kCmbThreads) void k_combine(SolverState S, const int32_t *__restrict__ flist,
                                                         const double2 *__restrict__ ycoef,
                                                         const int32_t *__restrict__ order,
                                                         double2 *__restrict__ X, int gtiles, int jchunks,
                                                         int ntiles) {
  __shared__ double2 yt[kCmbK][kCmbJ];
  __shared__ int sj[kCmbJ], sk[kCmbJ];
  int b = blockIdx.x;
  const int xcd = b % kXcds;
  b /= kXcds;
  const int jc = b % jchunks;
  const int tile = (b / jchunks) * kXcds + xcd;
  if (tile >= ntiles) return;
  const int gt = tile % gtiles;
  const int f = tile / gtiles;
  const int slot = flist[f];
  const int nw = S.n_omega;
  const int j0 = jc * kCmbJ;
  if (threadIdx.x < kCmbJ) {
    const int jj = j0 + threadIdx.x;
    const int j = jj < nw ? order[(long)f * nw + jj] : -1;
    sj[threadIdx.x] = j;
    sk[threadIdx.x] = j >= 0 ? shift_dim(S, slot, j) : 0;
  }
  __syncthreads();
  int K = 0;  // the chunk's largest Krylov dimension
#pragma unroll
  for (int q = 0; q < kCmbJ; ++q) K = max(K, sk[q]);
  const int g = gt * kCmbThreads + threadIdx.x;
  double2 acc[kCmbJ];
#pragma unroll
  for (int q = 0; q < kCmbJ; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += kCmbK) {
    for (int i = threadIdx.x; i < kCmbK * kCmbJ; i += kCmbThreads) {
      const int kk = i / kCmbJ, q = i - kk * kCmbJ;
      const int k = k0 + kk, j = sj[q];
      // coefficients past a shift's own dimension are zero
      yt[kk][q] = (k < sk[q] && j >= 0) ? ycoef[((long)f * S.kmax + k) * nw + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (g < S.npw) {
      const int kend = min(kCmbK, K - k0);
      // kCmbU basis values are loaded before any is used; past kend they are 0 (and so are their
      // coefficients in yt), which leaves acc unchanged
      for (int kb = 0; kb < kend; kb += kCmbU) {
        double2 vk[kCmbU];
#pragma unroll
        for (int u = 0; u < kCmbU; ++u)
          vk[u] = kb + u < kend ? basis_vec(S, slot, k0 + kb + u)[g] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < kCmbU; ++u) {
#pragma unroll
          for (int q = 0; q < kCmbJ; ++q) {
            const double2 yc = yt[kb + u][q];
            acc[q].x = fma(yc.x, vk[u].x, fma(-yc.y, vk[u].y, acc[q].x));
            acc[q].y = fma(yc.x, vk[u].y, fma(yc.y, vk[u].x, acc[q].y));
          }
        }
      }
    }
    __syncthreads();
  }
  if (g < S.npw) {
#pragma unroll
    for (int q = 0; q < kCmbJ; ++q) {
      const int j = sj[q];
      if (j >= 0) X[((long)f * nw + j) * S.npw + g] = acc[q];
    }
  }
}

constexpr int kResBatch = 4;

// ---------------------------------------------------------------------------
// true FP64 residual r = b - (A0 - z_j) x_j with A0 x_j applied afresh; writes
// dpsi (caller order) and the per-solve info
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRowThreads) void k_residual(SolverState S, const int32_t *__restrict__ flist,
                                                          const double2 *__restrict__ X,
                                                          const double2 *__restrict__ AX,
                                                          const double2 *__restrict__ cp,
                                                          const int32_t *__restrict__ u2i,
                                                          double2 *__restrict__ dpsi,
                                                          sgw_solve_info *__restrict__ info, double tol,
                                                          int *__restrict__ n_bad) {
  __shared__ double sh[(kRowThreads / 64) * 3];
  const int fj = blockIdx.x;
  const int f = fj / S.n_omega, j = fj - f * S.n_omega;
  const int slot = flist[f];
  const int pair = S.pair[slot];
  const int npw = S.npw;
  const double2 *x = X + (long)fj * npw;
  const double2 *ax = AX + (long)fj * npw;  // H x + alpha P_occ x
  const double2 *b = S.bvec + (long)slot * npw;
  const double eps = S.eps[slot];
  const double zr = S.omega[j], zi = S.eta_j ? S.eta_j[j] : S.eta;
  double2 *out = dpsi + ((long)pair * S.n_omega + j) * npw;
  double acc[3] = {0.0, 0.0, 0.0};
  const double er = eps + zr;
  // kResBatch plane waves per thread at a time, their loads issued before any is used
  for (int gb = threadIdx.x; gb < npw; gb += kResBatch * kRowThreads) {
    double2 xg[kResBatch], ag[kResBatch], bg[kResBatch];
#pragma unroll
    for (int u = 0; u < kResBatch; ++u) {
      const int g = gb + u * kRowThreads;
      const bool ok = g < npw;
      xg[u] = ok ? x[g] : make_double2(0.0, 0.0);
      ag[u] = ok ? ax[g] : make_double2(0.0, 0.0);
      bg[u] = ok ? b[g] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kResBatch; ++u) {
      // (A0 - z) x = (H + alpha P_occ) x - (eps + z) x   (all zero past npw)
      double2 ox;
      ox.x = ag[u].x - (er * xg[u].x - zi * xg[u].y);
      ox.y = ag[u].y - (er * xg[u].y + zi * xg[u].x);
      const double2 r = c_sub(bg[u], ox);
      acc[0] = fma(r.x, r.x, fma(r.y, r.y, acc[0]));
      acc[1] = fma(xg[u].x, xg[u].x, fma(xg[u].y, xg[u].y, acc[1]));
    }
  }
  // the solution in the caller's order: coalesced writes, gathered reads (x was just written)
  for (int ub = threadIdx.x; ub < npw; ub += kResBatch * kRowThreads) {
    double2 xv[kResBatch];
#pragma unroll
    for (int u = 0; u < kResBatch; ++u) {
      const int c = ub + u * kRowThreads;
      xv[u] = c < npw ? x[u2i[c]] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kResBatch; ++u)
      if (ub + u * kRowThreads < npw) out[ub + u * kRowThreads] = xv[u];
  }
  // ||psi^* x||^2 from the overlaps
  double cc = 0.0;
  for (int i = threadIdx.x; i < S.n_occ; i += kRowThreads) {
    const double2 c = cp[(long)fj * S.n_occ + i];
    cc += c.x * c.x + c.y * c.y;
  }
  acc[2] = cc;
  double tot[3];
  block_sum_n<kRowThreads, 3>(acc, sh, tot);
  if (threadIdx.x == 0) {
    const double nb = S.beta[(long)slot * (S.kmax + 1)];
    const double rn = sqrt(tot[0]);
    const double relres = nb > 0.0 ? rn / nb : rn;
    const int st = S.status[slot];
    int flags = 0;
    if (st == SLOT_MAXITER) flags |= SGW_FLAG_MAXITER;
    if (st == SLOT_BREAKDOWN) flags |= SGW_FLAG_BREAKDOWN;
    if (st == SLOT_NONFINITE || !isfinite(relres)) flags |= SGW_FLAG_NONFINITE;
    if (st == SLOT_ZERO_RHS) flags |= SGW_FLAG_ZERO_RHS;
    if (relres <= tol && !(flags & SGW_FLAG_NONFINITE)) flags |= SGW_FLAG_CONVERGED;
    else atomicAdd(n_bad, 1);
    sgw_solve_info inf;
    const int cj = S.conv[(long)slot * S.n_omega + j];
    inf.iters = cj >= 0 ? cj : S.kcur[slot];
    inf.flags = flags;
    inf.relres = relres;
    inf.occ_leak = tot[1] > 0.0 ? sqrt(tot[2] / tot[1]) : 0.0;
    info[(long)pair * S.n_omega + j] = inf;
  }
}

// out[a] = e_{cols[a]} (caller's order): the sources of Green's function columns
__global__ void k_unit_columns(int npw, const int32_t *__restrict__ cols, double2 *__restrict__ out, int tiles) {
  const int a = blockIdx.x / tiles;
  const int g = (blockIdx.x - a * tiles) * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  out[(long)a * npw + g] = make_double2(g == cols[a] ? 1.0 : 0.0, 0.0);
}

__global__ void k_transpose_potential(const double *__restrict__ v, double *__restrict__ vt,
                                      float *__restrict__ vt32, int n0, int n1, int n2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)n0 * n1 * n2;
  if (i >= n) return;
  // i indexes vt[i2][i0][i1]
  const int i1 = i % n1;
  const int i0 = (i / n1) % n0;
  const int i2 = i / ((long)n0 * n1);
  const double x = v[((long)i0 * n1 + i1) * n2 + i2];
  vt[i] = x;
  vt32[i] = (float)x;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
sgw_status permute(sgw_ctx *ctx, int npw, int n_vec, const double2 *in, long ldin, double2 *out, long ldout,
                   const int32_t *perm, int scatter, double scale) {
  if (n_vec <= 0) return SGW_OK;
  const int tiles = (npw + 255) / 256;
  PendingTiming tm;
  timing_begin(ctx, K_PERMUTE, n_vec * (npw * 36.0), 0.0, &tm);
  hipLaunchKernelGGL(k_permute, dim3((long)tiles * n_vec), dim3(256), 0, ctx->stream, npw, n_vec, in, ldin, out,
                     ldout, perm, scatter, scale, tiles);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status permute_copy(sgw_ctx *ctx, int npw, int n_vec, VecSrc x, double2 *y, long ldy) {
  if (n_vec <= 0) return SGW_OK;
  const int tiles = (npw + 255) / 256;
  hipLaunchKernelGGL(k_copy, dim3((long)tiles * n_vec), dim3(256), 0, ctx->stream, npw, x, y, ldy, tiles);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status rhs_source(sgw_ctx *ctx, const sgw_ham *h_kq, const sgw_ham *h_k, int n_vec, const int32_t *pairs,
                      int n_pert, const int32_t *dvm, const double2 *psi_v, long ld_psi, double2 *s, long lds) {
  if (n_vec <= 0) return SGW_OK;
  const int npw = h_kq->n_pw;
  const int tiles = (npw + 255) / 256;
  PendingTiming tm;
  timing_begin(ctx, K_RHS, n_vec * (npw * 32.0), 0.0, &tm);
  hipLaunchKernelGGL(k_rhs_source, dim3((long)tiles * n_vec), dim3(256), 0, ctx->stream, npw, h_kq->d_miller_int,
                     h_k->d_box, make_int3(h_k->box_lo[0], h_k->box_lo[1], h_k->box_lo[2]),
                     make_int3(h_k->box_dim[0], h_k->box_dim[1], h_k->box_dim[2]), pairs, n_pert, dvm, psi_v,
                     ld_psi, s, lds, tiles);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status slot_init(sgw_ctx *ctx, const SolverState &S, int n_fill, const double2 *src, const double2 *proj,
                     const int32_t *fill_slots, const int32_t *fill_pairs) {
  if (n_fill <= 0) return SGW_OK;
  PendingTiming tm;
  timing_begin(ctx, K_INIT, n_fill * (S.npw * 64.0), 0.0, &tm);
  hipLaunchKernelGGL(k_init, dim3(n_fill), dim3(kRowThreads), 0, ctx->stream, S, src, proj, fill_slots, fill_pairs);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

static int lanczos_threads(int npw) {
  return npw <= 16 * kLzSmall ? kLzSmall : npw <= 16 * kLzLarge ? kLzLarge : kLzHuge;
}

static int lanczos_ept(int npw) {
  const int nt = lanczos_threads(npw);
  int e = 1;
  while (e * nt < npw) e *= 2;
  return e;
}

sgw_status lanczos_step(sgw_ctx *ctx, const SolverState &S, int n_active, const int32_t *list, const double2 *Y) {
  if (n_active <= 0) return SGW_OK;
  if (S.npw > 16 * kLzHuge) return fail(SGW_ERR_UNSUPPORTED, "too many plane waves for the Lanczos kernel");
  const int ept = lanczos_ept(S.npw);
  const int nt = lanczos_threads(S.npw);
  PendingTiming tm;
  timing_begin(ctx, K_LANCZOS, n_active * (S.npw * 16.0 * 4), 0.0, &tm);
  switch (ept) {
#define SGW_LZ(E)                                                                                          \
  case E:                                                                                                  \
    if (nt == kLzSmall)                                                                                    \
      hipLaunchKernelGGL((k_lanczos<E, kLzSmall>), dim3(n_active), dim3(kLzSmall), 0, ctx->stream, S, list, \
                         Y);                                                                               \
    else if (nt == kLzLarge)                                                                               \
      hipLaunchKernelGGL((k_lanczos<E, kLzLarge>), dim3(n_active), dim3(kLzLarge), 0, ctx->stream, S, list, \
                         Y);                                                                               \
    else                                                                                                   \
      hipLaunchKernelGGL((k_lanczos<E, kLzHuge>), dim3(n_active), dim3(kLzHuge), 0, ctx->stream, S, list,   \
                         Y);                                                                               \
    break;
    SGW_LZ(1) SGW_LZ(2) SGW_LZ(4) SGW_LZ(8) SGW_LZ(16)
#undef SGW_LZ
    default:
      return fail(SGW_ERR_UNSUPPORTED, "too many plane waves for the Lanczos kernel");
  }
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status tridiag(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, double2 *ycoef, double2 *cp,
                   int32_t *order) {
  if (nf <= 0) return SGW_OK;
  const int n = nf * S.n_omega;
  PendingTiming tm;
  timing_begin(ctx, K_TRIDIAG, 0.0, 0.0, &tm);
  hipLaunchKernelGGL(k_tridiag, dim3((n + 63) / 64), dim3(64), 0, ctx->stream, S, flist, nf, ycoef, cp, order);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status combine(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, const double2 *ycoef,
                   const int32_t *order, double2 *X, double est_kavg, double est_kshift) {
  if (nf <= 0) return SGW_OK;
  const int gtiles = (S.npw + kCmbThreads - 1) / kCmbThreads;
  const int nw = S.n_omega;
  const bool j20 = (nw + 19) / 20 * 20 < (nw + 15) / 16 * 16;
  const int cj = j20 ? 20 : 16;
  const int jchunks = (nw + cj - 1) / cj;
  PendingTiming tm;
  const double bytes = nf * (est_kavg * S.npw * 16.0 + (double)S.n_omega * S.npw * 16.0);
  timing_begin(ctx, K_COMBINE, bytes, 8.0 * nf * est_kshift * S.npw * S.n_omega, &tm);
  const int ntiles = nf * gtiles;
  const long groups = (long)(ntiles + kXcds - 1) / kXcds * kXcds * jchunks;
  if (j20)
    hipLaunchKernelGGL(k_combine<20>, dim3(groups), dim3(kCmbThreads), 0, ctx->stream, S, flist, ycoef, order, X,
                       gtiles, jchunks, ntiles);
  else
    hipLaunchKernelGGL(k_combine<16>, dim3(groups), dim3(kCmbThreads), 0, ctx->stream, S, flist, ycoef, order, X,
                       gtiles, jchunks, ntiles);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status residual(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, const double2 *X,
                    const double2 *AX, const double2 *cp, long rows, const int32_t *u2i, double2 *dpsi,
                    sgw_solve_info *info, double tol, int *n_bad) {
  if (nf <= 0) return SGW_OK;
  PendingTiming tm;
  timing_begin(ctx, K_RESIDUAL, (double)nf * S.n_omega * S.npw * 16.0 * 4, 0.0, &tm);
  hipLaunchKernelGGL(k_residual, dim3((long)nf * S.n_omega), dim3(kRowThreads), 0, ctx->stream, S, flist, X, AX, cp,
                     u2i, dpsi, info, tol, n_bad);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status unit_columns(sgw_ctx *ctx, int npw, int n_col, const int32_t *cols, double2 *out) {
  if (n_col <= 0) return SGW_OK;
  const int tiles = (npw + 255) / 256;
  hipLaunchKernelGGL(k_unit_columns, dim3((long)tiles * n_col), dim3(256), 0, ctx->stream, npw, cols, out, tiles);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status transpose_potential(sgw_ctx *ctx, const double *v, double *vt, float *vt32, const int n[3]) {
  const long tot = (long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_transpose_potential, dim3((tot + 255) / 256), dim3(256), 0, ctx->stream, v, vt, vt32, n[0],
                     n[1], n[2]);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

}  // namespace sgw
