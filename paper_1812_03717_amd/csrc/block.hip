// Block multishift solver (SGW_SOLVER_BLOCK): one block Krylov space per band over all its
// perturbations (Sec. 2.3, Eqs. 6-8; the shifted systems of Sec. 2.2).
//
// The perturbations p of band v share the operator A_v = H - eps_v + alpha P_occ, so the block Krylov
// space K_k(A_v, [b_1 .. b_s]) serves every right-hand side, and, being shift invariant, every
// frequency z_j.  Block Lanczos (three-term block recurrence, no reorthogonalisation):
//     V_0 R_0 = B,   A_j = V_j^H A_v V_j,   W = A_v V_j - V_{j-1} B_j^H - V_j A_j,   V_{j+1} B_{j+1} = W,
// the orthonormalisations by Cholesky QR done twice.  With T_k the Hermitian block tridiagonal matrix
// (diagonal A_j, sub-diagonal B_{j+1}), the FOM solution of shift z is X(z) = V Y(z) with
// (T_k - z) Y(z) = E_0 R_0, and its residual is V_k B_k (last block of Y(z)).  The last block follows
// from a forward block recurrence per shift, D_j = A_j - z - B_j D_{j-1}^-1 B_j^H, F_j = -B_j
// D_{j-1}^-1 F_{j-1}, Y_last = D_j^-1 F_j, so the residual estimates cost s x s work per step and
// shift; a shift stops at the step where its estimate meets the threshold.  At the end the block
// tridiagonal systems are solved per shift (block Thomas) over each shift's own step count, and
// X = V Y, (H + alpha P) X = (AV) Y and Psi^H X = (Psi^H V) Y come out of batched products, AV and
// Psi^H V being kept from the recurrence; the true FP64 residual of every solution decides, as in the
// other solvers.
//
// H.x and the occupied projector are the library's kernels; the s x s Gram products, the thin
// n_pw x s combinations, the Cholesky factors and the shift recurrences are kernels here; the final
// products are rocBLAS zgemm (plain library products on the FP64 matrix cores).  Blocks hold at most
// kBlockMaxPert perturbations.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fft_lds.h"
#include "sgw_internal.h"
#include "solver_state.h"

namespace sgw {
namespace {

constexpr size_t kBA = 256;
constexpr int kGramRows = 256;  // plane waves per partial sum of the skinny products
constexpr int kGramTile = 32;   // rows staged in LDS at a time
constexpr int kRunShifts = 32;  // shifts whose solutions are formed together at the end
constexpr int kSubBands = 8;    // bands whose solutions share one shift order and step counts
size_t up(size_t b) { return (b + kBA - 1) / kBA * kBA; }

// Workspace of one chunk of nbc bands; kb = block steps + 1 stored blocks
struct BlkLayout {
  int nbc = 0, kb = 0, s = 0, run = 0;
  size_t basis, abasis, pov, rhs, y, w, v2, gram, coef, part, rfac, rinv, ablk, bblk, r0, bnorm, res, thomas,
      ycat, xg, axg, qg, list, c, t, psi, omega, eps, conv, ord, dvm, bstep, kband, bad, total;
};

BlkLayout blk_layout(const sgw_ham *h, int n_occ, int nbc, int s, int n_omega, int kb) {
  BlkLayout L;
  L.nbc = nbc;
  L.kb = kb;
  L.s = s;
  const size_t npw = h->n_pw, nv = (size_t)nbc * s, ss = (size_t)s * s;
  L.run = std::min(n_omega, kRunShifts);
  const size_t no = std::max(n_occ, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += up(bytes);
    return o;
  };
  L.basis = take(16 * (size_t)kb * nv * npw);
  L.abasis = take(16 * (size_t)kb * nv * npw);
  L.pov = take(16 * (size_t)kb * nv * no);
  L.rhs = take(16 * nv * npw);
  L.y = take(16 * nv * npw);
  L.w = take(16 * nv * npw);
  L.v2 = take(16 * nv * npw);
  L.gram = take(16 * nbc * ss);
  L.coef = take(16 * 2 * (size_t)nbc * ss);
  L.part = take(16 * (size_t)((npw + kGramRows - 1) / kGramRows) * nbc * ss);
  L.rfac = take(16 * nbc * ss);
  L.rinv = take(16 * nbc * ss);
  L.ablk = take(16 * (size_t)kb * nbc * ss);
  L.bblk = take(16 * (size_t)(kb + 1) * nbc * ss);
  L.r0 = take(16 * nbc * ss);
  L.bnorm = take(8 * nv);
  L.res = take(8 * (size_t)nbc * n_omega);
  L.thomas = take(16 * 2 * (size_t)kb * nbc * n_omega * ss);
  L.ycat = take(16 * (size_t)kb * s * nv * n_omega);
  const size_t nvg = (size_t)std::min(nbc, kSubBands) * s;  // vectors of one group of bands
  L.xg = take(16 * nvg * L.run * npw);
  L.axg = take(16 * nvg * L.run * npw);
  L.qg = take(16 * nvg * L.run * no);
  L.list = take(4 * nv);
  L.c = take(16 * kProjChunks * nv * no);
  L.t = take(hx_tbuf_bytes(h, nv));
  L.psi = take(16 * (size_t)std::max(n_occ, 1) * npw);
  L.omega = take(16 * (size_t)n_omega);
  L.eps = take(8 * (size_t)nbc);
  L.conv = take(4 * (size_t)nbc * n_omega);
  L.ord = take(8 * (size_t)nbc * n_omega);
  L.dvm = take(4 * 3 * (size_t)s);
  L.bstep = take(4 * (size_t)nbc);
  L.kband = take(4 * (size_t)nbc);
  L.bad = take(8);
  L.total = off;
  return L;
}

// block steps allowed: max_iter, the limit on the operator applications to each right-hand side
int blk_steps(const sgw_opts &o) { return std::max(1, o.max_iter); }

// bands per chunk: the largest count (at most `cap` when cap > 0) whose layout fits `budget` (at least
// one), then evened out over the chunks that n_band needs
int blk_chunk(const sgw_ham *h, int n_occ, int n_band, int s, int n_omega, int kb, double budget, int cap) {
  int lo = 1, hi = cap > 0 ? std::min(cap, n_band) : n_band;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if ((double)blk_layout(h, n_occ, mid, s, n_omega, kb).total <= budget) lo = mid;
    else hi = mid - 1;
  }
  const int n_chunks = (n_band + lo - 1) / lo;
  return (n_band + n_chunks - 1) / n_chunks;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// list[b s + c] = index of vector c of band b's block j in the basis [b][kb][s][npw]
__global__ void k_blk_list(int32_t *list, int nbc, int s, int kb, int j) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nbc * s) return;
  const int b = a / s, c = a - b * s;
  list[a] = (b * kb + j) * s + c;
}

// Skinny products C_b = A_b^H B_b (s x s, column-major) of every band's n_pw x s blocks, in two
// deterministic passes: partial sums over chunks of kGramRows plane waves (one workgroup per chunk and
// band, rows staged through LDS with coalesced column loads), then the chunks summed in order.

__global__ __launch_bounds__(256) void k_blk_gram(int npw, int s, const double2 *__restrict__ A, long sa,
                                                  const double2 *__restrict__ B, long sb, double2 *__restrict__ part) {
  __shared__ double2 As[kGramTile][kBlockMaxPert + 1], Bs[kGramTile][kBlockMaxPert + 1];
  const int chunk = blockIdx.x, b = blockIdx.y, nb = gridDim.y;
  const double2 *a = A + (long)b * sa, *bb = B + (long)b * sb;
  const bool same = a == bb;  // a Gram matrix A^H A: one tile serves both sides
  const int t = threadIdx.x;
  double2 acc[4];
  for (int r = 0; r < 4; ++r) acc[r] = make_double2(0.0, 0.0);
  const int g_end = min(npw, (chunk + 1) * kGramRows);
  // the next tile's elements (at most kGramTile kBlockMaxPert / 256 = 4 per thread) are loaded into
  // registers while the current tile is multiplied
  static_assert(kGramTile * kBlockMaxPert <= 4 * 256, "four staged elements per thread");
  double2 pa[4], pb[4];
  auto fetch = [&](int g0) {
    const int rows = min(kGramTile, g_end - g0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, r = e % kGramTile, c = e / kGramTile;
      const bool in = c < s && r < rows;
      pa[q] = in ? a[(long)c * npw + g0 + r] : make_double2(0.0, 0.0);
      if (!same) pb[q] = in ? bb[(long)c * npw + g0 + r] : make_double2(0.0, 0.0);
    }
  };
  fetch(chunk * kGramRows);
  for (int g0 = chunk * kGramRows; g0 < g_end; g0 += kGramTile) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, r = e % kGramTile, c = e / kGramTile;
      if (c < s) {
        As[r][c] = pa[q];
        if (!same) Bs[r][c] = pb[q];
      }
    }
    __syncthreads();
    if (g0 + kGramTile < g_end) fetch(g0 + kGramTile);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      if (e < s * s) {
        const int i = e % s, j = e / s;
        double2 v = acc[q];
        for (int r = 0; r < kGramTile; ++r) {
          const double2 x = As[r][i], y = same ? As[r][j] : Bs[r][j];
          v.x += x.x * y.x + x.y * y.y;
          v.y += x.x * y.y - x.y * y.x;
        }
        acc[q] = v;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + 256 * q;
    if (e < s * s) part[((long)chunk * nb + b) * s * s + e] = acc[q];
  }
}

__global__ void k_blk_gram_sum(int n_chunks, int nb, int ss, const double2 *__restrict__ part, double2 *__restrict__ c) {
  const int b = blockIdx.x;
  for (int e = threadIdx.x; e < ss; e += blockDim.x) {
    double2 v[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                    make_double2(0.0, 0.0)};
    int k = 0;
    for (; k + 4 <= n_chunks; k += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = c_add(v[q], part[((long)(k + q) * nb + b) * ss + e]);
    for (; k < n_chunks; ++k) v[0] = c_add(v[0], part[((long)k * nb + b) * ss + e]);
    c[(long)b * ss + e] = c_add(c_add(v[0], v[1]), c_add(v[2], v[3]));
  }
}

// Thin combinations out_b = sgn src_b coef_b (+ base_b) for every band b (blockIdx.y): src_b is n_pw x K
// (K <= 2 s, columns n_pw apart), coef_b K x s column-major (band stride K s, staged in LDS), one plane
// wave per thread with its SM >= s outputs in registers; copy (may be NULL) receives base_b too.
template <int SM>
__global__ __launch_bounds__(256) void k_blk_comb(int npw, int s, int K, const double2 *__restrict__ src, long ssrc,
                                                  const double2 *__restrict__ coef, double sgn,
                                                  const double2 *__restrict__ base, long sbase,
                                                  double2 *__restrict__ out, long sout, double2 *__restrict__ copy,
                                                  long scopy) {
  __shared__ double2 Cs[2 * kBlockMaxPert][SM];
  const int b = blockIdx.y;
  const double2 *cb = coef + (long)b * K * s;
  for (int e = threadIdx.x; e < K * s; e += 256) Cs[e % K][e / K] = cb[e];
  __syncthreads();
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= npw) return;
  double2 acc[SM];
#pragma unroll
  for (int c = 0; c < SM; ++c) acc[c] = make_double2(0.0, 0.0);
  const double2 *sb = src + (long)b * ssrc + g;
  for (int l = 0; l < K; ++l) {
    const double2 x = sb[(long)l * npw];
#pragma unroll
    for (int c = 0; c < SM; ++c) {
      if (c < s) {
        const double2 m = Cs[l][c];
        acc[c].x += x.x * m.x - x.y * m.y;
        acc[c].y += x.x * m.y + x.y * m.x;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < SM; ++c) {
    if (c < s) {
      double2 v = make_double2(sgn * acc[c].x, sgn * acc[c].y);
      if (base) {
        const double2 y = base[(long)b * sbase + (long)c * npw + g];
        v = c_add(v, y);
        if (copy) copy[(long)b * scopy + (long)c * npw + g] = y;
      }
      out[(long)b * sout + (long)c * npw + g] = v;
    }
  }
}

// Per band: A_j = (G + G^H)/2 - eps I into ablk, and the coefficients of W = Y - [V_{j-1} V_j] coef,
// coef = [B_j^H ; (G + G^H)/2] (2s x s, column-major; j = 0: the lower block alone, s x s)
__global__ void k_blk_coef(int s, int j, const double2 *__restrict__ g, const double2 *__restrict__ bj,
                           const double *__restrict__ eps, double2 *__restrict__ aj, double2 *__restrict__ coef) {
  const int b = blockIdx.x;
  const long ss = (long)s * s;
  const int K = j > 0 ? 2 * s : s, off = j > 0 ? s : 0;
  const double2 *gb = g + b * ss;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    const int r = e % s, c = e / s;
    const double2 x = gb[r + c * s], y = gb[c + r * s];
    const double2 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    aj[b * ss + e] = r == c ? make_double2(h.x - eps[b], 0.0) : h;
    coef[(long)b * K * s + off + r + (long)c * K] = r == c ? make_double2(h.x, 0.0) : h;
    if (j > 0) {
      const double2 t = bj[b * ss + c + r * s];  // (B_j^H)[r][c] = conj(B_j[c][r])
      coef[(long)b * K * s + r + (long)c * K] = make_double2(t.x, -t.y);
    }
  }
}

// Cholesky G = R^H R (R upper) of each band's Gram matrix, R^-1, and rout = R rprev (or R); a pivot
// below 1e-26 of the largest diagonal entry (a block that lost rank) lowers bstep[band] to `step`, the
// index of the basis block being formed
__global__ __launch_bounds__(64) void k_blk_chol(const double2 *__restrict__ gram, const double2 *__restrict__ rprev,
                                                 double2 *__restrict__ rout, double2 *__restrict__ rinv, int s,
                                                 int *bstep, int step) {
  __shared__ double2 R[kBlockMaxPert][kBlockMaxPert + 1];
  __shared__ double2 Ri[kBlockMaxPert][kBlockMaxPert + 1];
  __shared__ int fail;
  const long base = (long)blockIdx.x * s * s;
  const int t = threadIdx.x;
  if (t == 0) fail = 0;
  for (int e = t; e < s * s; e += blockDim.x) {
    const int i = e % s, j = e / s;
    R[i][j] = i <= j ? gram[base + e] : make_double2(0.0, 0.0);
    Ri[i][j] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  double gmax = 0.0;
  for (int i = 0; i < s; ++i) gmax = fmax(gmax, R[i][i].x);
  for (int k = 0; k < s; ++k) {
    // R[k][k] and row k to the right; rows above k are final
    if (t == 0) {
      double d = R[k][k].x;
      for (int i = 0; i < k; ++i) d -= R[i][k].x * R[i][k].x + R[i][k].y * R[i][k].y;
      if (!(d > 1e-26 * gmax)) {
        fail = 1;
        d = 1e-26 * gmax + 1e-300;
      }
      R[k][k] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    for (int j = k + 1 + t; j < s; j += blockDim.x) {
      double2 v = R[k][j];
      for (int i = 0; i < k; ++i) v = c_sub(v, c_mul(c_conj(R[i][k]), R[i][j]));
      const double inv = 1.0 / R[k][k].x;
      R[k][j] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
  }
  // R^-1 column by column (back substitution), one thread per column
  for (int j = t; j < s; j += blockDim.x) {
    for (int i = j; i >= 0; --i) {
      double2 v = i == j ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
      for (int l = i + 1; l <= j; ++l) v = c_sub(v, c_mul(R[i][l], Ri[l][j]));
      const double inv = 1.0 / R[i][i].x;
      Ri[i][j] = make_double2(v.x * inv, v.y * inv);
    }
  }
  __syncthreads();
  for (int e = t; e < s * s; e += blockDim.x) {
    const int i = e % s, j = e / s;
    rinv[base + e] = Ri[i][j];
    double2 v = make_double2(0.0, 0.0);
    if (rprev) {
      for (int l = i; l <= j; ++l) v = c_add(v, c_mul(R[i][l], rprev[base + l + j * s]));
    } else {
      v = R[i][j];
    }
    rout[base + e] = v;
  }
  if (t == 0 && fail) atomicMin(bstep + blockIdx.x, step);
}

// s x s blocks in LDS, [row][col] with a padded row.  Every helper is entered and left by all
// threads of the block (256 threads: each holds at most 4 of the s^2 <= 1024 entries).
using Blk = double2 (*)[kBlockMaxPert + 1];
constexpr int kBlkThreads = 256;
static_assert(kBlkThreads * 4 >= kBlockMaxPert * kBlockMaxPert, "4 entries per thread");

__device__ __forceinline__ void blk_load(Blk M, const double2 *src, int s) {
  for (int e = threadIdx.x; e < s * s; e += kBlkThreads) M[e % s][e / s] = src[e];
  __syncthreads();
}

__device__ __forceinline__ void blk_store(double2 *dst, Blk M, int s) {
  for (int e = threadIdx.x; e < s * s; e += kBlkThreads) dst[e] = M[e % s][e / s];
  __syncthreads();
}

// C = sgn op(A) op(B) (mode 0) or C = C - op(A) op(B) (mode 1), op = ^H where ha / hb; C may be
// A or B: the products are formed in registers before any entry is written
__device__ void blk_mm(Blk C, Blk A, bool ha, Blk B, bool hb, int s, double sgn, int mode) {
  double2 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = threadIdx.x + kBlkThreads * r;
    if (e < s * s) {
      const int i = e % s, j = e / s;
      double2 v = make_double2(0.0, 0.0);
      for (int l = 0; l < s; ++l) {
        const double2 a = ha ? c_conj(A[l][i]) : A[i][l];
        const double2 b = hb ? c_conj(B[j][l]) : B[l][j];
        v = c_add(v, c_mul(a, b));
      }
      acc[r] = mode ? c_sub(C[i][j], v) : make_double2(sgn * v.x, sgn * v.y);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = threadIdx.x + kBlkThreads * r;
    if (e < s * s) C[e % s][e / s] = acc[r];
  }
  __syncthreads();
}

// M = A - M - z I (M holds a product, A a block in global memory)
__device__ __forceinline__ void blk_diff_shift(Blk M, const double2 *A, double2 z, int s) {
  for (int e = threadIdx.x; e < s * s; e += kBlkThreads) {
    const int i = e % s, j = e / s;
    double2 v = c_sub(A[e], M[i][j]);
    if (i == j) v = c_sub(v, z);
    M[i][j] = v;
  }
  __syncthreads();
}

// in-place inverse of M by Gauss-Jordan elimination with partial pivoting (row exchanges recorded in
// perm, undone on the columns at the end)
__device__ void blk_inverse(Blk M, int s, int *perm) {
  for (int i = threadIdx.x; i < s; i += kBlkThreads) perm[i] = i;
  __syncthreads();
  __shared__ int piv;
  for (int k = 0; k < s; ++k) {
    // pivot: the largest |M[i][k]| over rows i >= k (s <= 32 rows: one wave, butterfly argmax)
    if (threadIdx.x < 64) {
      const int i = k + threadIdx.x;
      double a = -1.0;
      int idx = s;
      if (i < s) {
        a = M[i][k].x * M[i][k].x + M[i][k].y * M[i][k].y;
        idx = i;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double oa = __shfl_xor(a, off);
        const int oi = __shfl_xor(idx, off);
        if (oa > a || (oa == a && oi < idx)) {
          a = oa;
          idx = oi;
        }
      }
      if (threadIdx.x == 0) piv = idx;
    }
    __syncthreads();
    const int p = piv;
    if (p != k) {  // the same for the whole block
      for (int j = threadIdx.x; j < s; j += kBlkThreads) {
        const double2 tmp = M[k][j];
        M[k][j] = M[p][j];
        M[p][j] = tmp;
      }
      if (threadIdx.x == 0) {
        const int tp = perm[k];
        perm[k] = perm[p];
        perm[p] = tp;
      }
      __syncthreads();
    }
    const double2 d = M[k][k];
    const double q = 1.0 / (d.x * d.x + d.y * d.y);
    const double2 dinv = make_double2(d.x * q, -d.y * q);
    __syncthreads();  // every thread holds the pivot before row k is scaled
    for (int j = threadIdx.x; j < s; j += kBlkThreads) M[k][j] = j == k ? dinv : c_mul(M[k][j], dinv);
    __syncthreads();
    // rows i != k: columns j != k lose M[i][k] times the scaled pivot row ...
    for (int e = threadIdx.x; e < s * s; e += kBlkThreads) {
      const int i = e % s, j = e / s;
      if (i != k && j != k) M[i][j] = c_sub(M[i][j], c_mul(M[i][k], M[k][j]));
    }
    __syncthreads();
    // ... and column k becomes -M[i][k] / pivot
    for (int i = threadIdx.x; i < s; i += kBlkThreads)
      if (i != k) M[i][k] = c_mul(make_double2(-M[i][k].x, -M[i][k].y), M[k][k]);
    __syncthreads();
  }
  // inverse of A = (inverse of the row-exchanged matrix) with its columns put back: column l goes to
  // perm[l] (up to 4 entries per thread, read before any is written)
  double2 v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = threadIdx.x + kBlkThreads * r;
    if (e < s * s) v[r] = M[e % s][e / s];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = threadIdx.x + kBlkThreads * r;
    if (e < s * s) M[e % s][perm[e / s]] = v[r];
  }
  __syncthreads();
}

// Per (band, shift), one block of 256 threads: step j of the forward block recurrence of (T - z) and
// the residual estimate of the FOM solutions after j + 1 block steps.  ablk = A_j, bprev = B_j
// (j > 0), bnext = B_{j+1} of every band; the (band, shift)'s history in hist (kb steps of D_i^-1 and
// F_i) holds D_{j-1}^-1, F_{j-1} and takes D_j^-1, F_j, kept for the final block solve.
// res[band][shift] = largest over the block's columns c of ||B_{j+1} D_j^-1 F_j e_c|| / ||b_c||; once it is at most tol_int, conv[band][shift] = j + 1 and the
// shift's recurrence stops (its FOM solution is taken at that step).
__global__ __launch_bounds__(kBlkThreads) void k_blk_shift(int s, int n_omega, int j,
                                                         const double2 *__restrict__ ablk,
                                                         const double2 *__restrict__ bprev,
                                                         const double2 *__restrict__ bnext,
                                                         const double2 *__restrict__ r0,
                                                         const double *__restrict__ bnorm,
                                                         const double2 *__restrict__ zs, double2 *__restrict__ hist,
                                                         int kb, double *__restrict__ res,
                                                         int32_t *__restrict__ conv, double tol_int) {
  __shared__ double2 X1[kBlockMaxPert][kBlockMaxPert + 1], X2[kBlockMaxPert][kBlockMaxPert + 1],
      X3[kBlockMaxPert][kBlockMaxPert + 1];
  __shared__ int perm[kBlockMaxPert];
  __shared__ double cres[kBlockMaxPert];
  const int b = blockIdx.x / n_omega, k = blockIdx.x - b * n_omega;
  if (conv[(long)b * n_omega + k] >= 0) return;  // the whole block leaves together
  const long ss = (long)s * s, bo = (long)b * ss;
  double2 *hk = hist + ((long)b * n_omega + k) * 2 * kb * ss;  // step i: D_i^-1, then F_i
  if (j == 0) {
    blk_load(X1, r0 + bo, s);  // F_0 = R_0
    for (int e = threadIdx.x; e < s * s; e += kBlkThreads) X3[e % s][e / s] = make_double2(0.0, 0.0);
    __syncthreads();
  } else {
    blk_load(X1, hk + (long)(j - 1) * 2 * ss, s);
    blk_load(X2, bprev + bo, s);
    blk_mm(X3, X2, false, X1, false, s, 1.0, 0);   // L = B_j D_{j-1}^-1
    blk_load(X1, hk + (long)(j - 1) * 2 * ss + ss, s);
    blk_mm(X1, X3, false, X1, false, s, -1.0, 0);  // F_j = -L F_{j-1}
    blk_mm(X3, X3, false, X2, true, s, 1.0, 0);    // L B_j^H
  }
  blk_diff_shift(X3, ablk + bo, zs[k], s);  // D_j = A_j - L B_j^H - z
  blk_inverse(X3, s, perm);
  blk_store(hk + (long)j * 2 * ss, X3, s);
  blk_store(hk + (long)j * 2 * ss + ss, X1, s);
  blk_mm(X2, X3, false, X1, false, s, 1.0, 0);  // last block of Y = D_j^-1 F_j
  blk_load(X1, bnext + bo, s);
  blk_mm(X1, X1, false, X2, false, s, 1.0, 0);  // B_{j+1} Y_last
  for (int c = threadIdx.x; c < s; c += kBlkThreads) {
    double n2 = 0.0;
    for (int i = 0; i < s; ++i) n2 += X1[i][c].x * X1[i][c].x + X1[i][c].y * X1[i][c].y;
    const double nb = bnorm[b * s + c];
    cres[c] = nb > 0.0 ? sqrt(n2) / nb : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int c = 0; c < s; ++c) m = fmax(m, isfinite(cres[c]) ? cres[c] : 1e300);
    res[(long)b * n_omega + k] = m;
    if (m <= tol_int) conv[(long)b * n_omega + k] = j + 1;
  }
}

// Per (band, shift): block LU solve of (T_k - z) Y = E_0 R_0 over the shift's own step count kk (conv,
// else the band's kband): the forward sweep (D_i^-1, G_i) is the one k_blk_shift kept in scratch, the
// backward one is Y_{kk-1} = D_{kk-1}^-1 G_{kk-1}, Y_i = D_i^-1 (G_i - B_{i+1}^H Y_{i+1}).  Y goes
// to ycat[b] at rows i s + r, column pos[b][shift] s + c (leading dimension ldy); rows kk s .. k s - 1
// are zeroed.
__global__ __launch_bounds__(kBlkThreads) void k_blk_solve(int s, int n_omega, int k, int kb, int nbc,
                                                         const double2 *__restrict__ bblk,
                                                         const double2 *__restrict__ scratch,
                                                         double2 *__restrict__ ycat, long ldy, long ycat_stride,
                                                         const int32_t *__restrict__ conv,
                                                         const int32_t *__restrict__ pos,
                                                         const int32_t *__restrict__ kband) {
  __shared__ double2 X1[kBlockMaxPert][kBlockMaxPert + 1], X2[kBlockMaxPert][kBlockMaxPert + 1],
      X3[kBlockMaxPert][kBlockMaxPert + 1];
  const int b = blockIdx.x / n_omega, sh = blockIdx.x - b * n_omega;
  const long ss = (long)s * s;
  // the forward recurrence of k_blk_shift: step i holds D_i^-1, then G_i (= F_i)
  const double2 *scr = scratch + ((long)b * n_omega + sh) * 2 * kb * ss;
  const int cv = conv[(long)b * n_omega + sh], kbb = kband[b];
  const int kk = cv >= 0 && cv <= kbb ? cv : kbb;  // a band whose block lost rank keeps its valid steps
  const long col0 = (long)pos[(long)b * n_omega + sh] * s;
  double2 *yb = ycat + (long)b * ycat_stride;
  for (int e = threadIdx.x; e < (k - kk) * s * s; e += kBlkThreads) {
    const int r = e % ((k - kk) * s), c = e / ((k - kk) * s);
    yb[(long)(kk * s + r) + (col0 + c) * ldy] = make_double2(0.0, 0.0);
  }
  for (int i = kk - 1; i >= 0; --i) {
    blk_load(X1, scr + (long)i * 2 * ss + ss, s);  // G_i
    if (i < kk - 1) {
      blk_load(X3, bblk + ((long)(i + 1) * nbc + b) * ss, s);
      blk_mm(X1, X3, true, X2, false, s, 1.0, 1);  // G_i - B_{i+1}^H Y_{i+1}
    }
    blk_load(X3, scr + (long)i * 2 * ss, s);
    blk_mm(X2, X3, false, X1, false, s, 1.0, 0);  // Y_i
    for (int e = threadIdx.x; e < s * s; e += kBlkThreads) {
      const int r = e % s, c = e / s;
      yb[(long)(i * s + r) + (col0 + c) * ldy] = X2[r][c];
    }
    __syncthreads();
  }
}

// Per solution of a run of shifts (positions p0 .. p0 + len - 1 of the order ord): its true FP64
// residual from X = V Y and (H + alpha P) X = (AV) Y, both formed from the stored products, and the
// solution in the caller's order and sign.  Block a: band b, position p0 + l, perturbation c for
// a = (b len + l) s + c, the caller's perturbation pert0 + c of n_pert; x, ax at vector (b run + l) s + c
// of xg, axg (q: the overlaps psi^H x).
// relres = ||b - (ax - eps x - z x)|| / ||b||, occ_leak = ||q|| / ||x||, iters = the shift's step count
// (conv, else the band's kband; MAXITER when the residual misses tol after the step limit (maxed), no
// flag for a band whose block lost rank, so that it is refined per shift); dpsi[g] = -x[u2i[g]].
constexpr int kFinThreads = 1024, kFinUnroll = 4;  // threads per solution of k_blk_final, elements in flight
__global__ __launch_bounds__(kFinThreads) void k_blk_final(int npw, int n_occ, int s, int n_pert, int pert0, int n_omega,
                                                   int len, int p0, int run,
                                                   const double2 *__restrict__ xg, const double2 *__restrict__ axg,
                                                   const double2 *__restrict__ qg, const double2 *__restrict__ rhs,
                                                   const double *__restrict__ eps, const double2 *__restrict__ zs,
                                                   const int32_t *__restrict__ ord, const int32_t *__restrict__ conv,
                                                   const int32_t *__restrict__ kband, int k_final, int maxed,
                                                   double tol,
                                                   const int32_t *__restrict__ u2i,
                                                   double2 *__restrict__ dpsi, sgw_solve_info *info, int *bad) {
  __shared__ double red[4][kFinThreads];
  const long a = blockIdx.x;
  const int c = (int)(a % s);
  const long bl = a / s;
  const int b = (int)(bl / len), l = (int)(bl - (long)b * len);
  const int sh = ord[p0 + l];
  const long xv = ((long)b * run + l) * s + c;
  const double2 *xa = xg + xv * npw, *ya = axg + xv * npw, *ba = rhs + ((long)b * s + c) * npw;
  const double2 z = zs[sh];
  const double e = eps[b];
  const long o = ((long)b * n_pert + pert0 + c) * n_omega + sh;  // caller's (band, perturbation, shift)
  double2 *out = dpsi + o * npw;
  // one pass: the residual terms in the internal order, the solution gathered into the caller's;
  // kFinUnroll elements per thread in flight (the gather waits on its index load)
  double rr = 0.0, bb = 0.0, xx = 0.0, qq = 0.0;
  for (int g0 = threadIdx.x; g0 < npw; g0 += kFinUnroll * kFinThreads) {
    int src[kFinUnroll];
    double2 x[kFinUnroll], y[kFinUnroll], bv[kFinUnroll], xo[kFinUnroll];
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) {
      const int g = g0 + u * kFinThreads;
      if (g < npw) {
        src[u] = u2i[g];
        x[u] = xa[g];
        y[u] = ya[g];
        bv[u] = ba[g];
      }
    }
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u)
      if (g0 + u * kFinThreads < npw) xo[u] = xa[src[u]];
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) {
      const int g = g0 + u * kFinThreads;
      if (g < npw) {
        // (A - z) x = y - eps x - z x
        const double ax = y[u].x - e * x[u].x - (z.x * x[u].x - z.y * x[u].y);
        const double ay = y[u].y - e * x[u].y - (z.x * x[u].y + z.y * x[u].x);
        const double rx = bv[u].x - ax, ry = bv[u].y - ay;
        rr += rx * rx + ry * ry;
        bb += bv[u].x * bv[u].x + bv[u].y * bv[u].y;
        xx += x[u].x * x[u].x + x[u].y * x[u].y;
        out[g] = make_double2(-xo[u].x, -xo[u].y);
      }
    }
  }
  for (int i = threadIdx.x; i < n_occ; i += kFinThreads) {
    const double2 q = qg[xv * n_occ + i];
    qq += q.x * q.x + q.y * q.y;
  }
  red[0][threadIdx.x] = rr;
  red[1][threadIdx.x] = bb;
  red[2][threadIdx.x] = xx;
  red[3][threadIdx.x] = qq;
  __syncthreads();
  for (int h = kFinThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double occ = red[3][0];
    const int kbb = kband[b];
    const int cv = conv[(long)b * n_omega + sh] <= kbb ? conv[(long)b * n_omega + sh] : -1;
    const double nb = sqrt(red[1][0]), nx = sqrt(red[2][0]);
    const double rel = nb > 0.0 ? sqrt(red[0][0]) / nb : 0.0;
    sgw_solve_info r;
    r.iters = cv >= 0 ? cv : kbb;
    r.relres = rel;
    r.occ_leak = nx > 0.0 ? sqrt(occ) / nx : 0.0;
    int fl = 0;
    if (!isfinite(rel)) fl |= SGW_FLAG_NONFINITE;
    else if (nb == 0.0) fl |= SGW_FLAG_CONVERGED | SGW_FLAG_ZERO_RHS;
    else if (rel <= tol) fl |= SGW_FLAG_CONVERGED;
    else fl |= cv < 0 && maxed && kbb == k_final ? SGW_FLAG_MAXITER : 0;  // a band that lost rank: refined
    r.flags = fl;
    info[o] = r;
    if (!(fl & SGW_FLAG_CONVERGED)) atomicOr(bad, 1);
  }
}

// ---------------------------------------------------------------------------
// rocBLAS
// ---------------------------------------------------------------------------
rocblas_handle blas(sgw_ctx *ctx) {
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    ctx->blas = h;
  }
  rocblas_handle h = (rocblas_handle)ctx->blas;
  rocblas_set_stream(h, ctx->stream);
  return h;
}

// C_b = alpha op(A_b) B_b + beta C_b over nbatch (column-major, strides in elements); kid >= 0: the
// launch is timed under that id with its algorithmic bytes (A, B read, C written) and flops
sgw_status zgemm(sgw_ctx *ctx, rocblas_operation ta, rocblas_operation tb, int m, int n, int k, double2 alpha,
                 const double2 *A, long lda, long sa, const double2 *B, long ldb, long sb, double2 beta, double2 *C,
                 long ldc, long sc, int nbatch, int kid = -1) {
  rocblas_handle h = blas(ctx);
  if (!h) return fail(SGW_ERR_HIP, "block solver: rocblas_create_handle failed");
  const rocblas_double_complex al(alpha.x, alpha.y), be(beta.x, beta.y);
  PendingTiming tm;
  if (kid >= 0)
    timing_begin(ctx, kid, 16.0 * nbatch * ((double)m * k + (double)k * n + (double)m * n),
                 8.0 * nbatch * (double)m * n * k, &tm);
  const rocblas_status r = rocblas_zgemm_strided_batched(
      h, ta, tb, m, n, k, &al, (const rocblas_double_complex *)A, lda, sa, (const rocblas_double_complex *)B, ldb, sb,
      &be, (rocblas_double_complex *)C, ldc, sc, nbatch);
  if (kid >= 0) timing_end(ctx, &tm);
  if (r != rocblas_status_success) return fail(SGW_ERR_HIP, "block solver: rocblas_zgemm_strided_batched failed");
  return SGW_OK;
}

// Split the shifts, in order ord (step counts k[ord[p]] non-increasing), into at most kGroups runs
// [cut[g], cut[g + 1]) minimising the sum over runs of (length x the run's first step count): the work
// of the products X = V Y taken run by run.
constexpr int kGroups = 6;
std::vector<int> shift_runs(const std::vector<int> &ord, const std::vector<int> &k) {
  const int n = (int)ord.size();
  const int G = std::min(kGroups, n);
  const double inf = 1e300;
  // best[g][p]: least cost of the first p shifts in g runs
  std::vector<std::vector<double>> best(G + 1, std::vector<double>(n + 1, inf));
  std::vector<std::vector<int>> from(G + 1, std::vector<int>(n + 1, 0));
  best[0][0] = 0.0;
  for (int g = 1; g <= G; ++g)
    for (int p = 1; p <= n; ++p)
      for (int q = 0; q < p; ++q) {
        if (best[g - 1][q] >= inf) continue;
        const double c = best[g - 1][q] + (double)(p - q) * k[ord[q]];
        if (c < best[g][p]) {
          best[g][p] = c;
          from[g][p] = q;
        }
      }
  int g = 1;
  for (int h = 1; h <= G; ++h)
    if (best[h][n] < best[g][n]) g = h;
  std::vector<int> cut;
  for (int p = n; g > 0; --g) {
    cut.push_back(p);
    p = from[g][p];
  }
  cut.push_back(0);
  std::reverse(cut.begin(), cut.end());
  return cut;
}

// out_b = sgn src_b coef_b (+ base_b, copied to copy_b when copy is given) for the nb bands
sgw_status comb(sgw_ctx *ctx, int npw, int s, int nb, int K, const double2 *src, long ssrc, const double2 *coef,
                double sgn, const double2 *base, long sbase, double2 *out, long sout, double2 *copy = nullptr,
                long scopy = 0) {
  const dim3 grid((npw + 255) / 256, nb);
#define SGW_COMB(SM)                                                                                            \
  hipLaunchKernelGGL(k_blk_comb<SM>, grid, dim3(256), 0, ctx->stream, npw, s, K, src, ssrc, coef, sgn, base, sbase, \
                     out, sout, copy, scopy)
  if (s <= 8) SGW_COMB(8);
  else if (s <= 16) SGW_COMB(16);
  else if (s <= 20) SGW_COMB(20);
  else if (s <= 24) SGW_COMB(24);
  else SGW_COMB(32);
#undef SGW_COMB
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

// C_b = A_b^H B_b for the nb bands' n_pw x s blocks (band strides sa, sb), C contiguous s x s blocks
sgw_status gram(sgw_ctx *ctx, int npw, int s, int nb, const double2 *A, long sa, const double2 *B, long sb,
                double2 *part, double2 *C) {
  const int n_chunks = (npw + kGramRows - 1) / kGramRows;
  hipLaunchKernelGGL(k_blk_gram, dim3(n_chunks, nb), dim3(256), 0, ctx->stream, npw, s, A, sa, B, sb, part);
  hipLaunchKernelGGL(k_blk_gram_sum, dim3(nb), dim3(256), 0, ctx->stream, n_chunks, nb, s * s,
                     (const double2 *)part, C);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

// blocks of at most kBlockMaxPert perturbations, as equal as possible: group g of n_groups starts at
// first(g) and holds size(g) perturbations
struct PertGroups {
  int n_pert, n_groups;
  explicit PertGroups(int n) : n_pert(n), n_groups(std::max(1, (n + kBlockMaxPert - 1) / kBlockMaxPert)) {}
  int size(int g) const { return n_pert / n_groups + (g < n_pert % n_groups ? 1 : 0); }
  int first(int g) const { return g * (n_pert / n_groups) + std::min(g, n_pert % n_groups); }
  int largest() const { return size(0); }
};

}  // namespace

void blas_release(sgw_ctx *ctx) {
  if (ctx && ctx->blas) {
    rocblas_destroy_handle((rocblas_handle)ctx->blas);
    ctx->blas = nullptr;
  }
}

size_t block_workspace_bytes(const sgw_ham *h_kq, int n_occ, int n_band, int n_pert, int n_omega,
                             const sgw_opts &o) {
  if (n_band <= 0 || n_pert <= 0) return 256;
  const int kb = blk_steps(o) + 1;
  const int s = PertGroups(n_pert).largest();
  const int nbc = blk_chunk(h_kq, n_occ, n_band, s, n_omega, kb, kBlockBudget, o.slots);
  return blk_layout(h_kq, n_occ, nbc, s, n_omega, kb).total;
}

namespace {

// The perturbations pert0 .. pert0 + s - 1 of the caller's n_pert (dv_miller: theirs, s rows) as one
// block per band; dpsi and info are the caller's whole arrays.
sgw_status block_group(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq, const sgw_ham *h_k,
                       int n_band, const sgw_c128 *psi_v, const double *eps_v, int n_pert, int pert0, int s,
                       const int32_t *dv_miller, int n_omega, const double *omega, double eta, double tol,
                       const sgw_opts &o, void *workspace, size_t workspace_bytes, sgw_c128 *dpsi,
                       sgw_solve_info *info) {
  if (s > kBlockMaxPert || s < 1) return fail(SGW_ERR_INVALID_ARG, "block solver: bad block size");
  const int npw = h_kq->n_pw;
  const int kb = blk_steps(o) + 1;
  const int nbc = blk_chunk(h_kq, n_occ, n_band, s, n_omega, kb, (double)workspace_bytes, o.slots);
  const BlkLayout L = blk_layout(h_kq, n_occ, nbc, s, n_omega, kb);
  if (L.total > workspace_bytes) return fail(SGW_ERR_WORKSPACE, "block solver: workspace too small for one band");
  char *Wb = (char *)workspace;
  auto P = [&](size_t off) { return (double2 *)(Wb + off); };
  double2 *basis = P(L.basis), *rhs = P(L.rhs), *Y = P(L.y), *Wv = P(L.w), *V2 = P(L.v2), *gbuf = P(L.gram), *cbuf = P(L.coef),
          *part = P(L.part),
          *rfac = P(L.rfac), *rinv = P(L.rinv), *ablk = P(L.ablk), *bblk = P(L.bblk), *r0 = P(L.r0),
          *thomas = P(L.thomas), *ycat = P(L.ycat), *xg = P(L.xg),
          *axg = P(L.axg), *qg = P(L.qg), *abasis = P(L.abasis), *pov = P(L.pov), *C = P(L.c), *psi = P(L.psi),
          *zs = P(L.omega);
  double *bnorm = (double *)(Wb + L.bnorm), *res = (double *)(Wb + L.res), *deps = (double *)(Wb + L.eps);
  int32_t *list = (int32_t *)(Wb + L.list), *conv = (int32_t *)(Wb + L.conv), *dpos = (int32_t *)(Wb + L.ord);
  int *bad = (int *)(Wb + L.bad), *bstep = (int *)(Wb + L.bstep), *kband = (int *)(Wb + L.kband);
  void *T = Wb + L.t;
  const long ss = (long)s * s;
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  sgw_status st;

  // shifts z_j = omega_j + i eta_j, occupied states in internal order, dv_miller on the device
  std::vector<double2> hz(n_omega);
  for (int j = 0; j < n_omega; ++j) hz[j] = make_double2(omega[j], o.shift_imag ? o.shift_imag[j] : eta);
  SGW_HIP(hipMemcpyAsync(zs, hz.data(), sizeof(double2) * n_omega, hipMemcpyHostToDevice, ctx->stream));
  if ((st = permute(ctx, npw, n_occ, (const double2 *)psi_occ_kq, npw, psi, npw, h_kq->d_i2u, 0)) != SGW_OK) return st;
  int32_t *ddvm = (int32_t *)(Wb + L.dvm);
  SGW_HIP(hipMemcpyAsync(ddvm, dv_miller, sizeof(int32_t) * 3 * s, hipMemcpyHostToDevice, ctx->stream));
  std::vector<int32_t> hpairs((size_t)nbc * s);
  bool any_bad = false;
  const double tol_int = tol * o.tol_safety;

  for (int b0 = 0; b0 < n_band; b0 += nbc) {
    const int nb = std::min(nbc, n_band - b0);
    const int nv = nb * s;
    SGW_HIP(hipMemsetAsync(bad, 0, 8, ctx->stream));
    SGW_HIP(hipMemsetAsync(conv, 0xff, sizeof(int32_t) * nb * n_omega, ctx->stream));  // -1: running
    SGW_HIP(hipMemsetAsync(bstep, 0x7f, sizeof(int) * nb, ctx->stream));                // no rank loss
    SGW_HIP(hipMemcpyAsync(deps, eps_v + b0, sizeof(double) * nb, hipMemcpyHostToDevice, ctx->stream));
    // right-hand sides in internal order: rhs = (1 - P) s (the solution is negated on the way out)
    for (int a = 0; a < nv; ++a) hpairs[a] = (b0 + a / s) * s + a % s;
    SGW_HIP(hipMemcpyAsync(list, hpairs.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, ctx->stream));
    if ((st = rhs_source(ctx, h_kq, h_k, nv, list, s, ddvm, (const double2 *)psi_v, h_k->n_pw, Y, npw)) != SGW_OK)
      return st;
    if ((st = proj_dot(ctx, npw, n_occ, psi, nv, contiguous(Y, npw), C, nv)) != SGW_OK) return st;
    if ((st = proj_apply(ctx, npw, n_occ, psi, nv, contiguous(Y, npw), C, nv, rhs, npw, 1.0, 0)) != SGW_OK) return st;
    // column norms of every band's block (for the residual estimates): diagonal of rhs^H rhs
    if ((st = gram(ctx, npw, s, nb, rhs, (long)s * npw, rhs, (long)s * npw, part, gbuf)) != SGW_OK) return st;
    {
      std::vector<double2> hg((size_t)nb * ss);
      SGW_HIP(hipMemcpyAsync(hg.data(), gbuf, sizeof(double2) * nb * ss, hipMemcpyDeviceToHost, ctx->stream));
      if ((st = sync(ctx)) != SGW_OK) return st;
      std::vector<double> hn(nv);
      for (int b = 0; b < nb; ++b)
        for (int c = 0; c < s; ++c) hn[b * s + c] = std::sqrt(std::max(hg[(size_t)b * ss + c + c * s].x, 0.0));
      SGW_HIP(hipMemcpyAsync(bnorm, hn.data(), sizeof(double) * nv, hipMemcpyHostToDevice, ctx->stream));
    }
    // V_0 R_0 = rhs (Cholesky QR twice)
    // (step: the index of the basis block formed; a band whose Cholesky fails keeps blocks 0 .. step - 1)
    auto orth = [&](const double2 *src, double2 *dst, double2 *rout, int step) -> sgw_status {
      sgw_status s2;
      if ((s2 = gram(ctx, npw, s, nb, src, (long)s * npw, src, (long)s * npw, part, gbuf)) != SGW_OK) return s2;
      hipLaunchKernelGGL(k_blk_chol, dim3(nb), dim3(64), 0, ctx->stream, gbuf, (const double2 *)nullptr, rfac, rinv,
                         s, bstep, step);
      if ((s2 = comb(ctx, npw, s, nb, s, src, (long)s * npw, rinv, 1.0, nullptr, 0, V2, (long)s * npw)) != SGW_OK)
        return s2;
      if ((s2 = gram(ctx, npw, s, nb, V2, (long)s * npw, V2, (long)s * npw, part, gbuf)) != SGW_OK) return s2;
      hipLaunchKernelGGL(k_blk_chol, dim3(nb), dim3(64), 0, ctx->stream, gbuf, (const double2 *)rfac, rout, rinv, s,
                         bstep, step);
      // dst (strided per band in the basis) = V2 R2^-1
      return comb(ctx, npw, s, nb, s, V2, (long)s * npw, rinv, 1.0, nullptr, 0, dst, (long)kb * s * npw);
    };
    if ((st = orth(rhs, basis, r0, 0)) != SGW_OK) return st;
    // block Lanczos steps with the residual estimates of every (band, shift).  A band whose block loses
    // rank (dependent right-hand sides, or a block space that stops growing in some direction) keeps
    // its valid blocks: its later steps are ignored, its solutions are taken at that step count and
    // any that miss tol are refined per shift.
    int k = 0;
    std::vector<double> hres((size_t)nb * n_omega);
    std::vector<int> hbstep(nb);
    SGW_HIP(hipMemcpyAsync(hbstep.data(), bstep, sizeof(int) * nb, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    bool all_lost = true;
    for (int b = 0; b < nb; ++b) all_lost = all_lost && hbstep[b] <= 0;
    // host polls: every step once a step is large enough to hide the round trip
    const int poll = (long)nv * npw >= (1L << 22) ? 1 : std::max(1, o.steps_per_sync);
    for (int j = 0; j + 1 < kb && !all_lost; ++j) {
      hipLaunchKernelGGL(k_blk_list, dim3((nv + 255) / 256), dim3(256), 0, ctx->stream, list, nb, s, kb, j);
      const VecSrc vj = listed(basis, npw, list);
      if ((st = proj_dot(ctx, npw, n_occ, psi, nv, vj, C, nv)) != SGW_OK) return st;
      if (n_occ > 0)  // psi^H V_j kept per band: [b][kb][s][n_occ]
        SGW_HIP(hipMemcpy2DAsync(pov + (long)j * s * n_occ, sizeof(double2) * kb * s * n_occ, C,
                                 sizeof(double2) * s * n_occ, sizeof(double2) * s * n_occ, nb,
                                 hipMemcpyDeviceToDevice, ctx->stream));
      if ((st = hx_batch(ctx, h_kq, nv, vj, Y, npw, T)) != SGW_OK) return st;
      if ((st = proj_apply(ctx, npw, n_occ, psi, nv, vj, C, nv, Y, npw, o.alpha_pv, 1)) != SGW_OK) return st;
      // Y = (H + alpha P) V_j; G = V_j^H Y; A_j = herm(G) - eps I;
      // W = Y - V_{j-1} B_j^H - V_j herm(G) = (H + alpha P - eps) V_j - V_{j-1} B_j^H - V_j A_j, and Y kept as AV
      double2 *vj_ptr = basis + (long)j * s * npw;  // band 0; bands strided by kb s npw
      double2 *aj = ablk + (long)j * nbc * ss;
      if ((st = gram(ctx, npw, s, nb, vj_ptr, (long)kb * s * npw, Y, (long)s * npw, part, gbuf)) != SGW_OK) return st;
      hipLaunchKernelGGL(k_blk_coef, dim3(nb), dim3(256), 0, ctx->stream, s, j, (const double2 *)gbuf,
                         (const double2 *)(bblk + (long)j * nbc * ss), (const double *)deps, aj, cbuf);
      if ((st = comb(ctx, npw, s, nb, j > 0 ? 2 * s : s, j > 0 ? vj_ptr - (long)s * npw : vj_ptr,
                     (long)kb * s * npw, cbuf, -1.0, Y, (long)s * npw, Wv, (long)s * npw,
                     abasis + (long)j * s * npw, (long)kb * s * npw)) != SGW_OK)
        return st;
      if ((st = orth(Wv, vj_ptr + (long)s * npw, bblk + (long)(j + 1) * nbc * ss, j + 1)) != SGW_OK) return st;
      hipLaunchKernelGGL(k_blk_shift, dim3(nb * n_omega), dim3(kBlkThreads), 0, ctx->stream, s, n_omega, j,
                         (const double2 *)aj, (const double2 *)(bblk + (long)j * nbc * ss),
                         (const double2 *)(bblk + (long)(j + 1) * nbc * ss), (const double2 *)r0,
                         (const double *)bnorm, (const double2 *)zs, thomas, kb, res, conv, tol_int);
      SGW_HIP(hipGetLastError());
      k = j + 1;
      if (k % poll == 0 || k + 1 >= kb) {
        SGW_HIP(hipMemcpyAsync(hres.data(), res, sizeof(double) * nb * n_omega, hipMemcpyDeviceToHost, ctx->stream));
        SGW_HIP(hipMemcpyAsync(hbstep.data(), bstep, sizeof(int) * nb, hipMemcpyDeviceToHost, ctx->stream));
        if ((st = sync(ctx)) != SGW_OK) return st;
        double worst = 0.0;
        for (int b = 0; b < nb; ++b) {
          if (hbstep[b] <= k) continue;  // lost rank: done at its valid steps
          for (int q = 0; q < n_omega; ++q) {
            const double r = hres[(size_t)b * n_omega + q];
            worst = std::max(worst, std::isfinite(r) ? r : 1e300);
          }
        }
        if (worst <= tol_int) break;
      }
    }
    // every band's valid step count
    SGW_HIP(hipMemcpyAsync(hbstep.data(), bstep, sizeof(int) * nb, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    std::vector<int32_t> hkband(nb);
    for (int b = 0; b < nb; ++b) hkband[b] = std::min(k, std::max(hbstep[b], 0));
    SGW_HIP(hipMemcpyAsync(kband, hkband.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, ctx->stream));
    int hbad = 0;
    // Solutions: Y(z) per (band, shift) at the shift's own step count, X = V Y per band.  Within each
    // group of kSubBands bands the shifts are ordered by their largest step count over the group and
    // split into up to kGroups runs (least total inner dimension), one batched product per run piece
    // with that run's inner dimension.
    std::vector<int32_t> hconv((size_t)nb * n_omega);
    SGW_HIP(hipMemcpyAsync(hconv.data(), conv, sizeof(int32_t) * nb * n_omega, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    const int nsb = (nb + kSubBands - 1) / kSubBands;
    std::vector<std::vector<int>> sb_ksh(nsb, std::vector<int>(n_omega, 0)), sb_ord(nsb), sb_cut(nsb);
    std::vector<int32_t> hmap((size_t)(nb + nsb) * n_omega);  // pos[b][shift], then ord[group][p]
    for (int q = 0; q < nsb; ++q) {
      const int b_lo = q * kSubBands, b_hi = std::min(nb, b_lo + kSubBands);
      std::vector<int> &ksh = sb_ksh[q], &ord = sb_ord[q];
      for (int b = b_lo; b < b_hi; ++b)
        for (int j = 0; j < n_omega; ++j) {
          const int c = hconv[(size_t)b * n_omega + j];
          ksh[j] = std::max(ksh[j], c >= 0 && c <= hkband[b] ? c : hkband[b]);
        }
      ord.resize(n_omega);
      for (int j = 0; j < n_omega; ++j) ord[j] = j;
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return ksh[x] > ksh[y]; });
      for (int p = 0; p < n_omega; ++p) {
        for (int b = b_lo; b < b_hi; ++b) hmap[(size_t)b * n_omega + ord[p]] = p;
        hmap[(size_t)(nb + q) * n_omega + p] = ord[p];
      }
      sb_cut[q] = shift_runs(ord, ksh);
    }
    SGW_HIP(hipMemcpyAsync(dpos, hmap.data(), sizeof(int32_t) * hmap.size(), hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_blk_solve, dim3(nb * n_omega), dim3(kBlkThreads), 0, ctx->stream, s, n_omega, k, kb, nbc,
                       (const double2 *)bblk, (const double2 *)thomas, ycat, (long)kb * s,
                       (long)kb * s * s * n_omega, (const int32_t *)conv, (const int32_t *)dpos,
                       (const int32_t *)kband);
    SGW_HIP(hipGetLastError());
    // per run piece of at most L.run shifts: X = V Y, (H + alpha P) X = (AV) Y and psi^H X = (psi^H V) Y,
    // then the true residuals and the output
    const long ldy = (long)kb * s, ystride = (long)kb * s * s * n_omega;
    for (int q = 0; q < nsb; ++q) {
      const int b_lo = q * kSubBands, nq = std::min(kSubBands, nb - b_lo);
      const std::vector<int> &cut = sb_cut[q], &ord = sb_ord[q], &ksh = sb_ksh[q];
      const int32_t *dord = dpos + (size_t)(nb + q) * n_omega;
      for (size_t g = 0; g + 1 < cut.size(); ++g) {
        for (int p0 = cut[g]; p0 < cut[g + 1]; p0 += L.run) {
          const int len = std::min(L.run, cut[g + 1] - p0), kg = ksh[ord[p0]];
          const double2 *yc = ycat + (long)b_lo * ystride + (long)p0 * s * ldy;
          const long vo = (long)b_lo * kb * s;  // first basis vector of the group
          if (kg == 0) {  // every band of the group lost rank at the start: X = 0, refined per shift
            const size_t xb = sizeof(double2) * (size_t)nq * s * L.run * npw;
            SGW_HIP(hipMemsetAsync(xg, 0, xb, ctx->stream));
            SGW_HIP(hipMemsetAsync(axg, 0, xb, ctx->stream));
            if (n_occ > 0)
              SGW_HIP(hipMemsetAsync(qg, 0, sizeof(double2) * (size_t)nq * s * L.run * n_occ, ctx->stream));
          } else {
            if ((st = zgemm(ctx, rocblas_operation_none, rocblas_operation_none, npw, len * s, kg * s, one,
                            basis + vo * npw, npw, (long)kb * s * npw, yc, ldy, ystride, zero, xg, npw,
                            (long)s * L.run * npw, nq, K_BLK_PRODUCT)) != SGW_OK)
              return st;
            if ((st = zgemm(ctx, rocblas_operation_none, rocblas_operation_none, npw, len * s, kg * s, one,
                            abasis + vo * npw, npw, (long)kb * s * npw, yc, ldy, ystride, zero, axg, npw,
                            (long)s * L.run * npw, nq, K_BLK_PRODUCT)) != SGW_OK)
              return st;
            if (n_occ > 0 &&
                (st = zgemm(ctx, rocblas_operation_none, rocblas_operation_none, n_occ, len * s, kg * s, one,
                            pov + vo * n_occ, n_occ, (long)kb * s * n_occ, yc, ldy, ystride, zero, qg, n_occ,
                            (long)s * L.run * n_occ, nq, K_BLK_PRODUCT)) != SGW_OK)
              return st;
          }
          hipLaunchKernelGGL(k_blk_final, dim3(nq * len * s), dim3(kFinThreads), 0, ctx->stream, npw, n_occ, s, n_pert,
                             pert0, n_omega, len, p0, L.run, (const double2 *)xg, (const double2 *)axg, (const double2 *)qg,
                             (const double2 *)(rhs + (long)b_lo * s * npw), (const double *)(deps + b_lo),
                             (const double2 *)zs, dord, (const int32_t *)(conv + (long)b_lo * n_omega),
                             (const int32_t *)(kband + b_lo), k, k + 1 >= kb ? 1 : 0, tol,
                             (const int32_t *)h_kq->d_u2i, (double2 *)dpsi + (long)(b0 + b_lo) * n_pert * n_omega * npw,
                             info + (long)(b0 + b_lo) * n_pert * n_omega, bad);
          SGW_HIP(hipGetLastError());
        }
      }
    }
    SGW_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    any_bad = any_bad || hbad;
  }
  return any_bad ? SGW_NOT_CONVERGED : SGW_OK;
}


}  // namespace

sgw_status block_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq, const sgw_ham *h_k,
                       int n_band, const sgw_c128 *psi_v, const double *eps_v, int n_pert, const int32_t *dv_miller,
                       int n_omega, const double *omega, double eta, double tol, const sgw_opts &o, void *workspace,
                       size_t workspace_bytes, sgw_c128 *dpsi, sgw_solve_info *info) {
  const PertGroups G(n_pert);
  bool missed = false;
  for (int g = 0; g < G.n_groups; ++g) {
    const sgw_status st = block_group(ctx, h_kq, n_occ, psi_occ_kq, h_k, n_band, psi_v, eps_v, n_pert, G.first(g),
                                      G.size(g), dv_miller + 3 * G.first(g), n_omega, omega, eta, tol, o, workspace,
                                      workspace_bytes, dpsi, info);
    if (st != SGW_OK && st != SGW_NOT_CONVERGED) return st;
    missed = missed || st == SGW_NOT_CONVERGED;
  }
  return missed ? SGW_NOT_CONVERGED : SGW_OK;
}

}  // namespace sgw
