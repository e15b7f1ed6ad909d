// Occupied-manifold projector on the FP64 matrix cores (Sec. 2.3, Eqs. 7-8).
//
//   overlaps:  C[a][i] = sum_g conj(psi[i][g]) x_a[g]      (n_occ x n_vec, K = n_pw)
//   apply:     y_a[g]  = x_a[g] - sum_i psi[i][g] C[a][i]   (mode 0: 1 - P_occ)
//              y_a[g] += alpha sum_i psi[i][g] C[a][i]     (mode 1: + alpha P_occ)
//              (C[a][i] scaled by s[i] first when a row scale is given)
//
// The same contraction applies the separable non-local pseudopotential in H.x
// (Sec. 2.1): psi -> the projectors beta_p, s -> their energies E_p, mode 1.
//
// Both are complex GEMMs done as four real 16x16x4 FP64 MFMAs per step
// (re*re, im*im, re*im, im*re).  Workgroups of four wavefronts own large output
// tiles so that every operand fetched from L2 feeds many MFMAs:
//  * overlaps: a tile of TO occupied states x TV vectors over one chunk of
//    kProjChunkLen plane waves; Psi and x are staged through LDS in blocks of
//    kDotKB plane waves (double-buffered, the next block's global loads issued
//    before the current block's MFMAs).  Each chunk writes its partial overlaps;
//    a second pass adds them in chunk order into chunk 0.  Chunk boundaries
//    depend on n_pw alone, and a vector's arithmetic does not depend on the
//    tile it falls in, so results do not depend on how many vectors a launch
//    holds (the solver's schedules give bit-identical results).
//  * apply: a tile of kApplyG plane waves x TV vectors, each wave a 32-wide
//    plane-wave strip; C is staged through LDS in blocks of kApplyKB occupied
//    states, Psi is read straight into MFMA operands (16 consecutive plane
//    waves per row), and the outputs land as 16 consecutive plane waves of
//    four vectors per instruction (coalesced rows of y).
// Workgroups that share operands (one overlap chunk, one apply strip) are given
// ids congruent modulo the 8 XCDs, so they run on one XCD and share its L2.
//
// MFMA operand layout (v_mfma_f64_16x16x4f64, wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it receives D[l / 16 + 4 r][l % 16]
// in accumulator element r.
#include "fft_lds.h"
#include "sgw_internal.h"

namespace sgw {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// v if c, else 0: selected per component (a select between two double2 objects is lowered through
// private memory)
__device__ __forceinline__ double2 keep_if(bool c, double2 v) { return make_double2(c ? v.x : 0.0, c ? v.y : 0.0); }

constexpr int kXcdCount = 8;   // the GPU's XCDs; workgroup ids are dealt to them round-robin
constexpr int kDotKB = 16;     // plane waves per LDS block of the overlap kernel

// ---------------------------------------------------------------------------
// overlaps: grid = ceil(n_chunks / 8) * (otiles * vtiles) * 8 workgroups of 256 threads
// ---------------------------------------------------------------------------
template <int TO, int TV>
__global__ __launch_bounds__(256) void k_proj_dot(int npw, int n_occ, const double2 *__restrict__ psi, VecSrc x,
                                                  int n_vec, int n_chunks, double2 *__restrict__ cp, long rows,
                                                  int otiles, int vtiles) {
  constexpr int WO = TO / 2, WV = TV / 2;  // a wave's block: rows wo0.., vectors wv0..
  constexpr int MO = WO / 16, MV = WV / 16;
  constexpr int LO = TO / 16, LV = TV / 16;  // rows / vectors each thread stages per block
  __shared__ double2 ps[2][kDotKB][TO + 1];
  __shared__ double2 xs[2][kDotKB][TV + 1];
  // workgroup -> (chunk, tile): every tile of a chunk on the chunk's XCD
  const int xcd = blockIdx.x % kXcdCount;
  const int r = blockIdx.x / kXcdCount;
  const int ntile = otiles * vtiles;
  const int t = r % ntile;
  const int chunk = (r / ntile) * kXcdCount + xcd;
  if (chunk >= n_chunks) return;
  const int o0 = (t / vtiles) * TO, v0 = (t % vtiles) * TV;
  const int g_begin = chunk * kProjChunkLen;
  const int g_end = min(npw, g_begin + kProjChunkLen);
  const int nblk = (g_end - g_begin + kDotKB - 1) / kDotKB;

  const int tid = threadIdx.x;
  const int lk = tid & 15, lr = tid >> 4;  // staging: plane wave lk of the block, row / vector lr + 16 j
  // staging: row lr + 16 j of the occupied tile and vector lr + 16 j of the vector tile at plane wave
  // g_begin + lk of each block.  Loads always hit valid memory (rows, vectors and plane waves are
  // clamped into range) and the values out of range are replaced by zero afterwards, so no select
  // between addresses is needed.
  const double2 *prow[LO];
  const double2 *xrow[LV];
  bool pok[LO], xok[LV];
#pragma unroll
  for (int j = 0; j < LO; ++j) {
    const int i = o0 + lr + 16 * j;
    pok[j] = i < n_occ;
    prow[j] = psi + (long)min(i, n_occ - 1) * npw;
  }
#pragma unroll
  for (int j = 0; j < LV; ++j) {
    const int a = v0 + lr + 16 * j;
    xok[j] = a < n_vec;
    xrow[j] = x.ptr(min(a, n_vec - 1));
  }
  const double2 zero = make_double2(0.0, 0.0);
  const int gl = g_begin + lk;  // this thread's plane wave in block 0
  double2 pv[LO], xv[LV];
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int wo0 = (wave & 1) * WO, wv0 = (wave >> 1) * WV;
  d4 re[MO][MV], im[MO][MV];
#pragma unroll
  for (int m = 0; m < MO; ++m)
#pragma unroll
    for (int n = 0; n < MV; ++n) {
      re[m][n] = d4{0.0, 0.0, 0.0, 0.0};
      im[m][n] = d4{0.0, 0.0, 0.0, 0.0};
    }

  // block 0 into LDS buffer 0.  Raw loaded values stay in pv / xv and are zeroed out of range only
  // when written to LDS, so the next block's loads stay in flight during the MFMAs.
  bool in = gl < g_end;
  {
    const int g = min(gl, g_end - 1);
#pragma unroll
    for (int j = 0; j < LO; ++j) pv[j] = prow[j][g];
#pragma unroll
    for (int j = 0; j < LV; ++j) xv[j] = xrow[j][g];
#pragma unroll
    for (int j = 0; j < LO; ++j) ps[0][lk][lr + 16 * j] = keep_if(in && pok[j], pv[j]);
#pragma unroll
    for (int j = 0; j < LV; ++j) xs[0][lk][lr + 16 * j] = keep_if(in && xok[j], xv[j]);
  }
  __syncthreads();
  for (int kb = 0; kb < nblk; ++kb) {
    const int buf = kb & 1;
    const bool more = kb + 1 < nblk;
    if (more) {  // the next block's global loads
      const int gn = gl + (kb + 1) * kDotKB;
      in = gn < g_end;
      const int g = min(gn, g_end - 1);
#pragma unroll
      for (int j = 0; j < LO; ++j) pv[j] = prow[j][g];
#pragma unroll
      for (int j = 0; j < LV; ++j) xv[j] = xrow[j][g];
    }
#pragma unroll
    for (int ks = 0; ks < kDotKB / 4; ++ks) {
      const int kk = 4 * ks + kq;
      double2 A[MO], B[MV];
#pragma unroll
      for (int m = 0; m < MO; ++m) A[m] = ps[buf][kk][wo0 + 16 * m + col];
#pragma unroll
      for (int n = 0; n < MV; ++n) B[n] = xs[buf][kk][wv0 + 16 * n + col];
#pragma unroll
      for (int m = 0; m < MO; ++m)
#pragma unroll
        for (int n = 0; n < MV; ++n) {
          re[m][n] = mfma(A[m].x, B[n].x, re[m][n]);
          im[m][n] = mfma(A[m].x, B[n].y, im[m][n]);
        }
#pragma unroll
      for (int m = 0; m < MO; ++m)
#pragma unroll
        for (int n = 0; n < MV; ++n) {
          re[m][n] = mfma(A[m].y, B[n].y, re[m][n]);
          im[m][n] = mfma(-A[m].y, B[n].x, im[m][n]);
        }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < LO; ++j) ps[buf ^ 1][lk][lr + 16 * j] = keep_if(in && pok[j], pv[j]);
#pragma unroll
      for (int j = 0; j < LV; ++j) xs[buf ^ 1][lk][lr + 16 * j] = keep_if(in && xok[j], xv[j]);
    }
    __syncthreads();
  }
  // partial overlaps of this chunk: lane holds rows wo0 + 16 m + kq + 4 e of vector wv0 + 16 n + col
  double2 *out = cp + (long)chunk * rows * n_occ;
#pragma unroll
  for (int n = 0; n < MV; ++n) {
    const int a = v0 + wv0 + 16 * n + col;
    if (a >= n_vec) continue;
#pragma unroll
    for (int m = 0; m < MO; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = o0 + wo0 + 16 * m + kq + 4 * e;
        if (i < n_occ) out[(long)a * n_occ + i] = make_double2(re[m][n][e], im[m][n][e]);
      }
  }
}

// cp[0][a][i] = sum over chunks c of cp[c][a][i], in chunk order
__global__ __launch_bounds__(256) void k_proj_reduce(double2 *__restrict__ cp, long rows, int n_vec, int n_occ,
                                                   int n_chunks) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n_vec * n_occ) return;
  constexpr int U = 16;  // partials loaded before they are added
  double2 s = make_double2(0.0, 0.0);
  for (int c0 = 0; c0 < n_chunks; c0 += U) {
    double2 part[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      part[u] = c0 + u < n_chunks ? cp[(long)(c0 + u) * rows * n_occ + e] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c0 + u < n_chunks) s = c_add(s, part[u]);
  }
  cp[e] = s;
}

// ---------------------------------------------------------------------------
// apply: grid = ceil(gtiles / 8) * vtiles * 8 workgroups of 256 threads
// ---------------------------------------------------------------------------
constexpr int kApplyG = 128;    // plane waves per workgroup (a 32-wide strip per wave)
constexpr int kApplyKB = 64;    // occupied states per LDS block of C
constexpr int kApplyPre = 2;    // occupied K-steps per group of Psi operands (double-buffered)

template <int TV>
__global__ __launch_bounds__(256) void k_proj_apply(int npw, int n_occ, const double2 *__restrict__ psi, VecSrc x,
                                                    int n_vec, const double2 *__restrict__ cp,
                                                    double2 *__restrict__ y, long ldy, double alpha, int mode,
                                                    const double *__restrict__ row_scale, int gtiles, int vtiles) {
  constexpr int MV = TV / 16;  // vector tiles per wave (rows of the MFMA output)
  __shared__ double2 cs[TV][kApplyKB + 1];  // C of the tile's vectors, one block of occupied states
  const int xcd = blockIdx.x % kXcdCount;
  const int r = blockIdx.x / kXcdCount;
  const int vt = r % vtiles;
  const int gt = (r / vtiles) * kXcdCount + xcd;
  if (gt >= gtiles) return;
  const int a0 = vt * TV;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int gw = gt * kApplyG + wave * 32;  // this wave's strip: plane waves gw .. gw + 31
  const double2 zero = make_double2(0.0, 0.0);
  // B operand rows: psi[i][gw + 16 h + col] for i = i0 + kq
  const int gb0 = gw + col, gb1 = gw + 16 + col;
  const bool in0 = gb0 < npw, in1 = gb1 < npw;
  const int gc0 = min(gb0, npw - 1), gc1 = min(gb1, npw - 1);  // clamped: loads stay in range
  d4 re[MV][2], im[MV][2];
#pragma unroll
  for (int n = 0; n < MV; ++n)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      re[n][h] = d4{0.0, 0.0, 0.0, 0.0};
      im[n][h] = d4{0.0, 0.0, 0.0, 0.0};
    }
  for (int ib = 0; ib < n_occ; ib += kApplyKB) {
    const int kb = min(kApplyKB, n_occ - ib);
    __syncthreads();  // the previous block's C is no longer read
    for (int e = tid; e < TV * kApplyKB; e += 256) {
      const int v = e / kApplyKB, i = e - v * kApplyKB;
      const int ic = ib + min(i, kb - 1);
      double2 t = cp[(long)min(a0 + v, n_vec - 1) * n_occ + ic];
      if (row_scale) {
        const double sc = row_scale[ic];
        t = make_double2(t.x * sc, t.y * sc);
      }
      cs[v][i] = keep_if(a0 + v < n_vec && i < kb, t);
    }
    __syncthreads();
    const int nks = (kb + 3) / 4;
    // Psi operands of kApplyPre K-steps per group; the next group's loads are issued before the
    // current group's MFMAs, and out-of-range values are zeroed only at use
    double2 pc[kApplyPre][2], pn[kApplyPre][2];
#pragma unroll
    for (int s = 0; s < kApplyPre; ++s) {
      const double2 *pr = psi + (long)min(ib + 4 * s + kq, n_occ - 1) * npw;
      pn[s][0] = pr[gc0];
      pn[s][1] = pr[gc1];
    }
    for (int k0 = 0; k0 < nks; k0 += kApplyPre) {
#pragma unroll
      for (int s = 0; s < kApplyPre; ++s) {
        pc[s][0] = pn[s][0];
        pc[s][1] = pn[s][1];
      }
      if (k0 + kApplyPre < nks) {
#pragma unroll
        for (int s = 0; s < kApplyPre; ++s) {
          const double2 *pr = psi + (long)min(ib + 4 * (k0 + kApplyPre + s) + kq, n_occ - 1) * npw;
          pn[s][0] = pr[gc0];
          pn[s][1] = pr[gc1];
        }
      }
#pragma unroll
      for (int s = 0; s < kApplyPre; ++s) {
        const int kk = 4 * (k0 + s) + kq;  // past kb: C is zero in LDS and Psi is zeroed here
        const bool iv = kk < kb;
        const double2 p0 = keep_if(iv && in0, pc[s][0]), p1 = keep_if(iv && in1, pc[s][1]);
        double2 A[MV];
#pragma unroll
        for (int n = 0; n < MV; ++n) A[n] = cs[16 * n + col][kk < kApplyKB ? kk : 0];
#pragma unroll
        for (int n = 0; n < MV; ++n) {
          re[n][0] = mfma(A[n].x, p0.x, re[n][0]);
          im[n][0] = mfma(A[n].x, p0.y, im[n][0]);
          re[n][1] = mfma(A[n].x, p1.x, re[n][1]);
          im[n][1] = mfma(A[n].x, p1.y, im[n][1]);
        }
#pragma unroll
        for (int n = 0; n < MV; ++n) {
          re[n][0] = mfma(-A[n].y, p0.y, re[n][0]);
          im[n][0] = mfma(A[n].y, p0.x, im[n][0]);
          re[n][1] = mfma(-A[n].y, p1.y, re[n][1]);
          im[n][1] = mfma(A[n].y, p1.x, im[n][1]);
        }
      }
    }
  }
  // lane holds vectors a0 + 16 n + kq + 4 e at plane wave gw + 16 h + col
#pragma unroll
  for (int n = 0; n < MV; ++n)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = a0 + 16 * n + kq + 4 * e;
      if (a >= n_vec) continue;
      const double2 *src = mode == 0 ? x.ptr(a) : y + (long)a * ldy;
      double2 *dst = y + (long)a * ldy;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int g = gw + 16 * h + col;
        if (g >= npw) continue;
        const double2 old = src[g];
        dst[g] = mode == 0 ? make_double2(old.x - re[n][h][e], old.y - im[n][h][e])
                           : make_double2(fma(alpha, re[n][h][e], old.x), fma(alpha, im[n][h][e], old.y));
      }
    }
}

// vector tile width of the overlaps with the least padding for n_vec vectors (ties: the wider tile)
inline int vec_tile(int n_vec) {
  const int p64 = (n_vec + 63) / 64 * 64, p32 = (n_vec + 31) / 32 * 32;
  return p64 <= p32 ? 64 : 32;
}

}  // namespace

int proj_chunks(int npw, int *kc) {
  *kc = kProjChunkLen;
  const int n = (npw + kProjChunkLen - 1) / kProjChunkLen;
  return n < 1 ? 1 : n;
}

sgw_status proj_dot(sgw_ctx *ctx, int npw, int n_occ, const double2 *psi, int n_vec, VecSrc x, double2 *cp,
                    long rows, int kid) {
  if (n_vec <= 0 || n_occ <= 0) return SGW_OK;
  int kc;
  const int nch = proj_chunks(npw, &kc);
  if (nch > kProjChunks) return fail(SGW_ERR_UNSUPPORTED, "projector: too many plane waves for the overlap chunks");
  // 64-row occupied tiles reuse each staged vector twice as often; 32-row tiles give twice the
  // workgroups, which pays while a launch has fewer than ~4 per CU (no vector's arithmetic depends
  // on the tiles)
  const int tv = vec_tile(n_vec);
  const int vtiles = (n_vec + tv - 1) / tv;
  const int to = (n_occ <= 32 || (long)((n_occ + 63) / 64) * vtiles * nch < 1024) ? 32 : 64;
  const int otiles = (n_occ + to - 1) / to;
  const long groups = (long)((nch + kXcdCount - 1) / kXcdCount) * otiles * vtiles * kXcdCount;
  PendingTiming tm;
  timing_begin(ctx, kid, n_vec * (npw * 16.0) + (double)n_occ * npw * 16.0, 8.0 * n_vec * npw * n_occ, &tm);
#define SGW_DOT(TO, TV)                                                                                       \
  hipLaunchKernelGGL((k_proj_dot<TO, TV>), dim3(groups), dim3(256), 0, ctx->stream, npw, n_occ, psi, x, n_vec, \
                     nch, cp, rows, otiles, vtiles)
  if (to == 32) {
    if (tv == 32) SGW_DOT(32, 32);
    else SGW_DOT(32, 64);
  } else {
    if (tv == 32) SGW_DOT(64, 32);
    else SGW_DOT(64, 64);
  }
#undef SGW_DOT
  if (nch > 1) {
    const long ne = (long)n_vec * n_occ;
    hipLaunchKernelGGL(k_proj_reduce, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, cp, rows, n_vec, n_occ, nch);
  }
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status proj_apply(sgw_ctx *ctx, int npw, int n_occ, const double2 *psi, int n_vec, VecSrc x, const double2 *cp,
                      long rows, double2 *y, long ldy, double alpha, int mode, const double *row_scale, int kid) {
  if (n_vec <= 0) return SGW_OK;
  if (n_occ <= 0) {
    if (mode == 1) return SGW_OK;
    // y = x: nothing to subtract
    return permute_copy(ctx, npw, n_vec, x, y, ldy);
  }
  constexpr int tv = 32;
  const int vtiles = (n_vec + tv - 1) / tv;
  const int gtiles = (npw + kApplyG - 1) / kApplyG;
  const long groups = (long)((gtiles + kXcdCount - 1) / kXcdCount) * vtiles * kXcdCount;
  PendingTiming tm;
  timing_begin(ctx, kid, n_vec * (npw * 32.0) + (double)n_occ * npw * 16.0, 8.0 * n_vec * npw * n_occ, &tm);
  hipLaunchKernelGGL(k_proj_apply<tv>, dim3(groups), dim3(256), 0, ctx->stream, npw, n_occ, psi, x, n_vec, cp, y,
                     ldy, alpha, mode, row_scale, gtiles, vtiles);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

}  // namespace sgw
