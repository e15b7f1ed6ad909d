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

// ---------------------------------------------------------------------------
// Split-BF16 variant (the FP32-potential phase of mixed-precision solves).
//
// Every FP64 operand value v is written as three BF16 terms, v ~ h + m + l
// (h = bf16(v), m = bf16(v - h), l = bf16(v - h - m); the differences are exact
// in FP64), and a real product a b as the six largest term products
// ah bh + ah bm + am bh + ah bl + am bm + al bh: the dropped ones are below
// 2^-24 relative, so the contraction carries FP32-level accuracy at BF16
// matrix-core rates (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
// The occupied states are split once per solve into two layouts (a row-major one
// for the overlaps' A operand, a transposed one for the apply's B operand);
// x and C are split as they are loaded.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (wave64): lane l supplies
// A[l % 16][8 q + j] and B[8 q + j][l % 16], q = l / 16, j = 0..7 (one 16-byte
// vector each); it receives D[4 q + r][l % 16] in accumulator element r.
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// three-term BF16 split of one value
__device__ __forceinline__ void split3(double v, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = (__bf16)(float)v;
  const double r = v - (double)(float)h;
  m = (__bf16)(float)r;
  l = (__bf16)(float)(r - (double)(float)m);
}

// the split of 8 complex values into (term, component) vectors: t[2 k + c], k = h/m/l, c = re/im
__device__ __forceinline__ void split8(const double2 (&v)[8], bf8 (&t)[6]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    __bf16 h, m, l;
    split3(v[j].x, h, m, l);
    t[0][j] = h;
    t[2][j] = m;
    t[4][j] = l;
    split3(v[j].y, h, m, l);
    t[1][j] = h;
    t[3][j] = m;
    t[5][j] = l;
  }
}

// acc += a b over the six largest term products; a[k], b[k]: term k of one real operand
__device__ __forceinline__ f4 mfma_split(const bf8 &ah, const bf8 &am, const bf8 &al, const bf8 &bh, const bf8 &bm,
                                         const bf8 &bl, f4 acc) {
  acc = mfma_bf(al, bh, acc);
  acc = mfma_bf(am, bm, acc);
  acc = mfma_bf(ah, bl, acc);
  acc = mfma_bf(am, bh, acc);
  acc = mfma_bf(ah, bm, acc);
  return mfma_bf(ah, bh, acc);
}

constexpr int kBfKPad = 32;     // plane waves of the row-major split / occupied of the transposed one
constexpr int kBfStrip = 64;    // plane waves per wave in the apply (four 16-wide column tiles)

__global__ __launch_bounds__(256) void k_split_psi(int npw, int n_occ, const double2 *__restrict__ psi,
                                                   __bf16 *__restrict__ rowb, __bf16 *__restrict__ colb, int occ_r,
                                                   int npw_r, int npw_c, int occ_c) {
  // rowb[t][c][i][g] over i < occ_r, g < npw_r;  colb[t][c][g][i] over g < npw_c, i < occ_c
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long n_row = (long)occ_r * npw_r, n_col = (long)npw_c * occ_c;
  if (e < n_row) {
    const int i = (int)(e / npw_r), g = (int)(e - (long)i * npw_r);
    const double2 v = (i < n_occ && g < npw) ? psi[(long)i * npw + g] : make_double2(0.0, 0.0);
    __bf16 h, m, l;
    split3(v.x, h, m, l);
    rowb[0 * n_row + e] = h;
    rowb[2 * n_row + e] = m;
    rowb[4 * n_row + e] = l;
    split3(v.y, h, m, l);
    rowb[1 * n_row + e] = h;
    rowb[3 * n_row + e] = m;
    rowb[5 * n_row + e] = l;
  }
  if (e < n_col) {
    const int g = (int)(e / occ_c), i = (int)(e - (long)g * occ_c);
    const double2 v = (i < n_occ && g < npw) ? psi[(long)i * npw + g] : make_double2(0.0, 0.0);
    __bf16 h, m, l;
    split3(v.x, h, m, l);
    colb[0 * n_col + e] = h;
    colb[2 * n_col + e] = m;
    colb[4 * n_col + e] = l;
    split3(v.y, h, m, l);
    colb[1 * n_col + e] = h;
    colb[3 * n_col + e] = m;
    colb[5 * n_col + e] = l;
  }
}

// overlaps, split BF16: grid = ceil(n_chunks / 8) * (passes * vgroups) * 8 workgroups of 256 threads;
// a wave owns 16 vectors x MO row tiles of one pass over one chunk; the partials go to cp as FP64
template <int MO>
__global__ __launch_bounds__(256) void k_proj_dot_bf(int npw, int n_occ, const __bf16 *__restrict__ rowb, int occ_r,
                                                     int npw_r, VecSrc x, int n_vec, int n_chunks,
                                                     double2 *__restrict__ cp, long rows, int passes, int vgroups) {
  const int xcd = blockIdx.x % kXcdCount;
  const int r = blockIdx.x / kXcdCount;
  const int ntile = passes * vgroups;
  const int t = r % ntile;
  const int chunk = (r / ntile) * kXcdCount + xcd;
  if (chunk >= n_chunks) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, q = lane >> 4;
  const int i0 = (t / vgroups) * (16 * MO);
  const int a = (t % vgroups) * 64 + wave * 16 + col;  // this lane's vector (B operand column)
  const bool aok = a < n_vec;
  const double2 *xr = x.ptr(min(a, n_vec - 1));
  const int g_begin = chunk * kProjChunkLen;
  const int g_end = min(npw, g_begin + kProjChunkLen);
  const long plane = (long)occ_r * npw_r;  // one (term, component) array of the row-major split
  f4 re[MO], ima[MO], imb[MO];
#pragma unroll
  for (int m = 0; m < MO; ++m) {
    re[m] = f4{0.f, 0.f, 0.f, 0.f};
    ima[m] = f4{0.f, 0.f, 0.f, 0.f};
    imb[m] = f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int g0 = g_begin; g0 < g_end; g0 += 32) {
    const int gq = g0 + 8 * q;
    double2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = xr[min(gq + j, g_end - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = keep_if(aok && gq + j < g_end, v[j]);
    bf8 b[6];
    split8(v, b);
#pragma unroll
    for (int m = 0; m < MO; ++m) {
      const int i = i0 + 16 * m + col;  // A operand row (occupied state), always inside the padded split
      const __bf16 *pa = rowb + (long)i * npw_r + gq;
      bf8 A[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) A[k] = *(const bf8 *)(pa + k * plane);
      // conj(psi) x: re += pr xr + pi xi ; im += pr xi - pi xr
      re[m] = mfma_split(A[0], A[2], A[4], b[0], b[2], b[4], re[m]);
      re[m] = mfma_split(A[1], A[3], A[5], b[1], b[3], b[5], re[m]);
      ima[m] = mfma_split(A[0], A[2], A[4], b[1], b[3], b[5], ima[m]);
      imb[m] = mfma_split(A[1], A[3], A[5], b[0], b[2], b[4], imb[m]);
    }
  }
  // lane holds rows i0 + 16 m + 4 q + e of vector a
  if (!aok) return;
  double2 *out = cp + (long)chunk * rows * n_occ + (long)a * n_occ;
#pragma unroll
  for (int m = 0; m < MO; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + 16 * m + 4 * q + e;
      if (i < n_occ) out[i] = make_double2((double)re[m][e], (double)ima[m][e] - (double)imb[m][e]);
    }
}

// apply, split BF16: grid = ceil(strips / 8) * vgroups * 8 workgroups of 256 threads; a wave owns
// 16 vectors (A operand rows: C) x 64 plane waves (four column tiles: the transposed split of psi)
__global__ __launch_bounds__(256) void k_proj_apply_bf(int npw, int n_occ, const __bf16 *__restrict__ colb, int npw_c,
                                                       int occ_c, VecSrc x, int n_vec, const double2 *__restrict__ cp,
                                                       double2 *__restrict__ y, long ldy, double alpha, int mode,
                                                       int strips, int vgroups) {
  const int xcd = blockIdx.x % kXcdCount;
  const int r = blockIdx.x / kXcdCount;
  const int vg = r % vgroups;
  const int st = (r / vgroups) * kXcdCount + xcd;
  if (st >= strips) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, q = lane >> 4;
  const int g0 = st * (4 * kBfStrip) + wave * kBfStrip;  // this wave's 64 plane waves
  if (g0 >= npw) return;
  const int a0 = vg * 16;
  const int aA = min(a0 + col, n_vec - 1);  // A operand row: vector a0 + col (clamped; zeroed below)
  const bool aok = a0 + col < n_vec;
  const double2 *crow = cp + (long)aA * n_occ;
  const long plane = (long)npw_c * occ_c;
  f4 rea[4], reb[4], im[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    rea[n] = f4{0.f, 0.f, 0.f, 0.f};
    reb[n] = f4{0.f, 0.f, 0.f, 0.f};
    im[n] = f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int k0 = 0; k0 < n_occ; k0 += 32) {
    const int iq = k0 + 8 * q;
    double2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = crow[min(iq + j, n_occ - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = keep_if(aok && iq + j < n_occ, v[j]);
    bf8 A[6];
    split8(v, A);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int g = g0 + 16 * n + col;  // B operand column (plane wave), inside the padded split
      const __bf16 *pb = colb + (long)g * occ_c + iq;
      bf8 B[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) B[k] = *(const bf8 *)(pb + k * plane);
      // C psi: re += cr pr - ci pi ; im += cr pi + ci pr
      rea[n] = mfma_split(A[0], A[2], A[4], B[0], B[2], B[4], rea[n]);
      reb[n] = mfma_split(A[1], A[3], A[5], B[1], B[3], B[5], reb[n]);
      im[n] = mfma_split(A[0], A[2], A[4], B[1], B[3], B[5], im[n]);
      im[n] = mfma_split(A[1], A[3], A[5], B[0], B[2], B[4], im[n]);
    }
  }
  // lane holds vectors a0 + 4 q + e at plane wave g0 + 16 n + col
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int a = a0 + 4 * q + e;
    if (a >= n_vec) continue;
    const double2 *src = mode == 0 ? x.ptr(a) : y + (long)a * ldy;
    double2 *dst = y + (long)a * ldy;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int g = g0 + 16 * n + col;
      if (g >= npw) continue;
      const double pr = (double)rea[n][e] - (double)reb[n][e], pi = (double)im[n][e];
      const double2 old = src[g];
      dst[g] = mode == 0 ? make_double2(old.x - pr, old.y - pi) : make_double2(fma(alpha, pr, old.x), fma(alpha, pi, old.y));
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

namespace {
// row tiles per wave of the split overlaps, and the padded extents of the two split layouts: the
// row-major one holds whole passes of 16 * MO occupied rows (zero rows past n_occ) and whole 32-wide
// K steps of plane waves; the transposed one whole 256-wide apply strips and 32-wide K steps of
// occupied states
int split_mo(int n_occ) { return n_occ <= 64 ? 4 : 8; }
struct SplitDims {
  int occ_r, npw_r, npw_c, occ_c;
  size_t row_elems;  // elements of the row-major layout, rounded up to 256 bytes
};
SplitDims split_dims(int npw, int n_occ) {
  SplitDims d;
  const int rows = 16 * split_mo(n_occ);
  d.occ_r = (n_occ + rows - 1) / rows * rows;
  d.npw_r = (npw + kBfKPad - 1) / kBfKPad * kBfKPad;
  d.npw_c = (npw + 4 * kBfStrip - 1) / (4 * kBfStrip) * (4 * kBfStrip);
  d.occ_c = (n_occ + kBfKPad - 1) / kBfKPad * kBfKPad;
  d.row_elems = ((6 * (size_t)d.occ_r * d.npw_r * sizeof(__bf16) + 255) / 256 * 256) / sizeof(__bf16);
  return d;
}
}  // namespace

size_t proj_split_bytes(int npw, int n_occ) {
  if (n_occ <= 0) return 256;
  const SplitDims d = split_dims(npw, n_occ);
  return d.row_elems * sizeof(__bf16) + 6 * (size_t)d.npw_c * d.occ_c * sizeof(__bf16);
}

sgw_status proj_split(sgw_ctx *ctx, int npw, int n_occ, const double2 *psi, void *split) {
  if (n_occ <= 0) return SGW_OK;
  const SplitDims d = split_dims(npw, n_occ);
  __bf16 *rowb = (__bf16 *)split, *colb = rowb + d.row_elems;
  const long n = std::max((long)d.occ_r * d.npw_r, (long)d.npw_c * d.occ_c);
  hipLaunchKernelGGL(k_split_psi, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, npw, n_occ, psi, rowb, colb,
                     d.occ_r, d.npw_r, d.npw_c, d.occ_c);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status proj_dot_bf16(sgw_ctx *ctx, int npw, int n_occ, const void *split, int n_vec, VecSrc x, double2 *cp,
                         long rows) {
  if (n_vec <= 0 || n_occ <= 0) return SGW_OK;
  int kc;
  const int nch = proj_chunks(npw, &kc);
  if (nch > kProjChunks) return fail(SGW_ERR_UNSUPPORTED, "projector: too many plane waves for the overlap chunks");
  const SplitDims d = split_dims(npw, n_occ);
  const __bf16 *rowb = (const __bf16 *)split;
  const int mo = split_mo(n_occ);
  const int passes = (n_occ + 16 * mo - 1) / (16 * mo);
  const int vgroups = (n_vec + 63) / 64;
  const long groups = (long)((nch + kXcdCount - 1) / kXcdCount) * passes * vgroups * kXcdCount;
  PendingTiming tm;
  timing_begin(ctx, K_PROJ_DOT, n_vec * (npw * 16.0) + (double)n_occ * npw * 12.0, 8.0 * n_vec * npw * n_occ, &tm);
  if (mo == 4)
    hipLaunchKernelGGL(k_proj_dot_bf<4>, dim3(groups), dim3(256), 0, ctx->stream, npw, n_occ, rowb, d.occ_r, d.npw_r, x,
                       n_vec, nch, cp, rows, passes, vgroups);
  else
    hipLaunchKernelGGL(k_proj_dot_bf<8>, dim3(groups), dim3(256), 0, ctx->stream, npw, n_occ, rowb, d.occ_r, d.npw_r, x,
                       n_vec, nch, cp, rows, passes, vgroups);
  if (nch > 1) {
    const long ne = (long)n_vec * n_occ;
    hipLaunchKernelGGL(k_proj_reduce, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, cp, rows, n_vec, n_occ, nch);
  }
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

sgw_status proj_apply_bf16(sgw_ctx *ctx, int npw, int n_occ, const void *split, int n_vec, VecSrc x,
                           const double2 *cp, double2 *y, long ldy, double alpha, int mode) {
  if (n_vec <= 0) return SGW_OK;
  if (n_occ <= 0) {
    if (mode == 1) return SGW_OK;
    return permute_copy(ctx, npw, n_vec, x, y, ldy);
  }
  const SplitDims d = split_dims(npw, n_occ);
  const __bf16 *colb = (const __bf16 *)split + d.row_elems;
  const int strips = (npw + 4 * kBfStrip - 1) / (4 * kBfStrip);
  const int vgroups = (n_vec + 15) / 16;
  const long groups = (long)((strips + kXcdCount - 1) / kXcdCount) * vgroups * kXcdCount;
  PendingTiming tm;
  timing_begin(ctx, K_PROJ_APPLY, n_vec * (npw * 32.0) + (double)n_occ * npw * 12.0, 8.0 * n_vec * npw * n_occ, &tm);
  hipLaunchKernelGGL(k_proj_apply_bf, dim3(groups), dim3(256), 0, ctx->stream, npw, n_occ, colb, d.npw_c, d.occ_c, x,
                     n_vec, cp, y, ldy, alpha, mode, strips, vgroups);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

}  // namespace sgw
