// Occupied-manifold projector on the FP64 matrix cores (Sec. 2.3, Eqs. 7-8).
//
//   overlaps:  C[a][i] = sum_g conj(psi[i][g]) x_a[g]      (n_occ x n_vec, K = n_pw)
//   apply:     y_a[g]  = x_a[g] - sum_i psi[i][g] C[a][i]   (mode 0: 1 - P_occ)
//              y_a[g] += alpha sum_i psi[i][g] C[a][i]     (mode 1: + alpha P_occ)
//
// Both are complex GEMMs done as four real 16x16x4 FP64 MFMAs per step
// (re*re, im*im, re*im, im*re).  One wavefront owns a 16 x 16 output tile:
// in the overlap kernel rows are occupied states and columns are vectors, in
// the apply kernel rows are plane waves and columns are vectors.  The overlap
// reduction over plane waves is split into chunks (one workgroup per chunk and
// vector tile, its four waves splitting the chunk again and reducing through
// LDS); a second pass adds the chunk partials in a fixed order into chunk 0,
// so the result is deterministic and consumers read one complete overlap.
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

constexpr int kOccTilesMax = 4;  // occupied tiles (of 16) held in accumulators per pass
constexpr int kDotWaves = 4;
constexpr int kDotDepth = 4;     // K-steps of operands kept in flight per wave

// grid: vtiles x n_chunks x occ passes, block: kDotWaves wavefronts
template <int NOT>
__global__ __launch_bounds__(64 * kDotWaves) void k_proj_dot(int npw, int n_occ, const double2 *__restrict__ psi,
                                                             VecSrc x, int n_vec, int kc, int n_chunks,
                                                             double2 *__restrict__ cp, long rows, int vtiles) {
  __shared__ d4 red[kDotWaves - 1][2][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  int b = blockIdx.x;
  const int vt = b % vtiles;
  b /= vtiles;
  const int chunk = b % n_chunks;
  const int pass = b / n_chunks;
  const int occ0 = pass * NOT * 16;
  const int a = vt * 16 + col;
  const bool va = a < n_vec;
  const double2 *xv = va ? x.ptr(a) : nullptr;
  // this wave's share of the chunk, in steps of 4 plane waves
  const int c0 = chunk * kc, c1 = min(npw, c0 + kc);
  const int nsteps = (c1 - c0 + 3) / 4;
  const int sper = (nsteps + kDotWaves - 1) / kDotWaves;
  const int g0 = c0 + 4 * min(nsteps, wave * sper);
  const int g1 = min(c1, c0 + 4 * min(nsteps, (wave + 1) * sper));
  d4 re[NOT], im[NOT];
#pragma unroll
  for (int t = 0; t < NOT; ++t) {
    re[t] = d4{0.0, 0.0, 0.0, 0.0};
    im[t] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const double2 *prow[NOT];
  bool vrow[NOT];
#pragma unroll
  for (int t = 0; t < NOT; ++t) {
    const int i = occ0 + t * 16 + col;
    vrow[t] = i < n_occ;
    prow[t] = psi + (long)(vrow[t] ? i : 0) * npw;
  }
  // ring of kDotDepth steps of operands
  double2 xr[kDotDepth], pr[kDotDepth][NOT];
  auto load = [&](int g, int slot) {
    const int gg = g + kq;
    const bool in = gg < g1;
    xr[slot] = (va && in) ? xv[gg] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < NOT; ++t) pr[slot][t] = (vrow[t] && in) ? prow[t][gg] : make_double2(0.0, 0.0);
  };
#pragma unroll
  for (int d = 0; d < kDotDepth; ++d) load(g0 + 4 * d, d);
  for (int g = g0; g < g1; g += 4 * kDotDepth) {
#pragma unroll
    for (int d = 0; d < kDotDepth; ++d) {
      const double2 xc = xr[d];
#pragma unroll
      for (int t = 0; t < NOT; ++t) {
        const double2 pc = pr[d][t];
        re[t] = mfma(pc.x, xc.x, re[t]);
        im[t] = mfma(pc.x, xc.y, im[t]);
        re[t] = mfma(pc.y, xc.y, re[t]);
        im[t] = mfma(-pc.y, xc.x, im[t]);
      }
      load(g + 4 * (d + kDotDepth), d);
    }
  }
  // reduce the waves' partial tiles through LDS, one occupied tile at a time
  double2 *out = cp + ((long)chunk * rows + (va ? a : 0)) * n_occ;
#pragma unroll
  for (int t = 0; t < NOT; ++t) {
    if (wave > 0) {
      red[wave - 1][0][lane] = re[t];
      red[wave - 1][1][lane] = im[t];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int w = 0; w < kDotWaves - 1; ++w) {
        re[t] += red[w][0][lane];
        im[t] += red[w][1][lane];
      }
      if (va) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = occ0 + t * 16 + kq + 4 * r;
          if (i < n_occ) out[i] = make_double2(re[t][r], im[t][r]);
        }
      }
    }
    __syncthreads();
  }
}

// cp[0][a][i] = sum over chunks c of cp[c][a][i], in chunk order
__global__ __launch_bounds__(256) void k_proj_reduce(double2 *__restrict__ cp, long rows, int n_vec, int n_occ,
                                                   int n_chunks) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n_vec * n_occ) return;
  const int a = (int)(e / n_occ), i = (int)(e - (long)a * n_occ);
  double2 part[kProjChunks];
#pragma unroll
  for (int c = 0; c < kProjChunks; ++c)
    part[c] = c < n_chunks ? cp[((long)c * rows + a) * n_occ + i] : make_double2(0.0, 0.0);
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int c = 0; c < kProjChunks; ++c) s = c_add(s, part[c]);
  cp[(long)a * n_occ + i] = s;
}

constexpr int kApplyWaves = 4;
constexpr int kApplyG = 256;   // plane waves per block (each wave: kApplyG / kApplyWaves / 16 tiles)
constexpr int kApplyBatch = 4; // occupied K-steps whose operands are loaded before their MFMAs

// grid: vtiles x gtiles, block: kApplyWaves wavefronts; dynamic LDS: 16 * n_occ complex
__global__ __launch_bounds__(64 * kApplyWaves) void k_proj_apply(int npw, int n_occ, const double2 *__restrict__ psi,
                                                                VecSrc x, int n_vec, const double2 *__restrict__ cp,
                                                                double2 *__restrict__ y, long ldy, double alpha,
                                                                int mode, int vtiles) {
  extern __shared__ double2 cs[];  // [16][n_occ]: C of the tile's vectors
  const int vt = blockIdx.x % vtiles;
  const int gt = blockIdx.x / vtiles;
  const int a0 = vt * 16;
  for (int e = threadIdx.x; e < 16 * n_occ; e += 64 * kApplyWaves) {
    const int v = e / n_occ;
    cs[e] = a0 + v < n_vec ? cp[(long)a0 * n_occ + e] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int a = a0 + col;
  const bool va = a < n_vec;
  const double2 *xa = (va && mode == 0) ? x.ptr(a) : nullptr;
  double2 *ya = y + (long)(va ? a : 0) * ldy;
  const double2 *src = mode == 0 ? xa : ya;  // the values this lane updates
  for (int sub = wave; sub < kApplyG / 16; sub += kApplyWaves) {
    const int gb = gt * kApplyG + sub * 16;
    if (gb >= npw) break;
    // loaded before the products, so that their latency overlaps the MFMAs
    double2 old[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int g = gb + kq + 4 * r;
      old[r] = make_double2(0.0, 0.0);
      if (va && g < npw) old[r] = src[g];
    }
    d4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
    const int ga = gb + col;  // A operand row (plane wave) of this lane
    const bool gin = ga < npw;
    for (int i0 = 0; i0 < n_occ; i0 += 4 * kApplyBatch) {
      double2 p[kApplyBatch], c[kApplyBatch];
#pragma unroll
      for (int s = 0; s < kApplyBatch; ++s) {
        const int i = i0 + 4 * s + kq;
        p[s] = (i < n_occ && gin) ? psi[(long)i * npw + ga] : make_double2(0.0, 0.0);
        c[s] = (i < n_occ) ? cs[col * n_occ + i] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int s = 0; s < kApplyBatch; ++s) {
        re = mfma(p[s].x, c[s].x, re);
        im = mfma(p[s].x, c[s].y, im);
        re = mfma(-p[s].y, c[s].y, re);
        im = mfma(p[s].y, c[s].x, im);
      }
    }
    if (!va) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int g = gb + kq + 4 * r;
      if (g < npw)
        ya[g] = mode == 0 ? make_double2(old[r].x - re[r], old[r].y - im[r])
                          : make_double2(fma(alpha, re[r], old[r].x), fma(alpha, im[r], old[r].y));
    }
  }
}

}  // namespace

int proj_chunks(int npw, int *kc) {
  int n = (npw + 255) / 256;
  n = n < 1 ? 1 : (n > kProjChunks ? kProjChunks : n);
  int k = (npw + n - 1) / n;
  k = (k + 3) / 4 * 4;
  *kc = k;
  return (npw + k - 1) / k;
}

sgw_status proj_dot(sgw_ctx *ctx, int npw, int n_occ, const double2 *psi, int n_vec, VecSrc x, double2 *cp,
                    long rows) {
  if (n_vec <= 0 || n_occ <= 0) return SGW_OK;
  int kc;
  const int nch = proj_chunks(npw, &kc);
  const int vtiles = (n_vec + 15) / 16;
  const int otiles = (n_occ + 15) / 16;
  int not_ = 1;
  while (not_ < otiles && not_ < kOccTilesMax) not_ *= 2;
  const int passes = (otiles + not_ - 1) / not_;
  PendingTiming tm;
  timing_begin(ctx, K_PROJ_DOT, n_vec * (npw * 16.0) + (double)n_occ * npw * 16.0, 8.0 * n_vec * npw * n_occ, &tm);
  const dim3 grid((long)vtiles * nch * passes), block(64 * kDotWaves);
#define SGW_DOT(NOT)                                                                                           \
  hipLaunchKernelGGL(k_proj_dot<NOT>, grid, block, 0, ctx->stream, npw, n_occ, psi, x, n_vec, kc, nch, cp, rows, \
                     vtiles)
  switch (not_) {
    case 1: SGW_DOT(1); break;
    case 2: SGW_DOT(2); break;
    case 4: SGW_DOT(4); break;
    default: SGW_DOT(8); break;
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
                      long rows, double2 *y, long ldy, double alpha, int mode) {
  if (n_vec <= 0) return SGW_OK;
  if (n_occ <= 0) {
    if (mode == 1) return SGW_OK;
    // y = x: nothing to subtract
    return permute_copy(ctx, npw, n_vec, x, y, ldy);
  }
  const int vtiles = (n_vec + 15) / 16;
  const int gtiles = (npw + kApplyG - 1) / kApplyG;
  PendingTiming tm;
  timing_begin(ctx, K_PROJ_APPLY, n_vec * (npw * 32.0) + (double)n_occ * npw * 16.0, 8.0 * n_vec * npw * n_occ, &tm);
  hipLaunchKernelGGL(k_proj_apply, dim3((long)vtiles * gtiles), dim3(64 * kApplyWaves), sizeof(double2) * 16 * n_occ,
                     ctx->stream, npw, n_occ, psi, x, n_vec, cp, y, ldy, alpha, mode, vtiles);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

}  // namespace sgw
