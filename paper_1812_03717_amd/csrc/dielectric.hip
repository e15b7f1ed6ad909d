// Consumers of the linear variations: the density response to the plane-wave perturbations
// (Sec. 2.3, Eq. 5), the dielectric matrix (Eq. 4) and the correlation part of the screened
// interaction (Sec. 2.4, Eq. 9) with the bare or spherically truncated Coulomb potential
// (Sec. 2.6, Eq. 12).
//
// Density response.  The Fourier component q + G of 2 sum_v u_v^* (du_v(z) + du_v(-z)) per unit
// cell is, on the plane-wave bases, (2 / Omega) sum_v < exp(i (q+G) . r) u_v | du_{v,G'}(z) +
// du_{v,G'}(-z) >: a contraction over plane waves, no transform needed.  The variations have no
// occupied component, so the bra may be projected, and (1 - P_occ) exp(i (q+G) . r) u_v = -b_{v,G}
// is minus the right-hand side of the solves.  Per band this is the overlap contraction of the
// occupied projector with the n_pert right-hand sides in the place of the occupied states and the
// n_pert * n_omega variations as the vectors (FP64 matrix cores), accumulated over bands.
//
// Dielectric matrix and W_bar: eps_{GG'} = delta - chi_{GG'} v(q+G') (the perturbing charge's
// Coulomb potential on the columns), W_bar = v(q+G) (eps^{-1} - 1) (rows), one workgroup per
// frequency inverting eps in LDS by Gauss-Jordan elimination with partial pivoting.
#include <cmath>
#include <vector>

#include "fft_lds.h"
#include "sgw_internal.h"

namespace sgw {
namespace {

constexpr int kMaxDielectric = 64;  // largest n_G of the in-LDS inversion

struct Buf {
  void *p = nullptr;
  ~Buf() {
    if (p) hipFree(p);
  }
};

sgw_status alloc(Buf &b, size_t bytes) {
  SGW_HIP(hipMalloc(&b.p, std::max<size_t>(bytes, 256)));
  return SGW_OK;
}

// chi[j][g][h] (+)= scale * c[(h * n_omega + j) * n_g + g]   (c: overlaps of one band)
__global__ void k_chi_accum(const double2 *__restrict__ c, int n_g, int n_omega, double scale, double2 *__restrict__ chi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_omega * n_g * n_g) return;
  const int j = e / (n_g * n_g), r = e - j * n_g * n_g, g = r / n_g, h = r - g * n_g;
  const double2 t = c[((long)h * n_omega + j) * n_g + g];
  double2 o = chi[e];
  o.x = fma(scale, t.x, o.x);
  o.y = fma(scale, t.y, o.y);
  chi[e] = o;
}

__global__ void k_zero(double2 *__restrict__ p, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = make_double2(0.0, 0.0);
}

__device__ __forceinline__ double2 c_div1(double2 a) {  // 1 / a
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// one frequency per workgroup of 256 threads
__global__ __launch_bounds__(256) void k_dielectric(int n, const double2 *__restrict__ chi,
                                                    const double *__restrict__ v, const int32_t *__restrict__ zero_row,
                                                    double2 *__restrict__ eps, double2 *__restrict__ eps_inv,
                                                    double2 *__restrict__ wbar) {
  __shared__ double2 a[kMaxDielectric][kMaxDielectric + 1];
  __shared__ int piv[kMaxDielectric];
  __shared__ int p_row;
  const int j = blockIdx.x, tid = threadIdx.x;
  const long base = (long)j * n * n;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e / n, c = e - r * n;
    const double2 x = chi[base + e];
    double2 m = make_double2(-x.x * v[c], -x.y * v[c]);
    if (r == c) m.x += 1.0;
    a[r][c] = m;
    if (eps) eps[base + e] = m;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {  // pivot: the largest |a[r][k]|, r >= k (first on ties), by one wavefront
      double best = -1.0;
      int br = k;
      for (int r = k + tid; r < n; r += 64) {
        const double m = a[r][k].x * a[r][k].x + a[r][k].y * a[r][k].y;
        if (m > best) {
          best = m;
          br = r;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int orr = __shfl_xor(br, off);
        if (ob > best || (ob == best && orr < br)) {
          best = ob;
          br = orr;
        }
      }
      if (tid == 0) {
        p_row = br;
        piv[k] = br;
      }
    }
    __syncthreads();
    const int p = p_row;
    if (p != k)
      for (int c = tid; c < n; c += 256) {
        const double2 t = a[k][c];
        a[k][c] = a[p][c];
        a[p][c] = t;
      }
    __syncthreads();
    const double2 d = c_div1(a[k][k]);
    __syncthreads();  // every thread has read the pivot before row k changes
    for (int c = tid; c < n; c += 256) a[k][c] = c_mul(c == k ? make_double2(1.0, 0.0) : a[k][c], d);
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int r = e / n, c = e - r * n;
      if (r == k) continue;
      const double2 f = a[r][k];
      if (c == k) continue;
      a[r][c] = c_sub(a[r][c], c_mul(f, a[k][c]));
    }
    __syncthreads();
    for (int r = tid; r < n; r += 256)
      if (r != k) a[r][k] = c_mul(make_double2(-1.0, 0.0), c_mul(a[r][k], a[k][k]));
    __syncthreads();
  }
  // undo the row interchanges on the columns, last first
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int r = tid; r < n; r += 256) {
        const double2 t = a[r][k];
        a[r][k] = a[r][p];
        a[r][p] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += 256) {
    const int r = e / n, c = e - r * n;
    const double2 x = a[r][c];
    if (eps_inv) eps_inv[base + e] = x;
    if (wbar) {
      double2 w = make_double2(v[r] * (x.x - (r == c ? 1.0 : 0.0)), v[r] * x.y);
      if (r != c && (zero_row[r] || zero_row[c])) w = make_double2(0.0, 0.0);
      wbar[base + e] = w;
    }
  }
}

}  // namespace
}  // namespace sgw

using namespace sgw;

extern "C" sgw_status sgw_density_response(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                           const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, int n_pert,
                                           const int32_t *dv_miller, int n_omega, const sgw_c128 *dpsi_plus,
                                           const sgw_c128 *dpsi_minus, double weight, int accumulate,
                                           sgw_c128 *chi) {
  if (!ctx || !h_kq || !h_k) return fail(SGW_ERR_INVALID_ARG, "sgw_density_response: NULL context or Hamiltonian");
  if (n_occ < 0 || n_band < 0 || n_pert < 0 || n_omega < 0)
    return fail(SGW_ERR_INVALID_ARG, "sgw_density_response: negative size");
  if (!std::isfinite(weight)) return fail(SGW_ERR_INVALID_ARG, "sgw_density_response: weight not finite");
  const long nchi = (long)n_omega * n_pert * n_pert;
  if (nchi == 0) return SGW_OK;
  if (!chi || !dv_miller || !dpsi_plus || !dpsi_minus || (n_band > 0 && !psi_v))
    return fail(SGW_ERR_INVALID_ARG, "sgw_density_response: NULL array");
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_status st;
  if (!accumulate) {
    hipLaunchKernelGGL(k_zero, dim3((nchi + 255) / 256), dim3(256), 0, ctx->stream, (double2 *)chi, nchi);
    SGW_HIP(hipGetLastError());
  }
  if (n_band == 0) return sync(ctx);
  const int npw = h_kq->n_pw;
  // the right-hand sides b_{v,G} of every band (caller's order)
  Buf b, c;
  const long nb = (long)n_band * n_pert;
  if ((st = alloc(b, sizeof(double2) * (size_t)nb * npw)) != SGW_OK) return st;
  if ((st = sgw_build_rhs(ctx, h_kq, n_occ, psi_occ_kq, h_k, n_band, psi_v, n_pert, dv_miller, (sgw_c128 *)b.p)) !=
      SGW_OK)
    return st;
  const int nv = n_pert * n_omega;
  if ((st = alloc(c, sizeof(double2) * kProjChunks * (size_t)nv * n_pert)) != SGW_OK) return st;
  // chi = (2 w / Omega) sum_v <-b_{v,G} | du(z) + du(-z)>
  double bdet = 0;
  {
    const double(*B)[3] = h_kq->recip;
    bdet = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
           B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  }
  const double volume = std::pow(2.0 * M_PI, 3) / std::fabs(bdet);
  const double scale = -2.0 * weight / volume;
  for (int v = 0; v < n_band; ++v) {
    const double2 *bv = (const double2 *)b.p + (long)v * n_pert * npw;
    for (int side = 0; side < 2; ++side) {
      const double2 *xv = (const double2 *)(side == 0 ? dpsi_plus : dpsi_minus) + (long)v * nv * npw;
      if ((st = proj_dot(ctx, npw, n_pert, bv, nv, contiguous(xv, npw), (double2 *)c.p, nv, K_CHI_DOT)) != SGW_OK)
        return st;
      hipLaunchKernelGGL(k_chi_accum, dim3((nchi + 255) / 256), dim3(256), 0, ctx->stream, (const double2 *)c.p,
                         n_pert, n_omega, scale, (double2 *)chi);
      SGW_HIP(hipGetLastError());
    }
  }
  return sync(ctx);
}

extern "C" sgw_status sgw_coulomb(const sgw_ham *h_kq, const sgw_ham *h_k, int n_pert, const int32_t *dv_miller,
                                  double r_cut, double *v) {
  if (!h_kq || !h_k || (n_pert > 0 && (!dv_miller || !v)))
    return fail(SGW_ERR_INVALID_ARG, "sgw_coulomb: NULL argument");
  if (!std::isfinite(r_cut)) return fail(SGW_ERR_INVALID_ARG, "sgw_coulomb: r_cut not finite");
  for (int p = 0; p < n_pert; ++p) {
    double qg[3];
    for (int d = 0; d < 3; ++d) {
      qg[d] = h_kq->kvec[d] - h_k->kvec[d];
      for (int i = 0; i < 3; ++i) qg[d] += dv_miller[3 * p + i] * h_kq->recip[i][d];
    }
    const double k2 = qg[0] * qg[0] + qg[1] * qg[1] + qg[2] * qg[2];
    if (r_cut > 0.0) {
      const double k = std::sqrt(k2);
      v[p] = k2 == 0.0 ? 2.0 * M_PI * r_cut * r_cut : 4.0 * M_PI / k2 * (1.0 - std::cos(k * r_cut));
    } else {
      if (k2 == 0.0)
        return fail(SGW_ERR_INVALID_ARG, "sgw_coulomb: q + G = 0 for perturbation " + std::to_string(p) +
                                             " needs a truncated potential (r_cut > 0)");
      v[p] = 4.0 * M_PI / k2;
    }
  }
  return SGW_OK;
}

extern "C" sgw_status sgw_screened_coulomb(sgw_ctx *ctx, const sgw_ham *h_kq, const sgw_ham *h_k, int n_pert,
                                           const int32_t *dv_miller, double r_cut, int n_omega, const sgw_c128 *chi,
                                           sgw_c128 *eps, sgw_c128 *eps_inv, sgw_c128 *wbar) {
  if (!ctx || !h_kq || !h_k) return fail(SGW_ERR_INVALID_ARG, "sgw_screened_coulomb: NULL context or Hamiltonian");
  if (n_pert < 0 || n_omega < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_screened_coulomb: negative size");
  if (n_pert > kMaxDielectric)
    return fail(SGW_ERR_UNSUPPORTED, "sgw_screened_coulomb: more than " + std::to_string(kMaxDielectric) +
                                         " wave vectors");
  if (n_pert == 0 || n_omega == 0) return SGW_OK;
  if (!chi) return fail(SGW_ERR_INVALID_ARG, "sgw_screened_coulomb: NULL chi");
  std::vector<double> v(n_pert);
  sgw_status st;
  if ((st = sgw_coulomb(h_kq, h_k, n_pert, dv_miller, r_cut, v.data())) != SGW_OK) return st;
  std::vector<int32_t> zr(n_pert);
  for (int p = 0; p < n_pert; ++p) {
    double qg2 = 0;
    for (int d = 0; d < 3; ++d) {
      double x = h_kq->kvec[d] - h_k->kvec[d];
      for (int i = 0; i < 3; ++i) x += dv_miller[3 * p + i] * h_kq->recip[i][d];
      qg2 += x * x;
    }
    zr[p] = qg2 == 0.0;
  }
  SGW_HIP(hipSetDevice(ctx->device));
  Buf dv, dz;
  if ((st = alloc(dv, sizeof(double) * n_pert)) != SGW_OK) return st;
  if ((st = alloc(dz, sizeof(int32_t) * n_pert)) != SGW_OK) return st;
  SGW_HIP(hipMemcpyAsync(dv.p, v.data(), sizeof(double) * n_pert, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dz.p, zr.data(), sizeof(int32_t) * n_pert, hipMemcpyHostToDevice, ctx->stream));
  PendingTiming tm;
  // Gauss-Jordan: n^3 complex multiply-adds per matrix (8 flops each), the matrices read and written
  timing_begin(ctx, K_DIELECTRIC, 64.0 * n_omega * n_pert * n_pert, 8.0 * n_omega * (double)n_pert * n_pert * n_pert,
               &tm);
  hipLaunchKernelGGL(k_dielectric, dim3(n_omega), dim3(256), 0, ctx->stream, n_pert, (const double2 *)chi,
                     (const double *)dv.p, (const int32_t *)dz.p, (double2 *)eps, (double2 *)eps_inv, (double2 *)wbar);
  timing_end(ctx, &tm);
  SGW_HIP(hipGetLastError());
  return sync(ctx);
}
