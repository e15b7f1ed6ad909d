// Per-shift solves of (A0 - z) x = b (A0 = H - eps_v + alpha P_occ, Sec. 2.3,
// Eqs. 6-7) by BiCGStab with right preconditioning, x = M u, M diagonal in
// the plane-wave basis.  A preconditioner or a non-zero initial guess breaks
// the collinearity of the shifted residuals, so these solves cannot share one
// Krylov space; they serve the tail of a multishift run and the learned
// preconditioner.  One workgroup per system; the operator application is the
// batched FFT H.x plus the MFMA projector (driver), and these kernels add the
// shift and do the BiCGStab vector updates with fused reductions.
//
// Diagonal preconditioners:
//   Teter:   M_G = K(T_G / E_ref), K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4)
//            (Teter, Payne, Allan, Phys. Rev. B 40, 12255 (1989)), E_ref = <b|T|b>/<b|b>
//   learned: (m, g) from the MLP of each plane wave's features, M_G = m_G, x0 = g (.) b
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "fft_lds.h"
#include "pershift.h"
#include "reduce.h"

namespace sgw {
namespace {

constexpr int kPsThreads = 256;

__device__ __forceinline__ double2 cz(const PsState &S, int i) { return make_double2(S.eps[i] + S.zr[i], S.zi[i]); }
// (Y - (eps + z) u)_g
__device__ __forceinline__ double2 shifted(double2 y, double2 u, double2 ez) {
  return make_double2(y.x - (ez.x * u.x - ez.y * u.y), y.y - (ez.x * u.y + ez.y * u.x));
}
__device__ __forceinline__ double2 c_div(double2 a, double2 b) {
  const double d = 1.0 / (b.x * b.x + b.y * b.y);
  return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}
// conj(a) * b accumulated into acc[0..1]
__device__ __forceinline__ void cdot_acc(double2 a, double2 b, double *acc) {
  acc[0] = fma(a.x, b.x, fma(a.y, b.y, acc[0]));
  acc[1] = fma(a.x, b.y, fma(-a.y, b.x, acc[1]));
}

__global__ void k_ps_setup(PsState S, int n, const int32_t *__restrict__ list, const int32_t *__restrict__ sys,
                           const double *__restrict__ eps_band, const double *__restrict__ omega, double eta,
                           const double *__restrict__ eta_j, int n_pert, int n_omega) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int i = list[a], y = sys[a];
  const int pair = y / n_omega, j = y - pair * n_omega;
  S.out_index[i] = y;
  S.pair[i] = pair;
  S.eps[i] = eps_band[pair / n_pert];
  S.zr[i] = omega[j];
  S.zi[i] = eta_j ? eta_j[j] : eta;
  S.status[i] = PS_RUNNING;
  S.iters[i] = 0;
}

__global__ __launch_bounds__(kPsThreads) void k_ps_load_x(PsState S, const int32_t *__restrict__ list,
                                                         const double2 *__restrict__ dpsi) {
  const int i = list[blockIdx.x];
  const double2 *src = dpsi + (long)S.out_index[i] * S.npw;
  double2 *x = S.x + (long)i * S.npw;
  for (int g = threadIdx.x; g < S.npw; g += kPsThreads) x[g] = src[S.i2u[g]];
}

__global__ __launch_bounds__(kPsThreads) void k_ps_rhs(PsState S, const int32_t *__restrict__ list,
                                                      const double2 *__restrict__ src,
                                                      const double2 *__restrict__ proj) {
  __shared__ double sh[(kPsThreads / 64) * 2];
  const int a = blockIdx.x, i = list[a];
  const double2 *sv = src + (long)a * S.npw, *pv = proj + (long)a * S.npw;
  double2 *b = S.b + (long)i * S.npw;
  double acc[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < S.npw; g += kPsThreads) {
    const double2 p = pv[g], s = sv[g];
    b[g] = make_double2(-p.x, -p.y);
    acc[0] += p.x * p.x + p.y * p.y;
    acc[1] += s.x * s.x + s.y * s.y;
  }
  double tot[2];
  wg_sum<kPsThreads, 2>(acc, sh, tot);
  double nb = sqrt(tot[0]);
  if (!(nb > kZeroRhsRel * sqrt(tot[1])) && isfinite(nb)) {
    nb = 0.0;
    for (int g = threadIdx.x; g < S.npw; g += kPsThreads) b[g] = make_double2(0.0, 0.0);
  }
  if (threadIdx.x == 0) S.bnorm[i] = nb;
}

// M (and the initial guess) per system
__global__ __launch_bounds__(kPsThreads) void k_ps_precond(PsState S, const int32_t *__restrict__ list,
                                                          const double *__restrict__ kin, int mode,
                                                          const uint16_t *__restrict__ wb, int guess) {
  __shared__ double sh[(kPsThreads / 64) * 2];
  __shared__ float w[kMlpParams];
  const int a = blockIdx.x, i = list[a];
  const int npw = S.npw;
  const double2 *b = S.b + (long)i * npw;
  double2 *m = S.m + (long)i * npw;
  double2 *x = S.x + (long)i * npw;
  if (mode == PC_LEARNED) {
    for (int e = threadIdx.x; e < kMlpParams; e += kPsThreads) w[e] = __uint_as_float((uint32_t)wb[e] << 16);
    __syncthreads();
  }
  double eref = 1.0;
  if (mode == PC_TETER) {
    double acc[2] = {0.0, 0.0};
    for (int g = threadIdx.x; g < npw; g += kPsThreads) {
      const double2 bg = b[g];
      const double nb2 = bg.x * bg.x + bg.y * bg.y;
      acc[0] = fma(kin[g], nb2, acc[0]);
      acc[1] += nb2;
    }
    double tot[2];
    wg_sum<kPsThreads, 2>(acc, sh, tot);
    eref = tot[1] > 0.0 ? tot[0] / tot[1] : 1.0;
    if (!(eref > 0.0)) eref = 1.0;
  }
  const double eps = S.eps[i], om = S.zr[i], eta = S.zi[i];
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    double2 mg = make_double2(1.0, 0.0);
    double2 gg = make_double2(0.0, 0.0);
    if (mode == PC_TETER) {
      const double t = kin[g] / eref;
      const double num = 27.0 + t * (18.0 + t * (12.0 + t * 8.0));
      mg = make_double2(num / (num + 16.0 * t * t * t * t), 0.0);
    } else if (mode == PC_LEARNED) {
      float f[kMlpIn], h1[kMlpHid], o[kMlpOut];
      mlp_features(kin[g], eps, om, eta, f);
#pragma unroll
      for (int j = 0; j < kMlpHid; ++j) {
        float s = w[kMlpB1 + j];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) s = fmaf(w[kMlpW1 + j * kMlpIn + k], f[k], s);
        h1[j] = tanhf(s);
      }
#pragma unroll
      for (int q = 0; q < kMlpOut; ++q) o[q] = w[kMlpB3 + q];
      for (int j = 0; j < kMlpHid; ++j) {
        float s = w[kMlpB2 + j];
#pragma unroll
        for (int k = 0; k < kMlpHid; ++k) s = fmaf(w[kMlpW2 + j * kMlpHid + k], h1[k], s);
        const float h2 = tanhf(s);
#pragma unroll
        for (int q = 0; q < kMlpOut; ++q) o[q] = fmaf(w[kMlpW3 + q * kMlpHid + j], h2, o[q]);
      }
      const double sc = 1.0 / (kin[g] + 1.0);
      mg = make_double2(o[0] * sc, o[1] * sc);
      gg = make_double2(o[2] * sc, o[3] * sc);
    }
    m[g] = mg;
    if (guess == 0) x[g] = make_double2(0.0, 0.0);
    else if (guess == 1) x[g] = c_mul(gg, b[g]);
  }
}

__global__ __launch_bounds__(kPsThreads) void k_ps_start(PsState S, const int32_t *__restrict__ list,
                                                        const double2 *__restrict__ Y, int has_x0) {
  __shared__ double sh[(kPsThreads / 64) * 2];
  const int a = blockIdx.x, i = list[a];
  const int npw = S.npw;
  const double2 ez = cz(S, i);
  const double2 *b = S.b + (long)i * npw, *x = S.x + (long)i * npw, *y = Y + (long)a * npw;
  double2 *r = S.r + (long)i * npw, *rh = S.rh + (long)i * npw;
  double2 *p = S.p + (long)i * npw, *v = S.v + (long)i * npw;
  const double nb = S.bnorm[i];
  if (nb == 0.0) {
    double2 *xw = S.x + (long)i * npw;
    for (int g = threadIdx.x; g < npw; g += kPsThreads) xw[g] = make_double2(0.0, 0.0);
    has_x0 = 0;
  }
  double acc[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    double2 rg = b[g];
    if (has_x0) rg = c_sub(rg, shifted(y[g], x[g], ez));
    r[g] = rg;
    rh[g] = rg;
    p[g] = make_double2(0.0, 0.0);
    v[g] = make_double2(0.0, 0.0);
    acc[0] += rg.x * rg.x + rg.y * rg.y;
  }
  double tot[2];
  wg_sum<kPsThreads, 2>(acc, sh, tot);
  if (threadIdx.x == 0) {
    const double rn = sqrt(tot[0]);
    S.rnorm[i] = rn;
    S.rho_cur[i] = make_double2(tot[0], 0.0);
    S.rho_prev[i] = make_double2(1.0, 0.0);
    S.alph[i] = make_double2(1.0, 0.0);
    S.omg[i] = make_double2(1.0, 0.0);
    S.iters[i] = 0;
    int st = PS_RUNNING;
    if (nb == 0.0) st = PS_ZERO;
    else if (!isfinite(rn)) st = PS_NONFINITE;
    else if (rn <= S.tol * nb) st = PS_CONVERGED;
    S.status[i] = st;
  }
}

// p = r + beta (p - omega v), ph = M p
__global__ __launch_bounds__(kPsThreads) void k_ps_k1(PsState S, const int32_t *__restrict__ list) {
  const int i = list[blockIdx.x];
  if (S.status[i] != PS_RUNNING) return;
  const int npw = S.npw;
  const double2 om = S.omg[i];
  const double2 beta = c_mul(c_div(S.rho_cur[i], S.rho_prev[i]), c_div(S.alph[i], om));
  const double2 *r = S.r + (long)i * npw, *v = S.v + (long)i * npw, *m = S.m + (long)i * npw;
  double2 *p = S.p + (long)i * npw, *ph = S.ph + (long)i * npw;
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 pg = c_add(r[g], c_mul(beta, c_sub(p[g], c_mul(om, v[g]))));
    p[g] = pg;
    ph[g] = c_mul(m[g], pg);
  }
  __syncthreads();
  if (threadIdx.x == 0) S.rho_prev[i] = S.rho_cur[i];
}

// v = A ph; alpha = rho / <rh, v>; s = r - alpha v; sh = M s
__global__ __launch_bounds__(kPsThreads) void k_ps_k2(PsState S, const int32_t *__restrict__ list,
                                                     const double2 *__restrict__ Y) {
  __shared__ double sh_[(kPsThreads / 64) * 2];
  const int a = blockIdx.x, i = list[a];
  if (S.status[i] != PS_RUNNING) return;
  const int npw = S.npw;
  const double2 ez = cz(S, i);
  const double2 *y = Y + (long)a * npw, *ph = S.ph + (long)i * npw, *rh = S.rh + (long)i * npw;
  const double2 *r = S.r + (long)i * npw, *m = S.m + (long)i * npw;
  double2 *v = S.v + (long)i * npw, *s = S.s + (long)i * npw, *shv = S.sh + (long)i * npw;
  double acc[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 vg = shifted(y[g], ph[g], ez);
    v[g] = vg;
    cdot_acc(rh[g], vg, acc);
  }
  double tot[2];
  wg_sum<kPsThreads, 2>(acc, sh_, tot);
  const double2 sigma = make_double2(tot[0], tot[1]);
  const bool brk = !(sigma.x * sigma.x + sigma.y * sigma.y > 0.0);
  const double2 alpha = brk ? make_double2(0.0, 0.0) : c_div(S.rho_cur[i], sigma);
  double acc2[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 sg = c_sub(r[g], c_mul(alpha, v[g]));
    s[g] = sg;
    shv[g] = c_mul(m[g], sg);
    acc2[0] += sg.x * sg.x + sg.y * sg.y;
  }
  double tot2[2];
  wg_sum<kPsThreads, 2>(acc2, sh_, tot2);
  const double sn = sqrt(tot2[0]);
  const bool done = sn <= S.tol * S.bnorm[i];
  if (done) {
    double2 *x = S.x + (long)i * npw;
    for (int g = threadIdx.x; g < npw; g += kPsThreads) x[g] = c_add(x[g], c_mul(alpha, ph[g]));
  }
  if (threadIdx.x == 0) {
    S.alph[i] = alpha;
    if (brk) S.status[i] = PS_BREAKDOWN;
    else if (!isfinite(sn)) S.status[i] = PS_NONFINITE;
    else if (done) {
      S.status[i] = PS_CONVERGED;
      S.rnorm[i] = sn;
      S.iters[i] += 1;
    }
  }
}

// t = A sh; omega = <t, s> / <t, t>; x += alpha ph + omega sh; r = s - omega t
__global__ __launch_bounds__(kPsThreads) void k_ps_k3(PsState S, const int32_t *__restrict__ list,
                                                     const double2 *__restrict__ Y) {
  __shared__ double sh_[(kPsThreads / 64) * 3];
  const int a = blockIdx.x, i = list[a];
  if (S.status[i] != PS_RUNNING) return;
  const int npw = S.npw;
  const double2 ez = cz(S, i);
  const double2 *y = Y + (long)a * npw, *shv = S.sh + (long)i * npw, *s = S.s + (long)i * npw;
  const double2 *ph = S.ph + (long)i * npw, *rh = S.rh + (long)i * npw;
  double2 *x = S.x + (long)i * npw, *r = S.r + (long)i * npw;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 tg = shifted(y[g], shv[g], ez);
    cdot_acc(tg, s[g], acc);
    acc[2] += tg.x * tg.x + tg.y * tg.y;
  }
  double tot[3];
  wg_sum<kPsThreads, 3>(acc, sh_, tot);
  const bool brk = !(tot[2] > 0.0);
  const double2 om = brk ? make_double2(0.0, 0.0) : make_double2(tot[0] / tot[2], tot[1] / tot[2]);
  const double2 alpha = S.alph[i];
  double acc2[3] = {0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 tg = shifted(y[g], shv[g], ez);
    x[g] = c_add(x[g], c_add(c_mul(alpha, ph[g]), c_mul(om, shv[g])));
    const double2 rg = c_sub(s[g], c_mul(om, tg));
    r[g] = rg;
    cdot_acc(rh[g], rg, acc2);
    acc2[2] += rg.x * rg.x + rg.y * rg.y;
  }
  const int it = S.iters[i] + 1;  // read before the barriers of wg_sum; thread 0 updates it after them
  double tot2[3];
  wg_sum<kPsThreads, 3>(acc2, sh_, tot2);
  if (it == S.hist_iter && S.hist_r) {
    double2 *hr = S.hist_r + (long)S.out_index[i] * npw, *hx = S.hist_x + (long)S.out_index[i] * npw;
    for (int g = threadIdx.x; g < npw; g += kPsThreads) {
      const int u = S.i2u[g];
      hr[u] = r[g];
      hx[u] = x[g];
    }
  }
  if (threadIdx.x == 0) {
    const double rn = sqrt(tot2[2]);
    S.omg[i] = om;
    S.rho_cur[i] = make_double2(tot2[0], tot2[1]);
    S.rnorm[i] = rn;
    S.iters[i] = it;
    int st = PS_RUNNING;
    if (!isfinite(rn)) st = PS_NONFINITE;
    else if (rn <= S.tol * S.bnorm[i]) st = PS_CONVERGED;
    else if (brk || !(om.x * om.x + om.y * om.y > 0.0) || !(tot2[0] * tot2[0] + tot2[1] * tot2[1] > 0.0))
      st = PS_BREAKDOWN;
    else if (it >= S.max_iter) st = PS_MAXITER;
    S.status[i] = st;
  }
}

// true FP64 residual with Y = (H + alpha P_occ) x, dpsi and info
__global__ __launch_bounds__(kPsThreads) void k_ps_final(PsState S, const int32_t *__restrict__ list,
                                                        const double2 *__restrict__ Y,
                                                        const double2 *__restrict__ cp,
                                                        double2 *__restrict__ dpsi,
                                                        sgw_solve_info *__restrict__ info, int *__restrict__ n_bad,
                                                        int extra_flags) {
  __shared__ double sh_[(kPsThreads / 64) * 3];
  const int a = blockIdx.x, i = list[a];
  const int npw = S.npw;
  const double2 ez = cz(S, i);
  const double2 *y = Y + (long)a * npw, *x = S.x + (long)i * npw, *b = S.b + (long)i * npw;
  double2 *out = dpsi + (long)S.out_index[i] * npw;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += kPsThreads) {
    const double2 xg = x[g];
    const double2 rg = c_sub(b[g], shifted(y[g], xg, ez));
    acc[0] += rg.x * rg.x + rg.y * rg.y;
    acc[1] += xg.x * xg.x + xg.y * xg.y;
    out[S.i2u[g]] = xg;
  }
  double cc = 0.0;
  for (int o = threadIdx.x; o < S.n_occ; o += kPsThreads) {
    const double2 c = cp[(long)a * S.n_occ + o];
    cc += c.x * c.x + c.y * c.y;
  }
  acc[2] = cc;
  double tot[3];
  wg_sum<kPsThreads, 3>(acc, sh_, tot);
  if (threadIdx.x == 0) {
    const double nb = S.bnorm[i];
    const double rn = sqrt(tot[0]);
    const double relres = nb > 0.0 ? rn / nb : rn;
    const int st = S.status[i];
    int flags = extra_flags;
    if (st == PS_MAXITER) flags |= SGW_FLAG_MAXITER;
    if (st == PS_BREAKDOWN) flags |= SGW_FLAG_BREAKDOWN;
    if (st == PS_NONFINITE || !isfinite(relres)) flags |= SGW_FLAG_NONFINITE;
    if (st == PS_ZERO) flags |= SGW_FLAG_ZERO_RHS;
    if (relres <= S.tol_final && !(flags & SGW_FLAG_NONFINITE)) flags |= SGW_FLAG_CONVERGED;
    else atomicAdd(n_bad, 1);
    sgw_solve_info inf;
    inf.iters = S.iters[i];
    inf.flags = flags;
    inf.relres = relres;
    inf.occ_leak = tot[1] > 0.0 ? sqrt(tot[2] / tot[1]) : 0.0;
    info[S.out_index[i]] = inf;
  }
}

}  // namespace

#define SGW_PS_LAUNCH(kern, n, ...)                                                               \
  do {                                                                                            \
    if ((n) <= 0) return SGW_OK;                                                                  \
    hipLaunchKernelGGL(kern, dim3(n), dim3(kPsThreads), 0, ctx->stream, __VA_ARGS__);             \
    SGW_HIP(hipGetLastError());                                                                   \
    return SGW_OK;                                                                                \
  } while (0)

sgw_status ps_setup(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const int32_t *sys,
                    const double *eps_band, const double *omega, double eta, const double *eta_j, int n_pert,
                    int n_omega) {
  if (n <= 0) return SGW_OK;
  hipLaunchKernelGGL(k_ps_setup, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, S, n, list, sys, eps_band, omega,
                     eta, eta_j, n_pert, n_omega);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}
sgw_status ps_load_x(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *dpsi) {
  SGW_PS_LAUNCH(k_ps_load_x, n, S, list, dpsi);
}
sgw_status ps_rhs(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *src,
                  const double2 *proj) {
  SGW_PS_LAUNCH(k_ps_rhs, n, S, list, src, proj);
}
sgw_status ps_precond(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double *kin, int mode,
                      const sgw_mlp *mlp, int guess) {
  if (mode == PC_LEARNED && (!mlp || !mlp->wb)) return fail(SGW_ERR_INVALID_ARG, "learned preconditioner without MLP");
  const uint16_t *wb = mode == PC_LEARNED ? mlp->wb : nullptr;
  SGW_PS_LAUNCH(k_ps_precond, n, S, list, kin, mode, wb, guess);
}
sgw_status ps_start(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y, int has_x0) {
  SGW_PS_LAUNCH(k_ps_start, n, S, list, Y, has_x0);
}
sgw_status ps_k1(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list) { SGW_PS_LAUNCH(k_ps_k1, n, S, list); }
sgw_status ps_k2(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y) {
  SGW_PS_LAUNCH(k_ps_k2, n, S, list, Y);
}
sgw_status ps_k3(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y) {
  SGW_PS_LAUNCH(k_ps_k3, n, S, list, Y);
}
sgw_status ps_final(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y,
                    const double2 *cp, long rows, double2 *dpsi, sgw_solve_info *info, int *n_bad,
                    int extra_flags) {
  SGW_PS_LAUNCH(k_ps_final, n, S, list, Y, cp, dpsi, info, n_bad, extra_flags);
}

}  // namespace sgw

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
namespace sgw {
namespace {

constexpr size_t kPsAlign = 256;
constexpr double kPsBudget = 24.0 * (1ull << 30);
constexpr int kPsMaxSlots = 8192;

struct PsLayout {
  int B = 0, F = 0;
  long crow = 0;
  size_t psi, omega, epsb, dvm;
  size_t status, iters, out_index, pair, eps, zr, zi, bnorm, rnorm, rho_prev, rho_cur, alph, omg;
  size_t vec[10];
  size_t l_fill, l_sys, l_pairs, l_active, l_final, Y, Y2, C, T, bad;
  size_t total = 0;
};

size_t ps_take(size_t &off, size_t bytes) {
  off = (off + kPsAlign - 1) / kPsAlign * kPsAlign;
  const size_t r = off;
  off += std::max<size_t>(bytes, 1);
  return r;
}

PsLayout ps_layout(const sgw_ham *h, int n_occ, int n_band, int n_pert, int n_omega, const sgw_opts &o,
                   long n_systems) {
  PsLayout L;
  const long npw = h->n_pw;
  const double per_slot = 12.0 * npw * 16.0 + (double)hx_tbuf_bytes(h, 1) +
                          16.0 * kProjChunks * std::max(n_occ, 1) + 160.0;
  long B = o.ps_slots > 0 ? o.ps_slots : (long)std::min<double>(kPsMaxSlots, std::max(1.0, kPsBudget / per_slot));
  B = std::max<long>(1, std::min<long>(B, std::max<long>(n_systems, 1)));
  L.B = (int)B;
  L.F = std::max(1, L.B / 4);
  L.crow = B;
  size_t off = 0;
  L.psi = ps_take(off, 16ul * std::max(n_occ, 1) * npw);
  L.omega = ps_take(off, 16ul * std::max(n_omega, 1));  // omega, then the per-shift imaginary parts
  L.epsb = ps_take(off, 8ul * std::max(n_band, 1));
  L.dvm = ps_take(off, 12ul * std::max(n_pert, 1));
  L.status = ps_take(off, 4ul * B);
  L.iters = ps_take(off, 4ul * B);
  L.out_index = ps_take(off, 4ul * B);
  L.pair = ps_take(off, 4ul * B);
  L.eps = ps_take(off, 8ul * B);
  L.zr = ps_take(off, 8ul * B);
  L.zi = ps_take(off, 8ul * B);
  L.bnorm = ps_take(off, 8ul * B);
  L.rnorm = ps_take(off, 8ul * B);
  L.rho_prev = ps_take(off, 16ul * B);
  L.rho_cur = ps_take(off, 16ul * B);
  L.alph = ps_take(off, 16ul * B);
  L.omg = ps_take(off, 16ul * B);
  for (int k = 0; k < 10; ++k) L.vec[k] = ps_take(off, 16ul * B * npw);
  L.l_fill = ps_take(off, 4ul * B);
  L.l_sys = ps_take(off, 4ul * B);
  L.l_pairs = ps_take(off, 4ul * B);
  L.l_active = ps_take(off, 4ul * B);
  L.l_final = ps_take(off, 4ul * B);
  L.Y = ps_take(off, 16ul * B * npw);
  L.Y2 = ps_take(off, 16ul * B * npw);
  L.C = ps_take(off, 16ul * kProjChunks * B * std::max(n_occ, 1));
  L.T = ps_take(off, hx_tbuf_bytes(h, B));
  L.bad = ps_take(off, 64);
  L.total = (off + kPsAlign - 1) / kPsAlign * kPsAlign;
  return L;
}

}  // namespace

size_t ps_workspace_bytes(const sgw_ham *h, int n_occ, int n_band, int n_pert, int n_omega, const sgw_opts &o,
                          int n_systems) {
  return ps_layout(h, n_occ, n_band, n_pert, n_omega, o, n_systems).total;
}

sgw_status ps_solve(sgw_ctx *ctx, const PsProblem &P, const sgw_opts &o, const std::vector<int32_t> &systems,
                    bool warm, void *workspace, size_t workspace_bytes, double2 *dpsi, sgw_solve_info *info,
                    int *n_bad_out) {
  const sgw_ham *h = P.h_kq;
  const int npw = h->n_pw, n_occ = P.n_occ;
  const long n_all = (long)P.n_band * P.n_pert * P.n_omega;
  std::vector<int32_t> queue = systems;
  if (queue.empty()) {
    queue.resize(n_all);
    std::iota(queue.begin(), queue.end(), 0);
  }
  // hardest (highest band energy) first, for load balance across the slots
  std::stable_sort(queue.begin(), queue.end(), [&](int32_t a, int32_t b) {
    return P.eps_v[a / P.n_omega / P.n_pert] > P.eps_v[b / P.n_omega / P.n_pert];
  });
  const PsLayout L = ps_layout(h, n_occ, P.n_band, P.n_pert, P.n_omega, o, (long)queue.size());
  if (!workspace || workspace_bytes < L.total)
    return fail(SGW_ERR_WORKSPACE, "per-shift solve: workspace needs " + std::to_string(L.total) + " bytes");
  char *W = (char *)workspace;
  const int B = L.B;
  PsState S;
  S.npw = npw;
  S.n_occ = n_occ;
  S.max_iter = o.ps_max_iter;
  S.tol = P.tol * o.tol_safety;
  S.tol_final = P.tol;
  S.status = (int32_t *)(W + L.status);
  S.iters = (int32_t *)(W + L.iters);
  S.out_index = (int32_t *)(W + L.out_index);
  S.pair = (int32_t *)(W + L.pair);
  S.eps = (double *)(W + L.eps);
  S.zr = (double *)(W + L.zr);
  S.zi = (double *)(W + L.zi);
  S.bnorm = (double *)(W + L.bnorm);
  S.rnorm = (double *)(W + L.rnorm);
  S.rho_prev = (double2 *)(W + L.rho_prev);
  S.rho_cur = (double2 *)(W + L.rho_cur);
  S.alph = (double2 *)(W + L.alph);
  S.omg = (double2 *)(W + L.omg);
  double2 **vecs[10] = {&S.b, &S.x, &S.r, &S.rh, &S.p, &S.v, &S.s, &S.ph, &S.sh, &S.m};
  for (int k = 0; k < 10; ++k) *vecs[k] = (double2 *)(W + L.vec[k]);
  S.hist_iter = (o.hist_iter > 0 && o.hist_r && o.hist_x) ? o.hist_iter : 0;
  S.hist_r = S.hist_iter ? (double2 *)o.hist_r : nullptr;
  S.hist_x = S.hist_iter ? (double2 *)o.hist_x : nullptr;
  S.i2u = h->d_i2u;
  double2 *psi = (double2 *)(W + L.psi);
  double *d_omega = (double *)(W + L.omega), *d_epsb = (double *)(W + L.epsb);
  int32_t *d_dvm = (int32_t *)(W + L.dvm);
  int32_t *d_fill = (int32_t *)(W + L.l_fill), *d_sys = (int32_t *)(W + L.l_sys);
  int32_t *d_pairs = (int32_t *)(W + L.l_pairs), *d_active = (int32_t *)(W + L.l_active);
  int32_t *d_final = (int32_t *)(W + L.l_final);
  double2 *Y = (double2 *)(W + L.Y), *Y2 = (double2 *)(W + L.Y2), *C = (double2 *)(W + L.C);
  double2 *T = (double2 *)(W + L.T);
  int *d_bad = (int *)(W + L.bad);
  const long crow = L.crow;

  sgw_status st;
  // pinned staging: status | fill | sys | pairs | active | final | bad
  if ((st = ensure_pinned(ctx, sizeof(int32_t) * (6ul * B + 16))) != SGW_OK) return st;
  int32_t *p_status = (int32_t *)ctx->pinned;
  int32_t *p_fill = p_status + B, *p_sys = p_fill + B, *p_pairs = p_sys + B, *p_active = p_pairs + B;
  int32_t *p_final = p_active + B, *p_bad = p_final + B;

  SGW_HIP(hipMemcpyAsync(d_omega, P.omega, sizeof(double) * P.n_omega, hipMemcpyHostToDevice, ctx->stream));
  const double *d_eta_j = nullptr;
  if (o.shift_imag) {
    d_eta_j = d_omega + P.n_omega;
    SGW_HIP(hipMemcpyAsync((void *)d_eta_j, o.shift_imag, sizeof(double) * P.n_omega, hipMemcpyHostToDevice,
                           ctx->stream));
  }
  SGW_HIP(hipMemcpyAsync(d_epsb, P.eps_v, sizeof(double) * P.n_band, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(d_dvm, P.dv_miller, sizeof(int32_t) * 3 * P.n_pert, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), ctx->stream));
  if ((st = permute(ctx, npw, n_occ, P.psi_occ_kq, npw, psi, npw, h->d_i2u, 0)) != SGW_OK) return st;

  // y_a = (H + alpha P_occ) x_a
  auto matvec = [&](int n, VecSrc src) -> sgw_status {
    sgw_status s2;
    if ((s2 = proj_dot(ctx, npw, n_occ, psi, n, src, C, crow)) != SGW_OK) return s2;
    if ((s2 = hx_batch(ctx, h, n, src, Y, npw, T)) != SGW_OK) return s2;
    return proj_apply(ctx, npw, n_occ, psi, n, src, C, crow, Y, npw, o.alpha_pv, 1);
  };
  const int mode = o.precond;
  const int guess = warm ? 2 : (o.guess == SGW_GUESS_LEARNED ? 1 : 0);
  const bool has_x0 = guess != 0;

  size_t next = 0, finished = 0;
  std::vector<int> free_slots, active, done;
  for (int s = B - 1; s >= 0; --s) free_slots.push_back(s);
  while (finished < queue.size()) {
    int nfill = 0;
    while (!free_slots.empty() && next < queue.size()) {
      const int s = free_slots.back();
      free_slots.pop_back();
      const int32_t y = queue[next++];
      p_fill[nfill] = s;
      p_sys[nfill] = y;
      p_pairs[nfill] = y / P.n_omega;
      ++nfill;
    }
    if (nfill > 0) {
      SGW_HIP(hipMemcpyAsync(d_fill, p_fill, sizeof(int32_t) * nfill, hipMemcpyHostToDevice, ctx->stream));
      SGW_HIP(hipMemcpyAsync(d_sys, p_sys, sizeof(int32_t) * nfill, hipMemcpyHostToDevice, ctx->stream));
      SGW_HIP(hipMemcpyAsync(d_pairs, p_pairs, sizeof(int32_t) * nfill, hipMemcpyHostToDevice, ctx->stream));
      if ((st = ps_setup(ctx, S, nfill, d_fill, d_sys, d_epsb, d_omega, P.eta, d_eta_j, P.n_pert, P.n_omega)) !=
          SGW_OK)
        return st;
      if ((st = rhs_source(ctx, h, P.h_k, nfill, d_pairs, P.n_pert, d_dvm, P.psi_v, P.h_k->n_pw, Y, npw)) != SGW_OK)
        return st;
      if ((st = proj_dot(ctx, npw, n_occ, psi, nfill, contiguous(Y, npw), C, crow)) != SGW_OK) return st;
      if ((st = proj_apply(ctx, npw, n_occ, psi, nfill, contiguous(Y, npw), C, crow, Y2, npw, 1.0, 0)) != SGW_OK)
        return st;
      if ((st = ps_rhs(ctx, S, nfill, d_fill, Y, Y2)) != SGW_OK) return st;
      if (warm && (st = ps_load_x(ctx, S, nfill, d_fill, dpsi)) != SGW_OK) return st;
      if ((st = ps_precond(ctx, S, nfill, d_fill, h->d_kin, mode, o.mlp, guess)) != SGW_OK) return st;
      if (has_x0) {
        if ((st = matvec(nfill, listed(S.x, npw, d_fill))) != SGW_OK) return st;
        if ((st = ps_start(ctx, S, nfill, d_fill, Y, 1)) != SGW_OK) return st;
      } else if ((st = ps_start(ctx, S, nfill, d_fill, Y, 0)) != SGW_OK) {
        return st;
      }
      // (the pinned fill lists are rewritten only after the poll below has synchronised)
      for (int k = 0; k < nfill; ++k) active.push_back(p_fill[k]);
    }
    if (!active.empty()) {
      const int na = (int)active.size();
      std::memcpy(p_active, active.data(), sizeof(int32_t) * na);
      SGW_HIP(hipMemcpyAsync(d_active, p_active, sizeof(int32_t) * na, hipMemcpyHostToDevice, ctx->stream));
      for (int step = 0; step < o.steps_per_sync; ++step) {
        if ((st = ps_k1(ctx, S, na, d_active)) != SGW_OK) return st;
        if ((st = matvec(na, listed(S.ph, npw, d_active))) != SGW_OK) return st;
        if ((st = ps_k2(ctx, S, na, d_active, Y)) != SGW_OK) return st;
        if ((st = matvec(na, listed(S.sh, npw, d_active))) != SGW_OK) return st;
        if ((st = ps_k3(ctx, S, na, d_active, Y)) != SGW_OK) return st;
      }
    }
    SGW_HIP(hipMemcpyAsync(p_status, S.status, sizeof(int32_t) * B, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    std::vector<int> still;
    for (int s : active) (p_status[s] == PS_RUNNING ? still : done).push_back(s);
    active.swap(still);
    const bool waiting = next < queue.size();
    if (!done.empty() && (active.empty() || (int)done.size() >= L.F || (waiting && (int)done.size() * 4 >= L.F))) {
      const int nf = (int)done.size();
      std::memcpy(p_final, done.data(), sizeof(int32_t) * nf);
      SGW_HIP(hipMemcpyAsync(d_final, p_final, sizeof(int32_t) * nf, hipMemcpyHostToDevice, ctx->stream));
      if ((st = matvec(nf, listed(S.x, npw, d_final))) != SGW_OK) return st;
      if ((st = ps_final(ctx, S, nf, d_final, Y, C, crow, dpsi, info, d_bad, SGW_FLAG_PER_SHIFT)) != SGW_OK)
        return st;
      if ((st = sync(ctx)) != SGW_OK) return st;
      for (int s : done) free_slots.push_back(s);
      finished += done.size();
      done.clear();
    }
  }
  SGW_HIP(hipMemcpyAsync(p_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if ((st = sync(ctx)) != SGW_OK) return st;
  *n_bad_out = *p_bad;
  return SGW_OK;
}

}  // namespace sgw

// ---------------------------------------------------------------------------
// test hook: the diagonal preconditioner and initial guess of the per-shift solves
// ---------------------------------------------------------------------------
namespace {
struct HookBuf {
  void *p = nullptr;
  ~HookBuf() {
    if (p) hipFree(p);
  }
};
}  // namespace

extern "C" sgw_status sgw_precond_values(sgw_ctx *ctx, const sgw_ham *ham, int precond, int guess,
                                         const sgw_mlp *mlp, int n_vec, const double *eps, const double *omega,
                                         double eta, const sgw_c128 *b, sgw_c128 *m_out, sgw_c128 *x0_out) {
  using namespace sgw;
  if (!ctx || !ham) return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: NULL context or Hamiltonian");
  if (n_vec < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: n_vec < 0");
  if (precond < SGW_PC_NONE || precond > SGW_PC_LEARNED)
    return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: unknown preconditioner");
  if (guess != SGW_GUESS_ZERO && guess != SGW_GUESS_LEARNED)
    return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: unknown initial guess");
  if ((precond == SGW_PC_LEARNED || guess == SGW_GUESS_LEARNED) && (!mlp || mlp->device != ctx->device))
    return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: the learned model needs an sgw_mlp of this device");
  if (n_vec == 0) return SGW_OK;
  if (!eps || !omega || !b || !m_out || !x0_out) return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: NULL array");
  if (!std::isfinite(eta)) return fail(SGW_ERR_INVALID_ARG, "sgw_precond_values: eta not finite");
  SGW_HIP(hipSetDevice(ctx->device));
  const int npw = ham->n_pw;
  const size_t vb = sizeof(double2) * (size_t)npw * n_vec;
  HookBuf vec, par, lst;
  SGW_HIP(hipMalloc(&vec.p, 3 * vb));
  SGW_HIP(hipMalloc(&par.p, 3 * sizeof(double) * n_vec));
  SGW_HIP(hipMalloc(&lst.p, sizeof(int32_t) * n_vec));
  PsState S{};
  S.npw = npw;
  S.b = (double2 *)vec.p;
  S.m = S.b + (size_t)npw * n_vec;
  S.x = S.m + (size_t)npw * n_vec;
  S.eps = (double *)par.p;
  S.zr = S.eps + n_vec;
  S.zi = S.zr + n_vec;
  std::vector<double> hp(3 * (size_t)n_vec);
  std::vector<int32_t> hl(n_vec);
  for (int a = 0; a < n_vec; ++a) {
    hp[a] = eps[a];
    hp[n_vec + a] = omega[a];
    hp[2 * n_vec + a] = eta;
    hl[a] = a;
  }
  SGW_HIP(hipMemcpyAsync(par.p, hp.data(), sizeof(double) * hp.size(), hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(lst.p, hl.data(), sizeof(int32_t) * n_vec, hipMemcpyHostToDevice, ctx->stream));
  sgw_status st;
  if ((st = permute(ctx, npw, n_vec, (const double2 *)b, npw, S.b, npw, ham->d_i2u, 0)) != SGW_OK) return st;
  if ((st = ps_precond(ctx, S, n_vec, (const int32_t *)lst.p, ham->d_kin, precond, mlp,
                       guess == SGW_GUESS_LEARNED ? 1 : 0)) != SGW_OK)
    return st;
  if ((st = permute(ctx, npw, n_vec, S.m, npw, (double2 *)m_out, npw, ham->d_i2u, 1)) != SGW_OK) return st;
  if ((st = permute(ctx, npw, n_vec, S.x, npw, (double2 *)x0_out, npw, ham->d_i2u, 1)) != SGW_OK) return st;
  return sync(ctx);
}
