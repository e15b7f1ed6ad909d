// Correlation self-energy (Sec. 2.4, Eq. 10) on the imaginary axis or the real axis, its rational
// continuation to the real axis by AAA (Sec. 2.7), the spectral function and the linearised
// quasiparticle energy (Sec. 2.8, Eqs. 16-17).
//
// The diagonal element of Eq. 10 in a state n, with G and W_bar expanded in the plane waves q + G of
// W_bar, is
//     Sigma_n(w) = (alpha / (2 pi Omega)) sum_j w_j sum_{G,G'} W_bar_{GG'}(w'_j - w) < t_G | G(z_j) | t_G' >,
// t_G = exp(-i (q+G) . r) u_n at k - q, alpha = -1 on the imaginary axis (z_j = mu + i w'_j) and i on the
// real axis (z_j = w'_j shifted off the axis by the caller).  The pair elements come from the multishift
// solver: with no occupied projector and a zero band energy, the solve of (H - z) x = -t_G' for all
// shifts z_j at once gives x = G(z_j) t_G' (each shift with its own imaginary part), and
// the bra is the same plane-wave shift of u_n (minus the right-hand side of that solve): an overlap
// contraction on the FP64 matrix cores, as for the density response.  The frequency convolution is a
// small reduction per (n, w) on the GPU.  AAA is a greedy sequence of small SVDs (a few hundred
// points, at most a few dozen support points per state); it runs in the library's host code, with a
// one-sided Jacobi SVD, and the approximant is evaluated for the spectral function on the GPU.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "fft_lds.h"
#include "sgw_internal.h"

namespace sgw {
namespace {

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

// m[j][g][h] = -c[(h * n_freq + j) * n_g + g]   (c: overlaps of one band with the minus right-hand sides)
__global__ void k_pair_store(const double2 *__restrict__ c, int n_g, int n_freq, double2 *__restrict__ m) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_freq * n_g * n_g) return;
  const int j = e / (n_g * n_g), r = e - j * n_g * n_g, g = r / n_g, h = r - g * n_g;
  const double2 t = c[((long)h * n_freq + j) * n_g + g];
  m[e] = make_double2(-t.x, -t.y);
}

// sigma[n][k] = scale * sum_j w_j sum_{g,h} wbar[idx[k][j]][g][h] m[n][j][g][h] (complex scale); one
// workgroup per (n, k)
__global__ __launch_bounds__(256) void k_sigma(int n_g, int n_freq, int n_out, const double2 *__restrict__ m,
                                               const double *__restrict__ wq, const double2 *__restrict__ wbar,
                                               const int32_t *__restrict__ idx, double2 scale,
                                               double2 *__restrict__ sigma) {
  __shared__ double2 part[256];
  const int n = blockIdx.x / n_out, k = blockIdx.x - n * n_out;
  const int gg = n_g * n_g;
  double2 acc = make_double2(0.0, 0.0);
  for (int e = threadIdx.x; e < n_freq * gg; e += 256) {
    const int j = e / gg, r = e - j * gg;
    const double2 w = wbar[(long)idx[k * n_freq + j] * gg + r];
    const double2 x = m[((long)n * n_freq + j) * gg + r];
    const double2 p = c_mul(w, x);
    acc.x = fma(wq[j], p.x, acc.x);
    acc.y = fma(wq[j], p.y, acc.y);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {  // fixed order: deterministic
    if (threadIdx.x < s) part[threadIdx.x] = c_add(part[threadIdx.x], part[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[(long)n * n_out + k] = c_mul(scale, part[0]);
}

// Sigma^c(w + i d) from each state's barycentric approximant, and A(w) of Eq. 16
__global__ void k_spectral(int n_band, int n_sup_max, const int32_t *__restrict__ n_sup,
                           const double2 *__restrict__ zs, const double2 *__restrict__ fs,
                           const double2 *__restrict__ ws, int n_omega, const double *__restrict__ omega,
                           double broad, const double *__restrict__ eps, const double *__restrict__ delta,
                           double2 *__restrict__ sigma, double *__restrict__ a) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_band * n_omega) return;
  const int n = (int)(e / n_omega), i = (int)(e - (long)n * n_omega);
  const double2 z = make_double2(omega[i], broad);
  const double2 *zn = zs + (long)n * n_sup_max, *fn = fs + (long)n * n_sup_max, *wn = ws + (long)n * n_sup_max;
  double2 num = make_double2(0.0, 0.0), den = make_double2(0.0, 0.0), hit = make_double2(0.0, 0.0);
  bool at_node = false;
  for (int s = 0; s < n_sup[n]; ++s) {
    const double2 d = c_sub(z, zn[s]);
    if (d.x == 0.0 && d.y == 0.0) {
      at_node = true;
      hit = fn[s];
      continue;
    }
    const double q = 1.0 / (d.x * d.x + d.y * d.y);
    const double2 inv = make_double2(d.x * q, -d.y * q);  // 1 / d
    const double2 wi = c_mul(wn[s], inv);
    den = c_add(den, wi);
    num = c_add(num, c_mul(wi, fn[s]));
  }
  double2 s;
  if (at_node) {
    s = hit;
  } else {
    const double q = 1.0 / (den.x * den.x + den.y * den.y);
    s = c_mul(num, make_double2(den.x * q, -den.y * q));
  }
  if (sigma) sigma[e] = s;
  if (a) {
    const double re = omega[i] - eps[n] - s.x - delta[n], im = -s.y;
    a[e] = -s.y / (M_PI * (re * re + im * im));
  }
}

using cplx = std::complex<double>;

// smallest right singular vector of the rows x cols matrix a (column-major, a[c * rows + r]) by
// one-sided Jacobi rotations of the columns
std::vector<cplx> smallest_right_singular_vector(std::vector<cplx> a, int rows, int cols) {
  std::vector<cplx> v((size_t)cols * cols, 0.0);
  for (int c = 0; c < cols; ++c) v[(size_t)c * cols + c] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        cplx *ap = &a[(size_t)p * rows], *aq = &a[(size_t)q * rows];
        double al = 0.0, be = 0.0;
        cplx ga = 0.0;
        for (int r = 0; r < rows; ++r) {
          al += std::norm(ap[r]);
          be += std::norm(aq[r]);
          ga += std::conj(ap[r]) * aq[r];
        }
        const double g = std::abs(ga);
        if (g == 0.0 || g <= 1e-15 * std::sqrt(al * be)) continue;
        off = std::max(off, g / std::sqrt(al * be));
        // remove the phase of the off-diagonal element, then a real rotation zeroes it
        const cplx ph = ga / g;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int r = 0; r < rows; ++r) {
          const cplx x = ap[r], y = aq[r] * std::conj(ph);
          ap[r] = cs * x - sn * y;
          aq[r] = sn * x + cs * y;
        }
        cplx *vp = &v[(size_t)p * cols], *vq = &v[(size_t)q * cols];
        for (int r = 0; r < cols; ++r) {
          const cplx x = vp[r], y = vq[r] * std::conj(ph);
          vp[r] = cs * x - sn * y;
          vq[r] = sn * x + cs * y;
        }
      }
    if (off <= 1e-15) break;
  }
  int best = 0;
  double bn = 1e300;
  for (int c = 0; c < cols; ++c) {
    double nrm = 0.0;
    for (int r = 0; r < rows; ++r) nrm += std::norm(a[(size_t)c * rows + r]);
    if (nrm < bn) {
      bn = nrm;
      best = c;
    }
  }
  return std::vector<cplx>(v.begin() + (size_t)best * cols, v.begin() + (size_t)(best + 1) * cols);
}

}  // namespace
}  // namespace sgw

using namespace sgw;

namespace {
size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// the pair-element workspace: the solver's, then the solutions, the right-hand sides, the overlap
// partial sums and (for a NULL info) the solve records
struct PairLayout {
  size_t solver, x, b, c, info, total;
};

sgw_status pair_layout(sgw_ctx *ctx, const sgw_ham *h_kmq, int n_band, int n_g, int n_freq, const sgw_opts *opts,
                       PairLayout *L) {
  sgw_status st;
  size_t ws = 0;
  if ((st = sternheimer_workspace_size(ctx, h_kmq, 0, n_band, n_g, n_freq, opts, &ws)) != SGW_OK) return st;
  const size_t npw = h_kmq->n_pw, nvec = (size_t)n_band * n_g * n_freq;
  L->solver = 0;
  L->x = up256(ws);
  L->b = L->x + up256(sizeof(double2) * nvec * npw);
  L->c = L->b + up256(sizeof(double2) * (size_t)n_band * n_g * npw);
  L->info = L->c + up256(sizeof(double2) * kProjChunks * (size_t)n_g * n_freq * n_g);
  L->total = L->info + up256(sizeof(sgw_solve_info) * nvec);
  return SGW_OK;
}
}  // namespace

extern "C" sgw_status sgw_green_pair_workspace_size(sgw_ctx *ctx, const sgw_ham *h_kmq, int n_band, int n_g,
                                                    int n_freq, const sgw_opts *opts, size_t *bytes) {
  if (!ctx || !h_kmq || !bytes) return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_workspace_size: NULL argument");
  if (n_band < 0 || n_g < 0 || n_freq < 0)
    return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_workspace_size: negative size");
  PairLayout L;
  const sgw_status st = pair_layout(ctx, h_kmq, n_band, n_g, n_freq, opts, &L);
  if (st != SGW_OK) return st;
  *bytes = L.total;
  return SGW_OK;
}

extern "C" sgw_status sgw_green_pair_elements(sgw_ctx *ctx, const sgw_ham *h_kmq, const sgw_ham *h_k, int n_band,
                                              const sgw_c128 *psi_n, int n_g, const int32_t *g_miller, int n_freq,
                                              const double *z_re, const double *z_im, double tol, const sgw_opts *opts,
                                              void *workspace, size_t workspace_bytes, sgw_c128 *m_out,
                                              sgw_solve_info *info) {
  if (!ctx || !h_kmq || !h_k) return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_elements: NULL context or Hamiltonian");
  if (n_band < 0 || n_g < 0 || n_freq < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_elements: negative size");
  if ((long)n_band * n_g * n_freq == 0) return SGW_OK;
  if (!psi_n || !g_miller || !z_re || !z_im || !m_out)
    return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_elements: NULL array");
  for (int j = 0; j < n_freq; ++j)
    if (!std::isfinite(z_re[j]) || !std::isfinite(z_im[j]))
      return fail(SGW_ERR_INVALID_ARG, "sgw_green_pair_elements: frequency not finite");
  sgw_opts o;
  if (opts) o = *opts;
  else sgw_opts_default(&o);
  o.shift_imag = z_im;
  PairLayout L;
  sgw_status st = pair_layout(ctx, h_kmq, n_band, n_g, n_freq, &o, &L);
  if (st != SGW_OK) return st;
  if (!workspace || workspace_bytes < L.total)
    return fail(SGW_ERR_WORKSPACE, "sgw_green_pair_elements: workspace missing or below "
                                   "sgw_green_pair_workspace_size");
  if ((uintptr_t)workspace % 256 != 0)
    return fail(SGW_ERR_WORKSPACE, "sgw_green_pair_elements: workspace not 256-byte aligned");
  SGW_HIP(hipSetDevice(ctx->device));
  char *w = (char *)workspace;
  double2 *x = (double2 *)(w + L.x), *b = (double2 *)(w + L.b), *c = (double2 *)(w + L.c);
  sgw_solve_info *inf_p = info ? info : (sgw_solve_info *)(w + L.info);
  std::vector<int32_t> dv(3 * (size_t)n_g);
  for (int i = 0; i < 3 * n_g; ++i) dv[i] = -g_miller[i];  // t_G = exp(-i (q+G) . r) u_n
  std::vector<double> zero_eps(n_band, 0.0);
  const int npw = h_kmq->n_pw;
  // x = (H - z_j)^{-1} (-t_G') = G(z_j) t_G' for z_j = z_re[j] + i z_im[j]
  const sgw_status solved = sternheimer_solve(ctx, h_kmq, 0, nullptr, h_k, n_band, psi_n, zero_eps.data(), n_g,
                                              dv.data(), n_freq, z_re, 0.0, tol, &o, w + L.solver, L.x,
                                              (sgw_c128 *)x, inf_p);
  if (solved < 0) return solved;
  // the right-hand sides b_G = -t_G of every band
  if ((st = sgw_build_rhs(ctx, h_kmq, 0, nullptr, h_k, n_band, psi_n, n_g, dv.data(), (sgw_c128 *)b)) != SGW_OK)
    return st;
  const int nv = n_g * n_freq;
  const long per_band = (long)n_freq * n_g * n_g;
  for (int v = 0; v < n_band; ++v) {
    const double2 *bv = b + (long)v * n_g * npw;
    const double2 *xv = x + (long)v * nv * npw;
    if ((st = proj_dot(ctx, npw, n_g, bv, nv, contiguous(xv, npw), c, nv, K_CHI_DOT)) != SGW_OK) return st;
    hipLaunchKernelGGL(k_pair_store, dim3((per_band + 255) / 256), dim3(256), 0, ctx->stream, (const double2 *)c, n_g,
                       n_freq, (double2 *)m_out + v * per_band);
    SGW_HIP(hipGetLastError());
  }
  if ((st = sync(ctx)) != SGW_OK) return st;
  return solved;
}

extern "C" sgw_status sgw_sigma_c(sgw_ctx *ctx, int n_band, int n_g, int n_freq, const sgw_c128 *m_elem,
                                  const double *weights, int n_w, const sgw_c128 *wbar, int n_out,
                                  const int32_t *w_index, double volume, double alpha_re, double alpha_im,
                                  sgw_c128 *sigma) {
  if (!ctx) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: NULL context");
  if (n_band < 0 || n_g < 0 || n_freq < 0 || n_w < 0 || n_out < 0)
    return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: negative size");
  if ((long)n_band * n_out == 0) return SGW_OK;
  if (!m_elem || !weights || !wbar || !w_index || !sigma) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: NULL array");
  if (!(volume > 0.0) || !std::isfinite(volume)) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: volume must be positive");
  if (!std::isfinite(alpha_re) || !std::isfinite(alpha_im)) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: alpha not finite");
  for (long e = 0; e < (long)n_out * n_freq; ++e)
    if (w_index[e] < 0 || w_index[e] >= n_w) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: w_index out of range");
  for (int j = 0; j < n_freq; ++j)
    if (!std::isfinite(weights[j])) return fail(SGW_ERR_INVALID_ARG, "sgw_sigma_c: weight not finite");
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_status st;
  Buf dw, di;
  if ((st = alloc(dw, sizeof(double) * n_freq)) != SGW_OK) return st;
  if ((st = alloc(di, sizeof(int32_t) * (size_t)n_out * n_freq)) != SGW_OK) return st;
  SGW_HIP(hipMemcpyAsync(dw.p, weights, sizeof(double) * n_freq, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(di.p, w_index, sizeof(int32_t) * (size_t)n_out * n_freq, hipMemcpyHostToDevice,
                         ctx->stream));
  hipLaunchKernelGGL(k_sigma, dim3((long)n_band * n_out), dim3(256), 0, ctx->stream, n_g, n_freq, n_out,
                     (const double2 *)m_elem, (const double *)dw.p, (const double2 *)wbar, (const int32_t *)di.p,
                     make_double2(alpha_re / (2.0 * M_PI * volume), alpha_im / (2.0 * M_PI * volume)),
                     (double2 *)sigma);
  SGW_HIP(hipGetLastError());
  return sync(ctx);
}

extern "C" sgw_status sgw_aaa_fit(int n, const sgw_c128 *z, const sgw_c128 *f, double tol, int max_terms, int *n_sup,
                                  sgw_c128 *z_sup, sgw_c128 *f_sup, sgw_c128 *w_sup) {
  if (n < 2 || !z || !f || !n_sup || !z_sup || !f_sup || !w_sup)
    return fail(SGW_ERR_INVALID_ARG, "sgw_aaa_fit: need two points and non-NULL arrays");
  if (!(tol >= 0.0) || max_terms < 1) return fail(SGW_ERR_INVALID_ARG, "sgw_aaa_fit: bad tol or max_terms");
  std::vector<cplx> zz(n), ff(n);
  double fmax = 0.0;
  cplx mean = 0.0;
  for (int i = 0; i < n; ++i) {
    zz[i] = cplx(z[i].re, z[i].im);
    ff[i] = cplx(f[i].re, f[i].im);
    if (!std::isfinite(zz[i].real()) || !std::isfinite(zz[i].imag()) || !std::isfinite(ff[i].real()) ||
        !std::isfinite(ff[i].imag()))
      return fail(SGW_ERR_INVALID_ARG, "sgw_aaa_fit: point not finite");
    fmax = std::max(fmax, std::abs(ff[i]));
    mean += ff[i];
  }
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k)
      if (zz[i] == zz[k]) return fail(SGW_ERR_INVALID_ARG, "sgw_aaa_fit: repeated point");
  mean /= (double)n;
  std::vector<char> rest(n, 1);
  std::vector<cplx> r(n, mean), w;
  std::vector<int> sup;
  const int mmax = std::min(max_terms, n - 1);
  for (int m = 0; m < mmax; ++m) {
    int j = -1;
    double worst = -1.0;
    for (int i = 0; i < n; ++i)
      if (rest[i] && std::abs(ff[i] - r[i]) > worst) {
        worst = std::abs(ff[i] - r[i]);
        j = i;
      }
    sup.push_back(j);
    rest[j] = 0;
    const int k = (int)sup.size();
    std::vector<int> rows;
    for (int i = 0; i < n; ++i)
      if (rest[i]) rows.push_back(i);
    const int nr = (int)rows.size();
    // Loewner matrix of the other points against the support points
    std::vector<cplx> a((size_t)nr * k);
    for (int s = 0; s < k; ++s)
      for (int ri = 0; ri < nr; ++ri) {
        const int i = rows[ri];
        a[(size_t)s * nr + ri] = (ff[i] - ff[sup[s]]) / (zz[i] - zz[sup[s]]);
      }
    w = smallest_right_singular_vector(a, nr, k);
    for (int i = 0; i < n; ++i) r[i] = ff[i];
    for (int i : rows) {
      cplx num = 0.0, den = 0.0;
      for (int s = 0; s < k; ++s) {
        const cplx cw = w[s] / (zz[i] - zz[sup[s]]);
        num += cw * ff[sup[s]];
        den += cw;
      }
      r[i] = num / den;
    }
    double err = 0.0;
    for (int i = 0; i < n; ++i) err = std::max(err, std::abs(ff[i] - r[i]));
    if (err <= tol * fmax) break;
  }
  *n_sup = (int)sup.size();
  for (int s = 0; s < *n_sup; ++s) {
    z_sup[s] = {zz[sup[s]].real(), zz[sup[s]].imag()};
    f_sup[s] = {ff[sup[s]].real(), ff[sup[s]].imag()};
    w_sup[s] = {w[s].real(), w[s].imag()};
  }
  return SGW_OK;
}

extern "C" sgw_status sgw_pade_fit(int n, const sgw_c128 *z, const sgw_c128 *f, sgw_c128 *a) {
  if (n < 1 || !z || !f || !a) return fail(SGW_ERR_INVALID_ARG, "sgw_pade_fit: need a point and non-NULL arrays");
  std::vector<cplx> zz(n), g(n);
  for (int i = 0; i < n; ++i) {
    zz[i] = cplx(z[i].re, z[i].im);
    g[i] = cplx(f[i].re, f[i].im);
    if (!std::isfinite(zz[i].real()) || !std::isfinite(zz[i].imag()) || !std::isfinite(g[i].real()) ||
        !std::isfinite(g[i].imag()))
      return fail(SGW_ERR_INVALID_ARG, "sgw_pade_fit: point not finite");
  }
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k)
      if (zz[i] == zz[k]) return fail(SGW_ERR_INVALID_ARG, "sgw_pade_fit: repeated point");
  // g_p(z_i) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_i)) / ((z_i - z_{p-1}) g_{p-1}(z_i)), a_p = g_p(z_p), in place
  a[0] = {g[0].real(), g[0].imag()};
  for (int p = 1; p < n; ++p) {
    const cplx gp = g[p - 1];
    for (int i = p; i < n; ++i) {
      if (g[i] == cplx(0.0, 0.0)) return fail(SGW_ERR_INVALID_ARG, "sgw_pade_fit: the continued fraction breaks down");
      g[i] = (gp - g[i]) / ((zz[i] - zz[p - 1]) * g[i]);
    }
    a[p] = {g[p].real(), g[p].imag()};
    // a zero coefficient would cut the fraction short of the later points
    if (g[p] == cplx(0.0, 0.0) && p < n - 1)
      return fail(SGW_ERR_INVALID_ARG, "sgw_pade_fit: the continued fraction breaks down");
  }
  return SGW_OK;
}

extern "C" sgw_status sgw_pade_eval(int n, const sgw_c128 *z, const sgw_c128 *a, int n_x, const sgw_c128 *x,
                                    sgw_c128 *out) {
  if (n < 1 || n_x < 0 || !z || !a || (n_x > 0 && (!x || !out)))
    return fail(SGW_ERR_INVALID_ARG, "sgw_pade_eval: bad arguments");
  for (int e = 0; e < n_x; ++e) {
    const cplx xv(x[e].re, x[e].im);
    // A_{k+1} = A_k + (x - z_k) a_{k+1} A_{k-1}, the same for B; C = A_n / B_n
    cplx ap(0.0, 0.0), ac(a[0].re, a[0].im), bp(1.0, 0.0), bc(1.0, 0.0);
    for (int k = 1; k < n; ++k) {
      const cplx t = (xv - cplx(z[k - 1].re, z[k - 1].im)) * cplx(a[k].re, a[k].im);
      const cplx an = ac + t * ap, bn = bc + t * bp;
      ap = ac;
      ac = an;
      bp = bc;
      bc = bn;
    }
    const cplx c = ac / bc;
    out[e] = {c.real(), c.imag()};
  }
  return SGW_OK;
}

extern "C" sgw_status sgw_spectral_function(sgw_ctx *ctx, int n_band, int n_sup_max, const int32_t *n_sup,
                                            const sgw_c128 *z_sup, const sgw_c128 *f_sup, const sgw_c128 *w_sup,
                                            int n_omega, const double *omega, double broad, const double *eps_n,
                                            const double *delta, sgw_c128 *sigma, double *a) {
  if (!ctx) return fail(SGW_ERR_INVALID_ARG, "sgw_spectral_function: NULL context");
  if (n_band < 0 || n_omega < 0 || n_sup_max < 1) return fail(SGW_ERR_INVALID_ARG, "sgw_spectral_function: bad size");
  if ((long)n_band * n_omega == 0) return SGW_OK;
  if (!n_sup || !z_sup || !f_sup || !w_sup || !omega || !eps_n || !delta || (!sigma && !a))
    return fail(SGW_ERR_INVALID_ARG, "sgw_spectral_function: NULL array");
  for (int n = 0; n < n_band; ++n)
    if (n_sup[n] < 1 || n_sup[n] > n_sup_max) return fail(SGW_ERR_INVALID_ARG, "sgw_spectral_function: bad n_sup");
  if (!std::isfinite(broad)) return fail(SGW_ERR_INVALID_ARG, "sgw_spectral_function: broadening not finite");
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_status st;
  Buf dn, dz, df, dw, dom, de, dd;
  const size_t ns = (size_t)n_band * n_sup_max;
  if ((st = alloc(dn, sizeof(int32_t) * n_band)) != SGW_OK) return st;
  if ((st = alloc(dz, sizeof(double2) * ns)) != SGW_OK) return st;
  if ((st = alloc(df, sizeof(double2) * ns)) != SGW_OK) return st;
  if ((st = alloc(dw, sizeof(double2) * ns)) != SGW_OK) return st;
  if ((st = alloc(dom, sizeof(double) * n_omega)) != SGW_OK) return st;
  if ((st = alloc(de, sizeof(double) * n_band)) != SGW_OK) return st;
  if ((st = alloc(dd, sizeof(double) * n_band)) != SGW_OK) return st;
  SGW_HIP(hipMemcpyAsync(dn.p, n_sup, sizeof(int32_t) * n_band, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dz.p, z_sup, sizeof(double2) * ns, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(df.p, f_sup, sizeof(double2) * ns, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dw.p, w_sup, sizeof(double2) * ns, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dom.p, omega, sizeof(double) * n_omega, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(de.p, eps_n, sizeof(double) * n_band, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dd.p, delta, sizeof(double) * n_band, hipMemcpyHostToDevice, ctx->stream));
  const long ne = (long)n_band * n_omega;
  hipLaunchKernelGGL(k_spectral, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, n_band, n_sup_max,
                     (const int32_t *)dn.p, (const double2 *)dz.p, (const double2 *)df.p, (const double2 *)dw.p,
                     n_omega, (const double *)dom.p, broad, (const double *)de.p, (const double *)dd.p,
                     (double2 *)sigma, a);
  SGW_HIP(hipGetLastError());
  return sync(ctx);
}

extern "C" sgw_status sgw_quasiparticle(int n_sup, const sgw_c128 *z_sup, const sgw_c128 *f_sup,
                                        const sgw_c128 *w_sup, double eps_n, double delta, double *eps_qp,
                                        double *z_factor) {
  if (n_sup < 1 || !z_sup || !f_sup || !w_sup || !eps_qp || !z_factor)
    return fail(SGW_ERR_INVALID_ARG, "sgw_quasiparticle: bad arguments");
  // r = N / D with N = sum w f / (x - z_s), D = sum w / (x - z_s); r' = (N' D - N D') / D^2
  const cplx x(eps_n, 0.0);
  cplx num = 0.0, den = 0.0, dnum = 0.0, dden = 0.0;
  for (int s = 0; s < n_sup; ++s) {
    const cplx d = x - cplx(z_sup[s].re, z_sup[s].im);
    if (d == cplx(0.0, 0.0)) return fail(SGW_ERR_INVALID_ARG, "sgw_quasiparticle: eps_n is a support point");
    const cplx w(w_sup[s].re, w_sup[s].im), f(f_sup[s].re, f_sup[s].im);
    num += w * f / d;
    den += w / d;
    dnum -= w * f / (d * d);
    dden -= w / (d * d);
  }
  const cplx r = num / den, dr = (dnum * den - num * dden) / (den * den);
  const double z = 1.0 / (1.0 - dr.real());
  *z_factor = z;
  *eps_qp = eps_n + z * (r.real() + delta);
  return SGW_OK;
}
