// Learned diagonal preconditioner and initial guess for per-shift solves:
// a 3-layer MLP (5 -> 64 -> 64 -> 4, tanh) evaluated per plane wave.
//
// Outputs o: m_G = (o0 + i o1) / (T_G + 1) (preconditioner), g_G = (o2 + i o3) /
// (T_G + 1) (initial guess x0 = g (.) b).  Training rows carry, besides the
// features, two complex pairs (u_m, w_m) and (u_g, w_g); the loss is
//     L = (1/n) sum_rows |m u_m - w_m|^2 + |g u_g - w_g|^2.
// The rows built here from residual histories make L the diagonal
// approximate-inverse objective (residual after one preconditioned step).
//
// FP32 master weights and Adam moments; inference inside the solver reads a
// BF16 copy.  Gradients: each workgroup forward/backward-propagates 64 rows
// (one per lane) and forms its weight-gradient tile products in LDS; tiles are
// summed in a fixed order, so the gradient is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "fft_lds.h"
#include "pershift.h"
#include "reduce.h"

namespace sgw {
namespace {

constexpr int kRows = 64;  // rows per gradient workgroup (one wavefront)

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fff + ((u >> 16) & 1);  // round to nearest even
  return (uint16_t)(u >> 16);
}

__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = to_bf16(w[i]);
}

struct Fwd {
  float h1[kMlpHid], h2[kMlpHid], o[kMlpOut];
};

__device__ __forceinline__ void forward(const float *w, const float *f, Fwd &a) {
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float s = w[kMlpB1 + j];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) s = fmaf(w[kMlpW1 + j * kMlpIn + k], f[k], s);
    a.h1[j] = tanhf(s);
  }
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float s = w[kMlpB2 + j];
#pragma unroll
    for (int k = 0; k < kMlpHid; ++k) s = fmaf(w[kMlpW2 + j * kMlpHid + k], a.h1[k], s);
    a.h2[j] = tanhf(s);
  }
#pragma unroll
  for (int q = 0; q < kMlpOut; ++q) {
    float s = w[kMlpB3 + q];
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) s = fmaf(w[kMlpW3 + q * kMlpHid + j], a.h2[j], s);
    a.o[q] = s;
  }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ wg, int n, const float *__restrict__ feat,
                                                     float *__restrict__ out) {
  __shared__ float w[kMlpParams];
  for (int e = threadIdx.x; e < kMlpParams; e += blockDim.x) w[e] = wg[e];
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float f[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) f[k] = feat[(long)r * kMlpIn + k];
  Fwd a;
  forward(w, f, a);
#pragma unroll
  for (int q = 0; q < kMlpOut; ++q) out[(long)r * kMlpOut + q] = a.o[q];
}

// per-workgroup gradient partials gpart[block][kMlpParams] and loss partials
__global__ __launch_bounds__(kRows) void k_mlp_grad(const float *__restrict__ wg, int n, const float *__restrict__ feat,
                                                    const float *__restrict__ tgt, float *__restrict__ gpart,
                                                    float *__restrict__ lpart) {
  __shared__ float w[kMlpParams];
  __shared__ float sf[kRows][kMlpIn];
  __shared__ float sh1[kRows][kMlpHid];
  __shared__ float sh2[kRows][kMlpHid];
  __shared__ float dz1[kRows][kMlpHid];
  __shared__ float dz2[kRows][kMlpHid];
  __shared__ float dout[kRows][kMlpOut];
  __shared__ double red[2];
  const int lane = threadIdx.x;
  for (int e = lane; e < kMlpParams; e += kRows) w[e] = wg[e];
  __syncthreads();
  const int r = blockIdx.x * kRows + lane;
  const bool valid = r < n;
  float f[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) f[k] = valid ? feat[(long)r * kMlpIn + k] : 0.0f;
  Fwd a;
  forward(w, f, a);
  // loss and d loss / d o
  double loss = 0.0;
  float d[kMlpOut] = {0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const float sc = 1.0f / (f[0] * 10.0f + 1.0f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float ur = tgt[(long)r * 8 + 4 * h], ui = tgt[(long)r * 8 + 4 * h + 1];
      const float wr = tgt[(long)r * 8 + 4 * h + 2], wi = tgt[(long)r * 8 + 4 * h + 3];
      const float mr = a.o[2 * h] * sc, mi = a.o[2 * h + 1] * sc;
      const float er = mr * ur - mi * ui - wr, ei = mr * ui + mi * ur - wi;
      loss += (double)er * er + (double)ei * ei;
      // e = s (o_a + i o_b) u - w:  d|e|^2/d o_a = 2 Re(conj(e) s u), d/d o_b = -2 Im(conj(e) s u)
      const float sur = sc * ur, sui = sc * ui;
      const float cr = er * sur + ei * sui, ci = er * sui - ei * sur;
      d[2 * h] = 2.0f * cr / n;
      d[2 * h + 1] = -2.0f * ci / n;
    }
  }
  // backward through the layers for this row
  float dh2[kMlpHid];
  for (int j = 0; j < kMlpHid; ++j) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < kMlpOut; ++q) s = fmaf(w[kMlpW3 + q * kMlpHid + j], d[q], s);
    dh2[j] = s * (1.0f - a.h2[j] * a.h2[j]);
  }
  for (int k = 0; k < kMlpHid; ++k) {
    float s = 0.0f;
#pragma unroll 8
    for (int j = 0; j < kMlpHid; ++j) s = fmaf(w[kMlpW2 + j * kMlpHid + k], dh2[j], s);
    dz1[lane][k] = s * (1.0f - a.h1[k] * a.h1[k]);
  }
  for (int j = 0; j < kMlpHid; ++j) {
    sh1[lane][j] = a.h1[j];
    sh2[lane][j] = a.h2[j];
    dz2[lane][j] = dh2[j];
  }
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) sf[lane][k] = f[k];
#pragma unroll
  for (int q = 0; q < kMlpOut; ++q) dout[lane][q] = d[q];
  // loss partial
  double tot = loss;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  __syncthreads();
  // weight-gradient tiles: sum over the 64 rows in a fixed order
  float *gp = gpart + (long)blockIdx.x * kMlpParams;
  for (int e = lane; e < kMlpParams; e += kRows) {
    float s = 0.0f;
    if (e < kMlpB1) {
      const int j = e / kMlpIn, k = e - j * kMlpIn;
      for (int rr = 0; rr < kRows; ++rr) s = fmaf(dz1[rr][j], sf[rr][k], s);
    } else if (e < kMlpW2) {
      const int j = e - kMlpB1;
      for (int rr = 0; rr < kRows; ++rr) s += dz1[rr][j];
    } else if (e < kMlpB2) {
      const int j = (e - kMlpW2) / kMlpHid, k = (e - kMlpW2) - j * kMlpHid;
      for (int rr = 0; rr < kRows; ++rr) s = fmaf(dz2[rr][j], sh1[rr][k], s);
    } else if (e < kMlpW3) {
      const int j = e - kMlpB2;
      for (int rr = 0; rr < kRows; ++rr) s += dz2[rr][j];
    } else if (e < kMlpB3) {
      const int q = (e - kMlpW3) / kMlpHid, j = (e - kMlpW3) - q * kMlpHid;
      for (int rr = 0; rr < kRows; ++rr) s = fmaf(dout[rr][q], sh2[rr][j], s);
    } else {
      const int q = e - kMlpB3;
      for (int rr = 0; rr < kRows; ++rr) s += dout[rr][q];
    }
    gp[e] = s;
  }
  if (lane == 0) lpart[blockIdx.x] = (float)(tot / n);
}

// grad[e] = sum over blocks of gpart[block][e] (fixed order); loss likewise
__global__ void k_mlp_reduce(const float *__restrict__ gpart, const float *__restrict__ lpart, int nb,
                             float *__restrict__ grad, float *__restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kMlpParams) {
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += gpart[(long)b * kMlpParams + e];
    grad[e] = s;
  }
  if (e == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += lpart[b];
    loss[0] = (float)s;
  }
}

__global__ void k_mlp_adam(float *__restrict__ w, float *__restrict__ m1, float *__restrict__ m2,
                           const float *__restrict__ g, float lr, float c1, float c2, uint16_t *__restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpParams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float ge = g[e];
  const float a = b1 * m1[e] + (1.0f - b1) * ge;
  const float b = b2 * m2[e] + (1.0f - b2) * ge * ge;
  m1[e] = a;
  m2[e] = b;
  const float wn = w[e] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  w[e] = wn;
  wb[e] = to_bf16(wn);
}

// Training rows from residuals (caller order).  Vector a with band energy eps[a]
// and shift z = omega[a] + i eta yields, for plane wave u = stride * t, two rows:
//   row 2t:   (D r, r, D b, b) / norms      row 2t+1: (sqrt(c) r, 0, sqrt(c) b, 0) / norms
// with D = diag_u - eps - z and c = off2_u the diagonal and the squared
// off-diagonal column norm of H + alpha P_occ.  Summed over the plane waves of
// a vector, the loss of these rows is the diagonal sparse-approximate-inverse
// objective sum_G |r_G|^2 (|1 - D_G m_G|^2 + c_G |m_G|^2) / ||r||^2.
__global__ __launch_bounds__(256) void k_mlp_rows(int npw, const int32_t *__restrict__ u2i,
                                                  const double *__restrict__ kin, const double *__restrict__ diag,
                                                  const double *__restrict__ off2, const double *__restrict__ eps,
                                                  const double *__restrict__ omega, double eta,
                                                  const double2 *__restrict__ rv, const double2 *__restrict__ bv,
                                                  int stride, int per_vec, float *__restrict__ feat,
                                                  float *__restrict__ tgt) {
  __shared__ double sh[8];
  const int a = blockIdx.x;
  const double2 *r = rv + (long)a * npw, *b = bv + (long)a * npw;
  double acc[2] = {0.0, 0.0};
  for (int t = threadIdx.x; t < per_vec; t += 256) {
    const double2 x = r[(long)t * stride], y = b[(long)t * stride];
    acc[0] += x.x * x.x + x.y * x.y;
    acc[1] += y.x * y.x + y.y * y.y;
  }
  double tot[2];
  wg_sum<256, 2>(acc, sh, tot);
  const double sr = tot[0] > 0.0 ? 1.0 / sqrt(tot[0]) : 0.0;
  const double sb = tot[1] > 0.0 ? 1.0 / sqrt(tot[1]) : 0.0;
  const double e = eps[a], om = omega[a];
  for (int t = threadIdx.x; t < per_vec; t += 256) {
    const int u = t * stride;
    float f[kMlpIn];
    mlp_features(kin[u2i[u]], e, om, eta, f);
    const double2 d = make_double2(diag[u] - e - om, -eta);
    const double c = sqrt(fmax(off2[u], 0.0));
    const double2 x = r[u], y = b[u];
    const double2 dx = c_mul(d, x), dy = c_mul(d, y);
    const long row = 2 * ((long)a * per_vec + t);
    float *f0 = feat + row * kMlpIn;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) f0[k] = f0[kMlpIn + k] = f[k];
    float *t0 = tgt + row * 8;
    t0[0] = (float)(dx.x * sr);
    t0[1] = (float)(dx.y * sr);
    t0[2] = (float)(x.x * sr);
    t0[3] = (float)(x.y * sr);
    t0[4] = (float)(dy.x * sb);
    t0[5] = (float)(dy.y * sb);
    t0[6] = (float)(y.x * sb);
    t0[7] = (float)(y.y * sb);
    t0[8] = (float)(c * x.x * sr);
    t0[9] = (float)(c * x.y * sr);
    t0[10] = 0.0f;
    t0[11] = 0.0f;
    t0[12] = (float)(c * y.x * sb);
    t0[13] = (float)(c * y.y * sb);
    t0[14] = 0.0f;
    t0[15] = 0.0f;
  }
}

// unit vectors e_{g0 + a} (internal order) for a < n
__global__ void k_unit(int npw, int g0, int n, double2 *__restrict__ x) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * npw) return;
  const int a = (int)(e / npw), g = (int)(e - (long)a * npw);
  x[e] = make_double2(g == g0 + a ? 1.0 : 0.0, 0.0);
}

// column statistics of the operator from y_a = A e_{g0+a}: diagonal and squared off-diagonal norm,
// written in the caller's order
__global__ __launch_bounds__(256) void k_colstats(int npw, int g0, const double2 *__restrict__ y,
                                                  const int32_t *__restrict__ i2u, double *__restrict__ diag,
                                                  double *__restrict__ off2) {
  __shared__ double sh[8];
  const int a = blockIdx.x, g = g0 + a;
  const double2 *ya = y + (long)a * npw;
  double acc[1] = {0.0};
  for (int k = threadIdx.x; k < npw; k += 256) {
    if (k == g) continue;
    const double2 v = ya[k];
    acc[0] += v.x * v.x + v.y * v.y;
  }
  double tot[1];
  wg_sum<256, 1>(acc, sh, tot);
  if (threadIdx.x == 0) {
    diag[i2u[g]] = ya[g].x;
    off2[i2u[g]] = tot[0];
  }
}

}  // namespace

sgw_status mlp_upload_bf16(sgw_ctx *ctx, sgw_mlp *m) {
  hipLaunchKernelGGL(k_to_bf16, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, m->w, m->wb, kMlpParams);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

static sgw_status mlp_grad_impl(sgw_ctx *ctx, sgw_mlp *m, int n, const float *feat, const float *tgt) {
  const int nb = (n + kRows - 1) / kRows;
  if (nb > m->gpart_blocks) {
    if (m->gpart) hipFree(m->gpart);
    if (m->loss) hipFree(m->loss);
    m->gpart = nullptr;
    m->loss = nullptr;
    m->gpart_blocks = 0;
    SGW_HIP(hipMalloc(&m->gpart, sizeof(float) * kMlpParams * (size_t)nb));
    SGW_HIP(hipMalloc(&m->loss, sizeof(float) * (size_t)(nb + 1)));
    m->gpart_blocks = nb;
  }
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kRows), 0, ctx->stream, m->w, n, feat, tgt, m->gpart, m->loss + 1);
  SGW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, m->gpart, m->loss + 1,
                     nb, m->grad, m->loss);
  SGW_HIP(hipGetLastError());
  return SGW_OK;
}

}  // namespace sgw

using namespace sgw;

extern "C" sgw_status sgw_mlp_create(sgw_ctx *ctx, const float *init_w, uint64_t seed, sgw_mlp **out) {
  if (!ctx || !out) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_create: NULL argument");
  *out = nullptr;
  std::vector<float> w(kMlpParams, 0.0f);
  if (init_w) {
    std::memcpy(w.data(), init_w, sizeof(float) * kMlpParams);
    for (float v : w)
      if (!std::isfinite(v)) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_create: non-finite weight");
  } else {
    // Glorot-uniform weights, zero biases; the preconditioner output starts at m = 1 / (T + 1)
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int fan_out, int fan_in) {
      const float lim = std::sqrt(6.0f / (fan_in + fan_out));
      std::uniform_real_distribution<float> d(-lim, lim);
      for (int i = 0; i < fan_out * fan_in; ++i) w[off + i] = d(rng);
    };
    fill(kMlpW1, kMlpHid, kMlpIn);
    fill(kMlpW2, kMlpHid, kMlpHid);
    fill(kMlpW3, kMlpOut, kMlpHid);
    w[kMlpB3 + 0] = 1.0f;
    w[kMlpB3 + 2] = 1.0f;
  }
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_mlp *m = new sgw_mlp();
  m->ctx = ctx;
  m->device = ctx->device;
  auto bad = [&](hipError_t e) {
    if (m->w) hipFree(m->w);
    if (m->wb) hipFree(m->wb);
    if (m->m1) hipFree(m->m1);
    if (m->m2) hipFree(m->m2);
    if (m->grad) hipFree(m->grad);
    delete m;
    return fail(SGW_ERR_HIP, std::string("sgw_mlp_create: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMalloc(&m->w, sizeof(float) * kMlpParams)) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&m->wb, sizeof(uint16_t) * kMlpParams)) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&m->m1, sizeof(float) * kMlpParams)) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&m->m2, sizeof(float) * kMlpParams)) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&m->grad, sizeof(float) * kMlpParams)) != hipSuccess) return bad(e);
  if ((e = hipMemcpyAsync(m->w, w.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess)
    return bad(e);
  if ((e = hipMemsetAsync(m->m1, 0, sizeof(float) * kMlpParams, ctx->stream)) != hipSuccess) return bad(e);
  if ((e = hipMemsetAsync(m->m2, 0, sizeof(float) * kMlpParams, ctx->stream)) != hipSuccess) return bad(e);
  sgw_status st = mlp_upload_bf16(ctx, m);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return bad(e);
  if (st != SGW_OK) {
    sgw_mlp_destroy(m);
    return st;
  }
  *out = m;
  return SGW_OK;
}

extern "C" sgw_status sgw_mlp_destroy(sgw_mlp *m) {
  if (!m) return SGW_OK;
  hipSetDevice(m->device);
  void *ptrs[] = {m->w, m->wb, m->m1, m->m2, m->grad, m->gpart, m->loss};
  for (void *p : ptrs)
    if (p) hipFree(p);
  delete m;
  return SGW_OK;
}

extern "C" sgw_status sgw_mlp_get_weights(const sgw_mlp *m, float *w) {
  if (!m || !w) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_get_weights: NULL argument");
  SGW_HIP(hipSetDevice(m->device));
  SGW_HIP(hipStreamSynchronize(m->ctx->stream));
  SGW_HIP(hipMemcpy(w, m->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return SGW_OK;
}

extern "C" sgw_status sgw_mlp_set_weights(sgw_mlp *m, const float *w) {
  if (!m || !w) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_set_weights: NULL argument");
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(w[i])) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_set_weights: non-finite weight");
  SGW_HIP(hipSetDevice(m->device));
  SGW_HIP(hipMemcpyAsync(m->w, w, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->ctx->stream));
  sgw_status st = mlp_upload_bf16(m->ctx, m);
  if (st != SGW_OK) return st;
  SGW_HIP(hipStreamSynchronize(m->ctx->stream));
  return SGW_OK;
}

extern "C" int32_t sgw_mlp_num_params(void) { return kMlpParams; }

extern "C" sgw_status sgw_mlp_forward(sgw_ctx *ctx, const sgw_mlp *m, int n_rows, const float *feat, float *out) {
  if (!ctx || !m) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_forward: NULL context or MLP");
  if (n_rows < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_forward: n_rows < 0");
  if (n_rows == 0) return SGW_OK;
  if (!feat || !out) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_forward: NULL array");
  SGW_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_mlp_forward, dim3((n_rows + 255) / 256), dim3(256), 0, ctx->stream, m->w, n_rows, feat, out);
  SGW_HIP(hipGetLastError());
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  return SGW_OK;
}

extern "C" sgw_status sgw_mlp_grad(sgw_ctx *ctx, const sgw_mlp *m, int n_rows, const float *feat, const float *tgt,
                                   float *grad_out, float *loss_out) {
  if (!ctx || !m) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_grad: NULL context or MLP");
  if (n_rows <= 0 || !feat || !tgt || !grad_out) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_grad: empty or NULL input");
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_mlp *mm = const_cast<sgw_mlp *>(m);
  sgw_status st = mlp_grad_impl(ctx, mm, n_rows, feat, tgt);
  if (st != SGW_OK) return st;
  SGW_HIP(hipMemcpyAsync(grad_out, mm->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, ctx->stream));
  if (loss_out) SGW_HIP(hipMemcpyAsync(loss_out, mm->loss, sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  return SGW_OK;
}

extern "C" sgw_status sgw_mlp_train_step(sgw_ctx *ctx, sgw_mlp *m, int n_rows, const float *feat, const float *tgt,
                                         float lr, float *loss_out) {
  if (!ctx || !m) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_train_step: NULL context or MLP");
  if (n_rows <= 0 || !feat || !tgt) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_train_step: empty or NULL input");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_train_step: lr must be positive");
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_status st = mlp_grad_impl(ctx, m, n_rows, feat, tgt);
  if (st != SGW_OK) return st;
  m->step += 1;
  const float c1 = 1.0f - std::pow(0.9f, (float)m->step), c2 = 1.0f - std::pow(0.999f, (float)m->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, m->w, m->m1, m->m2, m->grad,
                     lr, c1, c2, m->wb);
  SGW_HIP(hipGetLastError());
  if (loss_out) {
    SGW_HIP(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  }
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  return SGW_OK;
}

extern "C" sgw_status sgw_operator_columns(sgw_ctx *ctx, const sgw_ham *h, int n_occ, const sgw_c128 *psi,
                                           double alpha, double *diag, double *off2) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_operator_columns: NULL context or Hamiltonian");
  if (n_occ < 0 || n_occ > kMaxOcc) return fail(SGW_ERR_INVALID_ARG, "sgw_operator_columns: bad n_occ");
  if (!diag || !off2 || (n_occ > 0 && !psi)) return fail(SGW_ERR_INVALID_ARG, "sgw_operator_columns: NULL array");
  if (!std::isfinite(alpha)) return fail(SGW_ERR_INVALID_ARG, "sgw_operator_columns: alpha not finite");
  SGW_HIP(hipSetDevice(ctx->device));
  const int npw = h->n_pw;
  const int batch = std::min(npw, 512);
  const size_t vb = sizeof(double2) * (size_t)batch * npw;
  void *buf = nullptr;
  // [psi (internal order) | X | Y | T | C]
  const size_t psi_b = sizeof(double2) * (size_t)std::max(n_occ, 1) * npw;
  const size_t t_b = hx_tbuf_bytes(h, batch);
  const size_t c_b = sizeof(double2) * (size_t)kProjChunks * batch * std::max(n_occ, 1);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  SGW_HIP(hipMalloc(&buf, al(psi_b) + 2 * al(vb) + al(t_b) + al(c_b)));
  char *B = (char *)buf;
  double2 *ps = (double2 *)B;
  double2 *X = (double2 *)(B + al(psi_b));
  double2 *Y = (double2 *)(B + al(psi_b) + al(vb));
  double2 *T = (double2 *)(B + al(psi_b) + 2 * al(vb));
  double2 *Cp = (double2 *)(B + al(psi_b) + 2 * al(vb) + al(t_b));
  sgw_status st = permute(ctx, npw, n_occ, (const double2 *)psi, npw, ps, npw, h->d_i2u, 0);
  for (int g0 = 0; g0 < npw && st == SGW_OK; g0 += batch) {
    const int n = std::min(batch, npw - g0);
    const long tot = (long)n * npw;
    hipLaunchKernelGGL(k_unit, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, npw, g0, n, X);
    if (hipGetLastError() != hipSuccess) st = fail(SGW_ERR_HIP, "sgw_operator_columns: launch failed");
    if (st == SGW_OK) st = proj_dot(ctx, npw, n_occ, ps, n, contiguous(X, npw), Cp, batch);
    if (st == SGW_OK) st = hx_batch(ctx, h, n, contiguous(X, npw), Y, npw, T);
    if (st == SGW_OK) st = proj_apply(ctx, npw, n_occ, ps, n, contiguous(X, npw), Cp, batch, Y, npw, alpha, 1);
    if (st == SGW_OK) {
      hipLaunchKernelGGL(k_colstats, dim3(n), dim3(256), 0, ctx->stream, npw, g0, Y, h->d_i2u, diag, off2);
      if (hipGetLastError() != hipSuccess) st = fail(SGW_ERR_HIP, "sgw_operator_columns: launch failed");
    }
  }
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  hipFree(buf);
  if (st == SGW_OK && e != hipSuccess)
    st = fail(SGW_ERR_HIP, std::string("sgw_operator_columns: ") + hipGetErrorString(e));
  return st;
}

extern "C" sgw_status sgw_mlp_rows(sgw_ctx *ctx, const sgw_ham *h, const double *diag, const double *off2, int n_vec,
                                   const double *eps, const double *omega, double eta, const sgw_c128 *r,
                                   const sgw_c128 *b, int stride, float *feat, float *tgt) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_rows: NULL context or Hamiltonian");
  if (n_vec < 0 || stride <= 0) return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_rows: bad n_vec or stride");
  if (n_vec == 0) return SGW_OK;
  if (!diag || !off2 || !eps || !omega || !r || !b || !feat || !tgt)
    return fail(SGW_ERR_INVALID_ARG, "sgw_mlp_rows: NULL array");
  SGW_HIP(hipSetDevice(ctx->device));
  const int per_vec = (h->n_pw + stride - 1) / stride;
  double *d_eo = nullptr;
  SGW_HIP(hipMalloc(&d_eo, sizeof(double) * 2 * n_vec));
  hipMemcpyAsync(d_eo, eps, sizeof(double) * n_vec, hipMemcpyHostToDevice, ctx->stream);
  hipMemcpyAsync(d_eo + n_vec, omega, sizeof(double) * n_vec, hipMemcpyHostToDevice, ctx->stream);
  hipLaunchKernelGGL(k_mlp_rows, dim3(n_vec), dim3(256), 0, ctx->stream, h->n_pw, h->d_u2i, h->d_kin, diag, off2,
                     d_eo, d_eo + n_vec, eta, (const double2 *)r, (const double2 *)b, stride, per_vec, feat, tgt);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(ctx->stream);
  hipFree(d_eo);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(SGW_ERR_HIP, std::string("sgw_mlp_rows: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  return SGW_OK;
}
