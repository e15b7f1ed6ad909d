// C ABI of libsgw.so: contexts, Hamiltonians, test hooks and the Sternheimer
// solve driver (host-side scheduling of the device-resident Krylov slots).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "pershift.h"
#include "sgw_internal.h"
#include "solver_state.h"

namespace sgw {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
sgw_status fail(sgw_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

const char *kernel_name(int id) {
  static const char *names[K_COUNT] = {"hx_sticks_inv", "hx_planes", "hx_sticks_fwd", "proj_dot",
                                       "proj_apply",    "rhs_source", "slot_init",    "lanczos_step",
                                       "tridiag",       "combine",   "residual",     "permute",
                                       "nl_dot",        "nl_apply",  "chi_dot",      "dielectric",
                                       "blk_product"};
  return (id >= 0 && id < K_COUNT) ? names[id] : "?";
}

static hipEvent_t get_event(sgw_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void timing_begin(sgw_ctx *ctx, int kid, double bytes, double flops, PendingTiming *t) {
  t->kid = -1;
  if (!(ctx->profile_mask & (1u << kid))) return;
  t->kid = kid;
  t->bytes = bytes;
  t->flops = flops;
  t->start = get_event(ctx);
  t->stop = get_event(ctx);
  if (!t->start || !t->stop) {
    t->kid = -1;
    return;
  }
  hipEventRecord(t->start, ctx->stream);
}

void timing_end(sgw_ctx *ctx, PendingTiming *t) {
  if (t->kid < 0) return;
  hipEventRecord(t->stop, ctx->stream);
  ctx->pending.push_back(*t);
}

// Must be called after the stream has been synchronised.
sgw_status timing_collect(sgw_ctx *ctx) {
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      KernelStat &s = ctx->stats[p.kid];
      s.launches += 1;
      s.ms += ms;
      s.bytes += p.bytes;
      s.flops += p.flops;
    }
    ctx->event_pool.push_back(p.start);
    ctx->event_pool.push_back(p.stop);
  }
  ctx->pending.clear();
  return SGW_OK;
}

sgw_status ensure_pinned(sgw_ctx *ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return SGW_OK;
  if (ctx->pinned) hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  size_t nb = std::max<size_t>(bytes, 1 << 16);
  SGW_HIP(hipHostMalloc(&ctx->pinned, nb, hipHostMallocDefault));
  ctx->pinned_bytes = nb;
  return SGW_OK;
}

sgw_status sync(sgw_ctx *ctx) {
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  return timing_collect(ctx);
}

}  // namespace sgw

using namespace sgw;

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free H.x (sgw_apply_h_noalloc)
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
constexpr size_t kAlign256 = 256;
constexpr int kScratchDevices = 64;
}  // namespace

// One copy per device, held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels and copies take the address from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};        // device address of `scratch`, per device
hipError_t g_scratch_err[kScratchDevices] = {};   // the lookup's error, when it failed

// Looks up this device's copy of `scratch` once (the device must be current).  A failure is kept and
// reported by sgw_apply_h_noalloc; the rest of the library does not need the array.
void scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_scratch_ptr[device] = p;
  else g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

void *scratch_ptr(int device, hipError_t *err) {
  if (device < 0 || device >= kScratchDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}
}  // namespace

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
extern "C" const char *sgw_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *sgw_version(void) { return "sgw-mi355x 0.1 (gfx950)"; }

extern "C" sgw_status sgw_ctx_create(int device, void *hip_stream, sgw_ctx **out) {
  if (!out) return fail(SGW_ERR_INVALID_ARG, "sgw_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  SGW_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SGW_ERR_INVALID_ARG, "sgw_ctx_create: no such device");
  SGW_HIP(hipSetDevice(device));
  scratch_setup(device);
  sgw_ctx *c = new sgw_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return SGW_OK;
}

extern "C" sgw_status sgw_ctx_destroy(sgw_ctx *ctx) {
  if (!ctx) return SGW_OK;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  timing_collect(ctx);
  for (auto e : ctx->event_pool) hipEventDestroy(e);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  blas_release(ctx);
  delete ctx;
  return SGW_OK;
}

extern "C" sgw_status sgw_ctx_set_fft_planes(sgw_ctx *ctx, int fft_planes) {
  if (!ctx) return fail(SGW_ERR_INVALID_ARG, "ctx is NULL");
  if (fft_planes < SGW_FFT_AUTO || fft_planes > SGW_FFT_TRI)
    return fail(SGW_ERR_INVALID_ARG, "sgw_ctx_set_fft_planes: unknown plane kernel");
  ctx->fft_planes = fft_planes;
  return SGW_OK;
}

extern "C" sgw_status sgw_plane_kernel(sgw_ctx *ctx, const sgw_ham *ham, int precision, int32_t *out) {
  if (!ctx || !ham || !out) return fail(SGW_ERR_INVALID_ARG, "sgw_plane_kernel: NULL argument");
  if (precision != SGW_FP64 && precision != SGW_MIXED)
    return fail(SGW_ERR_INVALID_ARG, "sgw_plane_kernel: unknown precision mode");
  *out = hx_plane_kernel(ctx, ham, precision == SGW_MIXED);
  return SGW_OK;
}

extern "C" sgw_status sgw_ctx_set_profiling(sgw_ctx *ctx, const char *kernels) {
  if (!ctx) return fail(SGW_ERR_INVALID_ARG, "ctx is NULL");
  if (!kernels || !*kernels) {
    ctx->profile_mask = 0;
    return SGW_OK;
  }
  if (std::strcmp(kernels, "all") == 0) {
    ctx->profile_mask = (1u << K_COUNT) - 1;
    return SGW_OK;
  }
  unsigned mask = 0;
  std::string s(kernels);
  size_t pos = 0;
  while (pos <= s.size()) {
    size_t e = s.find(',', pos);
    if (e == std::string::npos) e = s.size();
    const std::string name = s.substr(pos, e - pos);
    int k = 0;
    for (; k < K_COUNT; ++k)
      if (name == kernel_name(k)) break;
    if (k == K_COUNT) return fail(SGW_ERR_INVALID_ARG, "sgw_ctx_set_profiling: unknown kernel " + name);
    mask |= 1u << k;
    pos = e + 1;
  }
  ctx->profile_mask = mask;
  return SGW_OK;
}

extern "C" sgw_status sgw_ctx_reset_stats(sgw_ctx *ctx) {
  if (!ctx) return fail(SGW_ERR_INVALID_ARG, "ctx is NULL");
  for (auto &s : ctx->stats) s = KernelStat();
  return SGW_OK;
}

extern "C" sgw_status sgw_kernel_stats(sgw_ctx *ctx, const char *name, int64_t *launches, double *total_ms,
                                       double *alg_bytes, double *alg_flops) {
  if (!ctx || !name) return fail(SGW_ERR_INVALID_ARG, "sgw_kernel_stats: NULL argument");
  for (int k = 0; k < K_COUNT; ++k) {
    if (std::strcmp(kernel_name(k), name) == 0) {
      const KernelStat &s = ctx->stats[k];
      if (launches) *launches = s.launches;
      if (total_ms) *total_ms = s.ms;
      if (alg_bytes) *alg_bytes = s.bytes;
      if (alg_flops) *alg_flops = s.flops;
      return SGW_OK;
    }
  }
  return fail(SGW_ERR_INVALID_ARG, std::string("sgw_kernel_stats: unknown kernel ") + name);
}

// ---------------------------------------------------------------------------
// Hamiltonian
// ---------------------------------------------------------------------------
static int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

template <class T>
static sgw_status upload(sgw_ctx *ctx, T **dst, const std::vector<T> &src) {
  *dst = nullptr;
  if (src.empty()) return SGW_OK;
  SGW_HIP(hipMalloc((void **)dst, sizeof(T) * src.size()));
  SGW_HIP(hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, ctx->stream));
  return SGW_OK;
}

static void ham_free(sgw_ham *h) {
  if (!h) return;
  void *ptrs[] = {h->d_i2u, h->d_u2i,  h->d_stick_off, h->d_rows, h->d_stick_ij, h->d_pw_stick,
                  h->d_pw_z, h->d_miller_int, h->d_kin, h->d_vt, h->d_box, h->d_tw,
                  h->d_vt32, h->d_tw32, h->d_beta, h->d_ekb};
  for (void *p : ptrs)
    if (p) hipFree(p);
  delete h;
}

extern "C" sgw_status sgw_ham_create(sgw_ctx *ctx, const sgw_ham_desc *d, sgw_ham **out) {
  if (!ctx || !d || !out) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: NULL argument");
  *out = nullptr;
  if (d->n_pw <= 0 || !d->miller) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: empty basis");
  if (!d->v_loc) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: v_loc is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!hx_grid_supported(d->grid[a]))
      return fail(SGW_ERR_UNSUPPORTED, "sgw_ham_create: grid size " + std::to_string(d->grid[a]) +
                                           " not in {16,24,32,48,64,72}");
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (!std::isfinite(d->recip[a][b])) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: recip not finite");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->kvec[a])) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: kvec not finite");
  const int npw = d->n_pw;
  const int *n = d->grid;
  int mmin[3] = {1 << 30, 1 << 30, 1 << 30}, mmax[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (int g = 0; g < npw; ++g)
    for (int a = 0; a < 3; ++a) {
      mmin[a] = std::min(mmin[a], d->miller[3 * g + a]);
      mmax[a] = std::max(mmax[a], d->miller[3 * g + a]);
    }
  for (int a = 0; a < 3; ++a) {
    const int amax = std::max(std::abs(mmin[a]), std::abs(mmax[a]));
    if (2 * amax + 1 > n[a])
      return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: grid too small for the basis along axis " +
                                           std::to_string(a) + " (need 2*max|m|+1 <= N)");
  }
  // lookup box and distinctness
  int box_dim[3];
  long box_vol = 1;
  for (int a = 0; a < 3; ++a) {
    box_dim[a] = mmax[a] - mmin[a] + 1;
    box_vol *= box_dim[a];
  }
  if (box_vol > (1L << 28)) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: Miller range too large");
  std::vector<int32_t> box(box_vol, -1);
  for (int g = 0; g < npw; ++g) {
    const int *m = d->miller + 3 * g;
    const long idx = ((long)(m[0] - mmin[0]) * box_dim[1] + (m[1] - mmin[1])) * box_dim[2] + (m[2] - mmin[2]);
    if (box[idx] >= 0) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_create: repeated Miller index");
    box[idx] = g;
  }
  // sticks along axis 2, sorted by (m0, m1); plane waves within a stick by m2
  std::vector<int> order(npw);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const int *ma = d->miller + 3 * a, *mb = d->miller + 3 * b;
    if (ma[0] != mb[0]) return ma[0] < mb[0];
    if (ma[1] != mb[1]) return ma[1] < mb[1];
    return ma[2] < mb[2];
  });
  std::vector<int32_t> i2u(npw), u2i(npw), pw_stick(npw), pw_z(npw), miller_int(3 * npw), stick_off, stick_ij;
  // per row m0 = mmin[0] + t: first stick and the m1 range (one contiguous run)
  std::vector<int4> rows(mmax[0] - mmin[0] + 1, make_int4(0, 1, 0, 0));
  std::vector<char> row_seen(rows.size(), 0);
  std::vector<double> kin(npw);
  int ns = 0;
  for (int gi = 0; gi < npw; ++gi) {
    const int u = order[gi];
    const int *m = d->miller + 3 * u;
    if (gi == 0 || m[0] != d->miller[3 * order[gi - 1]] || m[1] != d->miller[3 * order[gi - 1] + 1]) {
      stick_off.push_back(gi);
      stick_ij.push_back((imod(m[0], n[0]) << 16) | imod(m[1], n[1]));
      int4 &r = rows[m[0] - mmin[0]];
      if (!row_seen[m[0] - mmin[0]]) {
        row_seen[m[0] - mmin[0]] = 1;
        r = make_int4(ns, m[1], m[1], 0);
      } else if (m[1] != r.z + 1) {
        return fail(SGW_ERR_UNSUPPORTED, "sgw_ham_create: the sticks of row m0 = " + std::to_string(m[0]) +
                                             " do not form one contiguous m1 range (basis not sphere-like)");
      } else {
        r.z = m[1];
      }
      ++ns;
    }
    i2u[gi] = u;
    u2i[u] = gi;
    pw_stick[gi] = ns - 1;
    pw_z[gi] = imod(m[2], n[2]);
    for (int a = 0; a < 3; ++a) miller_int[3 * gi + a] = m[a];
    double kg[3];
    for (int c = 0; c < 3; ++c)
      kg[c] = d->kvec[c] + m[0] * d->recip[0][c] + m[1] * d->recip[1][c] + m[2] * d->recip[2][c];
    kin[gi] = 0.5 * (kg[0] * kg[0] + kg[1] * kg[1] + kg[2] * kg[2]);
  }
  stick_off.push_back(npw);
  // twiddle tables exp(-2 pi i t / N) for the three axes
  std::vector<double2> tw;
  std::vector<float2> tw32;
  int tw_off[3];
  for (int a = 0; a < 3; ++a) {
    tw_off[a] = (int)tw.size();
    for (int t = 0; t < n[a]; ++t) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * t / n[a];
      tw.push_back(make_double2((double)cosl(ang), (double)sinl(ang)));
      tw32.push_back(make_float2((float)cosl(ang), (float)sinl(ang)));
    }
  }
  SGW_HIP(hipSetDevice(ctx->device));
  sgw_ham *h = new sgw_ham();
  h->ctx = ctx;
  h->device = ctx->device;
  for (int a = 0; a < 3; ++a) {
    h->n[a] = n[a];
    h->kvec[a] = d->kvec[a];
    h->box_lo[a] = mmin[a];
    h->box_dim[a] = box_dim[a];
    h->tw_off[a] = tw_off[a];
    for (int b = 0; b < 3; ++b) h->recip[a][b] = d->recip[a][b];
  }
  h->n_pw = npw;
  h->n_stick = ns;
  h->m0_lo = mmin[0];
  h->n_row = mmax[0] - mmin[0] + 1;
  h->m1_lo = mmin[1];
  h->m1_hi = mmax[1];
  h->m2_lo = mmin[2];
  h->m2_hi = mmax[2];
  h->miller.assign(d->miller, d->miller + 3 * npw);
  sgw_status st = SGW_OK;
#define SGW_UP(dst, src)                                   \
  if ((st = upload(ctx, &(dst), (src))) != SGW_OK) {        \
    hipStreamSynchronize(ctx->stream);                      \
    ham_free(h);                                            \
    return st;                                              \
  }
  SGW_UP(h->d_i2u, i2u);
  SGW_UP(h->d_u2i, u2i);
  SGW_UP(h->d_stick_off, stick_off);
  SGW_UP(h->d_rows, rows);
  SGW_UP(h->d_stick_ij, stick_ij);
  SGW_UP(h->d_pw_stick, pw_stick);
  SGW_UP(h->d_pw_z, pw_z);
  SGW_UP(h->d_miller_int, miller_int);
  SGW_UP(h->d_kin, kin);
  SGW_UP(h->d_box, box);
  SGW_UP(h->d_tw, tw);
  SGW_UP(h->d_tw32, tw32);
#undef SGW_UP
  const long ntot = (long)n[0] * n[1] * n[2];
  hipError_t e = hipMalloc((void **)&h->d_vt, sizeof(double) * ntot);
  if (e == hipSuccess) e = hipMalloc((void **)&h->d_vt32, sizeof(float) * ntot);
  if (e != hipSuccess) {
    hipStreamSynchronize(ctx->stream);
    ham_free(h);
    return fail(SGW_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  st = transpose_potential(ctx, d->v_loc, h->d_vt, h->d_vt32, n);
  e = hipStreamSynchronize(ctx->stream);
  if (st != SGW_OK || e != hipSuccess) {
    ham_free(h);
    return st != SGW_OK ? st : fail(SGW_ERR_HIP, std::string("sgw_ham_create: ") + hipGetErrorString(e));
  }
  *out = h;
  return SGW_OK;
}

extern "C" sgw_status sgw_ham_destroy(sgw_ham *h) {
  if (!h) return SGW_OK;
  // the context may already be gone: only the device id is used (hipFree waits for the device)
  hipSetDevice(h->device);
  ham_free(h);
  return SGW_OK;
}

extern "C" int32_t sgw_ham_npw(const sgw_ham *h) { return h ? h->n_pw : -1; }

// Largest number of non-local projectors per Hamiltonian (bounds the overlap scratch of H.x).
static constexpr int kMaxProj = 4096;

extern "C" sgw_status sgw_ham_set_nonlocal(sgw_ctx *ctx, sgw_ham *h, int n_proj, const sgw_c128 *beta,
                                           const double *e_kb) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_set_nonlocal: NULL context or Hamiltonian");
  if (h->device != ctx->device)
    return fail(SGW_ERR_INVALID_ARG, "sgw_ham_set_nonlocal: the Hamiltonian lives on another device");
  if (n_proj < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_set_nonlocal: n_proj < 0");
  if (n_proj > kMaxProj)
    return fail(SGW_ERR_UNSUPPORTED, "sgw_ham_set_nonlocal: more than " + std::to_string(kMaxProj) + " projectors");
  if (n_proj > 0 && (!beta || !e_kb)) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_set_nonlocal: NULL beta or e_kb");
  for (int p = 0; p < n_proj; ++p)
    if (!std::isfinite(e_kb[p])) return fail(SGW_ERR_INVALID_ARG, "sgw_ham_set_nonlocal: e_kb not finite");
  SGW_HIP(hipSetDevice(ctx->device));
  // launches of earlier calls on this stream may still read the old projectors
  SGW_HIP(hipStreamSynchronize(ctx->stream));
  if (h->d_beta) hipFree(h->d_beta);
  if (h->d_ekb) hipFree(h->d_ekb);
  h->d_beta = nullptr;
  h->d_ekb = nullptr;
  h->n_proj = 0;
  if (n_proj == 0) return SGW_OK;
  const int npw = h->n_pw;
  double2 *db = nullptr;
  double *de = nullptr;
  hipError_t e = hipMalloc((void **)&db, sizeof(double2) * (size_t)n_proj * npw);
  if (e == hipSuccess) e = hipMalloc((void **)&de, sizeof(double) * n_proj);
  if (e == hipSuccess) e = hipMemcpyAsync(de, e_kb, sizeof(double) * n_proj, hipMemcpyHostToDevice, ctx->stream);
  sgw_status st = SGW_OK;
  if (e == hipSuccess) st = permute(ctx, npw, n_proj, (const double2 *)beta, npw, db, npw, h->d_i2u, 0);
  const hipError_t e2 = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess || st != SGW_OK || e2 != hipSuccess) {
    if (db) hipFree(db);
    if (de) hipFree(de);
    if (st != SGW_OK) return st;
    return fail(SGW_ERR_HIP, std::string("sgw_ham_set_nonlocal: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  h->d_beta = db;
  h->d_ekb = de;
  h->n_proj = n_proj;
  return SGW_OK;
}

extern "C" int32_t sgw_ham_nproj(const sgw_ham *h) { return h ? h->n_proj : -1; }

// ---------------------------------------------------------------------------
// test hooks
// ---------------------------------------------------------------------------
namespace {

// scratch of the test hooks; freed after the hook has synchronised its stream
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) hipFree(p);
  }
};

sgw_status alloc_async(DevBuf &b, size_t bytes, hipStream_t) {
  SGW_HIP(hipMalloc(&b.p, std::max<size_t>(bytes, 256)));
  return SGW_OK;
}

}  // namespace

extern "C" sgw_status sgw_apply_h(sgw_ctx *ctx, const sgw_ham *h, int n_vec, const sgw_c128 *x, sgw_c128 *y,
                                  int precision) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h: NULL context or Hamiltonian");
  if (n_vec < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h: n_vec < 0");
  if (precision != SGW_FP64 && precision != SGW_MIXED)
    return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h: unknown precision mode");
  if (n_vec == 0) return SGW_OK;
  if (!x || !y) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h: NULL vector");
  if (x == y) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h: x and y alias");
  SGW_HIP(hipSetDevice(ctx->device));
  const int npw = h->n_pw;
  const size_t vb = sizeof(double2) * (size_t)npw * n_vec;
  DevBuf xi, yi, tb;
  sgw_status st;
  if ((st = alloc_async(xi, vb, ctx->stream)) != SGW_OK) return st;
  if ((st = alloc_async(yi, vb, ctx->stream)) != SGW_OK) return st;
  if ((st = alloc_async(tb, hx_tbuf_bytes(h, n_vec), ctx->stream)) != SGW_OK)
    return st;
  if ((st = permute(ctx, npw, n_vec, (const double2 *)x, npw, (double2 *)xi.p, npw, h->d_i2u, 0)) != SGW_OK)
    return st;
  if ((st = hx_batch(ctx, h, n_vec, contiguous((double2 *)xi.p, npw), (double2 *)yi.p, npw, tb.p,
                     precision == SGW_MIXED)) != SGW_OK)
    return st;
  if ((st = permute(ctx, npw, n_vec, (double2 *)yi.p, npw, (double2 *)y, npw, h->d_i2u, 1)) != SGW_OK) return st;
  return sync(ctx);
}

extern "C" sgw_status sgw_apply_h_noalloc(sgw_ctx *ctx, const sgw_ham *h, int n_vec, const sgw_c128 *x,
                                          sgw_c128 *y, int precision) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h_noalloc: NULL context or Hamiltonian");
  if (n_vec < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h_noalloc: n_vec < 0");
  if (precision != SGW_FP64 && precision != SGW_MIXED)
    return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h_noalloc: unknown precision mode");
  if (n_vec == 0) return SGW_OK;
  if (!x || !y) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h_noalloc: NULL vector");
  if (x == y) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_h_noalloc: x and y alias");
  const int npw = h->n_pw;
  // scratch: x and y in the internal order, then the stick buffer (each part 256-byte aligned)
  auto up = [](size_t b) { return (b + kAlign256 - 1) / kAlign256 * kAlign256; };
  const size_t per_vec = sizeof(double2) * (size_t)npw;
  const size_t vb = up(per_vec * n_vec);
  const size_t tb = up(hx_tbuf_bytes(h, n_vec));
  if (2 * vb + tb > kNoAllocScratchBytes) {
    const size_t one = 2 * up(per_vec) + up(hx_tbuf_bytes(h, 1));
    return fail(SGW_ERR_WORKSPACE, "sgw_apply_h_noalloc: " + std::to_string(n_vec) + " vectors need " +
                                       std::to_string(2 * vb + tb) + " bytes of scratch; the fixed scratch holds " +
                                       std::to_string(kNoAllocScratchBytes) + " (about " +
                                       std::to_string(kNoAllocScratchBytes / one) +
                                       " vectors of this Hamiltonian per call)");
  }
  hipError_t serr = hipSuccess;
  char *base = (char *)scratch_ptr(ctx->device, &serr);
  if (!base)
    return fail(SGW_ERR_HIP, std::string("sgw_apply_h_noalloc: device scratch not available: ") +
                                 hipGetErrorString(serr));
  SGW_HIP(hipSetDevice(ctx->device));
  // no timing events here (creating one allocates); restored on every return
  struct MaskOff {
    sgw_ctx *c;
    unsigned saved;
    ~MaskOff() { c->profile_mask = saved; }
  } mask{ctx, ctx->profile_mask};
  ctx->profile_mask = 0;
  double2 *xi = (double2 *)base, *yi = (double2 *)(base + vb);
  void *tbuf = base + 2 * vb;
  sgw_status st;
  if ((st = permute(ctx, npw, n_vec, (const double2 *)x, npw, xi, npw, h->d_i2u, 0)) != SGW_OK) return st;
  if ((st = hx_batch(ctx, h, n_vec, contiguous(xi, npw), yi, npw, tbuf, precision == SGW_MIXED)) != SGW_OK)
    return st;
  if ((st = permute(ctx, npw, n_vec, yi, npw, (double2 *)y, npw, h->d_i2u, 1)) != SGW_OK) return st;
  return sync(ctx);
}

extern "C" sgw_status sgw_apply_projector(sgw_ctx *ctx, const sgw_ham *h, int n_occ, const sgw_c128 *psi,
                                          int n_vec, const sgw_c128 *x, sgw_c128 *y, double alpha, int mode) {
  if (!ctx || !h) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_projector: NULL context or Hamiltonian");
  if (n_vec < 0 || n_occ < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_projector: negative size");
  const bool split = (mode & SGW_PROJ_SPLIT_BF16) != 0;
  mode &= ~SGW_PROJ_SPLIT_BF16;
  if (mode != 0 && mode != 1) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_projector: mode must be 0 or 1");
  if (n_occ > kMaxOcc)
    return fail(SGW_ERR_UNSUPPORTED, "sgw_apply_projector: n_occ above " + std::to_string(kMaxOcc));
  if (n_vec == 0) return SGW_OK;
  if (!x || !y || (n_occ > 0 && !psi)) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_projector: NULL array");
  if (x == y) return fail(SGW_ERR_INVALID_ARG, "sgw_apply_projector: x and y alias");
  SGW_HIP(hipSetDevice(ctx->device));
  const int npw = h->n_pw;
  DevBuf cb;
  sgw_status st;
  if ((st = alloc_async(cb, sizeof(double2) * kProjChunks * (size_t)n_vec * std::max(n_occ, 1), ctx->stream)) !=
      SGW_OK)
    return st;
  if (split) {
    DevBuf sb;
    if ((st = alloc_async(sb, proj_split_bytes(npw, n_occ), ctx->stream)) != SGW_OK) return st;
    const VecSrc xs = contiguous((const double2 *)x, npw);
    if ((st = proj_split(ctx, npw, n_occ, (const double2 *)psi, sb.p)) != SGW_OK) return st;
    if ((st = proj_dot_bf16(ctx, npw, n_occ, sb.p, n_vec, xs, (double2 *)cb.p, n_vec)) != SGW_OK) return st;
    if ((st = proj_apply_bf16(ctx, npw, n_occ, sb.p, n_vec, xs, (double2 *)cb.p, (double2 *)y, npw, alpha, mode)) !=
        SGW_OK)
      return st;
    return sync(ctx);
  }
  if ((st = proj_dot(ctx, npw, n_occ, (const double2 *)psi, n_vec, contiguous((const double2 *)x, npw),
                     (double2 *)cb.p, n_vec)) != SGW_OK)
    return st;
  if ((st = proj_apply(ctx, npw, n_occ, (const double2 *)psi, n_vec, contiguous((const double2 *)x, npw),
                       (double2 *)cb.p, n_vec, (double2 *)y, npw, alpha, mode)) != SGW_OK)
    return st;
  return sync(ctx);
}

static sgw_status check_miller_shift(const int32_t *dvm, int n_pert) {
  for (int p = 0; p < n_pert; ++p)
    for (int a = 0; a < 3; ++a)
      if (std::abs(dvm[3 * p + a]) > (1 << 20)) return fail(SGW_ERR_INVALID_ARG, "dv_miller out of range");
  return SGW_OK;
}

extern "C" sgw_status sgw_build_rhs(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                    const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, int n_pert,
                                    const int32_t *dv_miller, sgw_c128 *b) {
  if (!ctx || !h_kq || !h_k) return fail(SGW_ERR_INVALID_ARG, "sgw_build_rhs: NULL context or Hamiltonian");
  if (n_occ < 0 || n_band < 0 || n_pert < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_build_rhs: negative size");
  if (n_occ > kMaxOcc) return fail(SGW_ERR_UNSUPPORTED, "sgw_build_rhs: n_occ above " + std::to_string(kMaxOcc));
  const int nvec = n_band * n_pert;
  if (nvec == 0) return SGW_OK;
  if (!psi_v || !dv_miller || !b || (n_occ > 0 && !psi_occ_kq))
    return fail(SGW_ERR_INVALID_ARG, "sgw_build_rhs: NULL array");
  sgw_status st;
  if ((st = check_miller_shift(dv_miller, n_pert)) != SGW_OK) return st;
  SGW_HIP(hipSetDevice(ctx->device));
  const int npw = h_kq->n_pw;
  DevBuf pairs, dvm, s, c, psi;
  if ((st = alloc_async(pairs, sizeof(int32_t) * nvec, ctx->stream)) != SGW_OK) return st;
  if ((st = alloc_async(dvm, sizeof(int32_t) * 3 * n_pert, ctx->stream)) != SGW_OK) return st;
  if ((st = alloc_async(s, sizeof(double2) * (size_t)nvec * npw, ctx->stream)) != SGW_OK) return st;
  if ((st = alloc_async(c, sizeof(double2) * kProjChunks * (size_t)nvec * std::max(n_occ, 1), ctx->stream)) !=
      SGW_OK)
    return st;
  if ((st = alloc_async(psi, sizeof(double2) * (size_t)std::max(n_occ, 1) * npw, ctx->stream)) != SGW_OK) return st;
  std::vector<int32_t> hp(nvec);
  std::iota(hp.begin(), hp.end(), 0);
  SGW_HIP(hipMemcpyAsync(pairs.p, hp.data(), sizeof(int32_t) * nvec, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(dvm.p, dv_miller, sizeof(int32_t) * 3 * n_pert, hipMemcpyHostToDevice, ctx->stream));
  // internal-order copy of the occupied states
  if ((st = permute(ctx, npw, n_occ, (const double2 *)psi_occ_kq, npw, (double2 *)psi.p, npw, h_kq->d_i2u, 0)) !=
      SGW_OK)
    return st;
  if ((st = rhs_source(ctx, h_kq, h_k, nvec, (int32_t *)pairs.p, n_pert, (int32_t *)dvm.p,
                       (const double2 *)psi_v, h_k->n_pw, (double2 *)s.p, npw)) != SGW_OK)
    return st;
  if ((st = proj_dot(ctx, npw, n_occ, (double2 *)psi.p, nvec, contiguous((double2 *)s.p, npw), (double2 *)c.p,
                     nvec)) != SGW_OK)
    return st;
  // b = -(s - psi^T c): y = s - psi^T c here, negated by the scatter to the caller's order
  DevBuf bi;
  if ((st = alloc_async(bi, sizeof(double2) * (size_t)nvec * npw, ctx->stream)) != SGW_OK) return st;
  if ((st = proj_apply(ctx, npw, n_occ, (double2 *)psi.p, nvec, contiguous((double2 *)s.p, npw), (double2 *)c.p,
                       nvec, (double2 *)bi.p, npw, 1.0, 0)) != SGW_OK)
    return st;
  if ((st = permute(ctx, npw, nvec, (double2 *)bi.p, npw, (double2 *)b, npw, h_kq->d_i2u, 1, -1.0)) != SGW_OK)
    return st;
  st = sync(ctx);
  return st;
}

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------
extern "C" sgw_status sgw_opts_default(sgw_opts *o) {
  if (!o) return fail(SGW_ERR_INVALID_ARG, "sgw_opts_default: NULL");
  std::memset(o, 0, sizeof(*o));
  o->precision = SGW_FP64;
  o->max_iter = 600;
  o->alpha_pv = 1.0;
  o->tol_safety = 0.5;
  o->slots = 0;
  o->finalize_batch = 0;
  o->steps_per_sync = 8;
  o->solver = SGW_SOLVER_MULTISHIFT;
  o->precond = SGW_PC_NONE;
  o->guess = SGW_GUESS_ZERO;
  o->tail_iter = 160;
  o->ps_max_iter = 2000;
  o->ps_slots = 0;
  o->mlp = nullptr;
  o->hist_r = nullptr;
  o->hist_x = nullptr;
  o->hist_iter = 0;
  o->mixed_switch = kMixedSwitch;
  o->graph = 0;
  o->fft_planes = SGW_FFT_AUTO;
  o->basis_blocks = 0;
  return SGW_OK;
}

namespace {

constexpr size_t kAlign = 256;
// pooled Krylov basis: 32 vectors per block; when the budget cannot give every pair a full-size
// basis, up to this many times the slots of full-size bases share a pool of the same memory
constexpr int kBasisBlockShift = 5;
constexpr int kPoolSlotFactor = 4;
// workspace budget that sizes the automatic slot count: half of one MI355X's 288 GB of HBM, the
// rest left to the caller's arrays (the 64-atom workload's solutions take 65 GB)
constexpr double kDefaultBudget = 144.0 * (1ull << 30);

struct Layout {
  int S = 0, F = 0, kmax = 0, M = 8;
  size_t psi, omega, epsb, dvm, pair, kcur, status, eps, alpha, beta, rho, res, maxres, conv, bvec, basis;
  size_t l_active, l_fill, l_fillpairs, l_final, Y, Y2, C, T, ycoef, cp, order, X, AX, bad, btab = 0;
  size_t psplit = 0;  // split-BF16 copy of the occupied states (mixed precision), 0: none
  long c_rows = 0;
  // pooled Krylov basis: blocks of 2^bshift vectors, nbmax per slot at most, nblk in the pool;
  // S_full: the slots that full-size bases would give
  bool pooled = false;
  int bshift = 0, nbmax = 0, nblk = 0, S_full = 0;
  size_t total = 0;
};

size_t take(size_t &off, size_t bytes) {
  off = (off + kAlign - 1) / kAlign * kAlign;
  size_t r = off;
  off += std::max<size_t>(bytes, 1);
  return r;
}

sgw_opts resolve_opts(const sgw_opts *in) {
  sgw_opts o;
  sgw_opts_default(&o);
  if (in) {
    o.precision = in->precision;
    if (in->max_iter > 0) o.max_iter = in->max_iter;
    if (in->alpha_pv > 0) o.alpha_pv = in->alpha_pv;
    if (in->tol_safety > 0) o.tol_safety = in->tol_safety;
    o.slots = in->slots;
    o.finalize_batch = in->finalize_batch;
    if (in->steps_per_sync > 0) o.steps_per_sync = in->steps_per_sync;
    o.solver = in->solver;
    o.precond = in->precond;
    o.guess = in->guess;
    if (in->tail_iter > 0) o.tail_iter = in->tail_iter;
    if (in->ps_max_iter > 0) o.ps_max_iter = in->ps_max_iter;
    o.ps_slots = in->ps_slots;
    o.mlp = in->mlp;
    o.hist_r = in->hist_r;
    o.hist_x = in->hist_x;
    o.hist_iter = in->hist_iter;
    o.graph = in->graph;
    o.fft_planes = in->fft_planes;
    o.basis_blocks = in->basis_blocks;
    if (in->mixed_switch > 0) o.mixed_switch = in->mixed_switch;
    o.shift_imag = in->shift_imag;
  }
  return o;
}

Layout make_layout(const sgw_ham *h, int n_occ, int n_band, int n_pert, int n_omega, const sgw_opts &o) {
  Layout L;
  const long npw = h->n_pw;
  const int n_pairs = n_band * n_pert;
  L.kmax = o.max_iter;
  L.M = o.steps_per_sync;
  L.F = o.finalize_batch > 0 ? o.finalize_batch : std::max(1, (4096 + n_omega - 1) / n_omega);
  L.F = std::max(1, std::min(L.F, std::max(n_pairs, 1)));
  const double per_slot = (double)(L.kmax + 3) * npw * 16.0 + (double)hx_tbuf_bytes(h, 1) +
                          (L.kmax * 2.0 + n_omega * 24.0 + 64.0);
  int S = o.slots;
  if (S <= 0) {
    const double fixed = (double)L.F * n_omega * (2.0 * npw * 16.0 + (double)hx_tbuf_bytes(h, 1));
    S = (int)std::max(1.0, (kDefaultBudget - fixed) / per_slot);
    S = std::min(S, 4096);
  }
  // Pooled basis (the caller sizes the pool with basis_blocks): the slots draw their Krylov vectors
  // from a pool in blocks of 2^bshift as they grow, instead of each holding max_iter + 1
  L.bshift = kBasisBlockShift;
  L.nbmax = (L.kmax + 1 + (1 << L.bshift) - 1) >> L.bshift;
  L.S_full = std::max(1, std::min(S, std::max(n_pairs, 1)));
  if (o.basis_blocks > 0) {
    L.pooled = true;
    L.nblk = o.basis_blocks;
  } else if (o.slots <= 0 && S < n_pairs) {
    // the budget cannot give every pair a full-size slot: more slots share a pool of the same size
    const double fixed = (double)L.F * n_omega * (2.0 * npw * 16.0 + (double)hx_tbuf_bytes(h, 1));
    const double blk_bytes = (double)(1 << L.bshift) * npw * 16.0;
    const double small = per_slot - (double)(L.kmax + 1) * npw * 16.0;  // a slot without its basis
    S = std::max(1, std::min({n_pairs, 4096, kPoolSlotFactor * S}));
    while (S > 1 && (kDefaultBudget - fixed - S * small) / blk_bytes < 2.0 * L.nbmax) --S;
    L.pooled = true;
    L.nblk = (int)std::max<double>(L.nbmax, (kDefaultBudget - fixed - S * small) / blk_bytes);
  }
  L.S = std::max(1, std::min(S, std::max(n_pairs, 1)));
  const long nfv = (long)L.F * n_omega;
  const long tv = std::max<long>(L.S, nfv);
  size_t off = 0;
  L.psi = take(off, 16ul * std::max(n_occ, 1) * npw);
  if (o.precision == SGW_MIXED && n_occ > 0) L.psplit = take(off, proj_split_bytes((int)npw, n_occ));
  L.omega = take(off, 16ul * n_omega);  // omega, then the per-shift imaginary parts
  L.epsb = take(off, 8ul * std::max(n_band, 1));
  L.dvm = take(off, 12ul * std::max(n_pert, 1));
  L.pair = take(off, 4ul * L.S);
  L.kcur = take(off, 4ul * L.S);
  L.status = take(off, 4ul * L.S);
  L.eps = take(off, 8ul * L.S);
  L.alpha = take(off, 8ul * L.S * L.kmax);
  L.beta = take(off, 8ul * L.S * (L.kmax + 1));
  L.rho = take(off, 16ul * L.S * n_omega);
  L.res = take(off, 8ul * L.S * n_omega);
  L.maxres = take(off, 8ul * L.S);
  L.conv = take(off, 4ul * L.S * n_omega);
  L.bvec = take(off, 16ul * L.S * npw);
  if (L.pooled) {
    L.basis = take(off, 16ul * (size_t)L.nblk * ((size_t)1 << L.bshift) * npw);
    L.btab = take(off, 4ul * L.S * L.nbmax);
  } else {
    L.basis = take(off, 16ul * L.S * (L.kmax + 1) * npw);
  }
  L.l_active = take(off, 4ul * L.S);
  L.l_fill = take(off, 4ul * L.S);
  L.l_fillpairs = take(off, 4ul * L.S);
  L.l_final = take(off, 4ul * L.S);
  L.Y = take(off, 16ul * L.S * npw);
  L.Y2 = take(off, 16ul * L.S * npw);
  L.c_rows = tv;
  L.C = take(off, 16ul * kProjChunks * tv * std::max(n_occ, 1));
  L.T = take(off, hx_tbuf_bytes(h, tv));
  L.ycoef = take(off, 16ul * L.F * L.kmax * n_omega);
  L.cp = take(off, 16ul * L.F * L.kmax * n_omega);
  L.order = take(off, 4ul * L.F * n_omega);
  L.X = take(off, 16ul * nfv * npw);
  L.AX = take(off, 16ul * nfv * npw);
  L.bad = take(off, 64);
  L.total = (off + kAlign - 1) / kAlign * kAlign;
  return L;
}

}  // namespace

static sgw_status validate_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                 const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, const double *eps_v,
                                 int n_pert, const int32_t *dv_miller, int n_omega, const double *omega, double eta,
                                 double tol, const sgw_opts &o) {
  SGW_CHECK(ctx && h_kq && h_k, "sternheimer_solve: NULL context or Hamiltonian");
  SGW_CHECK(h_kq->ctx == ctx && h_k->ctx == ctx, "sternheimer_solve: Hamiltonian of another context");
  SGW_CHECK(n_occ >= 0 && n_band >= 0 && n_pert >= 0 && n_omega >= 0, "sternheimer_solve: negative size");
  if (n_occ > kMaxOcc)
    return fail(SGW_ERR_UNSUPPORTED, "sternheimer_solve: n_occ above " + std::to_string(kMaxOcc));
  SGW_CHECK(n_occ < h_kq->n_pw, "sternheimer_solve: n_occ must be below the basis size");
  SGW_CHECK(o.precision == SGW_FP64 || o.precision == SGW_MIXED, "sternheimer_solve: unknown precision mode");
  SGW_CHECK(o.precision == SGW_FP64 || o.solver != SGW_SOLVER_PER_SHIFT,
            "sternheimer_solve: the per-shift solver runs in FP64 only");
  SGW_CHECK(o.max_iter >= 1 && o.max_iter <= 100000, "sternheimer_solve: max_iter out of range");
  if (o.shift_imag) {
    SGW_CHECK(std::isfinite(eta), "sternheimer_solve: eta not finite");
    for (int j = 0; j < n_omega; ++j)
      SGW_CHECK(std::isfinite(o.shift_imag[j]), "sternheimer_solve: shift_imag not finite");
  } else {
    SGW_CHECK(std::isfinite(eta) && eta != 0.0, "sternheimer_solve: eta must be finite and non-zero");
  }
  SGW_CHECK(std::isfinite(tol) && tol > 0.0, "sternheimer_solve: tol must be positive");
  SGW_CHECK(std::isfinite(o.alpha_pv) && o.alpha_pv > 0.0, "sternheimer_solve: alpha_pv must be positive");
  SGW_CHECK(o.solver >= SGW_SOLVER_MULTISHIFT && o.solver <= SGW_SOLVER_BLOCK, "sternheimer_solve: unknown solver");
  if (o.solver == SGW_SOLVER_BLOCK) {
    SGW_CHECK(o.precision == SGW_FP64, "sternheimer_solve: the block solver runs in FP64 only");
    SGW_CHECK(o.precond == SGW_PC_NONE && o.guess == SGW_GUESS_ZERO,
              "sternheimer_solve: the block solver takes no preconditioner or initial guess");
    SGW_CHECK(o.hist_iter == 0, "sternheimer_solve: the block solver keeps no residual history");
  }
  SGW_CHECK(o.precond >= SGW_PC_NONE && o.precond <= SGW_PC_LEARNED, "sternheimer_solve: unknown preconditioner");
  SGW_CHECK(o.guess == SGW_GUESS_ZERO || o.guess == SGW_GUESS_LEARNED, "sternheimer_solve: unknown initial guess");
  SGW_CHECK(o.fft_planes >= SGW_FFT_AUTO && o.fft_planes <= SGW_FFT_TRI, "sternheimer_solve: unknown plane kernel");
  SGW_CHECK(o.basis_blocks == 0 ||
                (o.basis_blocks > 0 && ((long)o.basis_blocks << kBasisBlockShift) >= (long)o.max_iter + 1),
            "sternheimer_solve: basis_blocks must hold one pair's max_iter + 1 Krylov vectors");
  // preconditioners and guesses act in per-shift solves only: the per-shift solver, and the per-shift
  // phases of TAIL and MIXED (the multishift phase itself never uses them)
  SGW_CHECK(o.solver != SGW_SOLVER_MULTISHIFT || o.precision == SGW_MIXED ||
                (o.precond == SGW_PC_NONE && o.guess == SGW_GUESS_ZERO),
            "sternheimer_solve: a preconditioner or initial guess breaks the shared Krylov space; "
            "use the per-shift or tail solver");
  SGW_CHECK(o.ps_max_iter >= 1 && o.ps_max_iter <= 100000, "sternheimer_solve: ps_max_iter out of range");
  if (o.precond == SGW_PC_LEARNED || (o.guess == SGW_GUESS_LEARNED && o.solver == SGW_SOLVER_PER_SHIFT)) {
    SGW_CHECK(o.mlp != nullptr, "sternheimer_solve: the learned preconditioner or guess needs opts.mlp");
    SGW_CHECK(o.mlp->device == ctx->device, "sternheimer_solve: opts.mlp lives on another device");
  }
  SGW_CHECK(o.hist_iter >= 0, "sternheimer_solve: hist_iter < 0");
  SGW_CHECK(o.hist_iter == 0 || (o.hist_r && o.hist_x), "sternheimer_solve: hist_iter > 0 needs hist_r and hist_x");
  if ((long)n_band * n_pert * n_omega == 0) return SGW_OK;
  SGW_CHECK(psi_v && eps_v && dv_miller && omega, "sternheimer_solve: NULL input array");
  SGW_CHECK(n_occ == 0 || psi_occ_kq, "sternheimer_solve: psi_occ_kq is NULL");
  for (int j = 0; j < n_omega; ++j) SGW_CHECK(std::isfinite(omega[j]), "sternheimer_solve: omega not finite");
  for (int v = 0; v < n_band; ++v) SGW_CHECK(std::isfinite(eps_v[v]), "sternheimer_solve: eps_v not finite");
  if (h_kq->n_pw > 16384) return fail(SGW_ERR_UNSUPPORTED, "sternheimer_solve: basis above 16384");
  return check_miller_shift(dv_miller, n_pert);
}

// A captured sequence of launches on one stream, replayed with hipGraphLaunch.  An event recorded
// after every replay marks when the executable graph is no longer in use: a re-capture and the
// destructor (also on error returns, with a replay possibly still queued) wait for it before the
// executable graph is destroyed.
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  int na = -1, n64 = -1;
  StepGraph() = default;
  StepGraph(const StepGraph &) = delete;
  StepGraph &operator=(const StepGraph &) = delete;
  ~StepGraph() {
    release();
    if (done) hipEventDestroy(done);
  }
  void release() {
    if (!exec) return;
    if (done) hipEventSynchronize(done);
    hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  sgw_status launch(hipStream_t stream) {
    if (!done) SGW_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    SGW_HIP(hipGraphLaunch(exec, stream));
    SGW_HIP(hipEventRecord(done, stream));
    return SGW_OK;
  }
  template <class F>
  sgw_status capture(hipStream_t stream, F &&launches) {
    release();
    na = -1;
    n64 = -1;
    SGW_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    const sgw_status st = launches();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &g);
    if (st != SGW_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(SGW_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      exec = nullptr;
      return fail(SGW_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
    return SGW_OK;
  }
};

// options of the multishift phase of a TAIL solve
static sgw_opts tail_phase_opts(const sgw_opts &o) {
  sgw_opts m = o;
  m.max_iter = std::min(o.max_iter, o.tail_iter);
  return m;
}

// Options of the FP64 per-shift refinement that may follow a plain multishift solve: as many per-shift
// slots as fit in the multishift phase's own workspace (few shifts need it; it must not enlarge the
// workspace), unless the caller set ps_slots.
static sgw_opts refine_opts(const sgw_ham *h_kq, int n_occ, int n_band, int n_pert, int n_omega,
                            const sgw_opts &o) {
  sgw_opts r = o;
  if (o.ps_slots > 0) return r;
  const size_t ms = o.solver == SGW_SOLVER_BLOCK ? block_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega, o)
                                                 : make_layout(h_kq, n_occ, n_band, n_pert, n_omega, o).total;
  const long n_sys = (long)n_band * n_pert * n_omega;
  const int n_sys_i = (int)std::min<long>(n_sys, 1L << 30);
  int B = (int)std::max<long>(1, std::min<long>(n_sys, 8192));
  for (;;) {
    r.ps_slots = B;
    if (B == 1 || ps_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega, r, n_sys_i) <= ms) break;
    B = std::max(1, B * 3 / 4);
  }
  return r;
}

static size_t solve_workspace_bytes(const sgw_ham *h_kq, int n_occ, int n_band, int n_pert, int n_omega,
                                    const sgw_opts &o) {
  const long n_sys = (long)n_band * n_pert * n_omega;
  const int n_sys_i = (int)std::min<long>(n_sys, 1L << 30);
  switch (o.solver) {
    case SGW_SOLVER_BLOCK:  // the per-shift refinement reuses the workspace, as after the multishift solver
      return std::max(block_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega, o),
                      ps_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega,
                                         refine_opts(h_kq, n_occ, n_band, n_pert, n_omega, o), n_sys_i));
    case SGW_SOLVER_PER_SHIFT:
      return ps_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega, o, n_sys_i);
    case SGW_SOLVER_TAIL:
      return std::max(make_layout(h_kq, n_occ, n_band, n_pert, n_omega, tail_phase_opts(o)).total,
                      ps_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega, o, n_sys_i));
    default:  // FP64 per-shift refinement after the multishift phase reuses the workspace
      return std::max(make_layout(h_kq, n_occ, n_band, n_pert, n_omega, o).total,
                      ps_workspace_bytes(h_kq, n_occ, n_band, n_pert, n_omega,
                                         o.precision == SGW_MIXED
                                             ? o
                                             : refine_opts(h_kq, n_occ, n_band, n_pert, n_omega, o),
                                         n_sys_i));
  }
}

extern "C" sgw_status sternheimer_workspace_size(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, int n_band,
                                                 int n_pert, int n_omega, const sgw_opts *opts, size_t *bytes) {
  if (!ctx || !h_kq || !bytes) return fail(SGW_ERR_INVALID_ARG, "sternheimer_workspace_size: NULL argument");
  if (n_occ < 0 || n_band < 0 || n_pert < 0 || n_omega < 0)
    return fail(SGW_ERR_INVALID_ARG, "sternheimer_workspace_size: negative size");
  const sgw_opts o = resolve_opts(opts);
  if (o.solver < SGW_SOLVER_MULTISHIFT || o.solver > SGW_SOLVER_BLOCK)
    return fail(SGW_ERR_INVALID_ARG, "sternheimer_workspace_size: unknown solver");
  *bytes = solve_workspace_bytes(h_kq, n_occ, n_band, n_pert, std::max(n_omega, 1), o);
  return SGW_OK;
}

// The multishift solve proper (arguments validated, workspace checked).
static sgw_status multishift_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                   const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, const double *eps_v,
                                   int n_pert, const int32_t *dv_miller, int n_omega, const double *omega,
                                   double eta, double tol, const sgw_opts &o, void *workspace, sgw_c128 *dpsi,
                                   sgw_solve_info *info) {
  sgw_status st;
  const int n_pairs = n_band * n_pert;
  const Layout L = make_layout(h_kq, n_occ, n_band, n_pert, n_omega, o);
  char *W = (char *)workspace;
  const int npw = h_kq->n_pw;
  const int S = L.S, F = L.F;

  SolverState Sx;
  Sx.npw = npw;
  Sx.n_occ = n_occ;
  Sx.n_omega = n_omega;
  Sx.n_pert = n_pert;
  Sx.kmax = L.kmax;
  Sx.slot_stride = (long)(L.kmax + 1) * npw;
  Sx.psi = (double2 *)(W + L.psi);
  Sx.basis = (double2 *)(W + L.basis);
  Sx.bvec = (double2 *)(W + L.bvec);
  Sx.alpha_t = (double *)(W + L.alpha);
  Sx.beta = (double *)(W + L.beta);
  Sx.rho = (double2 *)(W + L.rho);
  Sx.res = (double *)(W + L.res);
  Sx.maxres = (double *)(W + L.maxres);
  Sx.conv = (int32_t *)(W + L.conv);
  Sx.pair = (int32_t *)(W + L.pair);
  Sx.kcur = (int32_t *)(W + L.kcur);
  Sx.status = (int32_t *)(W + L.status);
  Sx.eps = (double *)(W + L.eps);
  Sx.eps_band = (double *)(W + L.epsb);
  Sx.omega = (double *)(W + L.omega);
  Sx.eta = eta;
  Sx.alpha = o.alpha_pv;
  int32_t *d_btab = L.pooled ? (int32_t *)(W + L.btab) : nullptr;
  if (L.pooled) {
    Sx.btab = d_btab;
    Sx.nbmax = L.nbmax;
    Sx.bshift = L.bshift;
  }
  // Mixed precision: a matvec error at step k enters the shifted solutions weighted by their step-k
  // coefficients, which shrink with the residual (inexact Krylov theory); so a slot switches to
  // FP32 potential matvecs (~3e-8 relative error) once all its shifts' estimates are below
  // kMixedSwitch * tol, and the true FP64 residual decides afterwards.
  const bool mixed = o.precision == SGW_MIXED;
  const double switch_res = o.mixed_switch * tol;
  Sx.tol_int = tol * o.tol_safety;
  int32_t *d_active = (int32_t *)(W + L.l_active);
  int32_t *d_fill = (int32_t *)(W + L.l_fill);
  int32_t *d_fillpairs = (int32_t *)(W + L.l_fillpairs);
  int32_t *d_final = (int32_t *)(W + L.l_final);
  int32_t *d_dvm = (int32_t *)(W + L.dvm);
  double2 *Y = (double2 *)(W + L.Y);
  double2 *C = (double2 *)(W + L.C);   // overlap partials [kProjChunks][c_rows][n_occ]
  double2 *Y2 = (double2 *)(W + L.Y2);
  const long crow = L.c_rows;
  double2 *T = (double2 *)(W + L.T);
  double2 *ycoef = (double2 *)(W + L.ycoef);
  double2 *cp = (double2 *)(W + L.cp);
  int32_t *sorder = (int32_t *)(W + L.order);
  double2 *X = (double2 *)(W + L.X);
  double2 *AX = (double2 *)(W + L.AX);
  int *d_bad = (int *)(W + L.bad);

  // pinned staging: status[S] | active[S] | fill[S] | fillpairs[S] | final[S] | bad[16] | maxres[S]
  // | block table[S][nbmax] (pooled basis)
  const size_t ntab = L.pooled ? (size_t)S * L.nbmax : 0;
  if ((st = ensure_pinned(ctx, sizeof(int32_t) * (5ul * S + 16 + ntab) + sizeof(double) * (S + 1))) != SGW_OK)
    return st;
  int32_t *p_status = (int32_t *)ctx->pinned;
  int32_t *p_active = p_status + S;
  int32_t *p_fill = p_active + S;
  int32_t *p_fillpairs = p_fill + S;
  int32_t *p_final = p_fillpairs + S;
  int32_t *p_bad = p_final + S;
  double *p_maxres = (double *)(((uintptr_t)(p_bad + 16) + 7) & ~(uintptr_t)7);
  int32_t *p_btab = (int32_t *)(p_maxres + S);
  std::vector<char> slot_fp32(S, 0);

  // parameters
  SGW_HIP(hipMemcpyAsync((void *)Sx.omega, omega, sizeof(double) * n_omega, hipMemcpyHostToDevice, ctx->stream));
  if (o.shift_imag) {
    Sx.eta_j = Sx.omega + n_omega;
    SGW_HIP(hipMemcpyAsync((void *)Sx.eta_j, o.shift_imag, sizeof(double) * n_omega, hipMemcpyHostToDevice,
                           ctx->stream));
  }
  SGW_HIP(hipMemcpyAsync((void *)Sx.eps_band, eps_v, sizeof(double) * n_band, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemcpyAsync(d_dvm, dv_miller, sizeof(int32_t) * 3 * n_pert, hipMemcpyHostToDevice, ctx->stream));
  SGW_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), ctx->stream));
  if ((st = permute(ctx, npw, n_occ, (const double2 *)psi_occ_kq, npw, (double2 *)Sx.psi, npw, h_kq->d_i2u, 0)) !=
      SGW_OK)
    return st;
  // mixed precision: the slots in their FP32 phase apply the projector as a split-BF16 contraction
  void *psplit = L.psplit ? (void *)(W + L.psplit) : nullptr;
  if (psplit && (st = proj_split(ctx, npw, n_occ, Sx.psi, psplit)) != SGW_OK) return st;

  // work queue: the highest bands (slowest to converge) first
  std::vector<int> queue(n_pairs);
  std::iota(queue.begin(), queue.end(), 0);
  std::stable_sort(queue.begin(), queue.end(), [&](int a, int b) { return eps_v[a / n_pert] > eps_v[b / n_pert]; });
  size_t next = 0;
  std::vector<int> slot_pair(S, -1), free_slots, active, done;
  for (int s = S - 1; s >= 0; --s) free_slots.push_back(s);
  const VecSrc cur{Sx.basis, npw, d_active, Sx.kcur, Sx.slot_stride, Sx.btab, Sx.nbmax, Sx.bshift};
  const VecSrc xsrc = contiguous(X, npw);
  StepGraph graph;
  size_t finalized = 0;
  double ksum = 0;
  long kcount = 0;
  std::vector<int32_t> kc_host(S);
  std::vector<int32_t> conv_host;  // convergence steps read back for the timing statistics

  // Pooled basis: block table (host copy uploaded before the launches that read it), blocks owned
  // per slot, free blocks; pairs restarted after an eviction wait in requeue.  kcn: a slot's
  // Krylov dimension as of the last poll (0 when filled).
  std::vector<int32_t> htab;
  std::vector<int> nown, free_blk, kcn;
  std::deque<int> requeue;
  bool tab_dirty = false, stalled_prev = false;
  if (L.pooled) {
    htab.assign(ntab, 0);
    nown.assign(S, 0);
    kcn.assign(S, 0);
    for (int b = L.nblk - 1; b >= 0; --b) free_blk.push_back(b);
  }
  // maps Krylov vectors 0..kneed of slot s; false (blocks taken so far kept) when the pool is empty
  auto grow = [&](int s, int kneed) -> bool {
    const int need = (kneed >> L.bshift) + 1;
    while (nown[s] < need) {
      if (free_blk.empty()) return false;
      htab[(size_t)s * L.nbmax + nown[s]++] = free_blk.back();
      free_blk.pop_back();
      tab_dirty = true;
    }
    return true;
  };
  auto release = [&](int s) {
    for (int i = 0; i < nown[s]; ++i) free_blk.push_back(htab[(size_t)s * L.nbmax + i]);
    nown[s] = 0;
  };
  // Admission by expected growth: a pair enters only if the pool can carry every admitted pair to
  // its expected final Krylov dimension: max_iter until 16 pairs have finished, then the 90th
  // percentile of theirs (the queue runs from the slowest bands down, so this overestimates).
  // (a pool the caller sized admits whenever blocks for the first steps are free)
  const bool careful = L.pooled && o.basis_blocks <= 0;
  std::vector<int> kfin;
  int kest = L.kmax;
  auto expect_blocks = [&](int k_now) {
    const int k = std::min(L.kmax, std::max(k_now + L.M, kest));
    return (k >> L.bshift) + 1;
  };

  auto finalize = [&](std::vector<int> &list) -> sgw_status {
    for (size_t off = 0; off < list.size(); off += F) {
      const int nf = (int)std::min<size_t>(F, list.size() - off);
      double kavg = 0;
      for (int f = 0; f < nf; ++f) kavg += kc_host[list[off + f]];
      kavg /= nf;
      // mean dimension of the shifts' own solutions, for the combination's flop count (only while
      // its launches are timed: it reads the convergence steps back)
      double kshift = kavg;
      if (ctx->profile_mask & (1u << K_COMBINE)) {
        conv_host.resize((size_t)S * n_omega);
        SGW_HIP(hipMemcpyAsync(conv_host.data(), Sx.conv, sizeof(int32_t) * conv_host.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
        SGW_HIP(hipStreamSynchronize(ctx->stream));
        double ks = 0;
        for (int f = 0; f < nf; ++f) {
          const int sl = list[off + f], K = kc_host[sl];
          for (int j = 0; j < n_omega; ++j) {
            const int c = conv_host[(size_t)sl * n_omega + j];
            ks += (c >= 1 && c < K) ? c : K;
          }
        }
        kshift = ks / ((double)nf * n_omega);
      }
      std::memcpy(p_final, list.data() + off, sizeof(int32_t) * nf);
      SGW_HIP(hipMemcpyAsync(d_final, p_final, sizeof(int32_t) * nf, hipMemcpyHostToDevice, ctx->stream));
      sgw_status s2;
      if ((s2 = tridiag(ctx, Sx, d_final, nf, ycoef, cp, sorder)) != SGW_OK) return s2;
      if ((s2 = combine(ctx, Sx, d_final, nf, ycoef, sorder, X, kavg, kshift)) != SGW_OK) return s2;
      const int nv = nf * n_omega;
      if ((s2 = proj_dot(ctx, npw, n_occ, Sx.psi, nv, xsrc, C, crow)) != SGW_OK) return s2;
      if ((s2 = hx_batch(ctx, h_kq, nv, xsrc, AX, npw, T)) != SGW_OK) return s2;
      if ((s2 = proj_apply(ctx, npw, n_occ, Sx.psi, nv, xsrc, C, crow, AX, npw, o.alpha_pv, 1)) != SGW_OK) return s2;
      if ((s2 = residual(ctx, Sx, d_final, nf, X, AX, C, crow, h_kq->d_u2i, (double2 *)dpsi, info, tol, d_bad)) !=
          SGW_OK)
        return s2;
      // the pinned final list is reused by the next chunk: wait for the upload
      if ((s2 = sync(ctx)) != SGW_OK) return s2;
    }
    for (int s : list) {
      slot_pair[s] = -1;
      free_slots.push_back(s);
      if (L.pooled) release(s);
    }
    finalized += list.size();
    list.clear();
    return SGW_OK;
  };

  while (finalized < (size_t)n_pairs) {
    // refill free slots; with a pooled basis a pair is admitted only with blocks for its first steps,
    // and none while running pairs wait for blocks
    int nfill = 0;
    long committed = 0;  // blocks the admitted pairs are expected to need (pooled basis)
    if (L.pooled) {
      for (int s : active) committed += std::max(nown[s], expect_blocks(kcn[s]));
      for (int s : done) committed += nown[s];
    }
    while (!free_slots.empty() && (next < queue.size() || !requeue.empty()) && !(L.pooled && stalled_prev)) {
      const int s = free_slots.back();
      if (careful && committed + expect_blocks(0) > L.nblk && !(active.empty() && done.empty() && nfill == 0))
        break;
      if (L.pooled && !grow(s, std::min(L.M, L.kmax))) {
        release(s);
        break;
      }
      if (L.pooled) committed += expect_blocks(0);
      free_slots.pop_back();
      int pr;
      if (!requeue.empty()) {
        pr = requeue.front();
        requeue.pop_front();
      } else {
        pr = queue[next++];
      }
      slot_pair[s] = pr;
      if (L.pooled) kcn[s] = 0;
      p_fill[nfill] = s;
      p_fillpairs[nfill] = pr;
      ++nfill;
    }
    // the slots that take steps in this pass of the scheduler: with a pooled basis, those whose next steps' vectors
    // are mapped; when none of the running pairs can grow (and none was just admitted), the least
    // advanced one gives its blocks back and restarts later
    std::vector<int> run;
    if (L.pooled) {
      for (;;) {
        run.clear();
        for (int s : active)
          if (grow(s, std::min(kcn[s] + L.M, L.kmax))) run.push_back(s);
        if (!run.empty() || active.empty() || nfill > 0) break;
        if (!done.empty()) {  // finished pairs still hold blocks: finalise them first
          if ((st = finalize(done)) != SGW_OK) return st;
          continue;
        }
        int e = active[0];
        for (int s : active)
          if (kcn[s] < kcn[e]) e = s;
        release(e);
        requeue.push_front(slot_pair[e]);
        slot_pair[e] = -1;
        free_slots.push_back(e);
        active.erase(std::find(active.begin(), active.end(), e));
      }
      stalled_prev = run.size() < active.size();
      if (tab_dirty) {
        std::memcpy(p_btab, htab.data(), sizeof(int32_t) * ntab);
        SGW_HIP(hipMemcpyAsync(d_btab, p_btab, sizeof(int32_t) * ntab, hipMemcpyHostToDevice, ctx->stream));
        tab_dirty = false;
      }
    } else {
      run = active;
    }
    if (nfill > 0) {
      SGW_HIP(hipMemcpyAsync(d_fill, p_fill, sizeof(int32_t) * nfill, hipMemcpyHostToDevice, ctx->stream));
      SGW_HIP(hipMemcpyAsync(d_fillpairs, p_fillpairs, sizeof(int32_t) * nfill, hipMemcpyHostToDevice, ctx->stream));
      if ((st = rhs_source(ctx, h_kq, h_k, nfill, d_fillpairs, n_pert, d_dvm, (const double2 *)psi_v, h_k->n_pw, Y,
                           npw)) != SGW_OK)
        return st;
      if ((st = proj_dot(ctx, npw, n_occ, Sx.psi, nfill, contiguous(Y, npw), C, crow)) != SGW_OK) return st;
      if ((st = proj_apply(ctx, npw, n_occ, Sx.psi, nfill, contiguous(Y, npw), C, crow, Y2, npw, 1.0, 0)) != SGW_OK)
        return st;
      if ((st = slot_init(ctx, Sx, nfill, Y, Y2, d_fill, d_fillpairs)) != SGW_OK) return st;
      for (int i = 0; i < nfill; ++i) {
        active.push_back(p_fill[i]);
        run.push_back(p_fill[i]);
        slot_fp32[p_fill[i]] = 0;
      }
    }
    if (!run.empty()) {
      // FP64 slots first, then the slots whose matvecs run with the FP32 potential
      int n64 = 0;
      for (int s : run)
        if (!slot_fp32[s]) p_active[n64++] = s;
      int k32 = n64;
      for (int s : run)
        if (slot_fp32[s]) p_active[k32++] = s;
      const int na = (int)run.size();
      SGW_HIP(hipMemcpyAsync(d_active, p_active, sizeof(int32_t) * na, hipMemcpyHostToDevice, ctx->stream));
      const VecSrc cur32{Sx.basis, npw, d_active + n64, Sx.kcur, Sx.slot_stride, Sx.btab, Sx.nbmax, Sx.bshift};
      auto steps = [&]() -> sgw_status {
        sgw_status s2;
        for (int step = 0; step < L.M; ++step) {
          // FP64 slots [0, n64), FP32-phase slots [n64, na): the overlaps of the latter go to rows n64..
          // of C, their projector runs split-BF16
          double2 *C32 = C + (long)n64 * n_occ;
          double2 *Y32 = Y + (long)n64 * npw;
          if ((s2 = proj_dot(ctx, npw, n_occ, Sx.psi, n64, cur, C, crow)) != SGW_OK) return s2;
          if (na > n64 && (s2 = proj_dot_bf16(ctx, npw, n_occ, psplit, na - n64, cur32, C32, crow)) != SGW_OK) return s2;
          if ((s2 = hx_batch(ctx, h_kq, n64, cur, Y, npw, T)) != SGW_OK) return s2;
          if ((s2 = hx_batch(ctx, h_kq, na - n64, cur32, Y32, npw, T, true)) != SGW_OK) return s2;
          if ((s2 = proj_apply(ctx, npw, n_occ, Sx.psi, n64, cur, C, crow, Y, npw, o.alpha_pv, 1)) != SGW_OK) return s2;
          if (na > n64 &&
              (s2 = proj_apply_bf16(ctx, npw, n_occ, psplit, na - n64, cur32, C32, Y32, npw, o.alpha_pv, 1)) != SGW_OK)
            return s2;
          if ((s2 = lanczos_step(ctx, Sx, na, d_active, Y)) != SGW_OK) return s2;
        }
        return SGW_OK;
      };
      // The launches read the active list from device memory, so a captured
      // sequence depends only on the number of active slots (and of FP64 ones).
      // The legacy default stream cannot be captured: launches stay eager there.
      if (o.graph && ctx->profile_mask == 0 && ctx->stream != nullptr) {
        if (graph.na != na || graph.n64 != n64) {
          if ((st = graph.capture(ctx->stream, steps)) != SGW_OK) return st;
          graph.na = na;
          graph.n64 = n64;
        }
        if ((st = graph.launch(ctx->stream)) != SGW_OK) return st;
      } else if ((st = steps()) != SGW_OK) {
        return st;
      }
    }
    // poll
    SGW_HIP(hipMemcpyAsync(p_status, Sx.status, sizeof(int32_t) * S, hipMemcpyDeviceToHost, ctx->stream));
    SGW_HIP(hipMemcpyAsync(kc_host.data(), Sx.kcur, sizeof(int32_t) * S, hipMemcpyDeviceToHost, ctx->stream));
    if (mixed)
      SGW_HIP(hipMemcpyAsync(p_maxres, Sx.maxres, sizeof(double) * S, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != SGW_OK) return st;
    if (L.pooled)
      for (int s : active) kcn[s] = kc_host[s];
    if (mixed)
      for (int s : active) slot_fp32[s] = slot_fp32[s] || p_maxres[s] <= switch_res;
    std::vector<int> still;
    for (int s : active) {
      if (p_status[s] == SLOT_RUNNING) still.push_back(s);
      else {
        done.push_back(s);
        ksum += kc_host[s];
        ++kcount;
        if (L.pooled) kfin.push_back(kc_host[s]);
      }
    }
    if (L.pooled && kfin.size() >= 16) {
      std::vector<int> t = kfin;
      const size_t q = t.size() * 9 / 10;
      std::nth_element(t.begin(), t.begin() + q, t.end());
      kest = std::min(L.kmax, t[q]);
    }
    active.swap(still);
    const bool refill_waiting = next < queue.size() || !requeue.empty();
    if (!done.empty() && (active.empty() || (int)done.size() >= F || (refill_waiting && (int)done.size() * 4 >= F) ||
                          (L.pooled && stalled_prev))) {
      if ((st = finalize(done)) != SGW_OK) return st;
    }
  }
  SGW_HIP(hipMemcpyAsync(p_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if ((st = sync(ctx)) != SGW_OK) return st;
  return *p_bad > 0 ? SGW_NOT_CONVERGED : SGW_OK;
}

// Validation of one problem with resolved options (no GPU work).
static sgw_status check_problem(sgw_ctx *ctx, const sgw_problem &p, const sgw_opts &o) {
  sgw_status st = validate_solve(ctx, p.h_kq, p.n_occ, p.psi_occ_kq, p.h_k, p.n_band, p.psi_v, p.eps_v, p.n_pert,
                                 p.dv_miller, p.n_omega, p.omega, p.eta, p.tol, o);
  if (st != SGW_OK) return st;
  const long n_sys = (long)p.n_band * p.n_pert * p.n_omega;
  if (n_sys == 0) return SGW_OK;
  SGW_CHECK(p.dpsi && p.info, "sternheimer_solve: NULL output array");
  SGW_CHECK(n_sys < (1L << 31), "sternheimer_solve: more than 2^31 solves in one call");
  return SGW_OK;
}

static size_t problem_workspace_bytes(const sgw_problem &p, const sgw_opts &o) {
  return solve_workspace_bytes(p.h_kq, p.n_occ, p.n_band, p.n_pert, std::max(p.n_omega, 1), o);
}

// The solve of a validated problem on ctx's stream, dispatched on the solver.
static sgw_status run_solve(sgw_ctx *ctx, const sgw_problem &p, const sgw_opts &o, void *workspace,
                            size_t workspace_bytes) {
  const long n_sys = (long)p.n_band * p.n_pert * p.n_omega;
  if (n_sys == 0) return SGW_OK;
  const size_t need = problem_workspace_bytes(p, o);
  if (!workspace || workspace_bytes < need)
    return fail(SGW_ERR_WORKSPACE, "sternheimer_solve: workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) % kAlign != 0)
    return fail(SGW_ERR_WORKSPACE, "sternheimer_solve: workspace must be 256-byte aligned");
  SGW_HIP(hipSetDevice(ctx->device));
  FftScope fft(ctx, o.fft_planes);
  sgw_status st;
  PsProblem P{p.h_kq, p.h_k, p.n_occ, (const double2 *)p.psi_occ_kq, p.n_band, (const double2 *)p.psi_v, p.eps_v,
              p.n_pert, p.dv_miller, p.n_omega, p.omega, p.eta, p.tol};
  if (o.solver == SGW_SOLVER_PER_SHIFT) {
    int n_bad = 0;
    if ((st = ps_solve(ctx, P, o, {}, false, workspace, workspace_bytes, (double2 *)p.dpsi, p.info, &n_bad)) !=
        SGW_OK)
      return st;
    return n_bad > 0 ? SGW_NOT_CONVERGED : SGW_OK;
  }
  // TAIL: multishift up to tail_iter; MIXED: multishift with FP32 potential matvecs.  Then the shifts
  // whose true FP64 residual is above tol continue per shift in FP64 from their multishift iterate.
  // Plain FP64 multishift: only the shifts whose recurrence estimate met the stopping threshold while
  // the true residual, recomputed from x, missed tol (rounding in the recurrence: tight tolerances
  // near the FP64 floor of kappa * eps) are refined that way; shifts that hit max_iter or met
  // non-finite values keep their flags.
  // The block solver is refined the same way as plain FP64 multishift.
  const bool plain = (o.solver == SGW_SOLVER_MULTISHIFT && o.precision == SGW_FP64) || o.solver == SGW_SOLVER_BLOCK;
  const sgw_opts o1 = o.solver == SGW_SOLVER_TAIL ? tail_phase_opts(o) : o;
  if (o.solver == SGW_SOLVER_BLOCK)
    st = block_solve(ctx, p.h_kq, p.n_occ, p.psi_occ_kq, p.h_k, p.n_band, p.psi_v, p.eps_v, p.n_pert, p.dv_miller,
                     p.n_omega, p.omega, p.eta, p.tol, o, workspace, workspace_bytes, p.dpsi, p.info);
  else
    st = multishift_solve(ctx, p.h_kq, p.n_occ, p.psi_occ_kq, p.h_k, p.n_band, p.psi_v, p.eps_v, p.n_pert,
                          p.dv_miller, p.n_omega, p.omega, p.eta, p.tol, o1, workspace, p.dpsi, p.info);
  if (st != SGW_OK && st != SGW_NOT_CONVERGED) return st;
  if (st == SGW_OK) return SGW_OK;
  std::vector<sgw_solve_info> hinfo(n_sys);
  SGW_HIP(hipMemcpyAsync(hinfo.data(), p.info, sizeof(sgw_solve_info) * n_sys, hipMemcpyDeviceToHost, ctx->stream));
  if ((st = sync(ctx)) != SGW_OK) return st;
  std::vector<int32_t> tail;
  bool left = false;  // a plain solve that stays unconverged whatever the refinement does
  for (long y = 0; y < n_sys; ++y) {
    const int fl = hinfo[y].flags;
    if (fl & SGW_FLAG_CONVERGED) continue;
    if (plain && (fl & (SGW_FLAG_MAXITER | SGW_FLAG_NONFINITE))) {
      left = true;
      continue;
    }
    tail.push_back((int32_t)y);
  }
  if (tail.empty()) return SGW_NOT_CONVERGED;
  int n_bad = 0;
  const sgw_opts o2 = plain ? refine_opts(p.h_kq, p.n_occ, p.n_band, p.n_pert, std::max(p.n_omega, 1), o) : o;
  if ((st = ps_solve(ctx, P, o2, tail, true, workspace, workspace_bytes, (double2 *)p.dpsi, p.info, &n_bad)) !=
      SGW_OK)
    return st;
  return (n_bad > 0 || left) ? SGW_NOT_CONVERGED : SGW_OK;
}

extern "C" sgw_status sternheimer_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                        const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, const double *eps_v,
                                        int n_pert, const int32_t *dv_miller, int n_omega, const double *omega,
                                        double eta, double tol, const sgw_opts *opts, void *workspace,
                                        size_t workspace_bytes, sgw_c128 *dpsi, sgw_solve_info *info) {
  sgw_problem p;
  std::memset(&p, 0, sizeof(p));
  p.h_kq = h_kq;
  p.h_k = h_k;
  p.n_occ = n_occ;
  p.n_band = n_band;
  p.n_pert = n_pert;
  p.n_omega = n_omega;
  p.psi_occ_kq = psi_occ_kq;
  p.psi_v = psi_v;
  p.eps_v = eps_v;
  p.dv_miller = dv_miller;
  p.omega = omega;
  p.eta = eta;
  p.tol = tol;
  p.dpsi = dpsi;
  p.info = info;
  const sgw_opts o = resolve_opts(opts);
  const sgw_status st = check_problem(ctx, p, o);
  if (st != SGW_OK) return st;
  return run_solve(ctx, p, o, workspace, workspace_bytes);
}

// ---------------------------------------------------------------------------
// Green's function columns (Sec. 2.2, Eqs. 2-3): (H_k - z_j) G_{.G'}(z_j) = -e_{G'}
// ---------------------------------------------------------------------------
namespace {

size_t up256(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// The Green's solve is the multishift solve with no occupied states, zero band energy, one
// perturbation with G_p = 0 and the unit vectors e_{G'} as the "states": its right-hand side is then
// b = -e_{G'} and its operator H - z.  Workspace: the solve's, then the unit vectors and the columns.
sgw_problem green_problem(const sgw_ham *h_k, int n_col, int n_omega, const double *omega, double eta, double tol,
                          const double *eps0, const int32_t *dvm0, sgw_c128 *g, sgw_solve_info *info) {
  sgw_problem p;
  std::memset(&p, 0, sizeof(p));
  p.h_kq = h_k;
  p.h_k = h_k;
  p.n_occ = 0;
  p.n_band = n_col;
  p.n_pert = 1;
  p.n_omega = n_omega;
  p.psi_occ_kq = nullptr;
  p.psi_v = nullptr;  // the unit vectors, set once they are on the device
  p.eps_v = eps0;
  p.dv_miller = dvm0;
  p.omega = omega;
  p.eta = eta;
  p.tol = tol;
  p.dpsi = g;
  p.info = info;
  return p;
}

}  // namespace

extern "C" sgw_status sgw_green_workspace_size(sgw_ctx *ctx, const sgw_ham *h_k, int n_col, int n_omega,
                                               const sgw_opts *opts, size_t *bytes) {
  if (!ctx || !h_k || !bytes) return fail(SGW_ERR_INVALID_ARG, "sgw_green_workspace_size: NULL argument");
  if (n_col < 0 || n_omega < 0) return fail(SGW_ERR_INVALID_ARG, "sgw_green_workspace_size: negative size");
  const sgw_opts o = resolve_opts(opts);
  if (o.solver < SGW_SOLVER_MULTISHIFT || o.solver > SGW_SOLVER_BLOCK)
    return fail(SGW_ERR_INVALID_ARG, "sgw_green_workspace_size: unknown solver");
  // block solver: the columns as the perturbations of one right-hand side family (see sgw_green_solve)
  const bool blk = o.solver == SGW_SOLVER_BLOCK;
  const size_t base = up256(solve_workspace_bytes(h_k, 0, blk ? 1 : n_col, blk ? n_col : 1, std::max(n_omega, 1), o));
  *bytes = base + up256(sizeof(double2) * (size_t)n_col * h_k->n_pw) + up256(sizeof(int32_t) * (size_t)n_col);
  return SGW_OK;
}

extern "C" sgw_status sgw_green_solve(sgw_ctx *ctx, const sgw_ham *h_k, int n_col, const int32_t *cols, int n_omega,
                                      const double *omega, double eta, double tol, const sgw_opts *opts,
                                      void *workspace, size_t workspace_bytes, sgw_c128 *g, sgw_solve_info *info) {
  SGW_CHECK(ctx && h_k, "sgw_green_solve: NULL context or Hamiltonian");
  SGW_CHECK(n_col >= 0 && n_omega >= 0, "sgw_green_solve: negative size");
  if ((long)n_col * n_omega == 0) return SGW_OK;
  SGW_CHECK(cols && omega && g && info, "sgw_green_solve: NULL array");
  const int npw = h_k->n_pw;
  for (int c = 0; c < n_col; ++c)
    SGW_CHECK(cols[c] >= 0 && cols[c] < npw, "sgw_green_solve: column index outside the basis");
  if (!workspace) return fail(SGW_ERR_WORKSPACE, "sgw_green_solve: workspace missing");
  const sgw_opts o = resolve_opts(opts);
  const std::vector<double> eps0(n_col, 0.0);
  const int32_t dvm0[3] = {0, 0, 0};
  sgw_problem p = green_problem(h_k, n_col, n_omega, omega, eta, tol, eps0.data(), dvm0, g, info);
  // Block solver: the operator H_k - z is the same for every column, so the columns are the
  // perturbations of one band: e_{G'} is the unit vector at G_0 = cols[0] shifted by G' - G_0, and the
  // n_col right-hand sides share one block Krylov space (the output layout is the same).
  const bool blk = o.solver == SGW_SOLVER_BLOCK;
  std::vector<int32_t> dvb;
  if (blk) {
    dvb.resize(3 * (size_t)n_col);
    const int32_t *m = h_k->miller.data();
    for (int c = 0; c < n_col; ++c)
      for (int a = 0; a < 3; ++a) dvb[3 * c + a] = m[3 * cols[c] + a] - m[3 * cols[0] + a];
    p.n_band = 1;
    p.n_pert = n_col;
    p.dv_miller = dvb.data();
  }
  // validation with a stand-in for the device unit vectors (only their presence is checked)
  p.psi_v = (const sgw_c128 *)workspace;
  sgw_status st = check_problem(ctx, p, o);
  if (st != SGW_OK) return st;
  const size_t base = up256(problem_workspace_bytes(p, o));
  const size_t need = base + up256(sizeof(double2) * (size_t)n_col * npw) + up256(sizeof(int32_t) * (size_t)n_col);
  if (!workspace || workspace_bytes < need)
    return fail(SGW_ERR_WORKSPACE, "sgw_green_solve: workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) % kAlign != 0)
    return fail(SGW_ERR_WORKSPACE, "sgw_green_solve: workspace must be 256-byte aligned");
  SGW_HIP(hipSetDevice(ctx->device));
  double2 *unit = (double2 *)((char *)workspace + base);
  int32_t *dcols = (int32_t *)((char *)unit + up256(sizeof(double2) * (size_t)n_col * npw));
  SGW_HIP(hipMemcpyAsync(dcols, cols, sizeof(int32_t) * n_col, hipMemcpyHostToDevice, ctx->stream));
  if ((st = unit_columns(ctx, npw, blk ? 1 : n_col, dcols, unit)) != SGW_OK) return st;
  p.psi_v = (const sgw_c128 *)unit;
  return run_solve(ctx, p, o, workspace, base);
}

// ---------------------------------------------------------------------------
// batches of systems and the autotuner
// ---------------------------------------------------------------------------
namespace {

// Options whose workspace fits `budget` bytes.  Multishift: the slot count (and the finalisation batch)
// are lowered from the requested or automatic values.  Block: the bands per chunk (slots) are the most
// that fit, at least one.
sgw_opts fit_to_budget(const sgw_problem &p, sgw_opts o, size_t budget) {
  if (o.solver == SGW_SOLVER_BLOCK) {
    int lo = 1, hi = std::max(1, o.slots > 0 ? std::min(o.slots, p.n_band) : p.n_band);
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      sgw_opts t = o;
      t.slots = mid;
      if (problem_workspace_bytes(p, t) <= budget) lo = mid;
      else hi = mid - 1;
    }
    o.slots = lo;
    return o;
  }
  if (o.solver != SGW_SOLVER_MULTISHIFT) return o;
  const int n_omega = std::max(p.n_omega, 1);
  Layout L = make_layout(p.h_kq, p.n_occ, p.n_band, p.n_pert, n_omega, o);
  o.slots = L.S_full;  // a worker's part holds full-size bases
  o.finalize_batch = L.F;
  L = make_layout(p.h_kq, p.n_occ, p.n_band, p.n_pert, n_omega, o);
  while (L.total > budget && (o.slots > 1 || o.finalize_batch > 1)) {
    if (o.slots > 1) o.slots = std::max(1, o.slots * 3 / 4);
    if (o.finalize_batch > 1 && (o.slots == 1 || (long)o.finalize_batch * n_omega > o.slots))
      o.finalize_batch = std::max(1, o.finalize_batch * 3 / 4);
    L = make_layout(p.h_kq, p.n_occ, p.n_band, p.n_pert, n_omega, o);
  }
  return o;
}

// A system whose launches alone fill the GPU (at least 128 (band, perturbation) pairs of at least
// 4,096 plane waves: 128 vectors give >= 6,000 plane workgroups on a 48-point grid) loses more to a
// worker's share of the workspace (fewer slots, hence fewer vectors per launch) than it gains from
// running beside others: in a batch over several workers such systems run first, one at a time over
// the whole workspace with the options of a single solve.
bool fills_gpu(const sgw_problem &p) { return p.h_kq->n_pw >= 4096 && (long)p.n_band * p.n_pert >= 128; }

double predicted_cost(const sgw_problem &p) {
  const double npw = p.h_kq->n_pw;
  const double grid = (double)p.h_kq->n[0] * p.h_kq->n[1] * p.h_kq->n[2];
  const double pairs = (double)p.n_band * p.n_pert;
  // Krylov steps (~100 per pair, each an FFT H.x and the projector) plus the residual of every shift
  return pairs * (100.0 + p.n_omega) * (grid * std::log2(std::max(grid, 2.0)) / 8.0 + npw * (p.n_occ + 8));
}

}  // namespace

extern "C" sgw_status sternheimer_batch_workspace_size(sgw_ctx *ctx, int n_sys, const sgw_problem *problems,
                                                       int n_workers, size_t *bytes) {
  if (!ctx || !bytes || (n_sys > 0 && !problems))
    return fail(SGW_ERR_INVALID_ARG, "sternheimer_batch_workspace_size: NULL argument");
  if (n_sys < 0 || n_workers < 1 || n_workers > kMaxWorkers)
    return fail(SGW_ERR_INVALID_ARG, "sternheimer_batch_workspace_size: bad n_sys or n_workers");
  const size_t budget = (size_t)(kDefaultBudget / n_workers) / kAlign * kAlign;
  size_t part = 0, alone = 0;
  for (int i = 0; i < n_sys; ++i) {
    if (!problems[i].h_kq) return fail(SGW_ERR_INVALID_ARG, "sternheimer_batch_workspace_size: NULL Hamiltonian");
    const sgw_opts o = resolve_opts(&problems[i].opts);
    if (n_workers > 1 && fills_gpu(problems[i])) {
      alone = std::max(alone, problem_workspace_bytes(problems[i], o));
    } else {
      part = std::max(part, problem_workspace_bytes(problems[i], fit_to_budget(problems[i], o, budget)));
    }
  }
  part = (part + kAlign - 1) / kAlign * kAlign;
  *bytes = std::max(part * n_workers, (alone + kAlign - 1) / kAlign * kAlign);
  return SGW_OK;
}

extern "C" sgw_status sternheimer_solve_batch(sgw_ctx *ctx, int n_sys, sgw_problem *problems, int n_workers,
                                              void *workspace, size_t workspace_bytes) {
  SGW_CHECK(ctx, "sternheimer_solve_batch: NULL context");
  SGW_CHECK(n_sys >= 0 && (n_sys == 0 || problems), "sternheimer_solve_batch: bad problem array");
  SGW_CHECK(n_workers >= 1 && n_workers <= kMaxWorkers, "sternheimer_solve_batch: n_workers out of range");
  if (n_sys == 0) return SGW_OK;
  SGW_CHECK(workspace && ((uintptr_t)workspace) % kAlign == 0, "sternheimer_solve_batch: workspace missing or unaligned");
  const size_t part = workspace_bytes / n_workers / kAlign * kAlign;
  const size_t whole = workspace_bytes / kAlign * kAlign;
  std::vector<sgw_opts> opts(n_sys);
  std::vector<char> alone(n_sys, 0);
  for (int i = 0; i < n_sys; ++i) {
    sgw_problem &p = problems[i];
    p.status = SGW_OK;
    p.worker = -1;
    p.ms = 0.0;
    const sgw_opts o = resolve_opts(&p.opts);
    sgw_status st = check_problem(ctx, p, o);
    if (st != SGW_OK) {
      p.status = st;
      return fail(st, "problem " + std::to_string(i) + ": " + sgw_last_error());
    }
    alone[i] = n_workers > 1 && fills_gpu(p);
    const size_t room = alone[i] ? whole : part;
    opts[i] = alone[i] && problem_workspace_bytes(p, o) <= whole ? o : fit_to_budget(p, o, room);
    if (problem_workspace_bytes(p, opts[i]) > room) {
      p.status = SGW_ERR_WORKSPACE;
      return fail(SGW_ERR_WORKSPACE, "sternheimer_solve_batch: problem " + std::to_string(i) +
                                         " does not fit the workspace of " + std::to_string(room) + " bytes");
    }
  }
  // longest predicted first: the systems that fill the GPU one at a time, then the others over the workers
  std::vector<int> order(n_sys);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return predicted_cost(problems[a]) > predicted_cost(problems[b]); });
  std::stable_partition(order.begin(), order.end(), [&](int i) { return alone[i] != 0; });
  const int n_alone = (int)std::count(alone.begin(), alone.end(), 1);
  SGW_HIP(hipSetDevice(ctx->device));
  // the workers' streams wait for the work already queued on the caller's stream
  hipEvent_t ready = nullptr;
  SGW_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  SGW_HIP(hipEventRecord(ready, ctx->stream));
  struct Worker {
    hipStream_t stream = nullptr;
    sgw_ctx *ctx = nullptr;
  };
  std::vector<Worker> workers(n_workers);
  sgw_status st = SGW_OK;
  for (int w = 0; w < n_workers && st == SGW_OK; ++w) {
    if (hipStreamCreateWithFlags(&workers[w].stream, hipStreamNonBlocking) != hipSuccess) {
      st = fail(SGW_ERR_HIP, "sternheimer_solve_batch: hipStreamCreate failed");
      break;
    }
    if ((st = sgw_ctx_create(ctx->device, workers[w].stream, &workers[w].ctx)) != SGW_OK) break;
    workers[w].ctx->fft_planes = ctx->fft_planes;
    workers[w].ctx->profile_mask = ctx->profile_mask;
    if (hipStreamWaitEvent(workers[w].stream, ready, 0) != hipSuccess)
      st = fail(SGW_ERR_HIP, "sternheimer_solve_batch: hipStreamWaitEvent failed");
  }
  std::atomic<int> next{n_alone};
  std::atomic<bool> abort_flag{false};
  std::mutex mu;
  std::string first_error;
  sgw_status first_status = SGW_OK;
  auto record = [&](int i, int w, sgw_status s, double ms) {
    problems[i].status = s;
    problems[i].worker = w;
    problems[i].ms = ms;
    if (s < 0) {
      std::lock_guard<std::mutex> lock(mu);
      if (first_status == SGW_OK) {
        first_status = s;
        first_error = "problem " + std::to_string(i) + ": " + sgw_last_error();
      }
      abort_flag = true;
    }
  };
  // the systems that fill the GPU, one at a time over the whole workspace on worker 0's stream; that
  // stream is drained before the workers' shares of the workspace are reused
  for (int k = 0; k < n_alone && st == SGW_OK && !abort_flag; ++k) {
    const int i = order[k];
    const auto t0 = std::chrono::steady_clock::now();
    const sgw_status s = run_solve(workers[0].ctx, problems[i], opts[i], workspace, whole);
    const auto t1 = std::chrono::steady_clock::now();
    record(i, 0, s, std::chrono::duration<double, std::milli>(t1 - t0).count());
  }
  if (st == SGW_OK && n_alone > 0 && hipStreamSynchronize(workers[0].stream) != hipSuccess)
    st = fail(SGW_ERR_HIP, "sternheimer_solve_batch: hipStreamSynchronize failed");
  auto work = [&](int w) {
    if (hipSetDevice(ctx->device) != hipSuccess) {
      abort_flag = true;
      return;
    }
    char *base = (char *)workspace + (size_t)w * part;
    while (!abort_flag) {
      const int k = next++;
      if (k >= n_sys) break;
      const int i = order[k];
      const auto t0 = std::chrono::steady_clock::now();
      const sgw_status s = run_solve(workers[w].ctx, problems[i], opts[i], base, part);
      const auto t1 = std::chrono::steady_clock::now();
      record(i, w, s, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
  };
  if (st == SGW_OK && !abort_flag) {
    std::vector<std::thread> threads;
    for (int w = 1; w < n_workers; ++w) threads.emplace_back(work, w);
    work(0);
    for (auto &t : threads) t.join();
  }
  for (auto &w : workers) {
    if (w.ctx) {
      hipStreamSynchronize(w.stream);
      timing_collect(w.ctx);
      for (int k = 0; k < K_COUNT; ++k) {
        ctx->stats[k].launches += w.ctx->stats[k].launches;
        ctx->stats[k].ms += w.ctx->stats[k].ms;
        ctx->stats[k].bytes += w.ctx->stats[k].bytes;
        ctx->stats[k].flops += w.ctx->stats[k].flops;
      }
      sgw_ctx_destroy(w.ctx);
    }
    if (w.stream) hipStreamDestroy(w.stream);
  }
  hipEventDestroy(ready);
  if (st != SGW_OK) return st;
  if (first_status != SGW_OK) return fail(first_status, first_error);
  for (int i = 0; i < n_sys; ++i)
    if (problems[i].status == SGW_NOT_CONVERGED) return SGW_NOT_CONVERGED;
  return SGW_OK;
}

extern "C" sgw_status sgw_autotune(sgw_ctx *ctx, const sgw_problem *problem, sgw_opts *best, double *tune_ms) {
  SGW_CHECK(ctx && problem && best, "sgw_autotune: NULL argument");
  const auto t_start = std::chrono::steady_clock::now();
  const sgw_problem &p = *problem;
  const sgw_opts base = resolve_opts(&p.opts);
  sgw_status st = validate_solve(ctx, p.h_kq, p.n_occ, p.psi_occ_kq, p.h_k, p.n_band, p.psi_v, p.eps_v, p.n_pert,
                                 p.dv_miller, p.n_omega, p.omega, p.eta, p.tol, base);
  if (st != SGW_OK) return st;
  SGW_CHECK(base.solver == SGW_SOLVER_MULTISHIFT, "sgw_autotune: tunes the multishift solver only");
  // system class: grid, and n_pw, n_occ, n_omega to within a factor sqrt(2)
  auto bucket = [](int n) { return std::to_string((int)std::lround(2.0 * std::log2(std::max(n, 1)))); };
  const std::string key = std::to_string(p.h_kq->n[0]) + "x" + std::to_string(p.h_kq->n[1]) + "x" +
                          std::to_string(p.h_kq->n[2]) + "/" + bucket(p.h_kq->n_pw) + "/" + bucket(p.n_occ) + "/" +
                          bucket(p.n_omega);
  auto hit = ctx->tuned.find(key);
  if (hit != ctx->tuned.end()) {
    *best = base;
    best->steps_per_sync = hit->second.steps_per_sync;
    best->graph = hit->second.graph;
    if (base.fft_planes == SGW_FFT_AUTO) best->fft_planes = hit->second.fft_planes;
    if (tune_ms) *tune_ms = 0.0;
    return SGW_OK;
  }
  *best = base;
  if ((long)p.n_band * p.n_pert * p.n_omega == 0) {
    if (tune_ms) *tune_ms = 0.0;
    return SGW_OK;
  }
  SGW_HIP(hipSetDevice(ctx->device));
  // sample: the two highest bands (the slowest pairs) and up to eight perturbations
  sgw_problem s = p;
  const int nb = std::min(p.n_band, 2), np = std::min(p.n_pert, 8);
  s.n_band = nb;
  s.psi_v = p.psi_v + (size_t)(p.n_band - nb) * p.h_k->n_pw;
  s.eps_v = p.eps_v + (p.n_band - nb);
  s.n_pert = np;
  const size_t n_sys = (size_t)nb * np * p.n_omega;
  const size_t ws_b = problem_workspace_bytes(s, base);
  void *buf = nullptr;
  const size_t out_b = (sizeof(sgw_c128) * n_sys * p.h_kq->n_pw + kAlign - 1) / kAlign * kAlign;
  const size_t info_b = (sizeof(sgw_solve_info) * n_sys + kAlign - 1) / kAlign * kAlign;
  SGW_HIP(hipMalloc(&buf, out_b + info_b + ws_b));
  s.dpsi = (sgw_c128 *)buf;
  s.info = (sgw_solve_info *)((char *)buf + out_b);
  void *ws = (char *)buf + out_b + info_b;
  // candidates run on a stream of their own, as the workers of a batch do (capturable, untimed)
  hipStream_t tstream = nullptr;
  sgw_ctx *tctx = nullptr;
  hipEvent_t ready = nullptr;
  if (hipStreamCreateWithFlags(&tstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, ctx->stream) != hipSuccess || hipStreamWaitEvent(tstream, ready, 0) != hipSuccess) {
    st = fail(SGW_ERR_HIP, "sgw_autotune: stream setup failed");
  } else {
    st = sgw_ctx_create(ctx->device, tstream, &tctx);
    if (st == SGW_OK) tctx->fft_planes = ctx->fft_planes;
  }
  // plane-pass kernel of the FP64 H.x: every kernel that applies to this grid, timed on a batch of
  // vectors the size of a typical step (the slots of up to 512 pairs), zeros as input
  int fft_best = base.fft_planes;
  if (st >= 0 && base.fft_planes == SGW_FFT_AUTO) {
    const sgw_ham *h = p.h_kq;
    const int nv = (int)std::min<long>(512, std::max<long>(1, (long)p.n_band * p.n_pert));
    const size_t vb = sizeof(double2) * (size_t)nv * h->n_pw;
    const size_t tb = hx_tbuf_bytes(h, nv);
    void *hb = nullptr;
    if (hipMalloc(&hb, 2 * vb + tb) != hipSuccess) {
      st = fail(SGW_ERR_HIP, "sgw_autotune: H.x buffers");
    } else if (hipMemsetAsync(hb, 0, 2 * vb, tstream) != hipSuccess) {
      st = fail(SGW_ERR_HIP, "sgw_autotune: H.x buffers");
    } else {
      double fft_ms = 1e300;
      const double2 *x = (const double2 *)hb;
      double2 *y = (double2 *)((char *)hb + vb);
      void *t = (char *)hb + 2 * vb;
      for (int v = SGW_FFT_LINE; v <= SGW_FFT_TRI && st >= 0; ++v) {
        FftScope fs(tctx, v);
        if (hx_plane_kernel(tctx, h, false) != v) continue;  // does not apply here
        double ms = 0;
        for (int rep = 0; rep < 4 && st >= 0; ++rep) {  // the first run is not timed
          const auto t0 = std::chrono::steady_clock::now();
          st = hx_batch(tctx, h, nv, contiguous(x, h->n_pw), y, h->n_pw, t);
          if (st >= 0 && hipStreamSynchronize(tstream) != hipSuccess)
            st = fail(SGW_ERR_HIP, "sgw_autotune: H.x timing");
          if (rep > 0)
            ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (st >= 0 && ms < fft_ms) {
          fft_ms = ms;
          fft_best = v;
        }
      }
    }
    if (hb) {
      hipStreamSynchronize(tstream);
      hipFree(hb);
    }
  }
  double best_ms = 1e300;
  sgw_opts winner = base;
  winner.fft_planes = fft_best;
  const int steps[] = {4, 8, 16};
  for (int warm = 1, c = 0; c < 6 && st >= 0; ++c) {
    sgw_opts o = base;
    o.fft_planes = fft_best;
    o.steps_per_sync = steps[c % 3];
    o.graph = c / 3;
    if (warm) {  // first launch of every kernel: not timed
      st = run_solve(tctx, s, o, ws, ws_b);
      warm = 0;
      if (st < 0) break;
    }
    const auto t0 = std::chrono::steady_clock::now();
    st = run_solve(tctx, s, o, ws, ws_b);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st >= 0 && ms < best_ms) {
      best_ms = ms;
      winner = o;
    }
  }
  const std::string err = st < 0 ? std::string(sgw_last_error()) : std::string();
  if (tstream) hipStreamSynchronize(tstream);
  if (tctx) sgw_ctx_destroy(tctx);
  if (tstream) hipStreamDestroy(tstream);
  if (ready) hipEventDestroy(ready);
  hipFree(buf);
  if (st < 0) return fail(st, err);
  *best = base;
  best->steps_per_sync = winner.steps_per_sync;
  best->graph = winner.graph;
  best->fft_planes = winner.fft_planes;
  ctx->tuned[key] = *best;
  if (tune_ms)
    *tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return SGW_OK;
}
