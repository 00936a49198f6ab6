// C ABI of the PTTK library (tt_kernel.h): handle lifecycle, argument checks,
// and the orchestration of the offline stage (Algorithm 2), the online stage
// (Algorithm 3) and the apply / backward calls on the caller's stream.
#include <algorithm>
#include <map>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>

#include "ttk_internal.h"

namespace ttk {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

tt_status fail(tt_status s, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {
struct Pool {
  std::multimap<size_t, void*> free;   // idle blocks by size
  std::vector<std::pair<void*, size_t>> pending;   // released since the last synchronisation
  size_t total = 0;
};
constexpr size_t POOL_CAP = (size_t)1 << 30;
Pool& pool_of(bool host, int dev) {
  // never destroyed: a buffer released while the process exits still finds it
  thread_local auto* pools = new std::map<std::pair<int, bool>, Pool>();
  return (*pools)[{dev, host}];
}
void pool_drop(void* p, bool host) {
  if (host) (void)hipHostFree(p);
  else (void)hipFree(p);
}
}  // namespace

void* pool_take(size_t* bytes, bool host, int dev) {
  Pool& pl = pool_of(host, dev);
  if (!pl.pending.empty()) {
    (void)hipDeviceSynchronize();   // every block released so far is idle after this (dev is current)
    for (auto& e : pl.pending) {
      pl.free.emplace(e.second, e.first);
      pl.total += e.second;
    }
    pl.pending.clear();
    while (pl.total > POOL_CAP && !pl.free.empty()) {   // the largest go first
      auto it = std::prev(pl.free.end());
      pl.total -= it->first;
      pool_drop(it->second, host);
      pl.free.erase(it);
    }
  }
  // the smallest block that fits, if it wastes at most half of itself
  auto it = pl.free.lower_bound(*bytes);
  if (it == pl.free.end() || it->first > 2 * *bytes + 4096) return nullptr;
  void* p = it->second;
  *bytes = it->first;
  pl.total -= it->first;
  pl.free.erase(it);
  return p;
}

void pool_give(void* p, size_t bytes, bool host, int dev) { pool_of(host, dev).pending.emplace_back(p, bytes); }

namespace {
// Frees every block of the pool (after the synchronisation that makes the
// released ones idle), so that an allocation that failed can be retried.
void pool_trim(bool host, int dev) {
  Pool& pl = pool_of(host, dev);
  if (!pl.pending.empty()) (void)hipDeviceSynchronize();
  for (auto& e : pl.pending) pool_drop(e.first, host);
  for (auto& e : pl.free) pool_drop(e.second, host);
  pl.pending.clear();
  pl.free.clear();
  pl.total = 0;
}
}  // namespace

template <bool HOST>
tt_status Buf<HOST>::alloc(size_t nbytes) {
  if (nbytes <= bytes && p) return TTK_OK;
  release();   // (to the pool: the next take synchronises before reusing it)
  if (nbytes == 0) nbytes = 16;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TTK_ERR_HIP, "no current device");
  }
  size_t got = nbytes;
  if (void* q = pool_take(&got, HOST, dev)) {
    p = q;
    bytes = got;
    return TTK_OK;
  }
  auto get = [&] { return HOST ? hipHostMalloc(&p, nbytes, hipHostMallocDefault) : hipMalloc(&p, nbytes); };
  if (get() != hipSuccess) {   // the pool's idle blocks go back, then once more
    (void)hipGetLastError();
    pool_trim(HOST, dev);
    if (get() != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(TTK_ERR_OOM, "%s allocation of %zu bytes failed", HOST ? "pinned host" : "device", nbytes);
    }
  }
  bytes = nbytes;
  return TTK_OK;
}
template struct Buf<false>;
template struct Buf<true>;


static int kind_dtheta(int kind) {
  switch (kind) {
    case TTK_MATERN: return 2;
    case TTK_LAPLACE3D: case TTK_LAPLACE2D: case TTK_BIHARMONIC: case TTK_THINPLATE: return 0;
    case TTK_SE: case TTK_EXPONENTIAL: case TTK_MATERN32: case TTK_MATERN52: case TTK_MATERN_NU:
    case TTK_MULTIQUADRIC: case TTK_TPS: case TTK_TEST_POLY: case TTK_TEST_SEP: return 1;
    default: return -1;
  }
}

static tt_status check_params(const tt_kernel_params* p) {
  if (!p) return fail(TTK_ERR_ARG, "params is NULL");
  if (p->d < 1 || p->d > 3) return fail(TTK_ERR_ARG, "d = %d outside 1..3", p->d);
  const int dt = kind_dtheta(p->kind);
  if (dt < 0) return fail(TTK_ERR_ARG, "unknown kernel kind %d", p->kind);
  if (p->d_theta != dt && p->d_theta != 0)
    return fail(TTK_ERR_ARG, "kernel kind %d needs d_theta = %d, or 0 with theta_fixed (got %d)", p->kind, dt,
                p->d_theta);
  if (p->d_theta == 0)   // non-parametric TTK at fixed theta: every parameter positive
    for (int j = 0; j < dt; ++j)
      if (!(p->theta_fixed[j] > 0)) return fail(TTK_ERR_ARG, "theta_fixed[%d] must be positive", j);
  if (p->n_spatial < 2 || p->n_spatial > MAXN) return fail(TTK_ERR_ARG, "n_spatial = %d outside 2..%d", p->n_spatial, MAXN);
  if (p->d_theta > 0 && (p->n_param < 2 || p->n_param > MAXN))
    return fail(TTK_ERR_ARG, "n_param = %d outside 2..%d", p->n_param, MAXN);
  for (int j = 0; j < p->d; ++j) {
    if (!(p->box_s[2 * j] < p->box_s[2 * j + 1])) return fail(TTK_ERR_ARG, "source box dimension %d is empty", j);
    if (!(p->box_t[2 * j] < p->box_t[2 * j + 1])) return fail(TTK_ERR_ARG, "target box dimension %d is empty", j);
  }
  for (int j = 0; j < p->d_theta; ++j)
    if (!(p->box_theta[2 * j] < p->box_theta[2 * j + 1])) return fail(TTK_ERR_ARG, "parameter box %d is empty", j);
  if (p->dtype != TTK_FP32 && p->dtype != TTK_FP64) return fail(TTK_ERR_ARG, "dtype %d unknown", p->dtype);
  if (p->max_rank > MAXR) return fail(TTK_ERR_ARG, "max_rank %d above %d", p->max_rank, MAXR);
  if (p->init_card != 0 && p->init_card != 1 && p->init_card != 2)
    return fail(TTK_ERR_ARG, "init_card must be 1 or 2");
  if (p->kind == TTK_MATERN_NU && !(p->kernel_const > 0)) return fail(TTK_ERR_ARG, "Matern nu must be positive");
  return TTK_OK;
}

tt_status make_grid(const tt_kernel_params* p, Grid* g) {
  g->d = p->d;
  g->dt = p->d_theta;
  g->D = 2 * p->d + p->d_theta;
  for (int j = 0; j < g->D; ++j) {
    int n;
    double lo, hi;
    if (j < g->d) { n = p->n_spatial; lo = p->box_s[2 * j]; hi = p->box_s[2 * j + 1]; }
    else if (j < g->d + g->dt) { n = p->n_param; lo = p->box_theta[2 * (j - g->d)]; hi = p->box_theta[2 * (j - g->d) + 1]; }
    else { n = p->n_spatial; lo = p->box_t[2 * (j - g->d - g->dt)]; hi = p->box_t[2 * (j - g->d - g->dt) + 1]; }
    g->n[j] = n;
    g->lo[j] = lo;
    g->hi[j] = hi;
    // eta_i = phi_[lo,hi](zeta_i), zeta_i = cos((2i+1) pi / (2n)), i = 0..n-1
    for (int i = 0; i < n; ++i) {
      const double z = std::cos((2.0 * i + 1.0) * M_PI / (2.0 * n));
      g->nodes[j * MAXN + i] = (lo - hi) / 2.0 * z + (lo + hi) / 2.0;
    }
  }
  return TTK_OK;
}

namespace {

// Coefficient-basis core Ghat[a, k, b] = sum_i C[k, i] G[a, i, b] with
// C[k, i] = (c_k / n) T_k(zeta_i), written in one of three layouts:
//  mode 0: chain stage, row-major [(a + k r0) r1 + b]     (source cores)
//  mode 1: chain stage transposed [(b + k r1) r0 + a]     (target cores)
//  mode 2: little-endian FP64 [a + k r0 + b r0 n]          (parameter cores)
template <class T>
__global__ void k_dct_core(const double* G, int r0, int n, int r1, const double* C, int mode, T* out) {
  const int64_t total = (int64_t)r0 * n * r1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r0);
    const int k = (int)((e / r0) % n);
    const int b = (int)(e / ((int64_t)r0 * n));
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += C[k + i * n] * G[a + (int64_t)i * r0 + (int64_t)b * r0 * n];
    int64_t o;
    if (mode == 0) o = (int64_t)(a + k * r0) * r1 + b;
    else if (mode == 1) o = (int64_t)(b + k * r1) * r0 + a;
    else o = e;
    out[o] = (T)s;
  }
}

__global__ void k_identity_batch(void* M, int r, int B, int fp32) {
  const int64_t total = (int64_t)r * r * B;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % ((int64_t)r * r);
    const double v = (q % r == q / r) ? 1.0 : 0.0;
    if (fp32) static_cast<float*>(M)[e] = (float)v;
    else static_cast<double*>(M)[e] = v;
  }
}

// out (k x rc, dtype, column-major) = U[:, :rc] (FP64, leading dimension k);
// lam_out (rc, dtype) = lam[:rc].
template <class T>
__global__ void k_g2_convert(const double* U, int k, int rc, const double* lam, T* out, T* lam_out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * rc;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (T)U[e];
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < rc; i += blockDim.x) lam_out[i] = (T)lam[i];
}

// Z (N x rc row-major, leading dimension ldz) = Y (N x rc column-major, ld N).
template <class T>
__global__ void k_g2_rows(const T* Y, int64_t N, int rc, T* Z, int64_t ldz) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * rc; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / rc;
    const int c = (int)(e - p * rc);
    Z[p * ldz + c] = Y[p + (int64_t)c * N];
  }
}

// B (n x m, ldb = n) = A^T for A (m x n, lda = m), FP64
__global__ void k_transpose_small(const double* A, int m, int n, double* B) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * n; e += gridDim.x * blockDim.x) {
    const int i = e % m, j = e / m;
    B[j + (size_t)i * n] = A[e];
  }
}

// W[i + b rc] *= lam[i]  (rc x B)
template <class T>
__global__ void k_g2_scale(T* W, const T* lam, int rc, int B) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)rc * B;
       e += (int64_t)gridDim.x * blockDim.x)
    W[e] *= lam[e % rc];
}

}  // namespace

}  // namespace ttk

using namespace ttk;

struct tt_kernel {
  tt_kernel_params P{};
  Grid g;
  int dtype = TTK_FP32;
  size_t es = 4;
  std::vector<int> ranks, cross_ranks;
  std::vector<std::vector<double>> cores;   // host copy (read back on request for a device build)
  std::vector<DBuf> dcores;                 // the rounded cores on the device
  CrossOut cross;
  tt_kernel_info info{};
  int64_t ns = 0, nt = 0;
  int rs = 0, rt = 0, ldu = 0, ldv = 0;
  DBuf U, V, nodes, dct, stage[6], pcore[2];
  DBuf work, Mbuf, dMbuf, Wbuf, Zbuf, Abuf, Pbuf;   // Pbuf: partial sums of the reduces
  // Global-1 (Algorithm 4): Q (N x kg row-major, dtype), R (kg x kg FP64)
  int kg = 0;
  DBuf Q, Rg, Gwork, M64, Wg;
  ParamCore pc[2];
  DBuf Cgemm;        // d_theta = 2, float32: the products C_{k1 k2} of the parameter cores
  OnlineGemm og;
  ChainStage src[3], tgt[3];
  KSpec ks{};
  // after Phase 4 (tt_kernel_phase4_round) U, V and the parameter cores are
  // the rounded ones; the spatial cores no longer match them
  bool phase4 = false;
};

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// The parameter cores in the coefficient basis (Algorithm 3 contracts them
// with T_k(t(theta))) from the nodal ones in h->dcores, and for d_theta = 2 in
// float32 the products C_{k1 k2} of the online core's matrix-core form.
static tt_status prepare_param_cores(tt_kernel* h, hipStream_t st) {
  const int d = h->g.d, dt = h->g.dt;
  const int ns_ = h->P.n_spatial;
  const double* Cp = h->dct.as<double>() + (size_t)ns_ * ns_;
  for (int j = 0; j < dt; ++j) {
    const int k = d + j;
    const int r0 = h->ranks[k], n = h->g.n[k], r1 = h->ranks[k + 1];
    const size_t cnt = (size_t)r0 * n * r1;
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((cnt + 255) / 256, 4096));
    TTK_TRY(h->pcore[j].alloc(cnt * sizeof(double)));
    hipLaunchKernelGGL(k_dct_core<double>, dim3(nb), dim3(256), 0, st, h->dcores[k].as<double>(), r0, n, r1, Cp, 2,
                       h->pcore[j].as<double>());
    h->pc[j] = ParamCore{h->pcore[j].as<double>(), r0, n, r1, h->g.lo[k], h->g.hi[k]};
  }
  if (dt == 2 && h->dtype == TTK_FP32) {
    const size_t cnt = (size_t)h->pc[0].r0 * h->pc[1].r1 * h->pc[0].n * h->pc[1].n;
    TTK_TRY(h->Cgemm.alloc(cnt * sizeof(float)));
    TTK_TRY(online_gemm_prepare(h->pc, h->Cgemm.as<float>(), st));
    h->og = OnlineGemm{h->Cgemm.as<float>(), h->pc[0].n * h->pc[1].n, h->pc[0].r0, h->pc[1].r1};
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// DCT the cores on the device, lay them out for Phase 3 and the online stage,
// and run Phase 3 for sources and targets.
static tt_status finish_build(tt_kernel* h, const void* X, const void* Y, hipStream_t st) {
  const int d = h->g.d, dt = h->g.dt, D = h->g.D;
  const size_t es = h->es;
  // basis-change matrices C[k, i] = (c_k / n) T_k(zeta_i), T_k(zeta_i) = cos(k (2i+1) pi / (2n))
  const int ns_ = h->P.n_spatial, np_ = dt > 0 ? h->P.n_param : 2;
  std::vector<double> C((size_t)ns_ * ns_ + (size_t)np_ * np_);
  auto fill_c = [](double* c, int n) {
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i)
        c[k + i * n] = (k == 0 ? 1.0 : 2.0) / n * std::cos(k * (2.0 * i + 1.0) * M_PI / (2.0 * n));
  };
  fill_c(C.data(), ns_);
  fill_c(C.data() + (size_t)ns_ * ns_, np_);
  TTK_TRY(h->dct.alloc(C.size() * sizeof(double)));
  TTK_HIP(hipMemcpyAsync(h->dct.p, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, st));
  const double* Cs = h->dct.as<double>();
  ChainStage* src = h->src;
  ChainStage* tgt = h->tgt;
  for (int k = 0; k < D; ++k) {
    const int r0 = h->ranks[k], n = h->g.n[k], r1 = h->ranks[k + 1];
    const size_t cnt = (size_t)r0 * n * r1;
    const double* gk = h->dcores[k].as<double>();
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((cnt + 255) / 256, 4096));
    if (k < d || k >= d + dt) {
      const int mode = (k < d) ? 0 : 1;
      const int si = (k < d) ? k : (D - 1 - k);   // stage index
      DBuf& sb = h->stage[(k < d) ? si : 3 + si];
      TTK_TRY(sb.alloc(cnt * es));
      if (h->dtype == TTK_FP32)
        hipLaunchKernelGGL(k_dct_core<float>, dim3(nb), dim3(256), 0, st, gk, r0, n, r1, Cs, mode, sb.as<float>());
      else
        hipLaunchKernelGGL(k_dct_core<double>, dim3(nb), dim3(256), 0, st, gk, r0, n, r1, Cs, mode, sb.as<double>());
      ChainStage& cs = (k < d) ? src[si] : tgt[si];
      cs.G2 = sb.p;
      cs.n = n;
      if (k < d) { cs.r_in = r0; cs.r_out = r1; cs.coord = k; }
      else { cs.r_in = r1; cs.r_out = r0; cs.coord = k - d - dt; }
      cs.lo = h->g.lo[k];
      cs.hi = h->g.hi[k];
    }
  }
  TTK_TRY(prepare_param_cores(h, st));
  TTK_HIP(hipStreamSynchronize(st));   // (Phase 3 is timed on its own below)
  h->rs = h->ranks[d];
  h->rt = h->ranks[d + dt];
  // float32 rows padded for the matrix-core apply (columns past r are never
  // read into a result); float64 rows packed
  h->ldu = h->dtype == TTK_FP32 ? mfma_ld(h->rs) : h->rs;
  h->ldv = h->dtype == TTK_FP32 ? mfma_ld(h->rt) : h->rt;
  TTK_TRY(h->U.alloc((size_t)std::max<int64_t>(h->ns, 1) * h->ldu * es));
  TTK_TRY(h->V.alloc((size_t)std::max<int64_t>(h->nt, 1) * h->ldv * es));
  auto t0 = std::chrono::steady_clock::now();
  TTK_TRY(factor_contract(h->dtype, src, d, X, h->ns, h->U.p, h->ldu, st));
  TTK_TRY(factor_contract(h->dtype, tgt, d, Y, h->nt, h->V.p, h->ldv, st));
  TTK_HIP(hipGetLastError());
  TTK_HIP(hipStreamSynchronize(st));
  h->info.t_factor_ms = ms_since(t0);
  return TTK_OK;
}

static tt_status begin_build(const tt_kernel_params* p, const void* X, int64_t n_src, const void* Y, int64_t n_tgt,
                             tt_kernel_t* out, std::unique_ptr<tt_kernel>* hh, hipStream_t st) {
  TTK_TRY(check_params(p));
  if (!out) return fail(TTK_ERR_ARG, "out handle pointer is NULL");
  if (n_src < 0 || n_tgt < 0) return fail(TTK_ERR_ARG, "negative point count");
  if ((n_src > 0 && !X) || (n_tgt > 0 && !Y)) return fail(TTK_ERR_ARG, "point array is NULL");
  std::unique_ptr<tt_kernel> h(new (std::nothrow) tt_kernel());
  if (!h) return fail(TTK_ERR_OOM, "handle allocation failed");
  h->P = *p;
  h->dtype = p->dtype;
  h->es = p->dtype == TTK_FP32 ? 4 : 8;
  h->ns = n_src;
  h->nt = n_tgt;
  make_grid(p, &h->g);
  TTK_TRY(h->nodes.alloc((size_t)MAXD * MAXN * sizeof(double)));
  TTK_HIP(hipMemcpyAsync(h->nodes.p, h->g.nodes, sizeof(h->g.nodes), hipMemcpyHostToDevice, st));
  h->ks = KSpec{p->kind, p->d, p->d_theta, h->g.D, p->kernel_const, h->nodes.as<double>(),
                {p->theta_fixed[0], p->theta_fixed[1]}};
  *hh = std::move(h);
  return TTK_OK;
}

// Algorithm 4 takes one point set in one box: Y must be X (or NULL).
static tt_status check_symmetric(const tt_kernel_params* p, const void* X, int64_t n_src, const void** Y,
                                 int64_t* n_tgt) {
  if (!p || !p->symmetric_psd) return TTK_OK;
  if (*Y == nullptr) {
    *Y = X;
    *n_tgt = n_src;
  }
  if (*Y != X || *n_tgt != n_src)
    return fail(TTK_ERR_ARG, "symmetric_psd needs Y == X (or Y = NULL) and n_tgt == n_src");
  for (int j = 0; j < 2 * p->d; ++j)
    if (p->box_s[j] != p->box_t[j]) return fail(TTK_ERR_ARG, "symmetric_psd needs box_t == box_s");
  return TTK_OK;
}

// Offline part of Algorithm 4: thin QR [U V] = Q R.
static tt_status finish_global(tt_kernel* h, hipStream_t st) {
  if (!h->P.symmetric_psd) return TTK_OK;
  h->kg = h->rs + h->rt;
  TTK_TRY(h->Q.alloc((size_t)std::max<int64_t>(h->ns, 1) * h->kg * h->es));
  TTK_TRY(h->Rg.alloc((size_t)h->kg * h->kg * sizeof(double)));
  auto t0 = std::chrono::steady_clock::now();
  const tt_status s =
      global_qr(h->dtype, h->U.p, h->ldu, h->rs, h->V.p, h->ldv, h->rt, h->ns, h->Q.p, h->Rg.as<double>(), st);
  if (s < 0) {
    h->kg = 0;
    return s;
  }
  h->info.t_factor_ms += ms_since(t0);
  return TTK_OK;
}

static void fill_info(tt_kernel* h) {
  tt_kernel_info& I = h->info;
  I.D = h->g.D;
  I.r_s = h->rs;
  I.r_t = h->rt;
  for (int k = 0; k <= h->g.D && k < 9; ++k) {
    I.ranks[k] = h->ranks[k];
    I.cross_ranks[k] = h->cross_ranks.empty() ? h->ranks[k] : h->cross_ranks[k];
  }
  I.kernel_evals = h->cross.evals;
  I.sweeps = h->cross.sweeps;
  I.n_decisions = (int)h->cross.log.size();
  I.sampled_error = h->cross.error;
  I.init_max_cond = h->cross.init_max_cond;
  I.min_margin = h->cross.min_margin;
  I.n_src = h->ns;
  I.n_tgt = h->nt;
  I.dtype = h->dtype;
}

// ---------------------------------------------------------- online core
// M(theta_b) (and dM/dtheta when dM is not NULL) for b < B into the given
// workspace: the matrix-core product with the precomputed C_{k1 k2} for
// float32 handles with d_theta = 2 and B >= ONLINE_GEMM_MIN_B, the per-theta
// kernels otherwise.  online_work_bytes gives the workspace either needs.
static bool online_uses_gemm(const tt_kernel* h, int B) { return h->og.C != nullptr && B >= ONLINE_GEMM_MIN_B; }
static size_t online_work_bytes(const tt_kernel* h, int B, bool want_d) {
  if (h->g.dt == 0) return 0;
  if (online_uses_gemm(h, B)) return online_gemm_work_floats(h->og, B, want_d) * sizeof(float);
  return online_work_doubles(h->pc, h->g.dt, B) * sizeof(double);
}
static tt_status online_into(const tt_kernel* h, const void* theta, int B, void* M, void* dM, void* work,
                             hipStream_t st) {
  const int dt = h->g.dt;
  if (dt == 0) {
    hipLaunchKernelGGL(k_identity_batch, dim3(256), dim3(256), 0, st, M, h->rs, B, h->dtype == TTK_FP32);
  } else if (online_uses_gemm(h, B)) {
    TTK_TRY(online_core_gemm(h->pc, h->og, static_cast<const float*>(theta), B, static_cast<float*>(M),
                             static_cast<float*>(dM), static_cast<float*>(work), st));
  } else {
    online_core(h->dtype, h->pc, dt, theta, B, M, dM, static_cast<double*>(work), st);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// ---------------------------------------------------------- batched apply
// Scratch of one batched apply: M(theta_b) for all b, W = V^T X (unless the
// caller keeps it), Z = M W, the reduction's partial sums and the online
// core's workspace.  Each piece is written before it is read within a call,
// so nothing has to start at zero.
struct ApplyScratch {
  void* M = nullptr;
  void* W = nullptr;
  void* Z = nullptr;
  void* part = nullptr;
  void* owork = nullptr;
};
struct ApplySizes {
  size_t M = 0, W = 0, Z = 0, part = 0, owork = 0;   // bytes, each rounded up to 256
};
static size_t up256(size_t b) { return (b + 255) / 256 * 256; }
static void apply_sizes(const tt_kernel* h, int B, bool need_w, ApplySizes* z) {
  z->M = up256((size_t)h->rs * h->rt * B * h->es);
  z->W = need_w ? up256((size_t)h->rt * B * h->es) : 0;
  z->Z = up256((size_t)h->rs * B * h->es);
  z->part = up256(apply_reduce_work(h->nt, h->rt, B));
  z->owork = up256(online_work_bytes(h, B, false));
}

static tt_status check_apply_args(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, const void* Y,
                                  int64_t ldy) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B < 0) return fail(TTK_ERR_ARG, "B < 0");
  if (B == 0) return TTK_OK;
  if (!X || !Y) return fail(TTK_ERR_ARG, "X or Y is NULL");
  if (ldx < h->nt || ldy < h->ns) return fail(TTK_ERR_ARG, "leading dimension too small");
  if (h->g.dt > 0 && !theta) return fail(TTK_ERR_ARG, "theta is NULL");
  return TTK_OK;
}

// y_b = U M(theta_b) V^T x_b for b < B with the given scratch (no allocation).
static tt_status apply_core(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                            int64_t ldy, const ApplyScratch& s, hipStream_t st) {
  TTK_TRY(online_into(h, theta, B, s.M, nullptr, s.owork, st));
  TTK_TRY(apply_reduce_matvec(h->dtype, h->V.p, h->ldv, h->nt, h->rt, X, ldx, B, s.W, s.M, h->rs, h->rt, 0, s.Z,
                              s.part, st));
  TTK_TRY(apply_expand(h->dtype, h->U.p, h->ldu, h->ns, h->rs, s.Z, B, Y, ldy, st));
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// The fixed scratch of tt_kernel_apply_noalloc: one array per device, for
// the life of the process.  Host code never passes the array's name to a
// kernel (in host code it is only a stand-in for the symbol): its device
// address is looked up once per device and kept.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static tt_status noalloc_scratch(void** out) {
  int dev = 0;
  TTK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(TTK_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    TTK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(TTK_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TTK_OK;
}

extern "C" {

const char* tt_kernel_last_error(void) { return g_err.c_str(); }

tt_status tt_kernel_build_offline(const tt_kernel_params* p, const void* X, int64_t n_src, const void* Y,
                                  int64_t n_tgt, void* stream, tt_kernel_t* out) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(check_symmetric(p, X, n_src, &Y, &n_tgt));
  std::unique_ptr<tt_kernel> h;
  TTK_TRY(begin_build(p, X, n_src, Y, n_tgt, out, &h, st));
  if (h->P.tol <= 0) return fail(TTK_ERR_ARG, "tol must be positive");
  tt_kernel_params cp = h->P;
  if (cp.init_card == 0) cp.init_card = 2;
  if (cp.max_rank <= 0) cp.max_rank = MAXR;
  auto t0 = std::chrono::steady_clock::now();
  TTK_TRY(run_cross(&cp, h->g, h->ks, st, &h->cross));
  h->info.t_cross_ms = ms_since(t0);
  h->cross_ranks = h->cross.ranks;
  h->dcores = std::move(h->cross.cores);
  h->ranks = h->cross.ranks;
  t0 = std::chrono::steady_clock::now();
  TTK_TRY(round_gauge(h->dcores, h->ranks, h->g, h->P.tol, st));
  h->info.t_round_ms = ms_since(t0);
  TTK_TRY(finish_build(h.get(), X, Y, st));
  TTK_TRY(finish_global(h.get(), st));
  fill_info(h.get());
  const tt_status s = h->cross.converged ? TTK_OK : TTK_WARN_NOT_CONVERGED;
  if (s != TTK_OK) set_error("cross stopped with sampled error %.3e > tol %.3e", h->cross.error, h->P.tol);
  *out = h.release();
  return s;
}

tt_status tt_kernel_build_from_cores(const tt_kernel_params* p, const int* ranks, const double* cores, const void* X,
                                     int64_t n_src, const void* Y, int64_t n_tgt, void* stream, tt_kernel_t* out) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(check_symmetric(p, X, n_src, &Y, &n_tgt));
  std::unique_ptr<tt_kernel> h;
  TTK_TRY(begin_build(p, X, n_src, Y, n_tgt, out, &h, st));
  if (!ranks || !cores) return fail(TTK_ERR_ARG, "ranks or cores is NULL");
  const int D = h->g.D;
  if (ranks[0] != 1 || ranks[D] != 1) return fail(TTK_ERR_ARG, "ranks must start and end with 1");
  h->ranks.assign(ranks, ranks + D + 1);
  size_t off = 0;
  h->cores.resize(D);
  h->dcores.clear();
  h->dcores.resize(D);
  for (int k = 0; k < D; ++k) {
    if (ranks[k + 1] < 1 || ranks[k + 1] > MAXR) return fail(TTK_ERR_ARG, "rank %d out of range", ranks[k + 1]);
    const size_t cnt = (size_t)ranks[k] * h->g.n[k] * ranks[k + 1];
    h->cores[k].assign(cores + off, cores + off + cnt);
    TTK_TRY(h->dcores[k].alloc(cnt * sizeof(double)));
    TTK_HIP(hipMemcpyAsync(h->dcores[k].p, h->cores[k].data(), cnt * sizeof(double), hipMemcpyHostToDevice, st));
    off += cnt;
  }
  h->cross_ranks = h->ranks;
  TTK_TRY(finish_build(h.get(), X, Y, st));
  TTK_TRY(finish_global(h.get(), st));
  fill_info(h.get());
  *out = h.release();
  return TTK_OK;
}

tt_status tt_kernel_factor_rows(tt_kernel_t h, int side, const void* P, int64_t n, void* out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (side != 0 && side != 1) return fail(TTK_ERR_ARG, "side must be 0 (sources) or 1 (targets)");
  if (n < 0 || (n > 0 && (!P || !out))) return fail(TTK_ERR_ARG, "bad points or output");
  if (n == 0) return TTK_OK;
  if (h->phase4) return fail(TTK_ERR_UNSUPPORTED, "after Phase 4 the spatial cores no longer give U and V");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int r = side == 0 ? h->rs : h->rt;
  return factor_contract(h->dtype, side == 0 ? h->src : h->tgt, h->g.d, P, n, out, r, st);
}

tt_status tt_kernel_online_core(tt_kernel_t h, const void* theta, int B, void* M_out, void* dM_out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B < 0 || (B > 0 && !M_out)) return fail(TTK_ERR_ARG, "bad B or M_out");
  if (B == 0) return TTK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->g.dt > 0 && !theta) return fail(TTK_ERR_ARG, "theta is NULL");
  const size_t wb = online_work_bytes(h, B, dM_out != nullptr);
  if (wb) TTK_TRY(h->work.alloc(wb));
  return online_into(h, theta, B, M_out, h->g.dt > 0 ? dM_out : nullptr, h->work.p, st);
}

static tt_status prepare_M(tt_kernel_t h, const void* theta, int B, bool with_dM, hipStream_t st) {
  const size_t msz = (size_t)h->rs * h->rt * B * h->es;
  TTK_TRY(h->Mbuf.alloc(msz));
  if (with_dM) TTK_TRY(h->dMbuf.alloc(msz * std::max(h->g.dt, 1)));
  return tt_kernel_online_core(h, theta, B, h->Mbuf.p, with_dM ? h->dMbuf.p : nullptr, st);
}

// W (r x B) = F^T X with the handle's partial-sum workspace
static tt_status reduce_into(tt_kernel_t h, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx,
                             int B, void* W, hipStream_t st) {
  const size_t wb = apply_reduce_work(N, r, B);
  if (wb) TTK_TRY(h->Pbuf.alloc(wb));
  return apply_reduce(h->dtype, F, ldf, N, r, X, ldx, B, W, wb ? h->Pbuf.p : nullptr, st);
}

tt_status tt_kernel_apply(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          void* W_save, void* stream) {
  TTK_TRY(check_apply_args(h, theta, B, X, ldx, Y, ldy));
  if (B == 0) return TTK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  ApplySizes z;
  apply_sizes(h, B, W_save == nullptr, &z);
  ApplyScratch s{};
  TTK_TRY(h->Mbuf.alloc(z.M));
  s.M = h->Mbuf.p;
  s.W = W_save;
  if (!W_save) {
    TTK_TRY(h->Wbuf.alloc(z.W));
    s.W = h->Wbuf.p;
  }
  TTK_TRY(h->Zbuf.alloc(z.Z));
  s.Z = h->Zbuf.p;
  if (z.part) {
    TTK_TRY(h->Pbuf.alloc(z.part));
    s.part = h->Pbuf.p;
  }
  if (z.owork) {
    TTK_TRY(h->work.alloc(z.owork));
    s.owork = h->work.p;
  }
  return apply_core(h, theta, B, X, ldx, Y, ldy, s, st);
}

tt_status tt_kernel_apply_noalloc(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                                  int64_t ldy, void* W_save, void* stream) {
  TTK_TRY(check_apply_args(h, theta, B, X, ldx, Y, ldy));
  if (B == 0) return TTK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  ApplySizes z;
  apply_sizes(h, B, W_save == nullptr, &z);
  const size_t need = z.M + z.W + z.Z + z.part + z.owork;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(TTK_ERR_ARG,
                "tt_kernel_apply_noalloc: B = %d needs %zu bytes of scratch (M(theta), W, Z, partial sums and the "
                "online workspace); the fixed scratch holds %zu bytes: split the thetas into smaller calls",
                B, need, (size_t)NOALLOC_SCRATCH_BYTES);
  char* base = nullptr;
  TTK_TRY(noalloc_scratch(reinterpret_cast<void**>(&base)));
  ApplyScratch s{};
  size_t off = 0;
  s.M = base + off;
  off += z.M;
  s.W = W_save;
  if (!W_save) {
    s.W = base + off;
    off += z.W;
  }
  s.Z = base + off;
  off += z.Z;
  if (z.part) s.part = base + off;
  off += z.part;
  if (z.owork) s.owork = base + off;
  return apply_core(h, theta, B, X, ldx, Y, ldy, s, st);
}

tt_status tt_kernel_project(tt_kernel_t h, int side, const void* X, int64_t ldx, int B, void* W, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (side != 0 && side != 1) return fail(TTK_ERR_ARG, "side must be 0 (U) or 1 (V)");
  if (B < 0) return fail(TTK_ERR_ARG, "B < 0");
  if (B == 0) return TTK_OK;
  const int64_t n = side == 0 ? h->ns : h->nt;
  if (!X || !W) return fail(TTK_ERR_ARG, "X or W is NULL");
  if (ldx < n) return fail(TTK_ERR_ARG, "ldx too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return side == 0 ? reduce_into(h, h->U.p, h->ldu, h->ns, h->rs, X, ldx, B, W, st)
                   : reduce_into(h, h->V.p, h->ldv, h->nt, h->rt, X, ldx, B, W, st);
}

tt_status tt_kernel_apply_plain(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                                int64_t ldy, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B <= 0) return B == 0 ? TTK_OK : fail(TTK_ERR_ARG, "B < 0");
  if (!X || !Y) return fail(TTK_ERR_ARG, "X or Y is NULL");
  if (ldx < h->nt || ldy < h->ns) return fail(TTK_ERR_ARG, "leading dimension too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(prepare_M(h, theta, B, false, st));
  TTK_TRY(h->Wbuf.alloc((size_t)h->rt * B * h->es));
  TTK_TRY(h->Zbuf.alloc((size_t)h->rs * B * h->es));
  const size_t es = h->es;
  for (int b = 0; b < B; ++b) {
    const char* xb = static_cast<const char*>(X) + (size_t)b * ldx * es;
    char* yb = static_cast<char*>(Y) + (size_t)b * ldy * es;
    char* wb = h->Wbuf.as<char>() + (size_t)b * h->rt * es;
    char* zb = h->Zbuf.as<char>() + (size_t)b * h->rs * es;
    const char* Mb = h->Mbuf.as<char>() + (size_t)b * h->rs * h->rt * es;
    TTK_TRY(reduce_into(h, h->V.p, h->ldv, h->nt, h->rt, xb, ldx, 1, wb, st));
    batched_matvec(h->dtype, Mb, h->rs, h->rt, 0, wb, 1, zb, st);
    TTK_TRY(apply_expand(h->dtype, h->U.p, h->ldu, h->ns, h->rs, zb, 1, yb, ldy, st));
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_apply_backward(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx,
                                   const void* W_saved, const void* G, int64_t ldg, void* dX, int64_t lddx,
                                   void* dtheta, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B <= 0) return B == 0 ? TTK_OK : fail(TTK_ERR_ARG, "B < 0");
  if (!G) return fail(TTK_ERR_ARG, "G is NULL");
  if (ldg < h->ns) return fail(TTK_ERR_ARG, "ldg too small");
  if (dX && lddx < h->nt) return fail(TTK_ERR_ARG, "lddx too small");
  const bool want_dth = dtheta != nullptr && h->g.dt > 0;
  if (want_dth && !W_saved && (!X || ldx < h->nt)) return fail(TTK_ERR_ARG, "X needed when W_saved is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(prepare_M(h, theta, B, want_dth, st));
  TTK_TRY(h->Abuf.alloc((size_t)h->rs * B * h->es));
  const void* W = W_saved;
  if (want_dth && !W) {
    TTK_TRY(h->Wbuf.alloc((size_t)h->rt * B * h->es));
    TTK_TRY(reduce_into(h, h->V.p, h->ldv, h->nt, h->rt, X, ldx, B, h->Wbuf.p, st));   // W = V^T x
    W = h->Wbuf.p;
  }
  if (dX) {
    // A = U^T G, M^T a and (with dtheta) a^T dM w in one pass over the partial sums
    TTK_TRY(h->Zbuf.alloc((size_t)std::max(h->rs, h->rt) * B * h->es));
    const size_t wb = apply_reduce_work(h->ns, h->rs, B);
    if (wb) TTK_TRY(h->Pbuf.alloc(wb));
    TTK_TRY(apply_reduce_matvec(h->dtype, h->U.p, h->ldu, h->ns, h->rs, G, ldg, B, h->Abuf.p, h->Mbuf.p, h->rs,
                                h->rt, 1, h->Zbuf.p, wb ? h->Pbuf.p : nullptr, st, want_dth ? h->dMbuf.p : nullptr,
                                W, h->g.dt, dtheta));
    TTK_TRY(apply_expand(h->dtype, h->V.p, h->ldv, h->nt, h->rt, h->Zbuf.p, B, dX, lddx, st));
  } else {
    TTK_TRY(reduce_into(h, h->U.p, h->ldu, h->ns, h->rs, G, ldg, B, h->Abuf.p, st));   // A = U^T G
    if (want_dth) batched_bilinear(h->dtype, h->Abuf.p, h->dMbuf.p, W, h->rs, h->rt, B, h->g.dt, dtheta, st);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_global_online(tt_kernel_t h, const void* theta, int B, void* W_out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!h->kg) return fail(TTK_ERR_ARG, "handle was not built with symmetric_psd");
  if (B < 0 || (B > 0 && !W_out)) return fail(TTK_ERR_ARG, "bad B or W_out");
  if (B == 0) return TTK_OK;
  if (h->g.dt > 0 && !theta) return fail(TTK_ERR_ARG, "theta is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t msz = (size_t)h->rs * h->rt * B;
  TTK_TRY(h->M64.alloc(msz * sizeof(double)));
  if (h->g.dt == 0) {
    hipLaunchKernelGGL(k_identity_batch, dim3(256), dim3(256), 0, st, h->M64.p, h->rs, B, false);
  } else {
    TTK_TRY(h->work.alloc(online_work_doubles(h->pc, h->g.dt, B) * sizeof(double)));
    online_core_mixed(h->dtype, TTK_FP64, h->pc, h->g.dt, theta, B, h->M64.p, nullptr, h->work.as<double>(), st);
  }
  TTK_TRY(h->Gwork.alloc(global_online_work(h->rs, h->rt, B) * sizeof(double)));
  global_online(h->Rg.as<double>(), h->rs, h->rt, h->M64.as<double>(), B, h->dtype, W_out, h->Gwork.as<double>(), st);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_global_apply(tt_kernel_t h, const void* theta, const void* W, int B, const void* X, int64_t ldx,
                                 void* Y, int64_t ldy, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!h->kg) return fail(TTK_ERR_ARG, "handle was not built with symmetric_psd");
  if (B <= 0) return B == 0 ? TTK_OK : fail(TTK_ERR_ARG, "B < 0");
  if (!X || !Y) return fail(TTK_ERR_ARG, "X or Y is NULL");
  if (ldx < h->ns || ldy < h->ns) return fail(TTK_ERR_ARG, "leading dimension too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int k = h->kg;
  if (!W) {
    TTK_TRY(h->Wg.alloc((size_t)k * k * B * h->es));
    TTK_TRY(tt_kernel_global_online(h, theta, B, h->Wg.p, stream));
    W = h->Wg.p;
  }
  TTK_TRY(h->Wbuf.alloc((size_t)k * B * h->es));
  TTK_TRY(h->Zbuf.alloc((size_t)k * B * h->es));
  TTK_TRY(reduce_into(h, h->Q.p, k, h->ns, k, X, ldx, B, h->Wbuf.p, st));        // Q^T x
  batched_matvec(h->dtype, W, k, k, 0, h->Wbuf.p, B, h->Zbuf.p, st);             // W (Q^T x)
  TTK_TRY(apply_expand(h->dtype, h->Q.p, k, h->ns, k, h->Zbuf.p, B, Y, ldy, st));          // Q (...)
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_global2_online(tt_kernel_t h, const void* theta, double eps, void* Z_out, int64_t ldz,
                                   void* lam_out, int* rc, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!h->kg) return fail(TTK_ERR_ARG, "handle was not built with symmetric_psd");
  if (!(eps > 0.0)) return fail(TTK_ERR_ARG, "eps must be positive");
  if (!Z_out || !lam_out || !rc) return fail(TTK_ERR_ARG, "Z_out, lam_out or rc is NULL");
  const int k = h->kg;
  if (ldz < k) return fail(TTK_ERR_ARG, "ldz (%lld) below r_s + r_t = %d", (long long)ldz, k);
  if (h->g.dt > 0 && !theta) return fail(TTK_ERR_ARG, "theta is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(h->M64.alloc((size_t)h->rs * h->rt * sizeof(double)));
  if (h->g.dt == 0) {
    hipLaunchKernelGGL(k_identity_batch, dim3(256), dim3(256), 0, st, h->M64.p, h->rs, 1, false);
  } else {
    TTK_TRY(h->work.alloc(online_work_doubles(h->pc, h->g.dt, 1) * sizeof(double)));
    online_core_mixed(h->dtype, TTK_FP64, h->pc, h->g.dt, theta, 1, h->M64.p, nullptr, h->work.as<double>(), st);
  }
  TTK_TRY(h->Gwork.alloc(global2_work(h->rs, h->rt) * sizeof(double)));
  double *Uh = nullptr, *lam = nullptr;
  int r = 0;
  TTK_TRY(global2_online(h->Rg.as<double>(), h->rs, h->rt, h->M64.as<double>(), eps, h->Gwork.as<double>(), &Uh,
                         &lam, &r, st));
  *rc = r;
  if (r == 0) return TTK_OK;
  // Z = Q Uhat: Q (N x k row-major) times Uhat[:, :rc] (k x rc), through the
  // apply's expand (column-major N x rc), then to rows
  const int64_t N = h->ns;
  TTK_TRY(h->Zbuf.alloc((size_t)k * r * h->es));
  TTK_TRY(h->Wbuf.alloc((size_t)std::max<int64_t>(N, 1) * r * h->es));
  const unsigned g1 = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, ((int64_t)k * r + 255) / 256));
  if (h->dtype == TTK_FP32)
    hipLaunchKernelGGL(k_g2_convert<float>, dim3(g1), dim3(256), 0, st, (const double*)Uh, k, r, (const double*)lam,
                       h->Zbuf.as<float>(), static_cast<float*>(lam_out));
  else
    hipLaunchKernelGGL(k_g2_convert<double>, dim3(g1), dim3(256), 0, st, (const double*)Uh, k, r,
                       (const double*)lam, h->Zbuf.as<double>(), static_cast<double*>(lam_out));
  TTK_TRY(apply_expand(h->dtype, h->Q.p, k, N, k, h->Zbuf.p, r, h->Wbuf.p, N, st));
  const unsigned g2 = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (N * r + 255) / 256));
  if (h->dtype == TTK_FP32)
    hipLaunchKernelGGL(k_g2_rows<float>, dim3(g2), dim3(256), 0, st, (const float*)h->Wbuf.p, N, r,
                       static_cast<float*>(Z_out), ldz);
  else
    hipLaunchKernelGGL(k_g2_rows<double>, dim3(g2), dim3(256), 0, st, (const double*)h->Wbuf.p, N, r,
                       static_cast<double*>(Z_out), ldz);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_global2_apply(tt_kernel_t h, const void* Z, int64_t ldz, const void* lam, int rc, int B,
                                  const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!h->kg) return fail(TTK_ERR_ARG, "handle was not built with symmetric_psd");
  if (B < 0 || rc < 0 || rc > h->kg) return fail(TTK_ERR_ARG, "bad B or rc");
  if (B == 0) return TTK_OK;
  if (!X || !Y || (rc > 0 && (!Z || !lam))) return fail(TTK_ERR_ARG, "NULL argument");
  if (ldx < h->ns || ldy < h->ns || (rc > 0 && ldz < rc)) return fail(TTK_ERR_ARG, "leading dimension too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (rc == 0) {
    for (int b = 0; b < B; ++b) fill_zero(static_cast<char*>(Y) + (size_t)b * ldy * h->es, (size_t)h->ns * h->es, st);
    return TTK_OK;
  }
  TTK_TRY(h->Wbuf.alloc((size_t)rc * B * h->es));
  TTK_TRY(reduce_into(h, Z, (int)ldz, h->ns, rc, X, ldx, B, h->Wbuf.p, st));   // Z^T x
  const unsigned g = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, ((int64_t)rc * B + 255) / 256));
  if (h->dtype == TTK_FP32)
    hipLaunchKernelGGL(k_g2_scale<float>, dim3(g), dim3(256), 0, st, h->Wbuf.as<float>(), static_cast<const float*>(lam),
                       rc, B);
  else
    hipLaunchKernelGGL(k_g2_scale<double>, dim3(g), dim3(256), 0, st, h->Wbuf.as<double>(),
                       static_cast<const double*>(lam), rc, B);
  TTK_TRY(apply_expand(h->dtype, Z, (int)ldz, h->ns, rc, h->Wbuf.p, B, Y, ldy, st));   // Z (lam Z^T x)
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_phase4_round(tt_kernel_t h, double eps, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!(eps > 0.0)) return fail(TTK_ERR_ARG, "eps must be positive");
  if (h->kg) return fail(TTK_ERR_ARG, "Phase 4 is for the U, V of the low-rank form, not a Global-1 handle");
  const int d = h->g.d, dt = h->g.dt, rs = h->rs, rt = h->rt;
  if (rs > 128 || rt > 128)
    return fail(TTK_ERR_UNSUPPORTED, "Phase 4: ranks %d, %d above the tall-skinny QR's 128", rs, rt);
  if (h->ns < rs || h->nt < rt)
    return fail(TTK_ERR_UNSUPPORTED, "Phase 4 needs at least r_s sources and r_t targets");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto t0 = std::chrono::steady_clock::now();
  // S = Q_S R_S, T = Q_T R_T (tall-skinny QR, float64)
  TsqrState qs, qt;
  DBuf Rs, Rt;
  TTK_TRY(Rs.alloc((size_t)rs * rs * sizeof(double)));
  TTK_TRY(Rt.alloc((size_t)rt * rt * sizeof(double)));
  TTK_TRY(tsqr_factor(h->dtype, h->U.p, h->ldu, 1, h->ns, rs, &qs, Rs.as<double>(), rs, st));
  TTK_TRY(tsqr_factor(h->dtype, h->V.p, h->ldv, 1, h->nt, rt, &qt, Rt.as<double>(), rt, st));
  // the small TT [R_S, G_{d+1}, ..., G_{d+d_theta}, R_T^T]: the TT of Phase 4
  // with its first and last cores' point index replaced by the columns of
  // Q_S and Q_T (orthonormal, so TT-Round of either is the same rounding)
  const int D2 = dt + 2;
  std::vector<DBuf> sc(D2);
  std::vector<int> sr(D2 + 1);
  sr[0] = 1;
  sr[1] = rs;
  for (int j = 0; j < dt; ++j) sr[2 + j] = h->ranks[d + j + 1];
  sr[D2] = 1;
  Grid g2 = h->g;
  g2.d = 1;
  g2.dt = dt;
  g2.D = D2;
  g2.n[0] = rs;
  for (int j = 0; j < dt; ++j) g2.n[1 + j] = h->g.n[d + j];
  g2.n[D2 - 1] = rt;
  TTK_TRY(sc[0].alloc((size_t)rs * rs * sizeof(double)));
  TTK_HIP(hipMemcpyAsync(sc[0].p, Rs.p, (size_t)rs * rs * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int j = 0; j < dt; ++j) {
    const size_t cnt = (size_t)h->ranks[d + j] * h->g.n[d + j] * h->ranks[d + j + 1];
    TTK_TRY(sc[1 + j].alloc(cnt * sizeof(double)));
    TTK_HIP(hipMemcpyAsync(sc[1 + j].p, h->dcores[d + j].p, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  TTK_TRY(sc[D2 - 1].alloc((size_t)rt * rt * sizeof(double)));   // (a, b) = R_T(b, a)
  hipLaunchKernelGGL(k_transpose_small, dim3((rt * rt + 255) / 256), dim3(256), 0, st, (const double*)Rt.as<double>(),
                     rt, rt, sc[D2 - 1].as<double>());
  TTK_HIP(hipGetLastError());
  TTK_TRY(round_gauge(sc, sr, g2, eps, st));
  const int rs2 = sr[1], rt2 = sr[D2 - 1];
  // U' = Q_S A_S (A_S = the first core, rs x rs2) and V' = Q_T A_T^T (the last
  // core, rt2 x rt)
  const int ldu2 = h->dtype == TTK_FP32 ? mfma_ld(rs2) : rs2;
  const int ldv2 = h->dtype == TTK_FP32 ? mfma_ld(rt2) : rt2;
  DBuf U2, V2, CT;
  TTK_TRY(U2.alloc((size_t)std::max<int64_t>(h->ns, 1) * ldu2 * h->es));
  TTK_TRY(V2.alloc((size_t)std::max<int64_t>(h->nt, 1) * ldv2 * h->es));
  TTK_TRY(CT.alloc((size_t)rt * rt2 * sizeof(double)));
  if (ldu2 > rs2) fill_zero(U2.p, (size_t)std::max<int64_t>(h->ns, 1) * ldu2 * h->es, st);
  if (ldv2 > rt2) fill_zero(V2.p, (size_t)std::max<int64_t>(h->nt, 1) * ldv2 * h->es, st);
  TTK_TRY(tsqr_apply(&qs, sc[0].as<double>(), rs, rs2, h->dtype, U2.p, ldu2, 1, st));
  hipLaunchKernelGGL(k_transpose_small, dim3((rt * rt2 + 255) / 256), dim3(256), 0, st,
                     (const double*)sc[D2 - 1].as<double>(), rt2, rt, CT.as<double>());
  TTK_TRY(tsqr_apply(&qt, CT.as<double>(), rt, rt2, h->dtype, V2.p, ldv2, 1, st));
  // the handle takes the rounded parameter cores, U' and V'
  for (int j = 0; j < dt; ++j) h->dcores[d + j] = std::move(sc[1 + j]);
  for (int j = 0; j <= dt; ++j) h->ranks[d + j] = sr[1 + j];
  TTK_TRY(prepare_param_cores(h, st));
  TTK_HIP(hipStreamSynchronize(st));   // the old U, V, cores and the QR state are released below
  h->U = std::move(U2);
  h->V = std::move(V2);
  h->rs = rs2;
  h->rt = rt2;
  h->ldu = ldu2;
  h->ldv = ldv2;
  h->phase4 = true;
  h->cores.clear();
  h->info.r_s = rs2;
  h->info.r_t = rt2;
  for (int k = 0; k <= h->g.D && k < 9; ++k) h->info.ranks[k] = h->ranks[k];
  h->info.t_factor_ms += ms_since(t0);
  return TTK_OK;
}

tt_status tt_kernel_global_factors(tt_kernel_t h, int* k, void* Q_out, double* R_out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (!h->kg) return fail(TTK_ERR_ARG, "handle was not built with symmetric_psd");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (k) *k = h->kg;
  if (Q_out && h->ns > 0)
    TTK_HIP(hipMemcpyAsync(Q_out, h->Q.p, (size_t)h->ns * h->kg * h->es, hipMemcpyDeviceToDevice, st));
  if (R_out) {
    TTK_HIP(hipMemcpyAsync(R_out, h->Rg.p, (size_t)h->kg * h->kg * sizeof(double), hipMemcpyDeviceToHost, st));
    TTK_HIP(hipStreamSynchronize(st));
  }
  return TTK_OK;
}

tt_status tt_kernel_eval_entries(const tt_kernel_params* p, const int32_t* idx, int64_t P, double* out, void* stream) {
  TTK_TRY(check_params(p));
  if (P < 0 || (P > 0 && (!idx || !out))) return fail(TTK_ERR_ARG, "bad idx/out");
  if (P == 0) return TTK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Grid g;
  make_grid(p, &g);
  DBuf nodes;
  TTK_TRY(nodes.alloc(sizeof(g.nodes)));
  TTK_HIP(hipMemcpyAsync(nodes.p, g.nodes, sizeof(g.nodes), hipMemcpyHostToDevice, st));
  KSpec ks{p->kind, p->d, p->d_theta, g.D, p->kernel_const, nodes.as<double>(), {p->theta_fixed[0], p->theta_fixed[1]}};
  eval_multi32(ks, idx, P, out, st);
  TTK_HIP(hipGetLastError());
  TTK_HIP(hipStreamSynchronize(st));   // nodes is freed on return
  return TTK_OK;
}

tt_status tt_kernel_eval_dense(const tt_kernel_params* p, const void* X, int64_t nx, const void* Y, int64_t ny,
                               const double* theta, void* K, int64_t ldk, void* stream) {
  TTK_TRY(check_params(p));
  if (nx < 0 || ny < 0 || ldk < nx) return fail(TTK_ERR_ARG, "bad sizes");
  if (nx == 0 || ny == 0) return TTK_OK;
  if (!X || !Y || !K || (p->d_theta > 0 && !theta)) return fail(TTK_ERR_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Grid g;
  make_grid(p, &g);
  KSpec ks{p->kind, p->d, p->d_theta, g.D, p->kernel_const, nullptr, {p->theta_fixed[0], p->theta_fixed[1]}};
  if (p->dtype == TTK_FP32)
    eval_dense_f32(ks, static_cast<const float*>(X), nx, static_cast<const float*>(Y), ny, theta,
                   static_cast<float*>(K), ldk, st);
  else
    eval_dense_f64(ks, static_cast<const double*>(X), nx, static_cast<const double*>(Y), ny, theta,
                   static_cast<double*>(K), ldk, st);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_get_info(tt_kernel_t h, tt_kernel_info* info) {
  if (!h || !info) return fail(TTK_ERR_ARG, "NULL argument");
  *info = h->info;
  return TTK_OK;
}

tt_status tt_kernel_get_factors(tt_kernel_t h, void* U_out, void* V_out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (U_out && h->ns > 0)
    TTK_HIP(hipMemcpy2DAsync(U_out, (size_t)h->rs * h->es, h->U.p, (size_t)h->ldu * h->es, (size_t)h->rs * h->es,
                             (size_t)h->ns, hipMemcpyDeviceToDevice, st));
  if (V_out && h->nt > 0)
    TTK_HIP(hipMemcpy2DAsync(V_out, (size_t)h->rt * h->es, h->V.p, (size_t)h->ldv * h->es, (size_t)h->rt * h->es,
                             (size_t)h->nt, hipMemcpyDeviceToDevice, st));
  return TTK_OK;
}

tt_status tt_kernel_get_cores(tt_kernel_t h, double* cores, int64_t capacity) {
  if (!h || !cores) return fail(TTK_ERR_ARG, "NULL argument");
  if (h->phase4) return fail(TTK_ERR_UNSUPPORTED, "after Phase 4 the cores are U, the parameter cores and V");
  const int D = h->g.D;
  if (h->cores.size() != (size_t)D) {   // a device build: read the rounded cores back once
    h->cores.assign(D, {});
    for (int k = 0; k < D; ++k) {
      h->cores[k].resize((size_t)h->ranks[k] * h->g.n[k] * h->ranks[k + 1]);
      TTK_HIP(hipMemcpy(h->cores[k].data(), h->dcores[k].p, h->cores[k].size() * sizeof(double),
                        hipMemcpyDeviceToHost));
    }
  }
  size_t need = 0;
  for (auto& c : h->cores) need += c.size();
  if ((size_t)capacity < need) return fail(TTK_ERR_ARG, "capacity %lld < %zu", (long long)capacity, need);
  size_t off = 0;
  for (auto& c : h->cores) {
    std::memcpy(cores + off, c.data(), c.size() * sizeof(double));
    off += c.size();
  }
  return TTK_OK;
}

tt_status tt_kernel_get_coeff_cores(tt_kernel_t h, double* cores, int64_t capacity) {
  if (!h || !cores) return fail(TTK_ERR_ARG, "NULL argument");
  if (h->phase4) return fail(TTK_ERR_UNSUPPORTED, "after Phase 4 the cores are U, the parameter cores and V");
  const int d = h->g.d, dt = h->g.dt, D = h->g.D;
  size_t need = 0;
  for (int k = 0; k < D; ++k) need += (size_t)h->ranks[k] * h->g.n[k] * h->ranks[k + 1];
  if ((size_t)capacity < need) return fail(TTK_ERR_ARG, "capacity %lld < %zu", (long long)capacity, need);
  std::vector<double> tmp;
  std::vector<float> tmpf;
  size_t off = 0;
  for (int k = 0; k < D; ++k) {
    const int r0 = h->ranks[k], n = h->g.n[k], r1 = h->ranks[k + 1];
    const size_t cnt = (size_t)r0 * n * r1;
    if (k >= d && k < d + dt) {   // parameter core: FP64, little-endian already
      TTK_HIP(hipMemcpy(cores + off, h->pcore[k - d].p, cnt * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      // Phase 3 layout: source stage (a + i r0) r1 + b, target stage (b + i r1) r0 + a
      const DBuf& sb = h->stage[k < d ? k : 3 + (D - 1 - k)];
      tmp.resize(cnt);
      if (h->dtype == TTK_FP32) {
        tmpf.resize(cnt);
        TTK_HIP(hipMemcpy(tmpf.data(), sb.p, cnt * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < cnt; ++e) tmp[e] = tmpf[e];
      } else {
        TTK_HIP(hipMemcpy(tmp.data(), sb.p, cnt * sizeof(double), hipMemcpyDeviceToHost));
      }
      for (int b = 0; b < r1; ++b)
        for (int i = 0; i < n; ++i)
          for (int a = 0; a < r0; ++a) {
            const size_t src = k < d ? ((size_t)a + (size_t)i * r0) * r1 + b : ((size_t)b + (size_t)i * r1) * r0 + a;
            cores[off + a + (size_t)i * r0 + (size_t)b * r0 * n] = tmp[src];
          }
    }
    off += cnt;
  }
  return TTK_OK;
}

tt_status tt_kernel_get_cross(tt_kernel_t h, int32_t* left, int32_t* right, tt_kernel_decision* decisions,
                              int max_decisions) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  const int D = h->g.D;
  if (left) {
    size_t off = 0;
    for (int k = 1; k < D && k < (int)h->cross.left.size(); ++k) {
      std::memcpy(left + off, h->cross.left[k].data(), h->cross.left[k].size() * sizeof(int32_t));
      off += h->cross.left[k].size();
    }
  }
  if (right) {
    size_t off = 0;
    for (int k = 1; k < D && k < (int)h->cross.right.size(); ++k) {
      std::memcpy(right + off, h->cross.right[k].data(), h->cross.right[k].size() * sizeof(int32_t));
      off += h->cross.right[k].size();
    }
  }
  if (decisions) {
    const int n = std::min<int>(max_decisions, (int)h->cross.log.size());
    for (int i = 0; i < n; ++i) decisions[i] = h->cross.log[i];
  }
  return TTK_OK;
}

tt_status tt_kernel_destroy(tt_kernel_t h) {
  delete h;
  return TTK_OK;
}

}  // extern "C"

// ===================================================================
// Interaction lists (tt_kernel_batch_*)
// ===================================================================

namespace {

// Canonical frame of a box pair: canonical axis j is the pair's axis perm[j],
// reflected when sign[j] < 0; canonical source box [0, hs], target box centred
// at hs/2 + |delta|.  identity: the pair's own boxes (test kernels).
struct Frame {
  int perm[3] = {0, 1, 2};
  int sign[3] = {1, 1, 1};
  double cbs[6] = {0}, cbt[6] = {0};
  std::vector<double> key;
};

bool isotropic_kind(int kind) { return kind != TTK_TEST_POLY && kind != TTK_TEST_SEP; }

double round12(double v) {
  char buf[64];
  snprintf(buf, sizeof(buf), "%.11e", v);
  return std::strtod(buf, nullptr);
}

Frame pair_frame(int kind, int d, const tt_kernel_pair& pr) {
  Frame f;
  if (!isotropic_kind(kind)) {
    for (int j = 0; j < 2 * d; ++j) {
      f.cbs[j] = pr.box_s[j];
      f.cbt[j] = pr.box_t[j];
      f.key.push_back(pr.box_s[j]);
      f.key.push_back(pr.box_t[j]);
    }
    f.key.push_back(-1.0);
    return f;
  }
  double hs[3], ht[3], dl[3];
  for (int i = 0; i < d; ++i) {
    hs[i] = pr.box_s[2 * i + 1] - pr.box_s[2 * i];
    ht[i] = pr.box_t[2 * i + 1] - pr.box_t[2 * i];
    dl[i] = 0.5 * (pr.box_t[2 * i] + pr.box_t[2 * i + 1]) - 0.5 * (pr.box_s[2 * i] + pr.box_s[2 * i + 1]);
  }
  auto tup = [&](int i) { return std::array<double, 3>{round12(hs[i]), round12(ht[i]), round12(std::fabs(dl[i]))}; };
  std::vector<int> ax(d);
  for (int i = 0; i < d; ++i) ax[i] = i;
  std::stable_sort(ax.begin(), ax.end(), [&](int a, int b) { return tup(a) < tup(b); });
  for (int j = 0; j < d; ++j) {
    const int i = ax[j];
    f.perm[j] = i;
    f.sign[j] = dl[i] >= 0.0 ? 1 : -1;
    f.cbs[2 * j] = 0.0;
    f.cbs[2 * j + 1] = hs[i];
    const double m = 0.5 * hs[i] + std::fabs(dl[i]);
    f.cbt[2 * j] = m - 0.5 * ht[i];
    f.cbt[2 * j + 1] = m + 0.5 * ht[i];
    const auto t = tup(i);
    f.key.insert(f.key.end(), t.begin(), t.end());
  }
  return f;
}

}  // namespace

struct tt_kernel_batch {
  tt_kernel_params P{};
  int dtype = TTK_FP32, d = 0, dt = 0, D = 0;
  size_t es = 4;
  std::vector<tt_kernel_pair> pairs;
  std::vector<int> cls;
  std::vector<std::unique_ptr<tt_kernel>> classes;
  std::vector<ChainStage> stages;          // per pair: d source stages, then d target stages
  std::vector<int64_t> uoff, voff;         // element offsets of the pair blocks of U and V
  int64_t nx = 0, ny = 0;
  DBuf U, V;
  FactorBatchPlan plan;
  const void* lastX = nullptr;
  const void* lastY = nullptr;
  int factor_grid = 0;                     // chosen persistent grid (0 = one per tile)
  bool converged = true;
  int cfg_graph = 1, cfg_factor_grid = 0, cfg_reduce_rows = 0;
  tt_kernel_batch_info info{};
  // apply state, prepared per B
  int prepB = -1, reduce_rows = 0;
  std::vector<BatchSide> hs, ht;
  DBuf dsides_s, dsides_t, dmoff, ddmoff;
  DBuf it_rt, it_rs, it_es, it_et;         // reduce over targets / sources, expand over sources / targets
  int64_t n_rt = 0, n_rs = 0, n_es = 0, n_et = 0;
  DBuf Mall, dMall, work, Wt, Zs, As, Zt, part;
  std::vector<int64_t> Moff, dMoff;        // per class
  // captured graph
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  ~tt_kernel_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

tt_status batch_phase3(tt_kernel_batch* b, const void* X, const void* Y, int grid, hipStream_t st) {
  const int d = b->d;
  if (X != b->lastX || Y != b->lastY) {
    b->plan.njobs = -1;   // the job list holds the point pointers
    b->lastX = X;
    b->lastY = Y;
  }
  const int np = (int)b->pairs.size();
  std::vector<FactorJob> jobs;
  jobs.reserve(2 * np);
  for (int p = 0; p < np; ++p) {
    const tt_kernel_pair& pr = b->pairs[p];
    const tt_kernel* c = b->classes[b->cls[p]].get();
    if (pr.n_src > 0)
      jobs.push_back(FactorJob{&b->stages[(size_t)p * 2 * d], d, static_cast<const char*>(X) + pr.src_off * b->es,
                               b->nx, pr.n_src, b->U.as<char>() + b->uoff[p] * b->es, c->rs});
    if (pr.n_tgt > 0)
      jobs.push_back(FactorJob{&b->stages[(size_t)p * 2 * d + d], d, static_cast<const char*>(Y) + pr.tgt_off * b->es,
                               b->ny, pr.n_tgt, b->V.as<char>() + b->voff[p] * b->es, c->rt});
  }
  return factor_contract_batch(b->dtype, jobs.data(), (int)jobs.size(), grid, st, &b->plan);
}

// Phase 3 with the launch shape chosen by timing when not fixed by the caller.
tt_status batch_phase3_tuned(tt_kernel_batch* b, const void* X, const void* Y, hipStream_t st) {
  if (b->cfg_factor_grid != 0) {
    b->factor_grid = b->cfg_factor_grid < 0 ? 0 : b->cfg_factor_grid;
    return batch_phase3(b, X, Y, b->factor_grid, st);
  }
  TTK_TRY(batch_phase3(b, X, Y, 0, st));
  if (!b->plan.persistent) {
    b->factor_grid = 0;
    return TTK_OK;
  }
  int dev = 0, cus = 256;
  TTK_HIP(hipGetDevice(&dev));
  TTK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int cand[5] = {0, cus, 2 * cus, 4 * cus, 8 * cus};
  hipEvent_t e0, e1;
  TTK_HIP(hipEventCreate(&e0));
  TTK_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_g = 0;
  for (int g : cand) {
    TTK_TRY(batch_phase3(b, X, Y, g, st));   // warm
    TTK_HIP(hipEventRecord(e0, st));
    TTK_TRY(batch_phase3(b, X, Y, g, st));
    TTK_HIP(hipEventRecord(e1, st));
    TTK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TTK_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; best_g = g; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->factor_grid = best_g;
  return batch_phase3(b, X, Y, best_g, st);
}

void make_items(const std::vector<BatchSide>& sides, int64_t rows, bool rank_tiles, int B,
                std::vector<BatchItem>* out) {
  out->clear();
  for (int s = 0; s < (int)sides.size(); ++s) {
    const BatchSide& sd = sides[s];
    const int nrt = rank_tiles ? (sd.r + 63) / 64 : 1;
    for (int64_t r0 = 0; r0 < sd.n; r0 += rows)
      for (int rt = 0; rt < nrt; ++rt)
        for (int b0 = 0; b0 < B; b0 += 64)
          out->push_back(BatchItem{r0, s, (int)std::min<int64_t>(rows, sd.n - r0), rt * 64, b0});
  }
}

tt_status upload_items(const std::vector<BatchItem>& v, DBuf* buf, int64_t* n, hipStream_t st) {
  *n = (int64_t)v.size();
  TTK_TRY(buf->alloc(std::max<size_t>(1, v.size()) * sizeof(BatchItem)));
  if (!v.empty()) TTK_HIP(hipMemcpyAsync(buf->p, v.data(), v.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st));
  return TTK_OK;
}

tt_status set_reduce_rows(tt_kernel_batch* b, int rows, int B, hipStream_t st) {
  std::vector<BatchItem> v;
  make_items(b->ht, rows, true, B, &v);
  TTK_TRY(upload_items(v, &b->it_rt, &b->n_rt, st));
  make_items(b->hs, rows, true, B, &v);
  TTK_TRY(upload_items(v, &b->it_rs, &b->n_rs, st));
  TTK_HIP(hipStreamSynchronize(st));   // host staging goes out of scope
  b->reduce_rows = rows;
  return TTK_OK;
}

// Buffers, side tables and work lists for B thetas; the reduction chunk is
// chosen by timing the target-side reduction on X when not fixed.
tt_status batch_prepare(tt_kernel_batch* b, int B, const void* X, int64_t ldx, hipStream_t st) {
  if (b->prepB == B) return TTK_OK;
  const int np = (int)b->pairs.size(), nc = (int)b->classes.size();
  const size_t es = b->es;
  b->hs.assign(np, BatchSide{});
  b->ht.assign(np, BatchSide{});
  std::vector<int64_t> moff(np), dmoff(np);
  b->Moff.assign(nc, 0);
  b->dMoff.assign(nc, 0);
  int64_t m = 0, dm = 0;
  size_t wmax = 16;
  for (int c = 0; c < nc; ++c) {
    const tt_kernel* k = b->classes[c].get();
    b->Moff[c] = m;
    b->dMoff[c] = dm;
    m += (int64_t)B * k->rs * k->rt;
    dm += (int64_t)B * std::max(b->dt, 1) * k->rs * k->rt;
    if (b->dt > 0) wmax = std::max(wmax, online_work_doubles(k->pc, b->dt, B));
  }
  int64_t ws = 0, wt = 0;
  for (int p = 0; p < np; ++p) {
    const tt_kernel_pair& pr = b->pairs[p];
    const tt_kernel* k = b->classes[b->cls[p]].get();
    b->hs[p] = BatchSide{b->uoff[p], pr.n_src, pr.src_off, ws, k->rs, 0};
    b->ht[p] = BatchSide{b->voff[p], pr.n_tgt, pr.tgt_off, wt, k->rt, 0};
    ws += (int64_t)k->rs * B;
    wt += (int64_t)k->rt * B;
    moff[p] = b->Moff[b->cls[p]];
    dmoff[p] = b->dMoff[b->cls[p]];
  }
  TTK_TRY(b->dsides_s.alloc(sizeof(BatchSide) * np));
  TTK_TRY(b->dsides_t.alloc(sizeof(BatchSide) * np));
  TTK_TRY(b->dmoff.alloc(sizeof(int64_t) * np));
  TTK_TRY(b->ddmoff.alloc(sizeof(int64_t) * np));
  TTK_HIP(hipMemcpyAsync(b->dsides_s.p, b->hs.data(), sizeof(BatchSide) * np, hipMemcpyHostToDevice, st));
  TTK_HIP(hipMemcpyAsync(b->dsides_t.p, b->ht.data(), sizeof(BatchSide) * np, hipMemcpyHostToDevice, st));
  TTK_HIP(hipMemcpyAsync(b->dmoff.p, moff.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice, st));
  TTK_HIP(hipMemcpyAsync(b->ddmoff.p, dmoff.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice, st));
  TTK_TRY(b->Mall.alloc(std::max<int64_t>(m, 1) * es));
  TTK_TRY(b->dMall.alloc(std::max<int64_t>(dm, 1) * es));
  TTK_TRY(b->work.alloc(wmax * sizeof(double)));
  TTK_TRY(b->Wt.alloc(std::max<int64_t>(wt, 1) * es));
  TTK_TRY(b->Zt.alloc(std::max<int64_t>(wt, 1) * es));
  TTK_TRY(b->Zs.alloc(std::max<int64_t>(ws, 1) * es));
  TTK_TRY(b->As.alloc(std::max<int64_t>(ws, 1) * es));
  TTK_TRY(b->part.alloc(std::max<size_t>(1, (size_t)B * std::max(b->dt, 1) * np) * sizeof(double)));
  std::vector<BatchItem> v;
  make_items(b->hs, 64, false, B, &v);
  TTK_TRY(upload_items(v, &b->it_es, &b->n_es, st));
  make_items(b->ht, 64, false, B, &v);
  TTK_TRY(upload_items(v, &b->it_et, &b->n_et, st));
  TTK_HIP(hipStreamSynchronize(st));
  if (b->cfg_reduce_rows > 0) {
    TTK_TRY(set_reduce_rows(b, b->cfg_reduce_rows, B, st));
  } else {
    // time the target-side reduction for each candidate chunk
    const int cand[4] = {256, 1024, 4096, 16384};
    hipEvent_t e0, e1;
    TTK_HIP(hipEventCreate(&e0));
    TTK_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int best_r = 1024;
    for (int rows : cand) {
      TTK_TRY(set_reduce_rows(b, rows, B, st));
      fill_zero(b->Wt.p, (size_t)std::max<int64_t>(wt, 1) * es, st);
      batch_reduce(b->dtype, b->V.p, b->dsides_t.as<BatchSide>(), b->it_rt.as<BatchItem>(), b->n_rt, X, ldx, B,
                   b->Wt.p, st);
      TTK_HIP(hipEventRecord(e0, st));
      fill_zero(b->Wt.p, (size_t)std::max<int64_t>(wt, 1) * es, st);
      batch_reduce(b->dtype, b->V.p, b->dsides_t.as<BatchSide>(), b->it_rt.as<BatchItem>(), b->n_rt, X, ldx, B,
                   b->Wt.p, st);
      TTK_HIP(hipEventRecord(e1, st));
      TTK_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      TTK_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; best_r = rows; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TTK_TRY(set_reduce_rows(b, best_r, B, st));
  }
  TTK_HIP(hipGetLastError());
  b->prepB = B;
  b->info.reduce_rows = b->reduce_rows;
  return TTK_OK;
}

// The whole apply (+ backward) on stream st: launches only, no allocation or
// synchronisation, so it can be captured.
tt_status batch_enqueue(tt_kernel_batch* b, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                        int64_t ldy, const void* G, int64_t ldg, void* dX, int64_t lddx, void* dtheta,
                        hipStream_t st) {
  const int np = (int)b->pairs.size();
  const int dt = b->dt;
  const size_t es = b->es;
  const bool want_dth = G && dtheta && dt > 0;
  for (int c = 0; c < (int)b->classes.size(); ++c) {
    tt_kernel* k = b->classes[c].get();
    char* Mc = b->Mall.as<char>() + b->Moff[c] * es;
    char* dMc = b->dMall.as<char>() + b->dMoff[c] * es;
    if (dt == 0)
      hipLaunchKernelGGL(k_identity_batch, dim3(64), dim3(256), 0, st, Mc, k->rs, B, b->dtype == TTK_FP32);
    else
      online_core(b->dtype, k->pc, dt, theta, B, Mc, want_dth ? dMc : nullptr, b->work.as<double>(), st);
  }
  int64_t wt = 0, ws = 0;
  for (int p = 0; p < np; ++p) {
    wt += (int64_t)b->ht[p].r * B;
    ws += (int64_t)b->hs[p].r * B;
  }
  const BatchSide* ss = b->dsides_s.as<BatchSide>();
  const BatchSide* ts = b->dsides_t.as<BatchSide>();
  // forward: W_p = V_p^T x_p, Z_p = M W_p, Y = sum_p U_p Z_p
  fill_zero(b->Wt.p, (size_t)std::max<int64_t>(wt, 1) * es, st);
  batch_reduce(b->dtype, b->V.p, ts, b->it_rt.as<BatchItem>(), b->n_rt, X, ldx, B, b->Wt.p, st);
  batch_small(b->dtype, b->Mall.p, b->dmoff.as<int64_t>(), ts, ss, 0, b->Wt.p, b->Zs.p, B, np, st);
  fill_cols(b->dtype, Y, b->nx, B, ldy, st);
  batch_expand(b->dtype, b->U.p, ss, b->it_es.as<BatchItem>(), b->n_es, b->Zs.p, B, Y, ldy, st);
  if (G) {
    // backward: A_p = U_p^T g_p; dX = sum_p V_p M^T A_p; dtheta = sum_p A_p^T dM W_p
    fill_zero(b->As.p, (size_t)std::max<int64_t>(ws, 1) * es, st);
    batch_reduce(b->dtype, b->U.p, ss, b->it_rs.as<BatchItem>(), b->n_rs, G, ldg, B, b->As.p, st);
    if (dX) {
      batch_small(b->dtype, b->Mall.p, b->dmoff.as<int64_t>(), ss, ts, 1, b->As.p, b->Zt.p, B, np, st);
      fill_cols(b->dtype, dX, b->ny, B, lddx, st);
      batch_expand(b->dtype, b->V.p, ts, b->it_et.as<BatchItem>(), b->n_et, b->Zt.p, B, dX, lddx, st);
    }
    if (want_dth)
      batch_dtheta(b->dtype, b->As.p, ss, b->dMall.p, b->ddmoff.as<int64_t>(), b->Wt.p, ts, B, dt, np,
                   b->part.as<double>(), dtheta, st);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

}  // namespace

extern "C" {

tt_status tt_kernel_batch_build(const tt_kernel_params* p, const tt_kernel_pair* pairs, int num_pairs, const void* X,
                                int64_t n_x, const void* Y, int64_t n_y, void* stream, tt_kernel_batch_t* out) {
  if (!out) return fail(TTK_ERR_ARG, "out handle pointer is NULL");
  if (!p || !pairs || num_pairs <= 0) return fail(TTK_ERR_ARG, "params, pairs or num_pairs invalid");
  if (p->symmetric_psd) return fail(TTK_ERR_UNSUPPORTED, "batches of Global-1 pairs are not supported");
  if (n_x < 0 || n_y < 0 || (n_x > 0 && !X) || (n_y > 0 && !Y)) return fail(TTK_ERR_ARG, "bad point arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d = p->d;
  for (int i = 0; i < num_pairs; ++i) {
    const tt_kernel_pair& pr = pairs[i];
    if (pr.n_src < 0 || pr.n_tgt < 0 || pr.src_off < 0 || pr.tgt_off < 0 || pr.src_off + pr.n_src > n_x ||
        pr.tgt_off + pr.n_tgt > n_y)
      return fail(TTK_ERR_ARG, "pair %d: point range outside the arrays", i);
    for (int j = 0; j < d && j < 3; ++j)
      if (!(pr.box_s[2 * j] < pr.box_s[2 * j + 1]) || !(pr.box_t[2 * j] < pr.box_t[2 * j + 1]))
        return fail(TTK_ERR_ARG, "pair %d: empty box along axis %d", i, j);
  }
  std::unique_ptr<tt_kernel_batch> b(new (std::nothrow) tt_kernel_batch());
  if (!b) return fail(TTK_ERR_OOM, "batch allocation failed");
  b->P = *p;
  b->dtype = p->dtype;
  b->es = p->dtype == TTK_FP32 ? 4 : 8;
  b->d = d;
  b->dt = p->d_theta;
  b->D = 2 * d + p->d_theta;
  b->nx = n_x;
  b->ny = n_y;
  b->pairs.assign(pairs, pairs + num_pairs);
  // classes
  std::vector<Frame> frames(num_pairs);
  std::vector<std::vector<double>> keys;
  std::vector<int> rep;   // representative pair of each class
  b->cls.resize(num_pairs);
  for (int i = 0; i < num_pairs; ++i) {
    frames[i] = pair_frame(p->kind, d, pairs[i]);
    int c = -1;
    for (int q = 0; q < (int)keys.size(); ++q)
      if (keys[q] == frames[i].key) { c = q; break; }
    if (c < 0) {
      c = (int)keys.size();
      keys.push_back(frames[i].key);
      rep.push_back(i);
    }
    b->cls[i] = c;
  }
  // one cross + rounding per class, in the class's canonical boxes, no points
  for (int c = 0; c < (int)keys.size(); ++c) {
    tt_kernel_params cp = *p;
    const Frame& f = frames[rep[c]];
    for (int j = 0; j < 2 * d; ++j) {
      cp.box_s[j] = f.cbs[j];
      cp.box_t[j] = f.cbt[j];
    }
    tt_kernel_t h = nullptr;
    const tt_status s = tt_kernel_build_offline(&cp, nullptr, 0, nullptr, 0, stream, &h);
    if (s < 0) return s;
    if (s == TTK_WARN_NOT_CONVERGED) b->converged = false;
    b->classes.emplace_back(h);
    b->info.kernel_evals += h->info.kernel_evals;
    b->info.t_cross_ms += h->info.t_cross_ms;
    b->info.t_round_ms += h->info.t_round_ms;
  }
  // per-pair stages: the class cores read through the pair's own axes and orientation
  b->stages.resize((size_t)num_pairs * 2 * d);
  b->uoff.resize(num_pairs);
  b->voff.resize(num_pairs);
  int64_t uo = 0, vo = 0;
  for (int i = 0; i < num_pairs; ++i) {
    const tt_kernel* k = b->classes[b->cls[i]].get();
    const Frame& f = frames[i];
    const tt_kernel_pair& pr = pairs[i];
    for (int side = 0; side < 2; ++side)
      for (int si = 0; si < d; ++si) {
        ChainStage cs = side == 0 ? k->src[si] : k->tgt[si];
        const int canon = cs.coord;
        const int ax = f.perm[canon];
        const double* box = side == 0 ? pr.box_s : pr.box_t;
        double lo = box[2 * ax], hi = box[2 * ax + 1];
        if (f.sign[canon] < 0) std::swap(lo, hi);
        cs.coord = ax;
        cs.lo = lo;
        cs.hi = hi;
        b->stages[(size_t)i * 2 * d + side * d + si] = cs;
      }
    b->uoff[i] = uo;
    b->voff[i] = vo;
    uo += pr.n_src * k->rs;
    vo += pr.n_tgt * k->rt;
    b->info.factor_rows += pr.n_src + pr.n_tgt;
  }
  TTK_TRY(b->U.alloc((size_t)std::max<int64_t>(uo, 1) * b->es));
  TTK_TRY(b->V.alloc((size_t)std::max<int64_t>(vo, 1) * b->es));
  auto t0 = std::chrono::steady_clock::now();
  TTK_TRY(batch_phase3_tuned(b.get(), X, Y, st));
  TTK_HIP(hipStreamSynchronize(st));
  b->info.t_factor_ms = ms_since(t0);
  b->info.num_pairs = num_pairs;
  b->info.num_classes = (int)b->classes.size();
  b->info.factor_grid = b->factor_grid;
  const tt_status s = b->converged ? TTK_OK : TTK_WARN_NOT_CONVERGED;
  if (s != TTK_OK) set_error("the cross of at least one class stopped above tol");
  *out = b.release();
  return s;
}

tt_status tt_kernel_batch_configure(tt_kernel_batch_t b, int use_graph, int factor_grid, int reduce_rows) {
  if (!b) return fail(TTK_ERR_ARG, "NULL batch");
  if (reduce_rows < 0) return fail(TTK_ERR_ARG, "reduce_rows must be >= 0");
  b->cfg_graph = use_graph ? 1 : 0;
  b->cfg_factor_grid = factor_grid;
  b->cfg_reduce_rows = reduce_rows;
  b->prepB = -1;   // work lists are rebuilt on the next apply
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  b->key.clear();
  return TTK_OK;
}

tt_status tt_kernel_batch_factor(tt_kernel_batch_t b, const void* X, const void* Y, void* stream) {
  if (!b) return fail(TTK_ERR_ARG, "NULL batch");
  if ((b->nx > 0 && !X) || (b->ny > 0 && !Y)) return fail(TTK_ERR_ARG, "NULL point array");
  if (b->cfg_factor_grid != 0) b->factor_grid = b->cfg_factor_grid < 0 ? 0 : b->cfg_factor_grid;
  b->info.factor_grid = b->factor_grid;
  return batch_phase3(b, X, Y, b->factor_grid, static_cast<hipStream_t>(stream));
}

tt_status tt_kernel_batch_get_info(tt_kernel_batch_t b, tt_kernel_batch_info* info, int* class_of_pair,
                                   int* class_ranks) {
  if (!b) return fail(TTK_ERR_ARG, "NULL batch");
  b->info.graph = b->cfg_graph;
  if (info) *info = b->info;
  if (class_of_pair)
    for (size_t i = 0; i < b->cls.size(); ++i) class_of_pair[i] = b->cls[i];
  if (class_ranks)
    for (size_t c = 0; c < b->classes.size(); ++c)
      for (int k = 0; k < 9; ++k)
        class_ranks[c * 9 + k] = k <= b->D ? b->classes[c]->ranks[k] : 0;
  return TTK_OK;
}

tt_status tt_kernel_batch_get_class(tt_kernel_batch_t b, int c, tt_kernel_t* h) {
  if (!b || !h) return fail(TTK_ERR_ARG, "NULL argument");
  if (c < 0 || c >= (int)b->classes.size()) return fail(TTK_ERR_ARG, "class %d out of range", c);
  *h = b->classes[c].get();
  return TTK_OK;
}

tt_status tt_kernel_batch_get_factors(tt_kernel_batch_t b, int pair, void* U_out, void* V_out, void* stream) {
  if (!b) return fail(TTK_ERR_ARG, "NULL batch");
  if (pair < 0 || pair >= (int)b->pairs.size()) return fail(TTK_ERR_ARG, "pair %d out of range", pair);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const tt_kernel* k = b->classes[b->cls[pair]].get();
  const tt_kernel_pair& pr = b->pairs[pair];
  if (U_out && pr.n_src > 0)
    TTK_HIP(hipMemcpyAsync(U_out, b->U.as<char>() + b->uoff[pair] * b->es, (size_t)pr.n_src * k->rs * b->es,
                           hipMemcpyDeviceToDevice, st));
  if (V_out && pr.n_tgt > 0)
    TTK_HIP(hipMemcpyAsync(V_out, b->V.as<char>() + b->voff[pair] * b->es, (size_t)pr.n_tgt * k->rt * b->es,
                           hipMemcpyDeviceToDevice, st));
  return TTK_OK;
}

tt_status tt_kernel_batch_apply(tt_kernel_batch_t b, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                                int64_t ldy, const void* G, int64_t ldg, void* dX, int64_t lddx, void* dtheta,
                                void* stream) {
  if (!b) return fail(TTK_ERR_ARG, "NULL batch");
  if (B <= 0) return B == 0 ? TTK_OK : fail(TTK_ERR_ARG, "B < 0");
  if (!X || !Y) return fail(TTK_ERR_ARG, "X or Y is NULL");
  if (b->dt > 0 && !theta) return fail(TTK_ERR_ARG, "theta is NULL");
  if (ldx < b->ny || ldy < b->nx) return fail(TTK_ERR_ARG, "leading dimension too small");
  if (G && ldg < b->nx) return fail(TTK_ERR_ARG, "ldg too small");
  if (G && dX && lddx < b->ny) return fail(TTK_ERR_ARG, "lddx too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(batch_prepare(b, B, X, ldx, st));
  if (!b->cfg_graph)
    return batch_enqueue(b, theta, B, X, ldx, Y, ldy, G, ldg, dX, lddx, dtheta, st);
  const std::vector<const void*> key = {theta, X, Y, G, dX, dtheta, reinterpret_cast<const void*>((intptr_t)B),
                                        reinterpret_cast<const void*>((intptr_t)ldx),
                                        reinterpret_cast<const void*>((intptr_t)ldy),
                                        reinterpret_cast<const void*>((intptr_t)ldg),
                                        reinterpret_cast<const void*>((intptr_t)lddx)};
  if (!b->exec || b->key != key) {
    if (b->exec) {
      TTK_HIP(hipGraphExecDestroy(b->exec));
      b->exec = nullptr;
    }
    if (!b->cap) TTK_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    TTK_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    const tt_status s = batch_enqueue(b, theta, B, X, ldx, Y, ldy, G, ldg, dX, lddx, dtheta, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (s < 0) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(TTK_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      b->exec = nullptr;
      return fail(TTK_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    b->key = key;
  }
  TTK_HIP(hipGraphLaunch(b->exec, st));
  return TTK_OK;
}

tt_status tt_kernel_batch_destroy(tt_kernel_batch_t b) {
  delete b;
  return TTK_OK;
}

}  // extern "C"
