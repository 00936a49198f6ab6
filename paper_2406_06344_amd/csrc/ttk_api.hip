// C ABI of the PTTK library (tt_kernel.h): handle lifecycle, argument checks,
// and the orchestration of the offline stage (Algorithm 2), the online stage
// (Algorithm 3) and the apply / backward calls on the caller's stream.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>

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

tt_status DBuf::alloc(size_t nbytes) {
  if (nbytes <= bytes && p) return TTK_OK;
  // work queued earlier may still read the old buffer
  if (p) (void)hipDeviceSynchronize();
  release();
  if (nbytes == 0) nbytes = 16;
  if (hipMalloc(&p, nbytes) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return fail(TTK_ERR_OOM, "device allocation of %zu bytes failed", nbytes);
  }
  bytes = nbytes;
  return TTK_OK;
}

tt_status HBuf::alloc(size_t nbytes) {
  if (nbytes <= bytes && p) return TTK_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
  if (nbytes == 0) nbytes = 16;
  if (hipHostMalloc(&p, nbytes, hipHostMallocDefault) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return fail(TTK_ERR_OOM, "pinned host allocation of %zu bytes failed", nbytes);
  }
  bytes = nbytes;
  return TTK_OK;
}

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
  if (p->d_theta != dt) return fail(TTK_ERR_ARG, "kernel kind %d needs d_theta = %d (got %d)", p->kind, dt, p->d_theta);
  if (p->n_spatial < 2 || p->n_spatial > MAXN) return fail(TTK_ERR_ARG, "n_spatial = %d outside 2..%d", p->n_spatial, MAXN);
  if (dt > 0 && (p->n_param < 2 || p->n_param > MAXN))
    return fail(TTK_ERR_ARG, "n_param = %d outside 2..%d", p->n_param, MAXN);
  for (int j = 0; j < p->d; ++j) {
    if (!(p->box_s[2 * j] < p->box_s[2 * j + 1])) return fail(TTK_ERR_ARG, "source box dimension %d is empty", j);
    if (!(p->box_t[2 * j] < p->box_t[2 * j + 1])) return fail(TTK_ERR_ARG, "target box dimension %d is empty", j);
  }
  for (int j = 0; j < dt; ++j)
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

}  // namespace

}  // namespace ttk

using namespace ttk;

struct tt_kernel {
  tt_kernel_params P{};
  Grid g;
  int dtype = TTK_FP32;
  size_t es = 4;
  std::vector<int> ranks, cross_ranks;
  std::vector<std::vector<double>> cores;
  CrossOut cross;
  tt_kernel_info info{};
  int64_t ns = 0, nt = 0;
  int rs = 0, rt = 0, ldu = 0, ldv = 0;
  DBuf U, V, nodes, dct, stage[6], pcore[2], gtmp;
  DBuf work, Mbuf, dMbuf, Wbuf, Zbuf, Abuf;
  // Global-1 (Algorithm 4): Q (N x kg row-major, dtype), R (kg x kg FP64)
  int kg = 0;
  DBuf Q, Rg, Gwork, M64, Wg;
  ParamCore pc[2];
  ChainStage src[3], tgt[3];
  KSpec ks{};
};

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
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
  const double* Cp = Cs + (size_t)ns_ * ns_;
  size_t maxc = 1;
  for (int k = 0; k < D; ++k) maxc = std::max(maxc, h->cores[k].size());
  TTK_TRY(h->gtmp.alloc(maxc * sizeof(double)));
  ChainStage* src = h->src;
  ChainStage* tgt = h->tgt;
  for (int k = 0; k < D; ++k) {
    const int r0 = h->ranks[k], n = h->g.n[k], r1 = h->ranks[k + 1];
    const size_t cnt = (size_t)r0 * n * r1;
    TTK_HIP(hipMemcpyAsync(h->gtmp.p, h->cores[k].data(), cnt * sizeof(double), hipMemcpyHostToDevice, st));
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((cnt + 255) / 256, 4096));
    if (k < d || k >= d + dt) {
      const int mode = (k < d) ? 0 : 1;
      const int si = (k < d) ? k : (D - 1 - k);   // stage index
      DBuf& sb = h->stage[(k < d) ? si : 3 + si];
      TTK_TRY(sb.alloc(cnt * es));
      if (h->dtype == TTK_FP32)
        hipLaunchKernelGGL(k_dct_core<float>, dim3(nb), dim3(256), 0, st, h->gtmp.as<double>(), r0, n, r1, Cs, mode,
                           sb.as<float>());
      else
        hipLaunchKernelGGL(k_dct_core<double>, dim3(nb), dim3(256), 0, st, h->gtmp.as<double>(), r0, n, r1, Cs, mode,
                           sb.as<double>());
      ChainStage& cs = (k < d) ? src[si] : tgt[si];
      cs.G2 = sb.p;
      cs.n = n;
      if (k < d) { cs.r_in = r0; cs.r_out = r1; cs.coord = k; }
      else { cs.r_in = r1; cs.r_out = r0; cs.coord = k - d - dt; }
      cs.lo = h->g.lo[k];
      cs.hi = h->g.hi[k];
    } else {
      const int j = k - d;
      TTK_TRY(h->pcore[j].alloc(cnt * sizeof(double)));
      hipLaunchKernelGGL(k_dct_core<double>, dim3(nb), dim3(256), 0, st, h->gtmp.as<double>(), r0, n, r1, Cp, 2,
                         h->pcore[j].as<double>());
      h->pc[j] = ParamCore{h->pcore[j].as<double>(), r0, n, r1, h->g.lo[k], h->g.hi[k]};
    }
    // the staging buffer is overwritten by the next core
    TTK_HIP(hipStreamSynchronize(st));
  }
  h->rs = h->ranks[d];
  h->rt = h->ranks[d + dt];
  h->ldu = h->rs;
  h->ldv = h->rt;
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
  h->ks = KSpec{p->kind, p->d, p->d_theta, h->g.D, p->kernel_const, h->nodes.as<double>()};
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
  h->cores = h->cross.cores;
  h->ranks = h->cross.ranks;
  t0 = std::chrono::steady_clock::now();
  TTK_TRY(round_gauge(h->cores, h->ranks, h->g, h->P.tol, st));
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
  for (int k = 0; k < D; ++k) {
    if (ranks[k + 1] < 1 || ranks[k + 1] > MAXR) return fail(TTK_ERR_ARG, "rank %d out of range", ranks[k + 1]);
    const size_t cnt = (size_t)ranks[k] * h->g.n[k] * ranks[k + 1];
    h->cores[k].assign(cores + off, cores + off + cnt);
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
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int r = side == 0 ? h->rs : h->rt;
  return factor_contract(h->dtype, side == 0 ? h->src : h->tgt, h->g.d, P, n, out, r, st);
}

tt_status tt_kernel_online_core(tt_kernel_t h, const void* theta, int B, void* M_out, void* dM_out, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B < 0 || (B > 0 && !M_out)) return fail(TTK_ERR_ARG, "bad B or M_out");
  if (B == 0) return TTK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dt = h->g.dt;
  if (dt == 0) {
    hipLaunchKernelGGL(k_identity_batch, dim3(256), dim3(256), 0, st, M_out, h->rs, B, h->dtype == TTK_FP32);
    TTK_HIP(hipGetLastError());
    return TTK_OK;
  }
  if (!theta) return fail(TTK_ERR_ARG, "theta is NULL");
  TTK_TRY(h->work.alloc(online_work_doubles(h->pc, dt, B) * sizeof(double)));
  online_core(h->dtype, h->pc, dt, theta, B, M_out, dM_out, h->work.as<double>(), st);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

static tt_status prepare_M(tt_kernel_t h, const void* theta, int B, bool with_dM, hipStream_t st) {
  const size_t msz = (size_t)h->rs * h->rt * B * h->es;
  TTK_TRY(h->Mbuf.alloc(msz));
  if (with_dM) TTK_TRY(h->dMbuf.alloc(msz * std::max(h->g.dt, 1)));
  return tt_kernel_online_core(h, theta, B, h->Mbuf.p, with_dM ? h->dMbuf.p : nullptr, st);
}

tt_status tt_kernel_apply(tt_kernel_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          void* W_save, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B <= 0) return B == 0 ? TTK_OK : fail(TTK_ERR_ARG, "B < 0");
  if (!X || !Y) return fail(TTK_ERR_ARG, "X or Y is NULL");
  if (ldx < h->nt || ldy < h->ns) return fail(TTK_ERR_ARG, "leading dimension too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTK_TRY(prepare_M(h, theta, B, false, st));
  void* W = W_save;
  if (!W) {
    TTK_TRY(h->Wbuf.alloc((size_t)h->rt * B * h->es));
    W = h->Wbuf.p;
  }
  TTK_TRY(h->Zbuf.alloc((size_t)h->rs * B * h->es));
  apply_reduce(h->dtype, h->V.p, h->ldv, h->nt, h->rt, X, ldx, B, W, st);
  batched_matvec(h->dtype, h->Mbuf.p, h->rs, h->rt, 0, W, B, h->Zbuf.p, st);
  apply_expand(h->dtype, h->U.p, h->ldu, h->ns, h->rs, h->Zbuf.p, B, Y, ldy, st);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
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
    apply_reduce(h->dtype, h->V.p, h->ldv, h->nt, h->rt, xb, ldx, 1, wb, st);
    batched_matvec(h->dtype, Mb, h->rs, h->rt, 0, wb, 1, zb, st);
    apply_expand(h->dtype, h->U.p, h->ldu, h->ns, h->rs, zb, 1, yb, ldy, st);
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
  apply_reduce(h->dtype, h->U.p, h->ldu, h->ns, h->rs, G, ldg, B, h->Abuf.p, st);   // A = U^T G
  if (dX) {
    TTK_TRY(h->Zbuf.alloc((size_t)std::max(h->rs, h->rt) * B * h->es));
    batched_matvec(h->dtype, h->Mbuf.p, h->rs, h->rt, 1, h->Abuf.p, B, h->Zbuf.p, st);   // M^T a
    apply_expand(h->dtype, h->V.p, h->ldv, h->nt, h->rt, h->Zbuf.p, B, dX, lddx, st);
  }
  if (want_dth) {
    const void* W = W_saved;
    if (!W) {
      TTK_TRY(h->Wbuf.alloc((size_t)h->rt * B * h->es));
      apply_reduce(h->dtype, h->V.p, h->ldv, h->nt, h->rt, X, ldx, B, h->Wbuf.p, st);
      W = h->Wbuf.p;
    }
    batched_bilinear(h->dtype, h->Abuf.p, h->dMbuf.p, W, h->rs, h->rt, B, h->g.dt, dtheta, st);
  } else if (dtheta && h->g.dt == 0) {
    // no parameters: nothing to write
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
  apply_reduce(h->dtype, h->Q.p, k, h->ns, k, X, ldx, B, h->Wbuf.p, st);          // Q^T x
  batched_matvec(h->dtype, W, k, k, 0, h->Wbuf.p, B, h->Zbuf.p, st);             // W (Q^T x)
  apply_expand(h->dtype, h->Q.p, k, h->ns, k, h->Zbuf.p, B, Y, ldy, st);          // Q (...)
  TTK_HIP(hipGetLastError());
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
  KSpec ks{p->kind, p->d, p->d_theta, g.D, p->kernel_const, nodes.as<double>()};
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
  KSpec ks{p->kind, p->d, p->d_theta, g.D, p->kernel_const, nullptr};
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
