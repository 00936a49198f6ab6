// TT greedy-cross on the grid tensor of f_kappa (Appendices A and B):
// index initialisation (Algorithm 7), update cross steps (Algorithm 5) swept
// left to right (Algorithm 6), the sampled stopping test and the
// interpolation formula for the cores.
//
// Split of the work.  The host keeps the (small, integer) index sets and the
// counter-based random stream and decides where pivots go; every kernel
// entry, every residual, every argmax and every FP64 factorisation runs on
// the device.  One update step costs one host round trip (the pivot it
// chose); the stopping test one more per sweep.
//
// Readings shared with the oracle: residual R = A(:,J) A(I,J)^{-1} A(I,:) - A;
// max{rows, cols} samples by Floyd's algorithm from the splitmix64 stream
// keyed (seed, 2, sweep, k), then the bit; argmax ties (within 1e-12 x the
// largest |entry| evaluated so far in the step) go to the lowest position;
// a pivot is added only if |R| exceeds that band, is new, and the rank is
// below the cap.  Stopping: max |X - X^| / max |X| over n_test fixed
// multi-indices (stream (seed, 3)), with cores from C_k = F_k P_k^{-1} (LU);
// final cores from the QR form C_k = Q Q[J,:]^{-1}.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "ttk_internal.h"
#include "ttk_rng.h"

namespace ttk {

namespace {

constexpr double TIE_REL = 1e-12;

// Result of one update step, written on the device, read back once.
struct StepRes {
  int32_t s_pos, l, t, q_pos;
  int32_t pivot_row, pivot_col, added, info;
  double s_max, s_margin, s_scale, s_tau;
  double q_max, q_margin, q_scale, q_tau;
  double pivot_abs, pad;
};

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Largest |value| over up to four buffers, combined with *base (if non-NULL).
__global__ void k_absmax(const double* a, int na, const double* b, int nb, const double* c, int nc,
                         const double* d, int nd, const double* base, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < na; i += blockDim.x) m = fmax(m, fabs(a[i]));
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, fabs(b[i]));
  for (int i = threadIdx.x; i < nc; i += blockDim.x) m = fmax(m, fabs(c[i]));
  for (int i = threadIdx.x; i < nd; i += blockDim.x) m = fmax(m, fabs(d[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = base ? fmax(*base, red[0]) : red[0];
}

// R[i] = sum_q L(i,q) Rm(q,i) - A[i], with L(i,q) = L[i*sli + q*slq] and
// Rm(q,i) = Rm[q*srq + i*sri] (a zero stride broadcasts).
__global__ void k_resid(const double* L, int64_t sli, int64_t slq, const double* Rm, int64_t srq,
                        int64_t sri, const double* A, int n, int r, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < r; ++q) s += L[i * sli + q * slq] * Rm[q * srq + i * sri];
  out[i] = s - A[i];
}

// Robust argmax of |R| (lowest index within tau of the max) and the
// relative top-2 margin; stage 0 = sample stage (also records row/col of the
// chosen sample), stage 1 = search stage.
__global__ void k_select(const double* R, int n, const int32_t* srow, const int32_t* scol, int stage,
                         StepRes* res) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  const double scale = stage == 0 ? res->s_scale : res->q_scale;
  const double tau = TIE_REL * scale;
  double m = -1.0;
  for (int i = tid; i < n; i += blockDim.x) m = fmax(m, fabs(R[i]));
  sv[tid] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sv[tid] = fmax(sv[tid], sv[tid + s]);
    __syncthreads();
  }
  const double mx = sv[0];
  __syncthreads();
  int pos = 0x7fffffff;
  for (int i = tid; i < n; i += blockDim.x)
    if (fabs(R[i]) >= mx - tau) { pos = i; break; }
  si[tid] = pos;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) si[tid] = min(si[tid], si[tid + s]);
    __syncthreads();
  }
  const int p = si[0];
  __syncthreads();
  double sec = 0.0;
  for (int i = tid; i < n; i += blockDim.x)
    if (i != p) sec = fmax(sec, fabs(R[i]));
  sv[tid] = sec;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sv[tid] = fmax(sv[tid], sv[tid + s]);
    __syncthreads();
  }
  if (tid == 0) {
    const double margin = mx > 0.0 ? (mx - sv[0]) / mx : 0.0;
    if (stage == 0) {
      res->s_pos = p; res->s_max = mx; res->s_margin = margin; res->s_tau = tau;
      res->l = srow[p]; res->t = scol[p];
    } else {
      res->q_pos = p; res->q_max = mx; res->q_margin = margin; res->q_tau = tau;
      res->pivot_abs = fabs(R[p]);
    }
  }
}

__global__ void k_finalize(StepRes* res, int bit, const int32_t* I, const int32_t* J, int rk,
                           int max_rank, const int32_t* info) {
  if (threadIdx.x != 0) return;
  const int row = bit ? res->l : res->q_pos;
  const int col = bit ? res->q_pos : res->t;
  res->pivot_row = row;
  res->pivot_col = col;
  bool fresh = true;
  for (int q = 0; q < rk; ++q)
    if (I[q] == row || J[q] == col) fresh = false;
  res->added = (res->pivot_abs > res->q_tau && fresh && rk < max_rank) ? 1 : 0;
  res->info = *info;
}

// 2-norm condition numbers of the 2x2 probes of the index initialisation.
// F (2-row-set fibre, (rl*n) x rr col-major) holds phi(left_s, j, right_t).
// mode 0 (left-to-right): M = [[F(a,j1,c), F(a,j1,c')], [F(b,j2,c), F(b,j2,c')]]
// mode 1 (right-to-left): M = [[F(a,j1,c), F(a,j2,c')], [F(b,j1,c), F(b,j2,c')]]
__global__ void k_init_cond(const double* F, int rl, int rr, int n, int mode, int excl_diag,
                            double* cond) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int j1 = e / n, j2 = e % n;   // linear position j1 * n + j2
  const int m = rl * n;
  const int sa = 0, sb = rl > 1 ? 1 : 0;
  const int ca = 0, cb = rr > 1 ? 1 : 0;
  double a, b, c, d;
  if (mode == 0) {
    a = F[sa + j1 * rl + ca * m]; b = F[sa + j1 * rl + cb * m];
    c = F[sb + j2 * rl + ca * m]; d = F[sb + j2 * rl + cb * m];
  } else {
    a = F[sa + j1 * rl + ca * m]; b = F[sa + j2 * rl + cb * m];
    c = F[sb + j1 * rl + ca * m]; d = F[sb + j2 * rl + cb * m];
  }
  // singular values of [[a, b], [c, d]]: (p +- q)/2 with
  // p = |(a + d, c - b)|, q = |(a - d, b + c)|
  const double p = hypot(a + d, c - b), q = hypot(a - d, b + c);
  const double s1 = 0.5 * (p + q), s2 = 0.5 * fabs(p - q);
  double cv = (s2 > 0.0) ? s1 / s2 : INFINITY;
  if (!(cv == cv)) cv = INFINITY;
  if (excl_diag && j1 == j2) cv = INFINITY;
  cond[e] = cv;
}

// Lowest position within a relative band 1e-12 of the minimum (excluded
// entries are +inf; if all are +inf, the lowest allowed position).
__global__ void k_select_min(const double* v, int n, int excl_diag, int nn, int32_t* out_pos,
                             double* out_val) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  double m = INFINITY;
  for (int i = tid; i < n; i += blockDim.x) m = fmin(m, v[i]);
  sv[tid] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sv[tid] = fmin(sv[tid], sv[tid + s]);
    __syncthreads();
  }
  const double mn = sv[0];
  __syncthreads();
  int pos = 0x7fffffff;
  for (int i = tid; i < n; i += blockDim.x) {
    const bool allowed = !(excl_diag && (i / nn) == (i % nn));
    if (!allowed) continue;
    if (isinf(mn) ? true : (v[i] <= mn * (1.0 + 1e-12))) { pos = i; break; }
  }
  si[tid] = pos;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) si[tid] = min(si[tid], si[tid + s]);
    __syncthreads();
  }
  if (tid == 0) { *out_pos = si[0]; *out_val = v[si[0]]; }
}

// P[a + b*r] = F[rows[a] + b*ldf]  (rows of F at the given positions)
__global__ void k_gather_rows(const double* F, int ldf, const int32_t* rows, int r, int c, double* P) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * c) return;
  const int a = e % r, b = e / r;
  P[a + b * r] = F[rows[a] + (int64_t)b * ldf];
}

// B (n x m) = A^T for A (m x n)
__global__ void k_transpose(const double* A, int m, int n, int lda, double* B, int ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  B[j + (int64_t)i * ldb] = A[i + (int64_t)j * lda];
}

// TT value at test multi-indices: cores given as CT_k (r_k x r_{k-1} n_k,
// column-major), entry C_k[s, i, t] = CT_k[t + (s + i r_{k-1}) r_k].
// One wave per point, the running vector in LDS.
struct TTView {
  const double* CT[MAXD];
  int r[MAXD + 1];
  int D;
};
__global__ void __launch_bounds__(256) k_tt_points(TTView tv, const int16_t* idx, int P, double* out) {
  __shared__ double buf[4][2][MAXR];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 4 + w;
  if (p >= P) return;
  double* v = buf[w][0];
  double* vn = buf[w][1];
  if (lane == 0) v[0] = 1.0;
  __builtin_amdgcn_wave_barrier();
  for (int k = 0; k < tv.D; ++k) {
    const int r0 = tv.r[k], r1 = tv.r[k + 1];
    const int i = idx[(int64_t)p * tv.D + k];
    const double* blk = tv.CT[k] + (int64_t)i * r0 * r1;   // r1 x r0 block
    for (int t = lane; t < r1; t += 64) {
      double s = 0.0;
      for (int q = 0; q < r0; ++q) s += blk[t + (int64_t)q * r1] * v[q];
      vn[t] = s;
    }
    __builtin_amdgcn_wave_barrier();
    double* tmp = v; v = vn; vn = tmp;
  }
  if (lane == 0) out[p] = v[0];
}

__global__ void k_err_max(const double* a, const double* b, int n, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(a[i] - b[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

inline int nblk(int64_t n, int bs) { return (int)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Key of a multi-index (node indices < 32, at most 8 dims: 5 bits each).
inline uint64_t mkey(const int32_t* e, int len) {
  uint64_t k = (uint64_t)len;
  for (int i = 0; i < len; ++i) k = (k << 5) | (uint64_t)e[i];
  return k;
}

class Cross {
 public:
  Cross(const tt_kernel_params* p, const Grid& g, const KSpec& ks, hipStream_t st)
      : P_(*p), g_(g), ks_(ks), st_(st), N_(g.D) {}

  tt_status run(CrossOut* out);

 private:
  // index sets: L_[k] = I^{<=k} (r_k rows of k ints), R_[k] = I^{>k} (rows of N-k ints)
  std::vector<std::vector<int32_t>> L_, R_;
  int rank(int k) const {
    if (k == 0 || k == N_) return 1;
    return (int)(L_[k].size() / (size_t)k);
  }

  tt_status upload_sets(int k_left, int k_right, int16_t* dl, int16_t* dr);
  tt_status init_sets();
  tt_status update_step(int k, int sweep, tt_kernel_decision* rec);
  tt_status build_cores(bool qr, std::vector<double*>* CT);
  tt_status sampled_error(double* err);
  Addr fibre_addr(int k) const;   // F_k, k = 1..N
  Addr super_addr(int k) const;   // super-core k, k = 1..N-1
  tt_status ensure(DBuf& b, size_t bytes) { return b.alloc(bytes); }
  tt_status sync() { TTK_HIP(hipStreamSynchronize(st_)); return TTK_OK; }

  tt_kernel_params P_;
  const Grid& g_;
  KSpec ks_;
  hipStream_t st_;
  int N_;
  int64_t evals_ = 0;
  double min_margin_ = 1.0;

  // device buffers
  DBuf d_left_, d_right_, d_idx_, d_vals_, d_lu_, d_piv_, d_info_, d_res_, d_scratch_, d_R_;
  DBuf d_test_idx_, d_test_val_, d_test_hat_, d_core_[MAXD], d_fib_, d_tmp_, d_P_, d_err_;
  HBuf h_stage_, h_res_;
  int n_test_ = 0;
  double test_max_ = 0.0;
  double init_max_cond_ = 0.0;
};

Addr Cross::fibre_addr(int k) const {
  Addr a{};
  a.left = d_left_.as<int16_t>();
  a.right = d_right_.as<int16_t>();
  a.rl = rank(k - 1);
  a.lk = k - 1;
  a.rr = rank(k);
  a.lr = N_ - k;
  a.nmid = 1;
  a.nm0 = g_.n[k - 1];
  a.nm1 = 1;
  return a;
}

Addr Cross::super_addr(int k) const {
  Addr a{};
  a.left = d_left_.as<int16_t>();
  a.right = d_right_.as<int16_t>();
  a.rl = rank(k - 1);
  a.lk = k - 1;
  a.rr = rank(k + 1);
  a.lr = N_ - k - 1;
  a.nmid = 2;
  a.nm0 = g_.n[k - 1];
  a.nm1 = g_.n[k];
  return a;
}

// Upload I^{<=k_left} and I^{>k_right} as int16 row-major arrays.
tt_status Cross::upload_sets(int k_left, int k_right, int16_t* dl, int16_t* dr) {
  const size_t nl = (k_left == 0) ? 0 : L_[k_left].size();
  const size_t nr = (k_right == N_) ? 0 : R_[k_right].size();
  TTK_TRY(h_stage_.alloc((nl + nr + 2) * sizeof(int16_t)));
  int16_t* h = h_stage_.as<int16_t>();
  for (size_t i = 0; i < nl; ++i) h[i] = (int16_t)L_[k_left][i];
  for (size_t i = 0; i < nr; ++i) h[nl + i] = (int16_t)R_[k_right][i];
  if (nl) TTK_HIP(hipMemcpyAsync(dl, h, nl * sizeof(int16_t), hipMemcpyHostToDevice, st_));
  if (nr) TTK_HIP(hipMemcpyAsync(dr, h + nl, nr * sizeof(int16_t), hipMemcpyHostToDevice, st_));
  // the staging buffer is reused by the next call: wait for the copies
  return sync();
}

tt_status Cross::init_sets() {
  const int N = N_;
  SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_INIT);
  L_.assign(N + 1, {});
  R_.assign(N + 1, {});
  if (P_.init_card == 1) {
    std::vector<int32_t> q(N);
    for (int j = 0; j < N; ++j) q[j] = (int32_t)g.below((uint64_t)g_.n[j]);
    for (int k = 1; k < N; ++k) {
      L_[k].assign(q.begin(), q.begin() + k);
      R_[k].assign(q.begin() + k, q.end());
    }
    return TTK_OK;
  }
  std::vector<int32_t> q1(N), q2(N);
  for (int j = 0; j < N; ++j) q1[j] = (int32_t)g.below((uint64_t)g_.n[j]);
  for (int j = 0; j < N; ++j) q2[j] = (int32_t)g.below((uint64_t)g_.n[j]);
  for (int k = 1; k < N; ++k) {
    R_[k].assign(q1.begin() + k, q1.end());
    R_[k].insert(R_[k].end(), q2.begin() + k, q2.end());
  }
  struct Snap { std::vector<std::vector<int32_t>> L, R; double maxc; };
  std::vector<Snap> snaps;
  TTK_TRY(d_left_.alloc(2 * MAXD * sizeof(int16_t)));
  TTK_TRY(d_right_.alloc(2 * MAXD * sizeof(int16_t)));
  TTK_TRY(d_fib_.alloc(2 * MAXN * 2 * sizeof(double)));
  TTK_TRY(d_tmp_.alloc(MAXN * MAXN * sizeof(double) + 64));
  TTK_TRY(d_res_.alloc(sizeof(StepRes)));
  TTK_TRY(h_res_.alloc(sizeof(StepRes)));
  double* cond = d_tmp_.as<double>();
  int32_t* dpos = reinterpret_cast<int32_t*>(d_res_.as<char>());
  double* dval = reinterpret_cast<double*>(d_res_.as<char>() + 8);
  auto probe = [&](int k, int mode, int kl, int kr, int* j1, int* j2, double* cv) -> tt_status {
    // two-row sets I^{<=kl} (kl = k-1) and I^{>kr} (kr = k): fibre of dimension k-1
    TTK_TRY(upload_sets(kl, kr, d_left_.as<int16_t>(), d_right_.as<int16_t>()));
    Addr a{};
    a.left = d_left_.as<int16_t>();
    a.right = d_right_.as<int16_t>();
    a.rl = (kl == 0) ? 1 : 2;
    a.lk = kl;
    a.rr = (kr == N) ? 1 : 2;
    a.lr = N - kr;
    a.nmid = 1;
    a.nm0 = g_.n[k - 1];
    a.nm1 = 1;
    const int n = g_.n[k - 1];
    eval_product(ks_, a, nullptr, a.rl * n, nullptr, a.rr, d_fib_.as<double>(), st_);
    evals_ += (int64_t)a.rl * n * a.rr;
    const int excl = (mode == 0) ? (k == 1) : (k == N);
    hipLaunchKernelGGL(k_init_cond, dim3(nblk(n * n, 256)), dim3(256), 0, st_, d_fib_.as<double>(), a.rl,
                       a.rr, n, mode, excl, cond);
    hipLaunchKernelGGL(k_select_min, dim3(1), dim3(1024), 0, st_, cond, n * n, excl, n, dpos, dval);
    TTK_HIP(hipMemcpyAsync(h_res_.p, d_res_.p, 16, hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
    const int pos = *h_res_.as<int32_t>();
    *cv = *reinterpret_cast<double*>(h_res_.as<char>() + 8);
    *j1 = pos / n;
    *j2 = pos % n;
    return TTK_OK;
  };
  const int max_it = P_.init_max_it > 0 ? P_.init_max_it : 10;
  for (int it = 0; it < max_it; ++it) {
    double mc = 0.0;
    for (int k = 1; k < N; ++k) {            // left to right
      int j1, j2;
      double cv;
      TTK_TRY(probe(k, 0, k - 1, k, &j1, &j2, &cv));
      mc = std::max(mc, cv);
      std::vector<int32_t> nl;
      const std::vector<int32_t> emp;
      const std::vector<int32_t>& prev = (k > 1) ? L_[k - 1] : emp;
      const int len = k - 1;
      nl.insert(nl.end(), prev.begin(), prev.begin() + len);
      nl.push_back(j1);
      nl.insert(nl.end(), prev.begin() + (k > 1 ? len : 0), prev.begin() + (k > 1 ? 2 * len : 0));
      nl.push_back(j2);
      L_[k] = nl;
    }
    snaps.push_back({L_, R_, mc});
    mc = 0.0;
    for (int k = N; k >= 2; --k) {           // right to left
      int j1, j2;
      double cv;
      TTK_TRY(probe(k, 1, k - 1, k, &j1, &j2, &cv));
      mc = std::max(mc, cv);
      const int len = N - k;
      std::vector<int32_t> nr;
      nr.push_back(j1);
      if (k < N) nr.insert(nr.end(), R_[k].begin(), R_[k].begin() + len);
      nr.push_back(j2);
      if (k < N) nr.insert(nr.end(), R_[k].begin() + len, R_[k].begin() + 2 * len);
      R_[k - 1] = nr;
    }
    snaps.push_back({L_, R_, mc});
  }
  // smallest maximum condition number, earliest within a relative band
  double best = INFINITY;
  for (auto& s : snaps) best = std::min(best, s.maxc);
  size_t pick = 0;
  for (size_t i = 0; i < snaps.size(); ++i) {
    if (std::isinf(best) ? std::isinf(snaps[i].maxc) : (snaps[i].maxc <= best * (1.0 + 1e-12))) {
      pick = i;
      break;
    }
  }
  L_ = snaps[pick].L;
  R_ = snaps[pick].R;
  init_max_cond_ = snaps[pick].maxc;
  return TTK_OK;
}


tt_status Cross::update_step(int k, int sweep, tt_kernel_decision* rec) {
  const int N = N_;
  const int rl = rank(k - 1), rr = rank(k + 1), rk = rank(k);
  const int nk = g_.n[k - 1], nk1 = g_.n[k];
  const int rows = rl * nk, cols = nk1 * rr;
  // pivot positions of I^{<=k} (rows) and I^{>k} (columns) in the unfolding
  std::unordered_map<uint64_t, int> lpos, rpos;
  for (int s = 0; s < rl; ++s) lpos[mkey(k > 1 ? &L_[k - 1][(size_t)s * (k - 1)] : nullptr, k - 1)] = s;
  for (int t = 0; t < rr; ++t)
    rpos[mkey(k + 1 < N ? &R_[k + 1][(size_t)t * (N - k - 1)] : nullptr, N - k - 1)] = t;
  std::vector<int32_t> I(rk), J(rk);
  for (int q = 0; q < rk; ++q) {
    const int32_t* e = &L_[k][(size_t)q * k];
    I[q] = lpos.at(mkey(e, k - 1)) + e[k - 1] * rl;
    const int32_t* f = &R_[k][(size_t)q * (N - k)];
    J[q] = f[0] + rpos.at(mkey(f + 1, N - k - 1)) * nk1;
  }
  SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_UPDATE, (uint64_t)sweep, (uint64_t)k);
  const int ns = std::max(rows, cols);
  std::vector<int64_t> lin = g.floyd((int64_t)rows * cols, ns);
  const int bit = g.bit();
  // upload the neighbouring sets and the integer lists
  TTK_TRY(d_left_.alloc(std::max<size_t>(2, L_[k - 1].size()) * sizeof(int16_t)));
  TTK_TRY(d_right_.alloc(std::max<size_t>(2, (k + 1 < N ? R_[k + 1].size() : 0)) * sizeof(int16_t)));
  TTK_TRY(upload_sets(k - 1, k + 1, d_left_.as<int16_t>(), d_right_.as<int16_t>()));
  const size_t nint = (size_t)2 * rk + 2 * (size_t)ns;
  TTK_TRY(d_idx_.alloc(nint * sizeof(int32_t)));
  TTK_TRY(h_stage_.alloc(nint * sizeof(int32_t)));
  int32_t* hi = h_stage_.as<int32_t>();
  std::copy(I.begin(), I.end(), hi);
  std::copy(J.begin(), J.end(), hi + rk);
  for (int i = 0; i < ns; ++i) {
    hi[2 * rk + i] = (int32_t)(lin[i] / cols);
    hi[2 * rk + ns + i] = (int32_t)(lin[i] % cols);
  }
  TTK_HIP(hipMemcpyAsync(d_idx_.p, hi, nint * sizeof(int32_t), hipMemcpyHostToDevice, st_));
  const int32_t* dI = d_idx_.as<int32_t>();
  const int32_t* dJ = dI + rk;
  const int32_t* dsr = dJ + rk;
  const int32_t* dsc = dsr + ns;
  // value buffers
  const size_t nsearch = std::max((size_t)rk + (size_t)rk * cols + cols, (size_t)rows * rk + rk + rows);
  const size_t nvals = (size_t)rk * rk + 2 * (size_t)ns * rk + ns + nsearch;
  TTK_TRY(d_vals_.alloc(nvals * sizeof(double)));
  TTK_TRY(d_R_.alloc((size_t)std::max(ns, std::max(rows, cols)) * sizeof(double)));
  TTK_TRY(d_piv_.alloc(MAXR * sizeof(int32_t)));
  TTK_TRY(d_info_.alloc(sizeof(int32_t)));
  TTK_TRY(d_res_.alloc(sizeof(StepRes)));
  TTK_TRY(h_res_.alloc(sizeof(StepRes)));
  double* AIJ = d_vals_.as<double>();
  double* AsJ = AIJ + (size_t)rk * rk;
  double* AIs = AsJ + (size_t)ns * rk;
  double* As = AIs + (size_t)rk * ns;
  double* S0 = As + ns;
  StepRes* dres = d_res_.as<StepRes>();
  const int32_t* d_l = &dres->l;
  const int32_t* d_t = &dres->t;
  const Addr a = super_addr(k);
  eval_product(ks_, a, dI, rk, dJ, rk, AIJ, st_);
  eval_product(ks_, a, dsr, ns, dJ, rk, AsJ, st_);
  eval_product(ks_, a, dI, rk, dsc, ns, AIs, st_);
  eval_list(ks_, a, dsr, dsc, ns, As, st_);
  evals_ += (int64_t)rk * rk + 2 * (int64_t)ns * rk + ns;
  hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st_, AIJ, rk * rk, AsJ, ns * rk, AIs, rk * ns, As, ns,
                     (const double*)nullptr, &dres->s_scale);
  lu_factor(AIJ, rk, rk, d_piv_.as<int32_t>(), d_info_.as<int32_t>(), st_);
  lu_solve(AIJ, rk, rk, d_piv_.as<int32_t>(), 0, AIs, rk, ns, st_);
  hipLaunchKernelGGL(k_resid, dim3(nblk(ns, 256)), dim3(256), 0, st_, AsJ, (int64_t)1, (int64_t)ns, AIs,
                     (int64_t)1, (int64_t)rk, As, ns, rk, d_R_.as<double>());
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st_, d_R_.as<double>(), ns, dsr, dsc, 0, dres);
  if (bit == 1) {   // search the row of the sample's pivot
    double* AlJ = S0;
    double* AIall = AlJ + rk;
    double* Alall = AIall + (size_t)rk * cols;
    eval_product(ks_, a, d_l, 1, dJ, rk, AlJ, st_);
    eval_product(ks_, a, dI, rk, nullptr, cols, AIall, st_);
    eval_product(ks_, a, d_l, 1, nullptr, cols, Alall, st_);
    evals_ += (int64_t)rk + (int64_t)rk * cols + cols;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st_, AlJ, rk, AIall, rk * cols, Alall, cols,
                       (const double*)nullptr, 0, &dres->s_scale, &dres->q_scale);
    lu_solve(AIJ, rk, rk, d_piv_.as<int32_t>(), 0, AIall, rk, cols, st_);
    hipLaunchKernelGGL(k_resid, dim3(nblk(cols, 256)), dim3(256), 0, st_, AlJ, (int64_t)0, (int64_t)1, AIall,
                       (int64_t)1, (int64_t)rk, Alall, cols, rk, d_R_.as<double>());
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st_, d_R_.as<double>(), cols, dsr, dsc, 1, dres);
  } else {          // search the column
    double* AallJ = S0;
    double* AIt = AallJ + (size_t)rows * rk;
    double* Aallt = AIt + rk;
    eval_product(ks_, a, nullptr, rows, dJ, rk, AallJ, st_);
    eval_product(ks_, a, dI, rk, d_t, 1, AIt, st_);
    eval_product(ks_, a, nullptr, rows, d_t, 1, Aallt, st_);
    evals_ += (int64_t)rows * rk + rk + rows;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st_, AallJ, rows * rk, AIt, rk, Aallt, rows,
                       (const double*)nullptr, 0, &dres->s_scale, &dres->q_scale);
    lu_solve(AIJ, rk, rk, d_piv_.as<int32_t>(), 0, AIt, rk, 1, st_);
    hipLaunchKernelGGL(k_resid, dim3(nblk(rows, 256)), dim3(256), 0, st_, AallJ, (int64_t)1, (int64_t)rows,
                       AIt, (int64_t)1, (int64_t)0, Aallt, rows, rk, d_R_.as<double>());
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st_, d_R_.as<double>(), rows, dsr, dsc, 1, dres);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st_, dres, bit, dI, dJ, rk,
                     std::min(P_.max_rank > 0 ? P_.max_rank : MAXR, MAXR), d_info_.as<int32_t>());
  TTK_HIP(hipGetLastError());
  TTK_HIP(hipMemcpyAsync(h_res_.p, d_res_.p, sizeof(StepRes), hipMemcpyDeviceToHost, st_));
  TTK_TRY(sync());
  const StepRes r = *h_res_.as<StepRes>();
  if (r.info != 0)
    return fail(TTK_ERR_SINGULAR_CROSS, "cross: intersection matrix of super-core %d singular (sweep %d)", k,
                sweep);
  rec->sweep = sweep;
  rec->k = k;
  rec->rank_before = rk;
  rec->sample_pos = lin[r.s_pos];
  rec->bit = bit;
  rec->pivot_row = r.pivot_row;
  rec->pivot_col = r.pivot_col;
  rec->added = r.added;
  rec->sample_max = r.s_max;
  rec->sample_margin = r.s_margin;
  rec->pivot_abs = r.pivot_abs;
  rec->search_margin = r.q_margin;
  rec->tau = r.q_tau;
  if (r.s_max > 0) min_margin_ = std::min(min_margin_, r.s_margin);
  if (r.q_max > 0) min_margin_ = std::min(min_margin_, r.q_margin);
  if (r.added) {
    const int l = r.pivot_row, t = r.pivot_col;
    const int s = l % rl, ik = l / rl;
    if (k > 1) L_[k].insert(L_[k].end(), L_[k - 1].begin() + (size_t)s * (k - 1),
                            L_[k - 1].begin() + (size_t)(s + 1) * (k - 1));
    L_[k].push_back(ik);
    const int i1 = t % nk1, tt = t / nk1;
    R_[k].push_back(i1);
    if (k + 1 < N)
      R_[k].insert(R_[k].end(), R_[k + 1].begin() + (size_t)tt * (N - k - 1),
                   R_[k + 1].begin() + (size_t)(tt + 1) * (N - k - 1));
  }
  return TTK_OK;
}

// Cores of the cross interpolant, stored transposed: CT_k = C_k^T (r_k x r_{k-1} n_k).
// qr = false: C_k = F_k P_k^{-1} (LU).  qr = true: C_k = Q Q[J,:]^{-1} with F_k = Q R.
tt_status Cross::build_cores(bool qr, std::vector<double*>* CT) {
  const int N = N_;
  CT->assign(N, nullptr);
  for (int k = 1; k <= N; ++k) {
    const int r0 = rank(k - 1), r1 = rank(k), n = g_.n[k - 1];
    const int m = r0 * n;
    TTK_TRY(d_left_.alloc(std::max<size_t>(2, L_[k - 1].size()) * sizeof(int16_t)));
    TTK_TRY(d_right_.alloc(std::max<size_t>(2, (k < N ? R_[k].size() : 0)) * sizeof(int16_t)));
    TTK_TRY(upload_sets(k - 1, k, d_left_.as<int16_t>(), d_right_.as<int16_t>()));
    TTK_TRY(d_fib_.alloc((size_t)m * r1 * sizeof(double)));
    TTK_TRY(d_core_[k - 1].alloc((size_t)m * r1 * sizeof(double)));
    double* F = d_fib_.as<double>();
    double* C = d_core_[k - 1].as<double>();
    eval_product(ks_, fibre_addr(k), nullptr, m, nullptr, r1, F, st_);
    evals_ += (int64_t)m * r1;
    if (k == N) {
      hipLaunchKernelGGL(k_transpose, dim3(nblk((int64_t)m * r1, 256)), dim3(256), 0, st_, F, m, r1, m, C, r1);
      (*CT)[k - 1] = C;
      continue;
    }
    // row positions of I^{<=k} among the rows (s + i r0) of F_k
    std::unordered_map<uint64_t, int> lpos;
    for (int s = 0; s < r0; ++s) lpos[mkey(k > 1 ? &L_[k - 1][(size_t)s * (k - 1)] : nullptr, k - 1)] = s;
    std::vector<int32_t> Jp(r1);
    for (int q = 0; q < r1; ++q) {
      const int32_t* e = &L_[k][(size_t)q * k];
      Jp[q] = lpos.at(mkey(e, k - 1)) + e[k - 1] * r0;
    }
    TTK_TRY(d_idx_.alloc((size_t)r1 * sizeof(int32_t)));
    TTK_TRY(h_stage_.alloc((size_t)r1 * sizeof(int32_t)));
    std::copy(Jp.begin(), Jp.end(), h_stage_.as<int32_t>());
    TTK_HIP(hipMemcpyAsync(d_idx_.p, h_stage_.p, (size_t)r1 * sizeof(int32_t), hipMemcpyHostToDevice, st_));
    TTK_TRY(d_P_.alloc(((size_t)r1 * r1 + (size_t)r1 * r1 + 64) * sizeof(double)));
    double* Pm = d_P_.as<double>();
    double* Rq = Pm + (size_t)r1 * r1;
    if (qr) {
      TTK_TRY(d_tmp_.alloc((size_t)(r1 + 64) * sizeof(double)));
      qr_thin(F, m, r1, m, Rq, r1, d_tmp_.as<double>(), st_);
    }
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk(r1 * r1, 256)), dim3(256), 0, st_, F, m, d_idx_.as<int32_t>(),
                       r1, r1, Pm);
    TTK_TRY(d_piv_.alloc(MAXR * sizeof(int32_t)));
    TTK_TRY(d_info_.alloc(sizeof(int32_t)));
    lu_factor(Pm, r1, r1, d_piv_.as<int32_t>(), d_info_.as<int32_t>(), st_);
    hipLaunchKernelGGL(k_transpose, dim3(nblk((int64_t)m * r1, 256)), dim3(256), 0, st_, F, m, r1, m, C, r1);
    lu_solve(Pm, r1, r1, d_piv_.as<int32_t>(), 1, C, r1, m, st_);
    int32_t info = 0;
    TTK_HIP(hipMemcpyAsync(&info, d_info_.p, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
    if (info != 0) return fail(TTK_ERR_SINGULAR_CROSS, "cross: P_%d singular in the interpolation formula", k);
    (*CT)[k - 1] = C;
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status Cross::sampled_error(double* err) {
  std::vector<double*> CT;
  TTK_TRY(build_cores(false, &CT));
  TTView tv{};
  tv.D = N_;
  for (int k = 0; k < N_; ++k) tv.CT[k] = CT[k];
  for (int k = 0; k <= N_; ++k) tv.r[k] = rank(k);
  hipLaunchKernelGGL(k_tt_points, dim3(nblk(n_test_, 4)), dim3(256), 0, st_, tv, d_test_idx_.as<int16_t>(),
                     n_test_, d_test_hat_.as<double>());
  hipLaunchKernelGGL(k_err_max, dim3(1), dim3(1024), 0, st_, d_test_val_.as<double>(),
                     d_test_hat_.as<double>(), n_test_, d_err_.as<double>());
  double e = 0.0;
  TTK_HIP(hipMemcpyAsync(&e, d_err_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
  TTK_TRY(sync());
  *err = test_max_ > 0 ? e / test_max_ : e;
  return TTK_OK;
}

tt_status Cross::run(CrossOut* out) {
  const int N = N_;
  TTK_TRY(init_sets());
  // fixed test multi-indices of the stopping rule
  int nmax = 0;
  for (int j = 0; j < N; ++j) nmax = std::max(nmax, g_.n[j]);
  n_test_ = P_.n_test > 0 ? P_.n_test : std::max(1000, 20 * N * nmax);
  {
    SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_TEST);
    std::vector<int16_t> idx((size_t)n_test_ * N);
    for (int p = 0; p < n_test_; ++p)
      for (int j = 0; j < N; ++j) idx[(size_t)p * N + j] = (int16_t)g.below((uint64_t)g_.n[j]);
    TTK_TRY(d_test_idx_.alloc(idx.size() * sizeof(int16_t)));
    TTK_TRY(d_test_val_.alloc((size_t)n_test_ * sizeof(double)));
    TTK_TRY(d_test_hat_.alloc((size_t)n_test_ * sizeof(double)));
    TTK_TRY(d_err_.alloc(2 * sizeof(double)));
    TTK_HIP(hipMemcpyAsync(d_test_idx_.p, idx.data(), idx.size() * sizeof(int16_t), hipMemcpyHostToDevice, st_));
    eval_multi16(ks_, d_test_idx_.as<int16_t>(), n_test_, d_test_val_.as<double>(), st_);
    evals_ += n_test_;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st_, d_test_val_.as<double>(), n_test_,
                       (const double*)nullptr, 0, (const double*)nullptr, 0, (const double*)nullptr, 0,
                       (const double*)nullptr, d_err_.as<double>());
    TTK_HIP(hipMemcpyAsync(&test_max_, d_err_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
  }
  double err = 0.0;
  TTK_TRY(sampled_error(&err));
  int sweep = 0;
  const int max_sweeps = P_.max_sweeps > 0 ? P_.max_sweeps : 200;
  while (err > P_.tol && sweep < max_sweeps) {
    int added = 0;
    for (int k = 1; k < N; ++k) {
      tt_kernel_decision rec{};
      TTK_TRY(update_step(k, sweep, &rec));
      out->log.push_back(rec);
      added += rec.added;
    }
    ++sweep;
    TTK_TRY(sampled_error(&err));
    if (added == 0) break;
  }
  std::vector<double*> CT;
  TTK_TRY(build_cores(true, &CT));
  out->ranks.assign(N + 1, 1);
  for (int k = 0; k <= N; ++k) out->ranks[k] = rank(k);
  out->cores.assign(N, {});
  for (int k = 1; k <= N; ++k) {
    const int r0 = rank(k - 1), r1 = rank(k), n = g_.n[k - 1];
    const size_t cnt = (size_t)r0 * n * r1;
    std::vector<double> ct(cnt);
    TTK_HIP(hipMemcpyAsync(ct.data(), CT[k - 1], cnt * sizeof(double), hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
    // G_k[a + i r0 + b r0 n] = C_k[(a + i r0), b] = CT[b + (a + i r0) r1]
    std::vector<double>& G = out->cores[k - 1];
    G.resize(cnt);
    for (int row = 0; row < r0 * n; ++row)
      for (int b = 0; b < r1; ++b) G[row + (size_t)b * r0 * n] = ct[b + (size_t)row * r1];
  }
  out->left.assign(N + 1, {});
  out->right.assign(N + 1, {});
  for (int k = 1; k < N; ++k) { out->left[k] = L_[k]; out->right[k] = R_[k]; }
  out->sweeps = sweep;
  out->error = err;
  out->converged = err <= P_.tol;
  out->init_max_cond = init_max_cond_;
  out->min_margin = min_margin_;
  out->evals = evals_;
  return TTK_OK;
}

}  // namespace

tt_status run_cross(const tt_kernel_params* p, const Grid& g, const KSpec& ks, hipStream_t st, CrossOut* out) {
  if (g.D < 2) return fail(TTK_ERR_ARG, "cross needs at least two dimensions");
  Cross c(p, g, ks, st);
  return c.run(out);
}

}  // namespace ttk
