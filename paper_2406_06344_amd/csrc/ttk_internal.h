// Internal declarations shared by the host-side translation units of the
// PTTK library.  Device code of one unit is launched only through the host
// wrappers declared here, so no relocatable device code is needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tt_kernel.h"

namespace ttk {

constexpr int MAXD = 8;    // 2 d + d_theta with d <= 3, d_theta <= 2
constexpr int MAXN = 32;   // Chebyshev nodes per dimension
constexpr int MAXR = 256;  // TT rank cap

// Kernel-function description passed by value to device code.
struct KSpec {
  int kind;
  int d, dt, D;
  double kconst;
  const double* nodes;  // device, D x MAXN: node eta_i of dimension j at j*MAXN + i
  double thfix[2];      // the kind's parameters when dt = 0 (non-parametric TTK)
};

// Thread-local error message behind tt_kernel_last_error().
void set_error(const char* fmt, ...);
tt_status fail(tt_status s, const char* fmt, ...);

#define TTK_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::ttk::fail(TTK_ERR_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                         __FILE__, __LINE__);                                          \
  } while (0)

#define TTK_TRY(expr)            \
  do {                           \
    tt_status s_ = (expr);       \
    if (s_ < 0) return s_;       \
  } while (0)

// Owning device buffer (DBuf) and pinned host staging buffer (HBuf,
// allocated, never registered).  Released memory goes back to a per-thread
// pool instead of being freed, and the next allocation on the same thread and
// device takes it from there.  A released block waits in the pool until the
// next take, which first synchronises the device once for all blocks
// released since the last one, so a block handed out is never still read or
// written by queued work, whatever stream that work is on.  The pool keeps
// at most 1 GiB per thread, device and kind; beyond that the largest blocks
// are freed.
// a block of at least *bytes for device dev (its size back in *bytes), or nullptr
void* pool_take(size_t* bytes, bool host, int dev);
void pool_give(void* p, size_t bytes, bool host, int dev);
template <bool HOST>
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;   // the device current when it was allocated (its pool)
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), bytes(o.bytes), dev(o.dev) { o.p = nullptr; o.bytes = 0; }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; dev = o.dev;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~Buf() { release(); }
  void release() { if (p) pool_give(p, bytes, HOST, dev); p = nullptr; bytes = 0; }
  tt_status alloc(size_t nbytes);          // grows only; contents undefined
  template <class T> T* as() const { return static_cast<T*>(p); }
};
using DBuf = Buf<false>;
using HBuf = Buf<true>;

// ---------------------------------------------------------------- problem
struct Grid {
  int d = 0, dt = 0, D = 0;
  int n[MAXD] = {0};
  double lo[MAXD] = {0}, hi[MAXD] = {0};   // box of dimension j in (x, theta, y) order
  double nodes[MAXD * MAXN] = {0};          // host copy of the node table
};
tt_status make_grid(const tt_kernel_params* p, Grid* g);

// ---------------------------------------------------------- kernel entries
// Entries of the super-core unfolding / fibre addressed through index sets
// (see ttk_eval.hip): multi-index = (left[s], mid..., right[t]).
struct Addr {
  const int16_t* left;   // rl x lk row-major (lk = number of leading dims)
  const int16_t* right;  // rr x lr row-major (lr = number of trailing dims)
  int rl, lk, rr, lr;
  int nmid;              // 1 (fibre) or 2 (super-core)
  int nm0, nm1;          // node counts of the middle dims
};
// out[i + j*nr] = A(rows[i], cols[j]) (out[j + i*nc] when trans_out); rows/cols
// NULL = all rows/cols.  amax (device, may be NULL): max |value| folded into
// AMAX_SLOTS slots as for eval_segs.
void eval_product(const KSpec& ks, const Addr& a, const int32_t* rows, int nr,
                  const int32_t* cols, int nc, double* out, hipStream_t st,
                  double* amax = nullptr, bool trans_out = false);
// One block of entries for eval_segs: mode 0 = product (i fastest), 1 = product
// with the column index fastest, 2 = list of (rows[i], cols[i]) with nc = 1.
struct EvalSeg {
  const int32_t* rows;
  const int32_t* cols;
  int nr, nc, mode;
  double* out;
};
// amax (device, may be NULL): AMAX_SLOTS doubles; block b folds its max
// |value| into slot b mod AMAX_SLOTS (one contended address would serialise).
constexpr int AMAX_SLOTS = 32;
void eval_segs(const KSpec& ks, const Addr& a, const EvalSeg* segs, int nseg, hipStream_t st,
               double* amax);
// out[i] = A(rows[i], cols[i]); amax as for eval_product
void eval_list(const KSpec& ks, const Addr& a, const int32_t* rows, const int32_t* cols,
               int np, double* out, hipStream_t st, double* amax = nullptr);
// out[i] = f_kappa at multi-index idx[i*D .. i*D+D-1] (int16 or int32)
void eval_multi16(const KSpec& ks, const int16_t* idx, int64_t P, double* out, hipStream_t st);
void eval_multi32(const KSpec& ks, const int32_t* idx, int64_t P, double* out, hipStream_t st);
// dense block K[i + j*ldk] = kappa(x_i, y_j; theta), T = float or double
void eval_dense_f32(const KSpec& ks, const float* X, int64_t nx, const float* Y, int64_t ny,
                    const double* theta, float* K, int64_t ldk, hipStream_t st);
void eval_dense_f64(const KSpec& ks, const double* X, int64_t nx, const double* Y, int64_t ny,
                    const double* theta, double* K, int64_t ldk, hipStream_t st);

// --------------------------------------------------- small dense FP64 algebra
// All column-major, one workgroup per call unless stated (ttk_linalg.hip).
void lu_factor(double* A, int n, int lda, int32_t* piv, int32_t* info, hipStream_t st);
// Solve A X = B (trans = 0) or A^T X = B (trans = 1) for nrhs columns, in place.
void lu_solve(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B,
              int ldb, int nrhs, hipStream_t st);
// Same with the right-hand-side index fastest: entry (k, c) of B at c + k * ldb,
// so one wave reads consecutive addresses.
void lu_solve_rm(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B,
                 int64_t ldb, int nrhs, hipStream_t st);
// Thin Householder QR of A (m x n, m >= n): A <- Q (m x n), R (n x n).
void qr_thin(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st);
// Blocked Householder QR (same result layout as qr_thin); work holds
// qr_blocked_work(m, n) doubles.
tt_status qr_blocked(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st);
size_t qr_blocked_work(int m, int n);
// The factorisation alone: the reflectors stay below the diagonal of A and
// their block factors in work (qr_blocked_work(m, n) doubles); R (n x n).
tt_status qr_factor(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st);
// C (m x nc, ldc) <- Q C with the Q of a qr_factor of A (m x n) and its work.
tt_status qr_apply_q(const double* A, int m, int n, int lda, double* work, double* C, int nc, int ldc,
                     hipStream_t st);
// R factors (n x n upper, ld ldr, at R + b sR) of `count` square matrices
// (A + b sA, ld lda, n <= 512, overwritten by their reflectors), all in one
// sequence of batched launches; work holds qr_r_batched_work(n, count).
size_t qr_r_batched_work(int n, int count);
tt_status qr_r_batched(double* A, int n, int lda, size_t sA, double* R, int ldr, size_t sR, double* work, int count,
                       hipStream_t st);
// Tall-skinny QR of an N x r matrix (r <= 512, N >= r): A(p, c) at
// A[p sp + c sc] in dtype.  tsqr_factor writes R (r x r upper, FP64, device,
// leading dimension ldr) and keeps the blocks' reflectors in *ts;
// tsqr_apply writes Q [C; 0] (N x c, c <= 512; C FP64 r x c on the device,
// leading dimension ldc) to Y(p, j) = Y[p sp + j sc] in out_dtype.
constexpr int TSQR_MAXLEV = 24;
struct TsqrState {
  int r = 0, nlev = 0, H = 0;
  int64_t N = 0;
  int nb[TSQR_MAXLEV] = {0};
  int64_t rows[TSQR_MAXLEV] = {0};
  DBuf A[TSQR_MAXLEV], tau[TSQR_MAXLEV], T[TSQR_MAXLEV];
  DBuf T64[TSQR_MAXLEV];   // 64-column block reflectors' T (levels of many 2048-row blocks)
  bool wide[TSQR_MAXLEV] = {false};
  DBuf V, Wp, D[2];
};
tt_status tsqr_factor(int dtype, const void* A, int64_t sp, int64_t sc, int64_t N, int r, TsqrState* ts, double* R,
                      int ldr, hipStream_t st);
tt_status tsqr_apply(TsqrState* ts, const double* C, int ldc, int c, int out_dtype, void* Y, int64_t sp, int64_t sc,
                     hipStream_t st);
// One-sided Jacobi SVD of A (n x n, lda): A <- U Sigma (columns), V (n x n),
// sigma (n); columns sorted by decreasing sigma.
void jacobi_svd(double* A, int n, int lda, double* V, int ldv, double* sigma, hipStream_t st);
// Same without the right vectors (A <- U Sigma normalised to U, sigma): in
// one workgroup's LDS when A fits, else by the block iteration over many
// workgroups (n <= 512; it waits for the stream between batches of sweeps).
// sigma's buffer holds jacobi_sigma_doubles(n).  false: nothing launched.
bool jacobi_svd_left(double* A, int n, int lda, double* sigma, hipStream_t st);
// count independent left-only SVDs by the block iteration together (one grid
// over every matrix's meetings; n <= 512): matrix b at A + b sA, its sigma
// and workspace at sigma + b sS (sS >= jacobi_sigma_doubles(n)).  false:
// nothing launched.
bool jacobi_svd_left_batched(double* A, int n, int lda, size_t sA, double* sigma, size_t sS, int count,
                             hipStream_t st);
// count independent SVDs, one workgroup each; matrix b at A + b sA, V + b sV,
// sigma (and its workspace) at sigma + b sS, sS >= jacobi_sigma_doubles(n).
void jacobi_svd_batched(double* A, int n, int lda, size_t sA, double* V, int ldv, size_t sV, double* sigma,
                        size_t sS, int count, hipStream_t st);
size_t jacobi_sigma_doubles(int n);
// C = alpha op(A) op(B) + beta C, small FP64 GEMM (many blocks).
void gemm64(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda,
            const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
// Frobenius norm of a vector into *out (device).
void nrm2(const double* x, int64_t n, double* out, hipStream_t st);

// ----------------------------------------------------------- the cross
struct CrossOut {
  std::vector<int> ranks;                     // r_0..r_D
  std::vector<DBuf> cores;                    // device FP64, little-endian r0 x n x r1
  std::vector<std::vector<int32_t>> left;     // I^{<=k}, k = 0..D
  std::vector<std::vector<int32_t>> right;    // I^{>k},  k = 0..D
  std::vector<tt_kernel_decision> log;
  int sweeps = 0;
  double error = 0.0, init_max_cond = 0.0, min_margin = 1.0;
  int64_t evals = 0;
  bool converged = false;
};
tt_status run_cross(const tt_kernel_params* p, const Grid& g, const KSpec& ks,
                    hipStream_t st, CrossOut* out);

// -------------------------------------------------- rounding and gauge
// TT-Round + gauge + signs of device FP64 cores (little-endian r0 x n x r1),
// in place: the buffers are reused for the rounded cores.
tt_status round_gauge(std::vector<DBuf>& cores, std::vector<int>& ranks, const Grid& g, double eps,
                      hipStream_t st);

// ----------------------------------------------------------- Phase 3
struct ChainStage {
  const void* G2;     // device, dtype, row-major (r_in * n) x r_out, row index a + k r_in
  int r_in, r_out, n;
  int coord;          // which coordinate of the point feeds this stage
  double lo, hi;      // box of that coordinate
};
tt_status factor_contract(int dtype, const ChainStage* stages, int nstages, const void* P_soa,
                          int64_t npts, void* out, int ldo, hipStream_t st);
// Phase 3 of many chains.  Job j: points with coordinate c of point q at
// P[c * ldp + q], q < npts, rows written to out (row-major, ldo).
struct FactorJob {
  const ChainStage* stages;
  int nstages;
  const void* P;
  int64_t ldp, npts;
  void* out;
  int ldo;
};
// Device copy of a job list (kept between calls with the same jobs).
struct FactorBatchPlan {
  DBuf desc, prefix;
  int njobs = -1;
  int64_t tiles = 0;
  bool persistent = false;
};
// FP32: one persistent launch of `grid` workgroups (0 = one per 64-point tile)
// striding over the tiles of all jobs; otherwise one launch per job.
tt_status factor_contract_batch(int dtype, const FactorJob* jobs, int njobs, int grid, hipStream_t st,
                                FactorBatchPlan* plan);

// ----------------------------------------------------------- online / apply
struct ParamCore {
  const double* Ghat;  // device FP64, coefficient-basis core, r0 x n x r1 little-endian
  int r0, n, r1;
  double lo, hi;
};
void online_core(int dtype, const ParamCore* pc, int dt, const void* theta, int B, void* M,
                 void* dM, double* work, hipStream_t st);
// Same with theta and the outputs in separate precisions (TTK_FP32 / TTK_FP64).
void online_core_mixed(int theta_dtype, int out_dtype, const ParamCore* pc, int dt, const void* theta, int B,
                       void* M, void* dM, double* work, hipStream_t st);
size_t online_work_doubles(const ParamCore* pc, int dt, int B);
// d_theta = 2, float32 outputs, as one matrix-core product: with the
// coefficient-basis parameter cores Ghat_1 (rs x n1 x rm) and Ghat_2
// (rm x n2 x rt), M(theta) = sum_{k1,k2} T_k1(t_1) T_k2(t_2) C_{k1 k2}, where
// C_{k1 k2} = Ghat_1[:, k1, :] Ghat_2[:, k2, :] is formed once per build
// (online_gemm_prepare), and the derivatives replace T_kj by T_kj'.
struct OnlineGemm {
  const float* C = nullptr;   // device, (rs rt) x nk row-major, row e = a + c rs, column k1 n2 + k2
  int nk = 0, rs = 0, rt = 0;
};
constexpr int ONLINE_GEMM_MIN_B = 32;   // below this the per-theta kernels are faster
tt_status online_gemm_prepare(const ParamCore* pc, float* C, hipStream_t st);   // C: rs rt n1 n2 floats
size_t online_gemm_work_floats(const OnlineGemm& og, int B, bool want_d);
tt_status online_core_gemm(const ParamCore* pc, const OnlineGemm& og, const float* theta, int B, float* M,
                           float* dM, float* work, hipStream_t st);

// W (r x B) = F^T X.  work: apply_reduce_work(N, r, B) bytes of device memory
// for the per-workgroup partial sums (may be NULL when that is 0); every
// byte the reduction reads from it is written first by the same call.
tt_status apply_reduce(int dtype, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx,
                       int B, void* W, void* work, hipStream_t st);
size_t apply_reduce_work(int64_t N, int r, int B);
tt_status apply_expand(int dtype, const void* F, int ldf, int64_t N, int r, const void* Z, int B,
                       void* Y, int64_t ldy, hipStream_t st);  // Y (N x B) = F Z
// Float32 matrix-core forms of the two wide contractions (ttk_apply_mfma.hip),
// taken for B > 16 and r <= MFMA_APPLY_MAXR.
constexpr int MFMA_APPLY_MAXR = 128;
bool apply_mfma_ok(int r, int B);
// Leading dimension for float32 U and V rows: the smallest ld >= r with
// ld % 32 == 16 (16-byte rows whose K-step reads hit disjoint LDS banks).
int mfma_ld(int r);
size_t apply_reduce_mfma_work(int64_t N, int r, int B);
tt_status apply_reduce_mfma(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B,
                            float* W, double* part, hipStream_t st);
// Y (N x B, ldy) = F Z (or += with accumulate), Z: r x B with leading dimension r.
tt_status apply_expand_mfma(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y,
                            int64_t ldy, hipStream_t st, bool accumulate = false);
// Float32 forms for 2 <= B <= 16 and r <= MFMA_APPLY_MAXR with 16-byte aligned
// rows of F (ldf % 4 == 0).  The reduce writes one float64 partial of W
// (r x B) per 256 rows, part[g r B + c + b r] for g < groups, groups >= N / 256.
bool skinny_mfma_ok(const void* F, int ldf, int r, int B);
bool skinny_expand_mfma_ok(const void* F, int ldf, int r, int B);   // and ldf <= 160
tt_status reduce_skinny_mfma(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B,
                             double* part, unsigned groups, hipStream_t st);
tt_status expand_skinny_mfma(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y,
                             int64_t ldy, hipStream_t st);
// W (r x B) = F^T X, then Z_b = op(M_b) W_b (r = the number of inputs of
// op(M)); work as for apply_reduce.  With dM (op = transpose only): also
// dtheta[b, j] = W_b^T dM_{b,j} Wv_b for j < dt (Wv: cols x B).  For skinny
// batches with M_b small enough for LDS the sum of the reduce's partials,
// the product and the bilinear forms are one launch.
tt_status apply_reduce_matvec(int dtype, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx,
                              int B, void* W, const void* M, int rows, int cols, int trans, void* Z, void* work,
                              hipStream_t st, const void* dM = nullptr, const void* Wv = nullptr, int dt = 0,
                              void* dtheta = nullptr);
void batched_matvec(int dtype, const void* M, int rows, int cols, int trans, const void* x,
                    int B, void* y, hipStream_t st);    // y_b = op(M_b) x_b
void batched_bilinear(int dtype, const void* A, const void* dM, const void* W, int rs, int rt,
                      int B, int dt, void* dtheta, hipStream_t st);  // dtheta[b,j] = a_b^T dM_bj w_b
void fill_zero(void* p, size_t bytes, hipStream_t st);
// ------------------------------------------ interaction-list batch apply
// One side (sources or targets) of one pair: its factor block F_p (n x r
// row-major at element offset foff), its first row in the N x B vectors and
// its r x B block of W / Z / A (column-major, element offset woff).
struct BatchSide {
  int64_t foff, n, roff, woff;
  int r, pad;
};
// Work item of the tall launches: rows row0 .. row0 + nrows - 1 of side
// `side`, rank columns r0 .. r0 + 63 (reduce only), thetas b0 .. b0 + 63.
struct BatchItem {
  int64_t row0;
  int side, nrows, r0, b0;
};
void batch_reduce(int dtype, const void* F, const BatchSide* sides, const BatchItem* items, int64_t nitems,
                  const void* X, int64_t ldx, int B, void* W, hipStream_t st);      // W_p += F_p^T X_p
void batch_expand(int dtype, const void* F, const BatchSide* sides, const BatchItem* items, int64_t nitems,
                  const void* Z, int B, void* Y, int64_t ldy, hipStream_t st);      // Y_p += F_p Z_p
void batch_small(int dtype, const void* M, const int64_t* moff, const BatchSide* in_s, const BatchSide* out_s,
                 int trans, const void* Win, void* Zout, int B, int npairs, hipStream_t st);
void batch_dtheta(int dtype, const void* A, const BatchSide* s_side, const void* dM, const int64_t* dmoff,
                  const void* W, const BatchSide* t_side, int B, int dt, int npairs, double* part, void* dtheta,
                  hipStream_t st);
void fill_cols(int dtype, void* Y, int64_t rows, int B, int64_t ldy, hipStream_t st);
// ----------------------------------------------- Global-1 (Algorithm 4)
// Thin QR of A = [U V] (N x k, k = rs + rt; U, V row-major in dtype) by
// blocked Householder QR in double precision.  Q: device, dtype, N x k
// row-major.  R: device, FP64, k x k column-major upper triangular.
// Synchronises st.
tt_status global_qr(int dtype, const void* U, int ldu, int rs, const void* V, int ldv, int rt, int64_t N,
                    void* Q, double* R, hipStream_t st);
// W_b = (Mh_b + |Mh_b|) / 2, the non-negative spectral part of
// Mh_b = R Hhat_b R^T, Hhat_b = [[0, M_b / 2], [M_b^T / 2, 0]], for M_b (FP64,
// rs x rt column-major at M + b rs rt).  W: device, out_dtype, B x k x k.
// work: global_online_work(rs, rt, B) doubles.
void global_online(const double* R, int rs, int rt, const double* M, int B, int out_dtype, void* W,
                   double* work, hipStream_t st);
size_t global_online_work(int rs, int rt, int B);
// Global-2 (Compress) for one theta, M (FP64 rs x rt): W_+ as above, its
// eigenpairs by a one-sided Jacobi (decreasing eigenvalues), and the
// truncation rank rc (the smallest r with sqrt(sum_{i > r} lambda_i^2) <=
// eps ||Mh||_F; 0 when no eigenvalue is positive).  On return *Uhat (k x k,
// column-major, inside work) holds the eigenvectors and *lam (inside work)
// the eigenvalues.  work: global2_work(rs, rt) doubles.  Synchronises st.
tt_status global2_online(const double* R, int rs, int rt, const double* M, double eps, double* work, double** Uhat,
                         double** lam, int* rc, hipStream_t st);
size_t global2_work(int rs, int rt);

}  // namespace ttk
