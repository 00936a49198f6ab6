// TT-Round (Algorithm 1) of the cross cores, then the gauge used by Phase 3:
// after the rounding sweep the cores G_1..G_{D-1} are left-orthonormal; the
// target cores G_D..G_{d+dt+1} are then right-orthonormalised (thin QR of
// (G^{1})^T, R pushed into the left neighbour), so the last parameter core
// carries the norm.  Signs: the largest-|.| entry of each column of a
// left-orthonormal G^{2} (row of a right-orthonormal G^{1}) is made positive,
// lowest index on ties, and the sign is pushed into the neighbour.
// Every factorisation runs on the device in double precision; the host only
// reads back singular values to choose the truncation rank.
//
// Readings: ||X||_F is taken as ||G_1||_F after the orthogonalisation sweep;
// the truncation keeps the smallest r' >= 1 whose discarded tail
// sqrt(sum_{i > r'} sigma_i^2) is <= delta = eps / sqrt(D - 1) ||X||_F; the
// mode-3 update of the orthogonalisation is G_{i-1}^{2} <- G_{i-1}^{2} R^T.
#include <cmath>

#include "ttk_internal.h"

namespace ttk {

namespace {

__global__ void k_transpose64(const double* A, int m, int n, int lda, double* B, int ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  B[j + (int64_t)i * ldb] = A[i + (int64_t)j * lda];
}

// W[a, b] = sigma[a] * V[b, a] for a < rp, b < r  (W = (Sigma V^T)[:rp, :], ld rp)
__global__ void k_sigma_vt(const double* sigma, const double* V, int r, int rp, double* W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rp * r) return;
  const int a = e % rp, b = e / rp;
  W[a + b * rp] = sigma[a] * V[b + a * r];
}

// Sign of the largest-|.| entry of each column of A (m x c), lowest row on ties.
__global__ void k_col_signs(const double* A, int m, int c, int lda, double* sg) {
  const int col = blockIdx.x;
  __shared__ double sv[256];
  __shared__ int si[256];
  double best = -1.0;
  int bi = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double v = fabs(A[i + (int64_t)col * lda]);
    if (v > best) { best = v; bi = i; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + s];
      if (b > a || (b == a && si[threadIdx.x + s] < si[threadIdx.x])) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = si[threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = A[si[0] + (int64_t)col * lda];
    sg[col] = v < 0.0 ? -1.0 : 1.0;
  }
}

// A[:, j] *= sg[j] (mode 0) or A[i, :] *= sg[i] (mode 1), A m x c.
__global__ void k_scale(double* A, int m, int c, int lda, const double* sg, int mode) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * c) return;
  const int i = (int)(e % m), j = (int)(e / m);
  A[i + (int64_t)j * lda] *= (mode == 0) ? sg[j] : sg[i];
}

// C (mc x nc, ldc) <- [S; 0] with S rows x nc (lds), rows <= mc.
__global__ void k_pad_rows(const double* S, int rows, int lds, double* C, int mc, int nc, int ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mc * nc) return;
  const int i = (int)(e % mc), j = (int)(e / mc);
  C[i + (int64_t)j * ldc] = i < rows ? S[i + (int64_t)j * lds] : 0.0;
}

inline int nb(int64_t n) { return (int)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

// Unfoldings taller than this are factored by the tall-skinny QR (blocks of
// at most 2048 rows, whose register panels hold a whole column block),
// shorter ones by the blocked Householder QR of one block.
constexpr int ROUND_TALL = 2048;

// I[:, :c] of an r x r identity (column-major, ld r)
__global__ void k_eye_cols(double* I, int r, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * c) return;
  I[e] = (e % r) == (e / r) ? 1.0 : 0.0;
}

struct Cores {
  std::vector<DBuf> g;       // device copies, core k as G^{2}/G^{1}-compatible memory
  std::vector<int> r;         // r_0..r_D
  std::vector<int> n;
};

// thin QR of (G_i^{1})^T, G_i <- Q^T, G_{i-1}^{2} <- G_{i-1}^{2} R^T.  When
// (G_i^{1})^T (n r1 x r0) is wide, the rank drops to n r1: the matrix is
// padded with zero rows to r0 x r0, whose Householder QR leaves the padding
// untouched (every reflector vanishes there), so the leading n r1 x n r1
// block of Q and the leading n r1 rows of R are the thin factors.
tt_status orth_right(Cores& c, int i, DBuf& A, DBuf& R, DBuf& T, DBuf& tau, hipStream_t st) {
  const int r0 = c.r[i], n = c.n[i], r1 = c.r[i + 1];
  const int m = n * r1;
  const int ma = std::max(m, r0);   // rows of the (padded) QR input
  const int rp = std::min(m, r0);   // new rank r_i
  TTK_TRY(A.alloc((size_t)ma * r0 * sizeof(double)));
  TTK_TRY(R.alloc((size_t)r0 * r0 * sizeof(double)));
  TTK_TRY(tau.alloc(qr_blocked_work(ma, r0) * sizeof(double)));
  double* G = c.g[i].as<double>();
  if (ma > m) fill_zero(A.p, (size_t)ma * r0 * sizeof(double), st);
  hipLaunchKernelGGL(k_transpose64, dim3(nb((int64_t)r0 * m)), dim3(256), 0, st, G, r0, m, r0, A.as<double>(),
                     ma);
  if (ma > ROUND_TALL) {   // Q[:, :rp] = Q [I[:, :rp]; 0] into A
    TsqrState ts;
    TTK_TRY(tsqr_factor(TTK_FP64, A.as<double>(), 1, ma, ma, r0, &ts, R.as<double>(), r0, st));
    DBuf E;
    TTK_TRY(E.alloc((size_t)r0 * rp * sizeof(double)));
    hipLaunchKernelGGL(k_eye_cols, dim3(nb((int64_t)r0 * rp)), dim3(256), 0, st, E.as<double>(), r0, rp);
    TTK_TRY(tsqr_apply(&ts, E.as<double>(), r0, rp, TTK_FP64, A.as<double>(), 1, ma, st));
  } else {
    TTK_TRY(qr_blocked(A.as<double>(), ma, r0, ma, R.as<double>(), r0, tau.as<double>(), st));
  }
  // G_i^{1} (rp x m) = Q[:m, :rp]^T
  hipLaunchKernelGGL(k_transpose64, dim3(nb((int64_t)rp * m)), dim3(256), 0, st, A.as<double>(), m, rp, ma, G, rp);
  const int q0 = c.r[i - 1], qn = c.n[i - 1];
  TTK_TRY(T.alloc((size_t)q0 * qn * rp * sizeof(double)));
  // G_{i-1}^{2} (q0 qn x r0) R[:rp, :]^T
  gemm64(0, 1, q0 * qn, rp, r0, 1.0, c.g[i - 1].as<double>(), q0 * qn, R.as<double>(), r0, 0.0, T.as<double>(),
         q0 * qn, st);
  TTK_HIP(hipMemcpyAsync(c.g[i - 1].p, T.p, (size_t)q0 * qn * rp * sizeof(double), hipMemcpyDeviceToDevice, st));
  c.r[i] = rp;   // (the work buffers are reserved at their largest size: nothing to wait for)
  return TTK_OK;
}

}  // namespace

tt_status round_gauge(std::vector<DBuf>& cores, std::vector<int>& ranks, const Grid& grid, double eps,
                      hipStream_t st) {
  const int D = (int)cores.size();
  Cores c;
  c.r = ranks;
  c.n.assign(grid.n, grid.n + D);
  c.g.resize(D);
  for (int k = 0; k < D; ++k) c.g[k] = std::move(cores[k]);   // rounded in place (ranks only fall)
  DBuf A, R, T, tau, tw, V, sig, W, nrm, sg, Cw;
  {
    // every work buffer at the largest size any step needs (the ranks only
    // fall from here), so that none is reallocated, which would wait for the
    // queued work, between the steps
    int rmax = 1, nmax = 1;
    for (int k = 0; k <= D; ++k) rmax = std::max(rmax, c.r[k]);
    for (int k = 0; k < D; ++k) nmax = std::max(nmax, c.n[k]);
    const size_t big = (size_t)rmax * rmax * nmax * sizeof(double), sq = (size_t)rmax * rmax * sizeof(double);
    TTK_TRY(A.alloc(big));
    TTK_TRY(T.alloc(big));
    TTK_TRY(Cw.alloc(big));
    TTK_TRY(R.alloc(sq));
    TTK_TRY(V.alloc(sq));
    TTK_TRY(W.alloc(sq));
    TTK_TRY(sig.alloc(sq + (3 * (size_t)rmax + 64) * sizeof(double)));
    TTK_TRY(tau.alloc(qr_blocked_work(rmax * nmax, rmax) * sizeof(double)));
    TTK_TRY(tw.alloc(qr_blocked_work(rmax, rmax) * sizeof(double)));
  }
  // right-to-left orthogonalisation
  for (int i = D - 1; i >= 1; --i) TTK_TRY(orth_right(c, i, A, R, T, tau, st));
  TTK_TRY(nrm.alloc(sizeof(double)));
  nrm2(c.g[0].as<double>(), (int64_t)c.r[0] * c.n[0] * c.r[1], nrm.as<double>(), st);
  double norm = 0.0;
  TTK_HIP(hipMemcpyAsync(&norm, nrm.p, sizeof(double), hipMemcpyDeviceToHost, st));
  TTK_HIP(hipStreamSynchronize(st));
  const double delta = eps / std::sqrt((double)std::max(D - 1, 1)) * norm;
  // left-to-right truncated SVD
  std::vector<double> hs;
  for (int i = 0; i < D - 1; ++i) {
    const int r0 = c.r[i], n = c.n[i], r1 = c.r[i + 1];
    const int m = r0 * n;
    // a wide G_i^{2} (after truncation of r_i) is padded with zero rows, as in orth_right
    const int ma = std::max(m, r1);
    TTK_TRY(A.alloc((size_t)ma * r1 * sizeof(double)));
    TTK_TRY(R.alloc((size_t)r1 * r1 * sizeof(double)));
    TTK_TRY(tau.alloc(qr_blocked_work(ma, r1) * sizeof(double)));
    TTK_TRY(V.alloc((size_t)r1 * r1 * sizeof(double)));
    TTK_TRY(sig.alloc(((size_t)r1 * r1 + 3 * (size_t)r1 + 64) * sizeof(double)));
    if (ma > m) fill_zero(A.p, (size_t)ma * r1 * sizeof(double), st);
    TTK_HIP(hipMemcpy2DAsync(A.p, (size_t)ma * sizeof(double), c.g[i].p, (size_t)m * sizeof(double),
                             (size_t)m * sizeof(double), (size_t)r1, hipMemcpyDeviceToDevice, st));
    const bool tall = ma > ROUND_TALL;
    TsqrState ts;
    if (tall) TTK_TRY(tsqr_factor(TTK_FP64, A.as<double>(), 1, ma, ma, r1, &ts, R.as<double>(), r1, st));
    else TTK_TRY(qr_factor(A.as<double>(), ma, r1, ma, R.as<double>(), r1, tau.as<double>(), st));
    // SVD of R.  Sigma V^T, pushed into the next core, is U^T R: with a copy of R
    // kept, only the left vectors are needed (V stays unaccumulated)
    TTK_HIP(hipMemcpyAsync(V.p, R.p, (size_t)r1 * r1 * sizeof(double), hipMemcpyDeviceToDevice, st));
    // The iteration runs on L = R2^T, where R^T = Q2 R2: R = L Q2^T, so L has
    // R's singular values and left vectors, and one QR step leaves L's
    // columns far closer to orthogonal (on these cores a few sweeps instead
    // of tens; the QR preconditioning of Drmac and Veselic without the
    // column pivoting)
    hipLaunchKernelGGL(k_transpose64, dim3(nb((int64_t)r1 * r1)), dim3(256), 0, st, (const double*)R.as<double>(),
                       r1, r1, r1, T.as<double>(), r1);
    TTK_TRY(qr_factor(T.as<double>(), r1, r1, r1, W.as<double>(), r1, tw.as<double>(), st));
    hipLaunchKernelGGL(k_transpose64, dim3(nb((int64_t)r1 * r1)), dim3(256), 0, st, (const double*)W.as<double>(),
                       r1, r1, r1, R.as<double>(), r1);
    const bool left_only = jacobi_svd_left(R.as<double>(), r1, r1, sig.as<double>(), st);
    if (!left_only) {   // (nothing was launched: the full SVD of R itself)
      TTK_HIP(hipMemcpyAsync(R.p, V.p, (size_t)r1 * r1 * sizeof(double), hipMemcpyDeviceToDevice, st));
      jacobi_svd(R.as<double>(), r1, r1, V.as<double>(), r1, sig.as<double>(), st);
    }
    hs.resize(r1);
    TTK_HIP(hipMemcpyAsync(hs.data(), sig.p, (size_t)r1 * sizeof(double), hipMemcpyDeviceToHost, st));
    TTK_HIP(hipStreamSynchronize(st));
    int rp = r1;
    {
      std::vector<double> tail(r1 + 1, 0.0);
      for (int j = r1 - 1; j >= 0; --j) tail[j] = tail[j + 1] + hs[j] * hs[j];
      for (int q = 1; q <= r1; ++q)
        if (std::sqrt(tail[q]) <= delta) { rp = q; break; }
    }
    rp = std::min(rp, m);   // a wide unfolding has at most m singular values
    // G_i^{2} <- Q[:m, :] U_R[:, :rp], the leading m rows of Q [U_R[:, :rp]; 0]: the
    // reflectors applied to the rp kept columns (Q itself is never formed)
    {
      double* Cq = c.g[i].as<double>();   // m x rp fits the core's buffer
      if (ma > m) {
        TTK_TRY(Cw.alloc((size_t)ma * rp * sizeof(double)));
        Cq = Cw.as<double>();
      }
      if (tall) {
        TTK_TRY(tsqr_apply(&ts, R.as<double>(), r1, rp, TTK_FP64, Cq, 1, ma, st));
      } else {
        hipLaunchKernelGGL(k_pad_rows, dim3(nb((int64_t)ma * rp)), dim3(256), 0, st, (const double*)R.as<double>(),
                           r1, r1, Cq, ma, rp, ma);
        TTK_TRY(qr_apply_q(A.as<double>(), ma, r1, ma, tau.as<double>(), Cq, rp, ma, st));
      }
      if (ma > m)
        TTK_HIP(hipMemcpy2DAsync(c.g[i].p, (size_t)m * sizeof(double), Cq, (size_t)ma * sizeof(double),
                                 (size_t)m * sizeof(double), (size_t)rp, hipMemcpyDeviceToDevice, st));
    }
    // G_{i+1}^{1} <- (Sigma V^T)[:rp, :] G_{i+1}^{1}
    const int n2 = c.n[i + 1], r2 = c.r[i + 2];
    TTK_TRY(W.alloc((size_t)rp * r1 * sizeof(double)));
    if (left_only)   // (Sigma V^T)[:rp, :] = U[:, :rp]^T R, R's copy in V
      gemm64(1, 0, rp, r1, r1, 1.0, R.as<double>(), r1, V.as<double>(), r1, 0.0, W.as<double>(), rp, st);
    else
      hipLaunchKernelGGL(k_sigma_vt, dim3(nb((int64_t)rp * r1)), dim3(256), 0, st, sig.as<double>(),
                         V.as<double>(), r1, rp, W.as<double>());
    TTK_TRY(T.alloc((size_t)rp * n2 * r2 * sizeof(double)));
    gemm64(0, 0, rp, n2 * r2, r1, 1.0, W.as<double>(), rp, c.g[i + 1].as<double>(), r1, 0.0, T.as<double>(), rp,
           st);
    TTK_HIP(hipMemcpyAsync(c.g[i + 1].p, T.p, (size_t)rp * n2 * r2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    c.r[i + 1] = rp;
  }
  // gauge: right-orthonormal target cores
  const int first_target = grid.d + grid.dt;
  for (int i = D - 1; i >= first_target && i >= 1; --i) TTK_TRY(orth_right(c, i, A, R, T, tau, st));
  // signs
  TTK_TRY(sg.alloc((size_t)MAXR * sizeof(double)));
  for (int i = 0; i + 1 < first_target; ++i) {
    const int r0 = c.r[i], n = c.n[i], r1 = c.r[i + 1];
    hipLaunchKernelGGL(k_col_signs, dim3(r1), dim3(256), 0, st, c.g[i].as<double>(), r0 * n, r1, r0 * n,
                       sg.as<double>());
    hipLaunchKernelGGL(k_scale, dim3(nb((int64_t)r0 * n * r1)), dim3(256), 0, st, c.g[i].as<double>(), r0 * n, r1,
                       r0 * n, sg.as<double>(), 0);
    const int n2 = c.n[i + 1], r2 = c.r[i + 2];
    hipLaunchKernelGGL(k_scale, dim3(nb((int64_t)r1 * n2 * r2)), dim3(256), 0, st, c.g[i + 1].as<double>(), r1,
                       n2 * r2, r1, sg.as<double>(), 1);
  }
  for (int i = D - 1; i >= first_target && i >= 1; --i) {
    const int r0 = c.r[i], n = c.n[i], r1 = c.r[i + 1];
    // rows of G^{1} (r0 x n r1) = columns of its transpose
    TTK_TRY(A.alloc((size_t)r0 * n * r1 * sizeof(double)));
    hipLaunchKernelGGL(k_transpose64, dim3(nb((int64_t)r0 * n * r1)), dim3(256), 0, st, c.g[i].as<double>(), r0,
                       n * r1, r0, A.as<double>(), n * r1);
    hipLaunchKernelGGL(k_col_signs, dim3(r0), dim3(256), 0, st, A.as<double>(), n * r1, r0, n * r1,
                       sg.as<double>());
    hipLaunchKernelGGL(k_scale, dim3(nb((int64_t)r0 * n * r1)), dim3(256), 0, st, c.g[i].as<double>(), r0, n * r1,
                       r0, sg.as<double>(), 1);
    const int q0 = c.r[i - 1], qn = c.n[i - 1];
    hipLaunchKernelGGL(k_scale, dim3(nb((int64_t)q0 * qn * r0)), dim3(256), 0, st, c.g[i - 1].as<double>(),
                       q0 * qn, r0, q0 * qn, sg.as<double>(), 0);
  }
  TTK_HIP(hipGetLastError());
  for (int k = 0; k < D; ++k) cores[k] = std::move(c.g[k]);
  TTK_HIP(hipStreamSynchronize(st));
  ranks = c.r;
  return TTK_OK;
}

}  // namespace ttk
