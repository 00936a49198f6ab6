// Small dense double-precision linear algebra for the cross and the rounding
// of the cores: LU with partial pivoting (solves with the intersection
// matrices of the cross), Householder QR (thin QR of the TT-Round sweeps and
// of the interpolation formula), one-sided Jacobi SVD (truncated SVD of
// TT-Round) and a small tiled GEMM.  Matrices are column-major.  The
// factorisations run in one workgroup: they are sequential in the column
// index and their sizes (<= 8192 x 256) keep them in L2.
#include <cstring>

#include "ttk_internal.h"
#include "ttk_wave.h"

namespace ttk {

namespace {

constexpr int BS = 1024;      // threads of the single-workgroup kernels
constexpr int NW = BS / 64;   // waves per workgroup

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NW; ++i) s += red[i];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------- LU
__global__ void __launch_bounds__(BS) k_lu(double* A, int n, int lda, int32_t* piv, int32_t* info) {
  __shared__ double wv[NW];
  __shared__ int wi[NW];
  __shared__ int s_piv;
  __shared__ double s_pv;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) *info = 0;
  for (int j = 0; j < n; ++j) {
    // partial pivoting: largest |A[i, j]|, i >= j, lowest row on ties
    double best = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += BS) {
      const double v = fabs(A[i + (size_t)j * lda]);
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { wv[w] = best; wi[w] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = wv[0];
      int p = wi[0];
      for (int q = 1; q < NW; ++q)
        if (wv[q] > b || (wv[q] == b && wi[q] < p)) { b = wv[q]; p = wi[q]; }
      s_piv = p;
      s_pv = b;
      piv[j] = p;
      if (b == 0.0 && *info == 0) *info = j + 1;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j)
      for (int c = tid; c < n; c += BS) {
        const double t = A[j + (size_t)c * lda];
        A[j + (size_t)c * lda] = A[p + (size_t)c * lda];
        A[p + (size_t)c * lda] = t;
      }
    __syncthreads();
    const double dg = A[j + (size_t)j * lda];
    if (dg != 0.0)
      for (int i = j + 1 + tid; i < n; i += BS) A[i + (size_t)j * lda] /= dg;
    __syncthreads();
    // trailing update, element-parallel with consecutive threads on consecutive rows
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += BS) {
      const int i = j + 1 + e % m, c = j + 1 + e / m;
      A[i + (size_t)c * lda] -= A[i + (size_t)j * lda] * A[j + (size_t)c * lda];
    }
    __syncthreads();
  }
}

// The same factorisation with the matrix held in LDS (n x n doubles).
template <int TB>
__global__ void __launch_bounds__(TB) k_lu_lds(double* Ag, int n, int lda, int32_t* piv, int32_t* info) {
  constexpr int BS = TB, NW = TB / 64;
  extern __shared__ double A[];
  __shared__ double wv[NW];
  __shared__ int wi[NW];
  __shared__ int s_piv;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < n * n; e += BS) A[e] = Ag[e % n + (size_t)(e / n) * lda];
  if (tid == 0) *info = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += BS) {
      const double v = fabs(A[i + j * n]);
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { wv[w] = best; wi[w] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = wv[0];
      int p = wi[0];
      for (int q = 1; q < NW; ++q)
        if (wv[q] > b || (wv[q] == b && wi[q] < p)) { b = wv[q]; p = wi[q]; }
      s_piv = p;
      piv[j] = p;
      if (b == 0.0 && *info == 0) *info = j + 1;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j)
      for (int c = tid; c < n; c += BS) {
        const double t = A[j + c * n];
        A[j + c * n] = A[p + c * n];
        A[p + c * n] = t;
      }
    __syncthreads();
    const double dg = A[j + j * n];
    if (dg != 0.0)
      for (int i = j + 1 + tid; i < n; i += BS) A[i + j * n] /= dg;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += BS) {
      const int i = j + 1 + e % m, c = j + 1 + e / m;
      A[i + c * n] -= A[i + j * n] * A[j + c * n];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += BS) Ag[e % n + (size_t)(e / n) * lda] = A[e];
}

// One thread per right-hand side: row swaps, then the two triangular solves.
__global__ void k_lu_solve(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B,
                           int ldb, int nrhs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double* b = B + (size_t)c * ldb;
  if (!trans) {
    for (int i = 0; i < n; ++i) {
      const int p = piv[i];
      if (p != i) { const double t = b[i]; b[i] = b[p]; b[p] = t; }
    }
    for (int i = 0; i < n; ++i) {            // L y = b, unit diagonal
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= LU[i + (size_t)k * lda] * b[k];
      b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {       // U x = y
      double s = b[i];
      for (int k = i + 1; k < n; ++k) s -= LU[i + (size_t)k * lda] * b[k];
      b[i] = s / LU[i + (size_t)i * lda];
    }
  } else {
    for (int i = 0; i < n; ++i) {            // U^T z = b
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= LU[k + (size_t)i * lda] * b[k];
      b[i] = s / LU[i + (size_t)i * lda];
    }
    for (int i = n - 1; i >= 0; --i) {       // L^T w = z
      double s = b[i];
      for (int k = i + 1; k < n; ++k) s -= LU[k + (size_t)i * lda] * b[k];
      b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      const int p = piv[i];
      if (p != i) { const double t = b[i]; b[i] = b[p]; b[p] = t; }
    }
  }
}

// Right-hand side c in one thread, b(k) at B[c + k ldb] (coalesced across a
// wave); the factor is staged in LDS when it fits.
__global__ void k_lu_solve_rm(const double* LUg, int n, int lda, const int32_t* piv, int trans, double* B,
                              int64_t ldb, int nrhs, int in_lds) {
  extern __shared__ double sLU[];
  const double* LU = LUg;
  int ld = lda;
  if (in_lds) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) sLU[e] = LUg[e % n + (size_t)(e / n) * lda];
    __syncthreads();
    LU = sLU;
    ld = n;
  }
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double* b = B + c;
#define BV(k) b[(int64_t)(k) * ldb]
  if (!trans) {
    for (int i = 0; i < n; ++i) {
      const int p = piv[i];
      if (p != i) { const double t = BV(i); BV(i) = BV(p); BV(p) = t; }
    }
    for (int i = 0; i < n; ++i) {
      double s = BV(i);
      for (int k = 0; k < i; ++k) s -= LU[i + k * ld] * BV(k);
      BV(i) = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = BV(i);
      for (int k = i + 1; k < n; ++k) s -= LU[i + k * ld] * BV(k);
      BV(i) = s / LU[i + i * ld];
    }
  } else {
    for (int i = 0; i < n; ++i) {
      double s = BV(i);
      for (int k = 0; k < i; ++k) s -= LU[k + i * ld] * BV(k);
      BV(i) = s / LU[i + i * ld];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = BV(i);
      for (int k = i + 1; k < n; ++k) s -= LU[k + i * ld] * BV(k);
      BV(i) = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      const int p = piv[i];
      if (p != i) { const double t = BV(i); BV(i) = BV(p); BV(p) = t; }
    }
  }
#undef BV
}

// Blocked solve with the LU factors for many right-hand sides.  A workgroup
// owns RB right-hand sides, kept in LDS as rows of the permuted system; the
// triangular solves go 16 rows at a time: a short serial solve of the 16 x 16
// diagonal block per right-hand side, then a parallel update of the rest.
// trans = 0 solves A x = b (P A = L U); trans = 1 solves A^T x = b.
// Entry (k, c) of B is at c + k ldb.
template <int RB>
__global__ void __launch_bounds__(256) k_lu_trsm(const double* LU, int n, int lda, const int32_t* piv, int trans,
                                                 double* B, int64_t ldb, int nrhs) {
  constexpr int NB = 16;
  extern __shared__ double smem[];
  double* X = smem;                                            // n x RB
  double* Pn = X + (size_t)n * RB;                              // NB x n coefficient panel
  int* perm = reinterpret_cast<int*>(Pn + (size_t)NB * n);      // n
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * RB;
  const int nc = min(RB, nrhs - c0);
  if (tid == 0) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 0; i < n; ++i) {
      const int p = piv[i];
      if (p != i) { const int t = perm[i]; perm[i] = perm[p]; perm[p] = t; }
    }
  }
  __syncthreads();
  for (int e = tid; e < n * RB; e += 256) {
    const int i = e / RB, c = e % RB;
    const int src = trans ? i : perm[i];
    X[i * RB + c] = (c < nc) ? B[(c0 + c) + (int64_t)src * ldb] : 0.0;
  }
  // coefficient of X[k] in row i: lower solve L[i,k] (trans 0) or U[k,i] (trans 1),
  // upper solve U[i,k] (trans 0) or L[k,i] (trans 1); staged as Pn[(k - i0) n + i]
  auto stage = [&](int i0, int i1, int ilo, int ihi) {
    const int nb = i1 - i0, cnt = ihi - ilo;
    if (!trans) {
      for (int e = tid; e < nb * cnt; e += 256) {
        const int i = ilo + e % cnt, kl = e / cnt;
        Pn[kl * n + i] = LU[i + (size_t)(i0 + kl) * lda];
      }
    } else {
      for (int e = tid; e < nb * cnt; e += 256) {
        const int kl = e % nb, i = ilo + e / nb;
        Pn[kl * n + i] = LU[(i0 + kl) + (size_t)i * lda];
      }
    }
  };
  __syncthreads();
  // lower solve: L (unit) for trans 0, U^T for trans 1
  for (int i0 = 0; i0 < n; i0 += NB) {
    const int i1 = min(i0 + NB, n);
    stage(i0, i1, i0, n);
    __syncthreads();
    if (tid < RB) {
      const int c = tid;
      for (int i = i0; i < i1; ++i) {
        double s = X[i * RB + c];
        for (int k = i0; k < i; ++k) s -= Pn[(k - i0) * n + i] * X[k * RB + c];
        X[i * RB + c] = trans ? s / Pn[(i - i0) * n + i] : s;
      }
    }
    __syncthreads();
    for (int e = tid; e < (n - i1) * RB; e += 256) {
      const int i = i1 + e / RB, c = e % RB;
      double s = X[i * RB + c];
      for (int k = i0; k < i1; ++k) s -= Pn[(k - i0) * n + i] * X[k * RB + c];
      X[i * RB + c] = s;
    }
    __syncthreads();
  }
  // upper solve: U for trans 0, L^T (unit) for trans 1
  for (int i1 = n; i1 > 0; i1 -= NB) {
    const int i0 = max(i1 - NB, 0);
    stage(i0, i1, 0, i1);
    __syncthreads();
    if (tid < RB) {
      const int c = tid;
      for (int i = i1 - 1; i >= i0; --i) {
        double s = X[i * RB + c];
        for (int k = i + 1; k < i1; ++k) s -= Pn[(k - i0) * n + i] * X[k * RB + c];
        X[i * RB + c] = trans ? s : s / Pn[(i - i0) * n + i];
      }
    }
    __syncthreads();
    for (int e = tid; e < i0 * RB; e += 256) {
      const int i = e / RB, c = e % RB;
      double s = X[i * RB + c];
      for (int k = i0; k < i1; ++k) s -= Pn[(k - i0) * n + i] * X[k * RB + c];
      X[i * RB + c] = s;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * RB; e += 256) {
    const int i = e / RB, c = e % RB;
    if (c < nc) {
      const int dst = trans ? perm[i] : i;
      B[(c0 + c) + (int64_t)dst * ldb] = X[i * RB + c];
    }
  }
}

// One right-hand side per single-wave workgroup: each substitution step is a
// dot product spread over the 64 lanes and reduced by shuffles.
__global__ void __launch_bounds__(64) k_lu_solve_wave(const double* LU, int n, int lda, const int32_t* piv,
                                                      int trans, double* B, int64_t ldb) {
  extern __shared__ double xw[];
  const int lane = threadIdx.x;
  double* b = B + blockIdx.x;               // entry k at b[k * ldb]
  for (int k = lane; k < n; k += 64) xw[k] = b[(int64_t)k * ldb];
  __syncthreads();
  if (!trans && lane == 0)
    for (int i = 0; i < n; ++i) {
      const int p = piv[i];
      if (p != i) { const double t = xw[i]; xw[i] = xw[p]; xw[p] = t; }
    }
  __syncthreads();
  // lower: L (unit) or U^T
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = lane; k < i; k += 64) s += (trans ? LU[k + (size_t)i * lda] : LU[i + (size_t)k * lda]) * xw[k];
    s = wave_sum(s);
    if (lane == 0) xw[i] = trans ? (xw[i] - s) / LU[i + (size_t)i * lda] : xw[i] - s;
    __syncthreads();
  }
  // upper: U or L^T (unit)
  for (int i = n - 1; i >= 0; --i) {
    double s = 0.0;
    for (int k = i + 1 + lane; k < n; k += 64) s += (trans ? LU[k + (size_t)i * lda] : LU[i + (size_t)k * lda]) * xw[k];
    s = wave_sum(s);
    if (lane == 0) xw[i] = trans ? xw[i] - s : (xw[i] - s) / LU[i + (size_t)i * lda];
    __syncthreads();
  }
  if (trans && lane == 0)
    for (int i = n - 1; i >= 0; --i) {
      const int p = piv[i];
      if (p != i) { const double t = xw[i]; xw[i] = xw[p]; xw[p] = t; }
    }
  __syncthreads();
  for (int k = lane; k < n; k += 64) b[(int64_t)k * ldb] = xw[k];
}

// ------------------------------------------------------------------- QR
// Householder reflectors H_j = I - tau_j v_j v_j^T with v_j(j) = 1, stored
// below the diagonal; then Q is formed in place by backward accumulation.
__global__ void __launch_bounds__(BS) k_qr(double* A, int m, int n, int lda, double* R, int ldr,
                                           double* tau) {
  __shared__ double red[NW];
  __shared__ double s_tau, s_alpha;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = 0; j < n; ++j) {
    double* aj = A + (size_t)j * lda;
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += BS) part += aj[i] * aj[i];
    const double tail = block_sum(part, red);
    if (tid == 0) {
      const double x0 = aj[j];
      const double nrm = sqrt(x0 * x0 + tail);
      if (tail == 0.0) {              // already upper triangular in this column
        s_tau = 0.0;
        s_alpha = x0;
      } else {
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        s_tau = (alpha - x0) / alpha;
        s_alpha = alpha;
        aj[j] = x0 - alpha;          // scaled below to make v(j) = 1
      }
    }
    __syncthreads();
    const double tj = s_tau;
    if (tj != 0.0) {
      const double v0 = aj[j];
      for (int i = j + 1 + tid; i < m; i += BS) aj[i] /= v0;
    }
    __syncthreads();
    if (tid == 0) { aj[j] = s_alpha; tau[j] = tj; }
    __syncthreads();
    if (tj != 0.0) {
      for (int c = j + 1 + w; c < n; c += NW) {   // one wave per trailing column
        double* ac = A + (size_t)c * lda;
        double dot = (lane == 0) ? ac[j] : 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) dot += aj[i] * ac[i];
        dot = wave_sum(dot) * tj;
        if (lane == 0) ac[j] -= dot;
        for (int i = j + 1 + lane; i < m; i += 64) ac[i] -= dot * aj[i];
      }
    }
    __syncthreads();
  }
  // R (upper triangle)
  for (int e = tid; e < n * n; e += BS) {
    const int i = e % n, c = e / n;
    R[i + (size_t)c * ldr] = (i <= c) ? A[i + (size_t)c * lda] : 0.0;
  }
  __syncthreads();
  // Q = H_0 ... H_{n-1} [I; 0], in place
  for (int j = n - 1; j >= 0; --j) {
    double* aj = A + (size_t)j * lda;
    const double tj = tau[j];
    if (j < n - 1) {
      if (tid == 0) aj[j] = 1.0;
      __syncthreads();
      for (int c = j + 1 + w; c < n; c += NW) {
        double* ac = A + (size_t)c * lda;
        double dot = 0.0;
        for (int i = j + lane; i < m; i += 64) dot += aj[i] * ac[i];
        dot = wave_sum(dot) * tj;
        for (int i = j + lane; i < m; i += 64) ac[i] -= dot * aj[i];
      }
      __syncthreads();
    }
    for (int i = j + 1 + tid; i < m; i += BS) aj[i] *= -tj;
    for (int i = tid; i < j; i += BS) aj[i] = 0.0;
    __syncthreads();
    if (tid == 0) aj[j] = 1.0 - tj;
    __syncthreads();
  }
}

// --------------------------------------------------- blocked Householder QR
// Panel factorisation (unblocked, one workgroup) of an m x jb panel: reflectors
// with v(j) = 1 below the diagonal, R's diagonal on it, tau out.
__global__ void __launch_bounds__(BS) k_qr_panel(double* A, int m, int jb, int lda, double* tau) {
  __shared__ double red[NW];
  __shared__ double s_tau, s_alpha;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = 0; j < jb && j < m; ++j) {
    double* aj = A + (size_t)j * lda;
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += BS) part += aj[i] * aj[i];
    const double tail = block_sum(part, red);
    if (tid == 0) {
      const double x0 = aj[j];
      const double nrm = sqrt(x0 * x0 + tail);
      if (tail == 0.0) {
        s_tau = 0.0;
        s_alpha = x0;
      } else {
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        s_tau = (alpha - x0) / alpha;
        s_alpha = alpha;
        aj[j] = x0 - alpha;
      }
    }
    __syncthreads();
    const double tj = s_tau;
    if (tj != 0.0) {
      const double v0 = aj[j];
      for (int i = j + 1 + tid; i < m; i += BS) aj[i] /= v0;
    }
    __syncthreads();
    if (tid == 0) { aj[j] = s_alpha; tau[j] = tj; }
    __syncthreads();
    if (tj != 0.0)
      for (int c = j + 1 + w; c < jb; c += NW) {
        double* ac = A + (size_t)c * lda;
        double dot = (lane == 0) ? ac[j] : 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) dot += aj[i] * ac[i];
        dot = wave_sum(dot) * tj;
        if (lane == 0) ac[j] -= dot;
        for (int i = j + 1 + lane; i < m; i += 64) ac[i] -= dot * aj[i];
      }
    __syncthreads();
  }
}

// V (m x jb, explicit): unit diagonal, reflectors below, zeros above.
__global__ void k_build_v(const double* A, int m, int jb, int lda, double* V, size_t sA, size_t sV) {
  A += blockIdx.y * sA;
  V += blockIdx.y * sV;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * jb) return;
  const int i = (int)(e % m), q = (int)(e / m);
  V[e] = (i == q) ? 1.0 : (i > q ? A[i + (size_t)q * lda] : 0.0);
}

// T (jb x jb upper) with H_0 ... H_{jb-1} = I - V T V^T (forward, columnwise).
__global__ void __launch_bounds__(BS) k_larft(const double* V, int m, int jb, const double* tau, double* T) {
  __shared__ double G[16][16];
  __shared__ double Ts[16][16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // G = V^T V (upper part)
  for (int pq = w; pq < jb * jb; pq += NW) {
    const int p = pq / jb, q = pq % jb;
    if (p > q) continue;
    double sdot = 0.0;
    for (int i = lane; i < m; i += 64) sdot += V[i + (size_t)p * m] * V[i + (size_t)q * m];
    sdot = wave_sum(sdot);
    if (lane == 0) G[p][q] = sdot;
  }
  __syncthreads();
  // column i of T from columns < i: T[r][i] = -tau_i sum_{r <= q < i} T[r][q] G[q][i]
  // for r < i, tau_i on the diagonal; rows in parallel
  for (int i = 0; i < jb; ++i) {
    if (tid < jb) {
      const int r = tid;
      double v = 0.0;
      if (r < i) {
        double acc = 0.0;
        for (int q = r; q < i; ++q) acc += Ts[r][q] * G[q][i];
        v = -tau[i] * acc;
      } else if (r == i) {
        v = tau[i];
      }
      Ts[r][i] = v;
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += BS) T[e % jb + (e / jb) * jb] = Ts[e % jb][e / jb];
}

// Register-resident panel factorisation for panels of at most PBT * RPT rows
// and 16 columns, PBT threads: thread t holds rows t + k PBT (k < RPT) of
// every column.
// Per column j, one block reduction (through LDS, no lane shuffles) of the
// sixteen sums D_c = sum_{i > j} a_j(i) a_c(i): D_j is the squared norm
// below the diagonal, and with the reflector v_j = e_j + s a_j(below j),
// s = 1 / (x0 - alpha), every other product follows without a second pass,
// v_j^T a_c = a_c(j) + s D_c: for c > j the update of the trailing panel
// columns, for c < j (a_c below row c holds v_c) the product v_c^T v_j, from
// which column j of T (H_0 ... H_{jb-1} = I - V T V^T) follows by the
// forward recurrence T(r, j) = -tau_j sum_{r <= q < j} T(r, q) v_q^T v_j.
// Row j of the panel (before H_j) comes from the thread that holds it.
// Writes the reflectors below the diagonal of the panel (unit diagonal
// implicit), R on and above it, tau, V explicit (mm x jb) and T (jb x jb).
constexpr int PB = 256;
// Batched (TSQR): blockIdx.y picks the matrix; A, tau, V and T are offset by
// their strides (0 for a single matrix).
template <int RPT, int PBT>
__global__ void __launch_bounds__(PBT) k_qr_panel_reg(double* A, int mm, int jb, int lda, double* tau, double* V,
                                                     double* T, size_t sA, size_t sTau, size_t sV, size_t sT) {
  A += blockIdx.y * sA;
  tau += blockIdx.y * sTau;
  V += blockIdx.y * sV;
  T += blockIdx.y * sT;
  constexpr int NB = 16, S = PBT / NB;   // S strips per column in the first reduction stage
  // block sums through LDS: every thread's partials in P (conflict-free
  // columns), then S partial sums per column in Q, then the sums in D
  __shared__ double P[NB][PBT], Q[NB][S];
  __shared__ double D[NB], rowj[2][NB], Ts[NB][NB];
  const int tid = threadIdx.x;
  const int rc = tid / S, rj = tid % S;   // (column, strip) of the first reduction stage
  double a[RPT][NB];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * PBT;
#pragma unroll
    for (int c = 0; c < NB; ++c) a[k][c] = (i < mm && c < jb) ? A[i + (size_t)c * lda] : 0.0;
  }
#pragma clang loop unroll(full)
  for (int j = 0; j < NB; ++j) {
    if (j >= jb) continue;   // uniform; the loop is fully unrolled (constant j)
    // row j (thread j) and every thread's partials of D_c over its rows below j
    if (tid == j)
#pragma unroll
      for (int c = 0; c < NB; ++c) rowj[j & 1][c] = a[0][c];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double part = 0.0;
      if (c < jb) {
#pragma unroll
        for (int k = 0; k < RPT; ++k)
          if (tid + k * PBT > j) part += a[k][j] * a[k][c];
      }
      P[c][tid] = part;
    }
    __syncthreads();
    {
      double sum = 0.0;
#pragma unroll
      for (int u = 0; u < PBT / S; ++u) sum += P[rc][u * S + rj];
      Q[rc][rj] = sum;
    }
    __syncthreads();
    if (tid < NB) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < S; ++q) sum += Q[tid][q];
      D[tid] = sum;
    }
    __syncthreads();
    const double tail = D[j], x0 = rowj[j & 1][j];
    double tj = 0.0, alpha = x0, scale = 0.0;
    if (tail != 0.0) {
      const double nrm = sqrt(x0 * x0 + tail);
      alpha = x0 >= 0.0 ? -nrm : nrm;
      tj = (alpha - x0) / alpha;
      scale = 1.0 / (x0 - alpha);
    }
    double sd[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) sd[c] = rowj[j & 1][c] + scale * D[c];
    // v_j: 1 at row j, the scaled column below it
    double v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * PBT;
      if (i > j && tj != 0.0) a[k][j] *= scale;
      v[k] = (i > j) ? a[k][j] : (i == j ? 1.0 : 0.0);
    }
    // apply H_j to the later columns; column j of T from the earlier ones
#pragma unroll
    for (int c = j + 1; c < NB; ++c) {
      if (c < jb) {
        const double f = tj * sd[c];
#pragma unroll
        for (int k = 0; k < RPT; ++k) a[k][c] -= f * v[k];
      }
    }
    if (tid < NB) {
      double t = 0.0;
      if (tid < j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q >= tid && q < j) acc += Ts[tid][q] * sd[q];
        t = -tj * acc;
      } else if (tid == j) {
        t = tj;
      }
      Ts[tid][j] = t;
    }
    if (tid == j) a[0][j] = alpha;   // R's diagonal entry
    if (tid == 0) tau[j] = tj;
    // (the next column's first barrier orders Ts, D and rowj: T's column j is
    // read only from the next column's recurrence on, after that barrier;
    // D is rewritten only after two more; rowj alternates by parity)
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * PBT;
    if (i < mm)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < jb) {
          A[i + (size_t)c * lda] = a[k][c];
          V[i + (size_t)c * mm] = (i > c) ? a[k][c] : (i == c ? 1.0 : 0.0);
        }
  }
  for (int e = tid; e < jb * jb; e += PBT) T[e % jb + (e / jb) * jb] = Ts[e % jb][e / jb];
}

// Launches the register panel for mm <= 16 PB rows; false if the panel is taller.
// Above 4 PB rows the panel takes 2 PB threads, four rows each (eight rows of
// sixteen columns per thread spill, slower at these heights); below, PB
// threads are faster (the block reductions dominate).  Above 8 PB rows, 2 PB
// threads of eight rows: the spills cost less than the single-workgroup
// panel without registers that those heights used before.
bool qr_panel_reg(double* A, int mm, int jb, int lda, double* tau, double* V, double* T, hipStream_t st,
                  int batch = 1, size_t sA = 0, size_t sTau = 0, size_t sV = 0, size_t sT = 0) {
  const dim3 g(1, batch);
  if (mm <= PB)
    hipLaunchKernelGGL((k_qr_panel_reg<1, PB>), g, dim3(PB), 0, st, A, mm, jb, lda, tau, V, T, sA, sTau, sV, sT);
  else if (mm <= 2 * PB)
    hipLaunchKernelGGL((k_qr_panel_reg<2, PB>), g, dim3(PB), 0, st, A, mm, jb, lda, tau, V, T, sA, sTau, sV, sT);
  else if (mm <= 4 * PB)
    hipLaunchKernelGGL((k_qr_panel_reg<4, PB>), g, dim3(PB), 0, st, A, mm, jb, lda, tau, V, T, sA, sTau, sV, sT);
  else if (mm <= 8 * PB)
    hipLaunchKernelGGL((k_qr_panel_reg<4, 2 * PB>), g, dim3(2 * PB), 0, st, A, mm, jb, lda, tau, V, T, sA, sTau, sV,
                       sT);
  else if (mm <= 16 * PB)   // (the rounding's unfoldings of 16 x 255 rows)
    hipLaunchKernelGGL((k_qr_panel_reg<8, 2 * PB>), g, dim3(2 * PB), 0, st, A, mm, jb, lda, tau, V, T, sA, sTau, sV,
                       sT);
  else
    return false;
  return true;
}

typedef double qdbl4 __attribute__((ext_vector_type(4)));

// C <- (I - V op(T) V^T) C for one panel of the blocked QR: V (mm x jb,
// explicit, ld mm), T (jb x jb, ld jb), op(T) = T^T (trans = 1: applying Q^T
// to the trailing matrix) or T (trans = 0: forming Q).  One block per 16
// columns of C, so the three products need no grid-wide ordering:
// W = V^T C (FP64 MFMA v_mfma_f64_16x16x4, the long dimension split over the
// sixteen waves, eight steps of loads in flight), W2 = op(T) W in LDS, and
// C -= V W2 by 16-row tiles (A at [l % 16][l / 16], B at [l / 16][l % 16],
// D row l / 16 + 4 v, column l % 16 in lane l, slot v).
// Batched (TSQR): blockIdx.y picks the matrix, V, T and C offset by their
// strides (0 for one matrix).
constexpr int QAW = 16;   // waves of k_qr_apply
__global__ void __launch_bounds__(QAW * 64) k_qr_apply(const double* V, int mm, int jb, const double* T, int trans,
                                                        double* C, int nc, int lda, size_t sV, size_t sT, size_t sC) {
  V += blockIdx.y * sV;
  T += blockIdx.y * sT;
  C += blockIdx.y * sC;
  constexpr int SBQ = 8;
  __shared__ double Wp[QAW][16][17], W2[16][17];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int c = blockIdx.x * 16 + li;
  const bool cok = c < nc, pok = li < jb;
  const int nst = (mm + 3) / 4;
  qdbl4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = wv * SBQ; s0 < nst; s0 += QAW * SBQ) {
    double a[SBQ], b[SBQ];
#pragma unroll
    for (int u = 0; u < SBQ; ++u) {
      const int i = 4 * (s0 + u) + lk;
      const bool ok = i < mm;
      a[u] = (ok && pok) ? V[i + (size_t)li * mm] : 0.0;
      b[u] = (ok && cok) ? C[i + (size_t)c * lda] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SBQ; ++u)
      if (s0 + u < nst) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Wp[wv][lk + 4 * v][li] = acc[v];
  __syncthreads();
  if (tid < 256) {
    const int p = tid >> 4, cc = tid & 15;
    double sum = 0.0;
    for (int w = 0; w < QAW; ++w) sum += Wp[w][p][cc];
    Wp[0][p][cc] = sum;
  }
  __syncthreads();
  if (tid < 256) {
    const int p = tid >> 4, cc = tid & 15;
    double sum = 0.0;
    if (p < jb)
      for (int q = 0; q < jb; ++q) sum += (trans ? T[q + p * jb] : T[p + q * jb]) * Wp[0][q][cc];
    W2[p][cc] = sum;
  }
  __syncthreads();
  // C -= V W2, two row tiles per wave at a time (their loads in flight together)
  const int ntile = (mm + 15) / 16;
  for (int rt = wv; rt < ntile; rt += 2 * QAW) {
    double av[2][4], cv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = rt + h * QAW;
      const int r = t * 16 + li;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int q = 4 * st + lk;
        av[h][st] = (t < ntile && r < mm && q < jb) ? V[r + (size_t)q * mm] : 0.0;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = t * 16 + lk + 4 * v;
        cv[h][v] = (t < ntile && row < mm && cok) ? C[row + (size_t)c * lda] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = rt + h * QAW;
      qdbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < 4; ++st) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][st], W2[4 * st + lk][li], d, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = t * 16 + lk + 4 * v;
        if (t < ntile && row < mm && cok) C[row + (size_t)c * lda] = cv[h][v] - d[v];
      }
    }
  }
}

// The same product split over row chunks of QRC rows as well as column tiles,
// for tall panels, where one block per 16 columns leaves the chip idle:
// k_qr_apply_w writes each chunk's W partial (V[chunk]^T C[chunk], 16 x 16,
// FP64 MFMA as above), k_qr_apply_sum folds the partials of a tile in chunk
// order when there are many, and k_qr_apply_c sums what is left in chunk
// order, forms W2 = op(T) W and updates its chunk, C -= V W2.  Partials
// live at Wp[(chunk * tiles + tile) * 256 + row * 16 + col].
constexpr int QRC = 128;   // rows per chunk
constexpr int QSW = 4;     // waves per block (QRC / 4 / QSW k-steps of four rows each)
constexpr int QSUM = 16;   // the update sums at most this many partials itself
static_assert(QSW * 64 == 256, "a thread per entry of the 16 x 16 products");
// (RC: rows per chunk, QRC by default; the batched tall-skinny QR takes
// 4 QRC, so a 2048-row block is 4 chunks and the grid four times smaller)
template <int RC = QRC>
__global__ void __launch_bounds__(QSW * 64) k_qr_apply_w(const double* V, int mm, int jb, const double* C, int nc,
                                                          int lda, double* Wp, size_t sV, size_t sC, size_t sW) {
  V += blockIdx.z * sV;   // (batched: blockIdx.z picks the matrix)
  C += blockIdx.z * sC;
  Wp += blockIdx.z * sW;
  constexpr int STEPS = RC / 4 / QSW;
  __shared__ double Ws[QSW][16][17];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = blockIdx.x, ch = blockIdx.y;
  const int c = ct * 16 + li;
  const bool cok = c < nc, pok = li < jb;
  const int r0 = ch * RC + wv * (RC / QSW);
  double a[STEPS], b[STEPS];
#pragma unroll
  for (int u = 0; u < STEPS; ++u) {
    const int i = r0 + 4 * u + lk;
    const bool ok = i < mm;
    a[u] = (ok && pok) ? V[i + (size_t)li * mm] : 0.0;
    b[u] = (ok && cok) ? C[i + (size_t)c * lda] : 0.0;
  }
  qdbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < STEPS; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) Ws[wv][lk + 4 * v][li] = acc[v];
  __syncthreads();
  double sum = 0.0;
#pragma unroll
  for (int w = 0; w < QSW; ++w) sum += Ws[w][tid >> 4][tid & 15];
  Wp[((size_t)ch * gridDim.x + ct) * 256 + tid] = sum;
}

// Sum of a tile's nch partials in chunk order, into chunk 0's slot (each
// thread reads and writes its own entry only; batched: blockIdx.y picks the
// matrix, its partials at Wp + b sW).
__global__ void __launch_bounds__(256) k_qr_apply_sum(double* Wp, int nch, int tiles, size_t sW = 0) {
  Wp += blockIdx.y * sW;
  const int ct = blockIdx.x, e = threadIdx.x;
  double sum = 0.0;
  for (int r = 0; r < nch; ++r) sum += Wp[((size_t)r * tiles + ct) * 256 + e];
  Wp[(size_t)ct * 256 + e] = sum;
}

template <int RC = QRC>
__global__ void __launch_bounds__(QSW * 64) k_qr_apply_c(const double* V, int mm, int jb, const double* T, int trans,
                                                          double* C, int nc, int lda, const double* Wp, int nparts,
                                                          size_t sV, size_t sT, size_t sC, size_t sW) {
  V += blockIdx.z * sV;   // (batched: blockIdx.z picks the matrix)
  T += blockIdx.z * sT;
  C += blockIdx.z * sC;
  Wp += blockIdx.z * sW;
  __shared__ double W[16][17], W2[16][17];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = blockIdx.x, ch = blockIdx.y;
  const int c = ct * 16 + li;
  const bool cok = c < nc;
  {
    double sum = 0.0;
    for (int r = 0; r < nparts; ++r) sum += Wp[((size_t)r * gridDim.x + ct) * 256 + tid];
    W[tid >> 4][tid & 15] = sum;
  }
  __syncthreads();
  {
    const int pr = tid >> 4, cc = tid & 15;
    double sum = 0.0;
    if (pr < jb)
      for (int q = 0; q < jb; ++q) sum += (trans ? T[q + pr * jb] : T[pr + q * jb]) * W[q][cc];
    W2[pr][cc] = sum;
  }
  __syncthreads();
  // the chunk's RC / 16 row tiles, RC / 16 / QSW per wave with their loads in flight together
  constexpr int TPW = RC / 16 / QSW;
  double av[TPW][4], cv[TPW][4];
#pragma unroll
  for (int h = 0; h < TPW; ++h) {
    const int t0 = ch * RC + (wv * TPW + h) * 16;
    const int r = t0 + li;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int q = 4 * st + lk;
      av[h][st] = (r < mm && q < jb) ? V[r + (size_t)q * mm] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = t0 + lk + 4 * v;
      cv[h][v] = (row < mm && cok) ? C[row + (size_t)c * lda] : 0.0;
    }
  }
#pragma unroll
  for (int h = 0; h < TPW; ++h) {
    const int t0 = ch * RC + (wv * TPW + h) * 16;
    qdbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 4; ++st) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][st], W2[4 * st + lk][li], d, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = t0 + lk + 4 * v;
      if (row < mm && cok) C[row + (size_t)c * lda] = cv[h][v] - d[v];
    }
  }
}

// C <- (I - V op(T) V^T) C: one block per 16 columns for short panels, the
// row-split kernels (partials in Wp) for tall ones.
void qr_apply(const double* V, int mm, int jb, const double* T, int trans, double* C, int nc, int lda, double* Wp,
              hipStream_t st) {
  const int tiles = (nc + 15) / 16;
  if (mm <= 4 * QRC) {
    hipLaunchKernelGGL(k_qr_apply, dim3(tiles), dim3(QAW * 64), 0, st, V, mm, jb, T, trans, C, nc, lda, (size_t)0,
                       (size_t)0, (size_t)0);
    return;
  }
  const int nch = (mm + QRC - 1) / QRC;
  hipLaunchKernelGGL(k_qr_apply_w<QRC>, dim3(tiles, nch), dim3(QSW * 64), 0, st, V, mm, jb, (const double*)C, nc, lda, Wp,
                     (size_t)0, (size_t)0, (size_t)0);
  int nparts = nch;
  if (nch > QSUM) {
    hipLaunchKernelGGL(k_qr_apply_sum, dim3(tiles), dim3(256), 0, st, Wp, nch, tiles, (size_t)0);
    nparts = 1;
  }
  hipLaunchKernelGGL(k_qr_apply_c<QRC>, dim3(tiles, nch), dim3(QSW * 64), 0, st, V, mm, jb, T, trans, C, nc, lda,
                     (const double*)Wp, nparts, (size_t)0, (size_t)0, (size_t)0, (size_t)0);
}

// Columns of Q for one panel from its reflectors (backward accumulation, as
// k_qr_panel_q), register-resident like k_qr_panel_reg: for j = jb-1 .. 0 the
// products v_j^T q_c with the already formed columns c > j are one block
// reduction through LDS, then q_c -= tau_j (v_j^T q_c) v_j and column j
// becomes H_j e_j.
template <int RPT, int PBT>
__global__ void __launch_bounds__(PBT) k_qr_panel_q_reg(double* A, int mm, int jb, int lda, const double* tau) {
  constexpr int NB = 16, S = PBT / NB;
  __shared__ double P[NB][PBT], Q[NB][S];
  __shared__ double sd[NB];
  const int tid = threadIdx.x;
  const int rc = tid / S, rj = tid % S;
  double a[RPT][NB];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * PBT;
#pragma unroll
    for (int c = 0; c < NB; ++c) a[k][c] = (i < mm && c < jb) ? A[i + (size_t)c * lda] : 0.0;
  }
#pragma clang loop unroll(full)
  for (int j = NB - 1; j >= 0; --j) {
    if (j >= jb) continue;   // uniform; the loop is fully unrolled (constant j)
    const double tj = tau[j];
    double v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * PBT;
      v[k] = (i > j) ? a[k][j] : (i == j ? 1.0 : 0.0);
    }
    if (j < jb - 1) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double sum = 0.0;
        if (c > j && c < jb)
#pragma unroll
          for (int k = 0; k < RPT; ++k) sum += v[k] * a[k][c];
        P[c][tid] = sum;
      }
      __syncthreads();
      {
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < PBT / S; ++u) sum += P[rc][u * S + rj];
        Q[rc][rj] = sum;
      }
      __syncthreads();
      if (tid < NB) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) sum += Q[tid][q];
        sd[tid] = sum;
      }
      __syncthreads();
#pragma unroll
      for (int c = j + 1; c < NB; ++c) {
        if (c < jb) {
          const double f = tj * sd[c];
#pragma unroll
          for (int k = 0; k < RPT; ++k) a[k][c] -= f * v[k];
        }
      }
      __syncthreads();   // sd is read by every thread before the next column writes P
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * PBT;
      a[k][j] = (i > j) ? -tj * v[k] : (i == j ? 1.0 - tj : 0.0);
    }
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * PBT;
    if (i < mm)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < jb) A[i + (size_t)c * lda] = a[k][c];
  }
}

// Launches the register form of the panel's Q for mm <= 8 PB rows; false otherwise.
bool qr_panel_q_reg(double* A, int mm, int jb, int lda, const double* tau, hipStream_t st) {
  if (mm <= PB)
    hipLaunchKernelGGL((k_qr_panel_q_reg<1, PB>), dim3(1), dim3(PB), 0, st, A, mm, jb, lda, tau);
  else if (mm <= 2 * PB)
    hipLaunchKernelGGL((k_qr_panel_q_reg<2, PB>), dim3(1), dim3(PB), 0, st, A, mm, jb, lda, tau);
  else if (mm <= 4 * PB)
    hipLaunchKernelGGL((k_qr_panel_q_reg<4, PB>), dim3(1), dim3(PB), 0, st, A, mm, jb, lda, tau);
  else if (mm <= 8 * PB)
    hipLaunchKernelGGL((k_qr_panel_q_reg<8, PB>), dim3(1), dim3(PB), 0, st, A, mm, jb, lda, tau);
  else if (mm <= 16 * PB)
    hipLaunchKernelGGL((k_qr_panel_q_reg<8, 2 * PB>), dim3(1), dim3(2 * PB), 0, st, A, mm, jb, lda, tau);
  else
    return false;
  return true;
}

// Columns of Q for one panel from its reflectors (backward accumulation), in place.
__global__ void __launch_bounds__(BS) k_qr_panel_q(double* A, int m, int jb, int lda, const double* tau) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = jb - 1; j >= 0; --j) {
    double* aj = A + (size_t)j * lda;
    const double tj = tau[j];
    if (j < jb - 1) {
      if (tid == 0) aj[j] = 1.0;
      __syncthreads();
      for (int c = j + 1 + w; c < jb; c += NW) {
        double* ac = A + (size_t)c * lda;
        double dot = 0.0;
        for (int i = j + lane; i < m; i += 64) dot += aj[i] * ac[i];
        dot = wave_sum(dot) * tj;
        for (int i = j + lane; i < m; i += 64) ac[i] -= dot * aj[i];
      }
      __syncthreads();
    }
    for (int i = j + 1 + tid; i < m; i += BS) aj[i] *= -tj;
    for (int i = tid; i < j; i += BS) aj[i] = 0.0;
    __syncthreads();
    if (tid == 0) aj[j] = 1.0 - tj;
    __syncthreads();
  }
}

__global__ void k_extract_r(const double* A, int n, int lda, double* R, int ldr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e % n, c = e / n;
  R[i + (size_t)c * ldr] = (i <= c) ? A[i + (size_t)c * lda] : 0.0;
}

__global__ void k_zero_rows(double* A, int rows, int cols, int lda) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  A[e % rows + (size_t)(e / rows) * lda] = 0.0;
}

// The rotation of a one-sided Jacobi step on columns (x, y) with squared
// norms al, be and inner product ga: the angle that zeroes the rotated pair's
// inner product, cot(2 theta) = (be - al) / (2 ga), taking the smaller root.
// With d = be - al, g = 2 ga, h = sqrt(d^2 + g^2) and w = |d| + h, the
// tangent is t = +-|g| / w and 1 + t^2 = 2h / w, so
//   c = w / sqrt(2 h w),  s = +-|g| / sqrt(2 h w)
// (one square root and one reciprocal square root on the dependent chain
// instead of two divisions and two roots).  The sign is that of d / g, +1 at
// d = 0.  d^2 and g^2 are fourth powers of the entries, far from overflow for
// the matrices here, as the convergence tests already assume.
__device__ inline void jacobi_rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g = 2.0 * ga;
  const double h = sqrt(d * d + g * g);
  const double w = fabs(d) + h;
  const double q = rsqrt(2.0 * h * w);
  c = w * q;
  s = (d == 0.0 || (d > 0.0) == (g > 0.0) ? 1.0 : -1.0) * fabs(g) * q;
}

// Singular values (column norms), normalised left vectors, columns sorted
// by decreasing sigma (stable in the column index); whole workgroup.
__device__ void jacobi_finish(double* A, int n, int lda, double* V, int ldv, double* sigma, double* work,
                              int32_t* order) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int c = w; c < n; c += NW) {
    double* ac = A + (size_t)c * lda;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += ac[i] * ac[i];
    s = sqrt(wave_sum(s));
    if (lane == 0) sigma[c] = s;
    if (s > 0.0)
      for (int i = lane; i < n; i += 64) ac[i] /= s;
  }
  __syncthreads();
  // order by decreasing sigma (stable in the column index)
  for (int c = tid; c < n; c += BS) {
    int rank = 0;
    const double sc = sigma[c];
    for (int o = 0; o < n; ++o) {
      const double so = sigma[o];
      if (so > sc || (so == sc && o < c)) ++rank;
    }
    order[rank] = c;
  }
  __syncthreads();
  double* tmp = work;  // n x n + n
  for (int e = tid; e < n * n; e += BS) tmp[e] = A[e % n + (size_t)order[e / n] * lda];
  __syncthreads();
  for (int e = tid; e < n * n; e += BS) A[e % n + (size_t)(e / n) * lda] = tmp[e];
  __syncthreads();
  if (V) {
    for (int e = tid; e < n * n; e += BS) tmp[e] = V[e % n + (size_t)order[e / n] * ldv];
    __syncthreads();
    for (int e = tid; e < n * n; e += BS) V[e % n + (size_t)(e / n) * ldv] = tmp[e];
  }
  for (int c = tid; c < n; c += BS) tmp[n * n + c] = sigma[order[c]];
  __syncthreads();
  for (int c = tid; c < n; c += BS) sigma[c] = tmp[n * n + c];
}

// ------------------------------------------------------------ Jacobi SVD
// One-sided (Hestenes) Jacobi on the columns of A (n x n): A V = U Sigma.
// Pairs follow a round-robin tournament so each round's rotations are
// disjoint; one wave per pair.
// Stopping: a pair rotates while its cosine |ga| / sqrt(al be) exceeds 1e-15.
// Cyclic Jacobi converges quadratically in the end, so after a sweep whose
// largest cosine stayed below JACOBI_LAST the cosines are of order its square
// (1e-12) or smaller, and the sweep that would follow rotates nothing or
// nearly nothing: rotations that small move the singular values at second
// order (1e-24 relative) and the columns' orthogonality at 1e-12.  The
// iteration stops after such a sweep instead of running that one.
constexpr double JACOBI_LAST = 1e-6;
__global__ void __launch_bounds__(BS) k_jacobi(double* A, int n, int lda, double* V, int ldv,
                                               double* sigma, size_t sA, size_t sV, size_t sS) {
  __shared__ int rotated, large;
  // one matrix per workgroup: A, V, sigma (+ its workspace) offset by the batch index
  A += blockIdx.x * sA;
  V += blockIdx.x * sV;
  sigma += blockIdx.x * sS;
  double* work = sigma + n;
  int32_t* order = reinterpret_cast<int32_t*>(work + (size_t)n * n + n);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < n * n; e += BS) V[e % n + (size_t)(e / n) * ldv] = (e % n == e / n) ? 1.0 : 0.0;
  const int np = (n + 1) & ~1;    // players, one dummy when n is odd
  // ||A||_F^2 (invariant under the rotations): pairs whose inner product is
  // below eps^2 of it are converged whatever their own norms, so columns at
  // rounding-noise level stop rotating among themselves
  __shared__ double red_nf[NW];
  double nf = 0.0;
  for (int e = tid; e < n * n; e += BS) {
    const double a = A[e % n + (size_t)(e / n) * lda];
    nf += a * a;
  }
  const double gfloor = 1e-30 * block_sum(nf, red_nf);
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = large = 0;
    __syncthreads();
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      for (int pr = w; pr < np / 2; pr += NW) {
        // circle method: player 0 fixed, others rotate
        int p = (pr == 0) ? 0 : 1 + (pr - 1 + rnd) % (np - 1);
        int q = 1 + (np - 2 - pr + rnd) % (np - 1);
        if (p > q) { const int t = p; p = q; q = t; }
        if (q >= n || p == q) continue;
        double* ap = A + (size_t)p * lda;
        double* aq = A + (size_t)q * lda;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < n; i += 64) {
          al += ap[i] * ap[i];
          be += aq[i] * aq[i];
          ga += ap[i] * aq[i];
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (fabs(ga) <= 1e-15 * sqrt(al * be) || fabs(ga) <= gfloor || ga == 0.0) continue;
        double c, s;
        jacobi_rotation(al, be, ga, c, s);
        for (int i = lane; i < n; i += 64) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = V + (size_t)p * ldv;
        double* vq = V + (size_t)q * ldv;
        for (int i = lane; i < n; i += 64) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
        if (lane == 0) {
          rotated = 1;
          if (fabs(ga) > JACOBI_LAST * sqrt(al * be)) large = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated || !large) break;
    __syncthreads();
  }
  jacobi_finish(A, n, lda, V, ldv, sigma, work, order);
}

// The same iteration with A in LDS: each round first rotates the column
// pairs of A in LDS and records the rotations, then all threads apply them to
// V in global memory in one parallel pass, so a round costs one global round
// trip instead of one per pair.  The rotations and their order are those of
// k_jacobi.  A pair is handled by G lanes (8 or 16), each holding E entries
// of both columns in registers (n <= G E): all of a lane's loads are issued
// at once (indices past n are clamped to n - 1, which rewrites that entry
// with the same value), so a round waits for LDS once before and once after
// the G-lane reductions.
template <int G>
__device__ inline double group_sum(double v) {
  return G == 8 ? row8_sum(v) : row16_sum(v);
}
template <int G, int E>
__global__ void __launch_bounds__(BS) k_jacobi_lds(double* Ag, int n, int lda, double* V, int ldv, double* sigma,
                                                   int want_v) {
  extern __shared__ double smj[];
  __shared__ int rotated, large;
  double* A = smj;                                  // n x n, leading dimension n
  const int np = (n + 1) & ~1;
  double* rc = A + (size_t)n * n;                   // np/2 cosines
  double* rs = rc + np / 2;                         // np/2 sines
  int* rp = reinterpret_cast<int*>(rs + np / 2);    // np/2 column pairs (p, q), p = -1: none
  int* rq = rp + np / 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double red_nf[NW];
  double nf = 0.0;
  for (int e = tid; e < n * n; e += BS) {
    const double a = Ag[e % n + (size_t)(e / n) * lda];
    A[e] = a;
    nf += a * a;
    if (want_v) V[e % n + (size_t)(e / n) * ldv] = (e % n == e / n) ? 1.0 : 0.0;
  }
  const double gfloor = 1e-30 * block_sum(nf, red_nf);   // as in k_jacobi
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = large = 0;
    __syncthreads();
    // a column pair per group of G lanes: a whole round of disjoint pairs
    // runs at once, with G-lane reductions
    const int grp = tid / G, gl = tid % G;
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      for (int pr = grp; pr < np / 2; pr += BS / G) {
        // the round-robin positions (both operands of the reduction are
        // below 2 (np - 1), so one conditional subtraction is the modulo)
        int p = 0;
        if (pr != 0) {
          const int x = pr - 1 + rnd;
          p = 1 + (x >= np - 1 ? x - (np - 1) : x);
        }
        const int y = np - 2 - pr + rnd;
        int q = 1 + (y >= np - 1 ? y - (np - 1) : y);
        if (p > q) { const int t = p; p = q; q = t; }
        int keep = 0;
        double c = 1.0, sn = 0.0;
        if (q < n && p != q) {
          double* ap = A + (size_t)p * n;
          double* aq = A + (size_t)q * n;
          double xv[E], yv[E];
#pragma unroll
          for (int u = 0; u < E; ++u) {
            const int i = min(gl + G * u, n - 1);
            xv[u] = ap[i];
            yv[u] = aq[i];
          }
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int u = 0; u < E; ++u) {   // (rows past n enter as zeros)
            const bool in = gl + G * u < n;
            const double x = in ? xv[u] : 0.0, y = in ? yv[u] : 0.0;
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
          al = group_sum<G>(al);
          be = group_sum<G>(be);
          ga = group_sum<G>(ga);
          // converged pair: |ga| <= 1e-15 sqrt(al be), compared squared (al,
          // be are squared column norms, far from the overflow range)
          if (!(ga * ga <= 1e-30 * (al * be) || fabs(ga) <= gfloor || ga == 0.0)) {
            jacobi_rotation(al, be, ga, c, sn);
#pragma unroll
            for (int u = 0; u < E; ++u) {
              const int i = min(gl + G * u, n - 1);
              ap[i] = c * xv[u] - sn * yv[u];
              aq[i] = sn * xv[u] + c * yv[u];
            }
            keep = 1;
            if (gl == 0) {
              rotated = 1;
              if (ga * ga > JACOBI_LAST * JACOBI_LAST * (al * be)) large = 1;
            }
          }
        }
        if (gl == 0) {
          rp[pr] = keep ? p : -1;
          rq[pr] = q;
          rc[pr] = c;
          rs[pr] = sn;
        }
      }
      __syncthreads();
      // V <- V G for this round's rotations (disjoint column pairs)
      const int npairs = want_v ? np / 2 : 0;
      for (int e = tid; e < npairs * n; e += BS) {
        const int pr = e / n, i = e % n;
        const int p = rp[pr];
        if (p < 0) continue;
        const int q = rq[pr];
        const double c = rc[pr], sn = rs[pr];
        double* vp = V + (size_t)p * ldv + i;
        double* vq = V + (size_t)q * ldv + i;
        const double x = *vp, y = *vq;
        *vp = c * x - sn * y;
        *vq = sn * x + c * y;
      }
      if (want_v) __syncthreads();
    }
    if (!rotated || !large) break;
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += BS) Ag[e % n + (size_t)(e / n) * lda] = A[e];
  __syncthreads();
  double* work = sigma + n;
  int32_t* order = reinterpret_cast<int32_t*>(work + (size_t)n * n + n);
  jacobi_finish(Ag, n, lda, want_v ? V : nullptr, ldv, sigma, work, order);
}

// Block form of the one-sided Jacobi iteration, for matrices whose n x n
// doubles do not fit one workgroup's LDS: the columns are split into blocks
// of JB_W, and the blocks meet in a round-robin tournament (the circle
// method over blocks, one dummy block when their number is odd).  Each
// meeting is one workgroup: it copies the 2 JB_W columns of its two blocks
// into LDS, runs one sweep of the column iteration over them (the circle
// method over the 2 JB_W columns, a pair per 32-lane group, rotations and
// convergence tests as in k_jacobi_lds), and writes them back.  A round of
// meetings is one launch; an outer sweep, in which every pair of columns
// meets at least once, is n_blocks - 1 launches followed by k_jb_check.
// The stopping rule is k_jacobi's, taken over the outer sweep: stop after a
// sweep with no rotation, or none whose cosine exceeded JACOBI_LAST.  The
// per-sweep flags and the squared Frobenius norm (the floor of the inner
// products) live past the workspace of jacobi_finish in sigma's buffer.
constexpr int JB_W = 16;    // columns per block
constexpr int JB_L = 32;    // lanes per column pair (E = ceil(n / 32) rows each)
constexpr int JB_T = JB_W * JB_L;   // threads: the JB_W pairs of 2 JB_W columns
__global__ void __launch_bounds__(BS) k_jb_init(const double* A, int n, int lda, double* aux, size_t sA, size_t sS) {
  A += blockIdx.x * sA;   // (batched: one matrix per workgroup)
  aux += blockIdx.x * sS;
  __shared__ double red[NW];
  double nf = 0.0;
  for (int e = threadIdx.x; e < n * n; e += BS) {
    const double a = A[e % n + (size_t)(e / n) * lda];
    nf += a * a;
  }
  nf = block_sum(nf, red);
  if (threadIdx.x == 0) {
    aux[0] = nf;
    int32_t* fl = reinterpret_cast<int32_t*>(aux + 1);
    fl[0] = fl[1] = fl[2] = 0;   // done, rotated, large
  }
}

__global__ void k_jb_check(double* aux, size_t sS) {
  aux += blockIdx.x * sS;
  int32_t* fl = reinterpret_cast<int32_t*>(aux + 1);
  if (threadIdx.x == 0) {
    if (!fl[1] || !fl[2]) fl[0] = 1;
    fl[1] = fl[2] = 0;
  }
}

// Whether every matrix of a batch has converged, as one int32 in the first
// matrix's spare aux word (aux[3]), so the host reads a single 4-byte word.
__global__ void __launch_bounds__(BS) k_jb_all_done(double* aux, size_t sS, int count) {
  int all = 1;
  for (int b = threadIdx.x; b < count; b += BS)
    all &= reinterpret_cast<const int32_t*>(aux + (size_t)b * sS + 1)[0] != 0;
  all = __syncthreads_and(all);
  if (threadIdx.x == 0) reinterpret_cast<int32_t*>(aux + 3)[0] = all;
}

template <int E>
__global__ void __launch_bounds__(JB_T) k_jacobi_block(double* A, int n, int lda, int nbp, int rnd, double* aux,
                                                        size_t sA, size_t sS) {
  A += blockIdx.y * sA;   // (batched: blockIdx.y picks the matrix, with its own flags)
  aux += blockIdx.y * sS;
  int32_t* fl = reinterpret_cast<int32_t*>(aux + 1);
  if (__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;   // converged
  constexpr int LDN = JB_L * E;    // LDS rows per column (n <= LDN)
  extern __shared__ double sj[];   // the 2 JB_W columns, leading dimension LDN
  __shared__ int s_rot, s_large;
  const int tid = threadIdx.x;
  if (tid == 0) s_rot = s_large = 0;
  // this workgroup's pair of blocks in round rnd
  int P = 0;
  if (blockIdx.x != 0) P = 1 + ((int)blockIdx.x - 1 + rnd) % (nbp - 1);
  int Q = 1 + (nbp - 2 - (int)blockIdx.x + rnd) % (nbp - 1);
  if (P > Q) { const int t = P; P = Q; Q = t; }
  const int nb = (n + JB_W - 1) / JB_W;
  auto gcol = [&](int c) {   // global column of local column c, -1 if none
    const int b = c < JB_W ? P : Q;
    const int g = b * JB_W + (c & (JB_W - 1));
    return (b < nb && g < n) ? g : -1;
  };
  {   // the 2 JB_W columns, each padded with zero rows to LDN: every load
      // issued before the first store, from clamped addresses with the
      // missing entries zeroed by a select (a copy loop of runtime length
      // waits for each load in turn)
    constexpr int CL = 2 * JB_W * LDN / JB_T;
    double v[CL];
#pragma unroll
    for (int u = 0; u < CL; ++u) {
      const int e = tid + u * JB_T;
      const int c = e / LDN, i = e - c * LDN;
      const int g = gcol(c);
      const double a = A[min(i, n - 1) + (size_t)max(g, 0) * lda];
      v[u] = (g >= 0 && i < n) ? a : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CL; ++u) sj[tid + u * JB_T] = v[u];
  }
  const double gfloor = 1e-30 * aux[0];
  __syncthreads();
  constexpr int NP = 2 * JB_W;
  const int grp = tid / JB_L, gl = tid % JB_L;
  int rot = 0, large = 0;
  for (int lr = 0; lr < NP - 1; ++lr) {
    int p = 0;
    if (grp != 0) {
      const int x = grp - 1 + lr;
      p = 1 + (x >= NP - 1 ? x - (NP - 1) : x);
    }
    const int y = NP - 2 - grp + lr;
    int q = 1 + (y >= NP - 1 ? y - (NP - 1) : y);
    if (p > q) { const int t = p; p = q; q = t; }
    if (gcol(p) >= 0 && gcol(q) >= 0) {
      double* ap = sj + p * LDN + gl;
      double* aq = sj + q * LDN + gl;
      double xv[E], yv[E];
#pragma unroll
      for (int u = 0; u < E; ++u) {
        xv[u] = ap[JB_L * u];
        yv[u] = aq[JB_L * u];
      }
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int u = 0; u < E; ++u) {   // (the padding rows are zeros and stay so)
        al = fma(xv[u], xv[u], al);
        be = fma(yv[u], yv[u], be);
        ga = fma(xv[u], yv[u], ga);
      }
      al = row32_sum(al);
      be = row32_sum(be);
      ga = row32_sum(ga);
      if (!(ga * ga <= 1e-30 * (al * be) || fabs(ga) <= gfloor || ga == 0.0)) {
        double c, sn;
        jacobi_rotation(al, be, ga, c, sn);
#pragma unroll
        for (int u = 0; u < E; ++u) {
          ap[JB_L * u] = c * xv[u] - sn * yv[u];
          aq[JB_L * u] = sn * xv[u] + c * yv[u];
        }
        rot = 1;
        if (ga * ga > JACOBI_LAST * JACOBI_LAST * (al * be)) large = 1;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2 * JB_W * LDN / JB_T; ++u) {
    const int e = tid + u * JB_T;
    const int c = e / LDN, i = e - c * LDN;
    const int g = gcol(c);
    if (g >= 0 && i < n) A[i + (size_t)g * lda] = sj[e];
  }
  if (rot) s_rot = 1;
  if (large) s_large = 1;
  __syncthreads();
  if (tid == 0) {
    if (s_rot) atomicOr(fl + 1, 1);
    if (s_large) atomicOr(fl + 2, 1);
  }
}

// Singular values, normalised left vectors and the ordering (jacobi_finish)
// of a matrix the block iteration has orthogonalised.
__global__ void __launch_bounds__(BS) k_jb_finish(double* A, int n, int lda, double* sigma, size_t sA, size_t sS) {
  A += blockIdx.x * sA;
  sigma += blockIdx.x * sS;
  double* work = sigma + n;
  int32_t* order = reinterpret_cast<int32_t*>(work + (size_t)n * n + n);
  jacobi_finish(A, n, lda, nullptr, 0, sigma, work, order);
}

// ----------------------------------------------------------------- GEMM
template <int TILE>
__global__ void k_gemm64(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda,
                         const double* B, int ldb, double beta, double* C, int ldc) {
  __shared__ double As[TILE][TILE + 1], Bs[TILE][TILE + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = blockIdx.x * TILE + tx, j = blockIdx.y * TILE + ty;
  double acc = 0.0;
  for (int k0 = 0; k0 < k; k0 += TILE) {
    // As[tx][ty] = op(A)(i, k0 + ty); Bs[tx][ty] = op(B)(k0 + tx, j)
    {
      const int kk = k0 + ty;
      double v = 0.0;
      if (i < m && kk < k) v = ta ? A[kk + (size_t)i * lda] : A[i + (size_t)kk * lda];
      As[tx][ty] = v;
    }
    {
      const int kk = k0 + tx;
      double v = 0.0;
      if (j < n && kk < k) v = tb ? B[j + (size_t)kk * ldb] : B[kk + (size_t)j * ldb];
      Bs[tx][ty] = v;
    }
    __syncthreads();
    for (int q = 0; q < TILE; ++q) acc += As[tx][q] * Bs[q][ty];
    __syncthreads();
  }
  if (i < m && j < n) {
    double* c = C + i + (size_t)j * ldc;
    *c = alpha * acc + (beta == 0.0 ? 0.0 : beta * *c);
  }
}

__global__ void k_nrm2(const double* x, int64_t n, double* out) {
  __shared__ double red[NW];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += BS) s += x[i] * x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = sqrt(s);
}

}  // namespace

void lu_factor(double* A, int n, int lda, int32_t* piv, int32_t* info, hipStream_t st) {
  // the matrix in LDS when it fits the workgroup's limit, else in global memory
  static int lds_limit = -1;
  if (lds_limit < 0) {
    int dev = 0, v = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      lds_limit = v;
    else
      lds_limit = 64 * 1024;
    (void)hipGetLastError();
  }
  const size_t sh = (size_t)n * n * sizeof(double);
  const size_t stat = 2 * NW * sizeof(double) + 64;   // static LDS of the kernel
  if (sh + stat <= (size_t)lds_limit) {
    bool ok = true;
    if (sh > 48 * 1024)
      ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lu_lds<256>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) == hipSuccess;
    if (ok) {
      hipLaunchKernelGGL(k_lu_lds<256>, dim3(1), dim3(256), sh, st, A, n, lda, piv, info);
      if (hipGetLastError() == hipSuccess) return;
    }
    (void)hipGetLastError();
  }
  hipLaunchKernelGGL(k_lu, dim3(1), dim3(BS), 0, st, A, n, lda, piv, info);
}

void lu_solve(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B, int ldb,
              int nrhs, hipStream_t st) {
  if (nrhs <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_lu_solve, dim3((nrhs + 63) / 64), dim3(64), 0, st, LU, n, lda, piv, trans, B, ldb,
                     nrhs);
}

void lu_solve_rm(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B, int64_t ldb,
                 int nrhs, hipStream_t st) {
  if (nrhs <= 0 || n <= 0) return;
  if (nrhs <= 8) {   // a handful of right-hand sides: one wave each
    hipLaunchKernelGGL(k_lu_solve_wave, dim3(nrhs), dim3(64), (size_t)n * sizeof(double), st, LU, n, lda, piv,
                       trans, B, ldb);
    return;
  }
  // 16 right-hand sides per workgroup (8 for the largest ranks, to stay
  // within 64 KB of LDS): enough workgroups to spread over the CUs
  if (n <= 248) {
    const size_t sh = (size_t)n * 16 * sizeof(double) + (size_t)16 * n * sizeof(double) + (size_t)n * sizeof(int);
    hipLaunchKernelGGL(k_lu_trsm<16>, dim3((nrhs + 15) / 16), dim3(256), sh, st, LU, n, lda, piv, trans, B, ldb,
                       nrhs);
  } else {
    const size_t sh = (size_t)n * 8 * sizeof(double) + (size_t)16 * n * sizeof(double) + (size_t)n * sizeof(int);
    hipLaunchKernelGGL(k_lu_trsm<8>, dim3((nrhs + 7) / 8), dim3(256), sh, st, LU, n, lda, piv, trans, B, ldb, nrhs);
  }
}

void qr_thin(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st) {
  hipLaunchKernelGGL(k_qr, dim3(1), dim3(BS), 0, st, A, m, n, lda, R, ldr, work);
}

// Blocked Householder QR, compact WY with panels of 16: the panel factors in
// one workgroup (registers when it has at most 2048 rows), the trailing update
// and the formation of Q are one qr_apply per panel.  qr_factor keeps the
// reflectors below the diagonal of A and the panels' T in work, for
// qr_blocked (Q formed in A) or qr_apply_q (Q applied to other columns).
namespace {
// The workspace of qr_blocked / qr_factor: tau (n), V (16 m), the panels' T
// (16 x 16 each), a spare 32 n + 64, then the row-split partials.
struct QrWork {
  double *tau, *V, *Tall, *Wp;
  QrWork(double* work, int m, int n) {
    tau = work;
    V = tau + n;
    Tall = V + (size_t)16 * m;
    Wp = Tall + (size_t)256 * ((n + 15) / 16) + 32 * (size_t)n + 64;
  }
};
}  // namespace

tt_status qr_factor(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st) {
  constexpr int NB = 16;
  if (m < n) return fail(TTK_ERR_ARG, "qr_factor needs m >= n");
  const QrWork w(work, m, n);
  const int npan = (n + NB - 1) / NB;
  for (int p = 0; p < npan; ++p) {
    const int j0 = p * NB, jb = std::min(NB, n - j0);
    const int mm = m - j0;
    double* Ap = A + j0 + (size_t)j0 * lda;
    double* T = w.Tall + (size_t)p * NB * NB;
    if (!qr_panel_reg(Ap, mm, jb, lda, w.tau + j0, w.V, T, st)) {
      hipLaunchKernelGGL(k_qr_panel, dim3(1), dim3(BS), 0, st, Ap, mm, jb, lda, w.tau + j0);
      hipLaunchKernelGGL(k_build_v, dim3((unsigned)(((int64_t)mm * jb + 255) / 256)), dim3(256), 0, st, Ap, mm, jb,
                         lda, w.V, (size_t)0, (size_t)0);
      hipLaunchKernelGGL(k_larft, dim3(1), dim3(BS), 0, st, w.V, mm, jb, w.tau + j0, T);
    }
    const int nc = n - j0 - jb;
    if (nc > 0) {
      double* A2 = A + j0 + (size_t)(j0 + jb) * lda;
      // A2 <- (I - V T^T V^T) A2
      qr_apply(w.V, mm, jb, T, 1, A2, nc, lda, w.Wp, st);
    }
  }
  hipLaunchKernelGGL(k_extract_r, dim3((n * n + 255) / 256), dim3(256), 0, st, A, n, lda, R, ldr);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status qr_blocked(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st) {
  constexpr int NB = 16;
  TTK_TRY(qr_factor(A, m, n, lda, R, ldr, work, st));
  const QrWork w(work, m, n);
  const int npan = (n + NB - 1) / NB;
  // Q = H_0 ... H_{n-1} [I; 0], panels from last to first
  for (int p = npan - 1; p >= 0; --p) {
    const int j0 = p * NB, jb = std::min(NB, n - j0);
    const int mm = m - j0;
    double* Ap = A + j0 + (size_t)j0 * lda;
    const double* T = w.Tall + (size_t)p * NB * NB;
    const int nc = n - j0 - jb;
    if (nc > 0) {
      hipLaunchKernelGGL(k_build_v, dim3((unsigned)(((int64_t)mm * jb + 255) / 256)), dim3(256), 0, st, Ap, mm, jb,
                         lda, w.V, (size_t)0, (size_t)0);
      double* Q2 = A + j0 + (size_t)(j0 + jb) * lda;
      // Q2 <- (I - V T V^T) Q2
      qr_apply(w.V, mm, jb, T, 0, Q2, nc, lda, w.Wp, st);
    }
    if (!qr_panel_q_reg(Ap, mm, jb, lda, w.tau + j0, st))
      hipLaunchKernelGGL(k_qr_panel_q, dim3(1), dim3(BS), 0, st, Ap, mm, jb, lda, w.tau + j0);
    if (j0 > 0)
      hipLaunchKernelGGL(k_zero_rows, dim3((j0 * jb + 255) / 256), dim3(256), 0, st, A + (size_t)j0 * lda, j0, jb,
                         lda);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status qr_apply_q(const double* A, int m, int n, int lda, double* work, double* C, int nc, int ldc,
                     hipStream_t st) {
  constexpr int NB = 16;
  if (nc <= 0) return TTK_OK;
  const QrWork w(work, m, n);
  const int npan = (n + NB - 1) / NB;
  // Q C = H_0 (H_1 (... H_{n-1} C)): the panels' block reflectors from last to first
  for (int p = npan - 1; p >= 0; --p) {
    const int j0 = p * NB, jb = std::min(NB, n - j0);
    const int mm = m - j0;
    hipLaunchKernelGGL(k_build_v, dim3((unsigned)(((int64_t)mm * jb + 255) / 256)), dim3(256), 0, st,
                       A + j0 + (size_t)j0 * lda, mm, jb, lda, w.V, (size_t)0, (size_t)0);
    qr_apply(w.V, mm, jb, w.Tall + (size_t)p * NB * NB, 0, C + j0, nc, ldc, w.Wp, st);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// ------------------------------------------------------------------ TSQR
namespace {

// Tall-skinny QR (Demmel, Grigori, Hoemmen & Langou, SIAM J. Sci. Comput.
// 2012) for N x r matrices with r <= 512: the rows are cut into blocks of H,
// every block is factored by the blocked Householder QR above (one batched
// launch per panel: the register panel and the trailing update with a
// batch index), the blocks' R factors are stacked and cut again, until one
// block is left; its R is the R of the whole matrix.  Q is never formed:
// Q [C; 0] is applied top-down, each level's reflectors (batched again) to
// the rows the level above hands down.  Each block's factorisation is
// Householder, so Q is orthonormal to working precision whatever the
// conditioning (a Gram-matrix route would square it; [U V] of Global-1 is
// numerically rank deficient).  H = 512 up to 128 columns (one k_qr_apply
// per trailing update), 2048 above (the register panel's limit; the update
// split over row chunks, at most 16, so their partials are summed in place).
inline int tsqr_h(int r) { return r <= 128 ? 512 : 2048; }
inline int tsqr_tr(int c) { return c <= 128 ? 32 : 8; }   // rows per LDS tile of the strided copies

// Level 0: the blocks Ab[b H r + i + c H] = A(g, c) for g = b H + i < N (A(g, c)
// at A[g sp + c sc]), 0 past N.  A tile of TR rows x r columns goes through
// LDS (TR (r + 1) doubles) so both sides are read and written along their
// contiguous direction.
template <class T>
__global__ void __launch_bounds__(256) k_tsqr_load(const T* A, int64_t sp, int64_t sc, int64_t N, int r, int H,
                                                   int TR, double* Ab) {
  extern __shared__ double tl[];
  const int64_t g0 = (int64_t)blockIdx.x * TR;
  for (int e = threadIdx.x; e < TR * r; e += 256) {
    const int i = e / r, c = e - i * r;
    const int64_t g = g0 + i;
    tl[i * (r + 1) + c] = g < N ? (double)A[g * sp + c * sc] : 0.0;
  }
  __syncthreads();
  const int64_t b = g0 / H;
  const int i0 = (int)(g0 - b * H);
  double* out = Ab + b * H * r;
  for (int e = threadIdx.x; e < TR * r; e += 256) {
    const int c = e / TR, i = e - c * TR;
    out[i0 + i + (int64_t)c * H] = tl[i * (r + 1) + c];
  }
}

// The output Y(p, j) = D0[p / H][p % H + j H] (p < N, j < c), to Y[p sp + j sc].
template <class T>
__global__ void __launch_bounds__(256) k_tsqr_store(const double* D, int64_t N, int c, int H, int TR, T* Y, int64_t sp,
                                                    int64_t sc) {
  extern __shared__ double tl[];
  const int64_t g0 = (int64_t)blockIdx.x * TR;
  const int64_t b = g0 / H;
  const int i0 = (int)(g0 - b * H);
  const double* in = D + b * H * c;
  for (int e = threadIdx.x; e < TR * c; e += 256) {
    const int j = e / TR, i = e - j * TR;
    tl[i * (c + 1) + j] = in[i0 + i + (int64_t)j * H];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TR * c; e += 256) {
    const int i = e / c, j = e - i * c;
    const int64_t g = g0 + i;
    if (g < N) Y[g * sp + j * sc] = (T)tl[i * (c + 1) + j];
  }
}

// Level l + 1 from level l: the stacked R factors (block b's R as rows
// b r .. b r + r - 1), cut into blocks of H rows, zero past `rows`.
__global__ void k_tsqr_stack(const double* Al, int r, int H, int64_t rows, int nbn, double* An) {
  const int64_t total = (int64_t)nbn * H * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bn = e / ((int64_t)H * r);
    const int64_t rem = e - bn * H * r;
    const int c = (int)(rem / H), i = (int)(rem % H);
    const int64_t g = bn * H + i;
    double v = 0.0;
    if (g < rows) {
      const int64_t b = g / r;
      const int ii = (int)(g - b * r);
      if (ii <= c) v = Al[b * H * r + ii + (int64_t)c * H];
    }
    An[e] = v;
  }
}

// Level l - 1's input from level l's result: block b gets rows b r .. b r + r - 1
// of the level above (which lie in its blocks of H rows), then zeros.
__global__ void k_tsqr_down(const double* Du, int c, int nb, int r, int H, double* Dl) {
  const int64_t total = (int64_t)nb * H * c;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ((int64_t)H * c);
    const int64_t rem = e - b * H * c;
    const int j = (int)(rem / H), i = (int)(rem % H);
    double v = 0.0;
    if (i < r) {
      const int64_t g = b * r + i;
      v = Du[(g / H) * H * c + (g % H) + (int64_t)j * H];
    }
    Dl[e] = v;
  }
}

// The top level's input [C; 0] (one block of H x c; C r x c, leading dimension ldc).
__global__ void k_tsqr_top(const double* C, int ldc, int r, int c, int H, double* D) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < H * c; e += gridDim.x * blockDim.x) {
    const int j = e / H, i = e % H;
    D[e] = i < r ? C[i + (size_t)j * ldc] : 0.0;
  }
}

inline unsigned tsqr_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

// ---- 64-column block reflectors for the 2048-row blocks
// An outer panel of OB columns (up to four 16-column register panels) is
// applied to the columns right of it, and in the application of Q, as one
// block reflector I - V op(T) V^T: V the outer panel's reflectors (kept
// below the diagonal of A by the register panels, unit diagonal) and T
// (OB x OB, upper triangular) built from the panels' own T and the products
// V_a^T V_b of their reflectors, so the trailing columns are read and
// written once per 64 columns instead of once per 16.
constexpr int OB = 64;

// V[i, c] of an outer panel whose diagonal starts at Vp (leading dimension
// ldv, mm rows, ob columns): the stored reflector below the diagonal, 1 on
// it, 0 above and past the extent
__device__ inline double vpan(const double* Vp, int ldv, int i, int c, int mm, int ob) {
  if (i >= mm || c >= ob || i < c) return 0.0;
  return i == c ? 1.0 : Vp[i + (size_t)c * ldv];
}

// T of the outer panel, one workgroup per block (blockIdx.x, strides sV,
// sT, s64): the panels' T_s (p0 + s, js x js column-major) on the diagonal,
// and column block s above it -T_(s) (V_(s)^T V_s) T_s, T_(s) the part
// already built (the forward, column-wise combination of compact-WY
// factors).  The products V_a^T V_b (a < b) run on FP64 MFMA.
__global__ void __launch_bounds__(256) k_qr_t64(const double* Vp, int ldv, size_t sV, int mm, int ob, const double* T,
                                                size_t sT, int p0, double* T64, size_t s64) {
  Vp += blockIdx.x * sV;
  T += blockIdx.x * sT;
  T64 += blockIdx.x * s64;
  __shared__ double G[OB][OB + 1], Tt[OB][OB + 1], Y[OB][17];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ns = (ob + 15) / 16;
  // the products V_a^T V_b (a < b, up to 6 pairs): the waves take the rows'
  // 4-row steps in turn, each step's 4 column blocks loaded once for all
  // pairs; the waves' sums then meet in G one wave at a time
  qdbl4 g[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) g[q] = qdbl4{0.0, 0.0, 0.0, 0.0};
  constexpr int TB = 4;
  const int nsteps = (mm + 3) / 4;
  for (int k0 = wv * TB; k0 < nsteps; k0 += 4 * TB) {
    double v[TB][4];
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int a = 0; a < 4; ++a) v[u][a] = a < ns ? vpan(Vp, ldv, 4 * (k0 + u) + lk, 16 * a + li, mm, ob) : 0.0;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      int q = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b, ++q)
          if (b < ns) g[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][a], v[u][b], g[q], 0, 0, 0);
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
      int q = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b, ++q)
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            double& dst = G[16 * a + lk + 4 * vv][16 * b + li];
            dst = (w == 0 ? 0.0 : dst) + g[q][vv];
          }
    }
    __syncthreads();
  }
  for (int e = tid; e < OB * OB; e += 256) Tt[e / OB][e % OB] = 0.0;
  __syncthreads();
  for (int s = 0; s < ns; ++s) {
    const int js = min(16, ob - 16 * s);
    const double* Ts = T + (size_t)(p0 + s) * 256;
    for (int e = tid; e < js * js; e += 256) Tt[16 * s + e % js][16 * s + e / js] = Ts[e];
  }
  __syncthreads();
  for (int s = 1; s < ns; ++s) {
    const int js = min(16, ob - 16 * s), ms = 16 * s;
    for (int e = tid; e < ms * js; e += 256) {   // Y = (V_(s)^T V_s) T_s
      const int i = e % ms, j = e / ms;
      double y = 0.0;
      for (int q = 0; q <= j; ++q) y += G[i][ms + q] * Tt[ms + q][ms + j];
      Y[i][j] = y;
    }
    __syncthreads();
    for (int e = tid; e < ms * js; e += 256) {   // column block s: -T_(s) Y (T_(s) upper triangular)
      const int i = e % ms, j = e / ms;
      double x = 0.0;
      for (int q = i; q < ms; ++q) x += Tt[i][q] * Y[q][j];
      Tt[i][ms + j] = -x;
    }
    __syncthreads();
  }
  for (int e = tid; e < ob * ob; e += 256) T64[e % ob + (size_t)(e / ob) * OB] = Tt[e % ob][e / ob];
}

// The block reflector's products walk the rows in chunks of QRC: a
// workgroup takes one chunk of one block, stages the chunk's V (QRC x 64,
// masked as vpan) in LDS once, and its waves take the 16-column tiles of C
// in turn, so V is read once per chunk whatever the width of C.
constexpr int WQ = QRC;   // rows per chunk of the wide products

// Vs[i][c] = vpan(Vp, ldv, r0 + i, c, mm, ob) for the chunk's WQ x OB panel,
// 256 threads.  Every read is from a clamped, valid entry of the panel and
// is turned into 0 or 1 arithmetically (v 0 + 1 on the diagonal, v 0 off the
// reflectors), eight per thread at a time: written as vpan() the reads
// compiled to one conditional load and wait per element.  (A zero of either
// sign contributes nothing to the products that read Vs.)
__device__ inline void stage_vpan(const double* Vp, int ldv, int r0, int mm, int ob, double (*Vs)[OB + 1], int tid) {
  constexpr int NE = WQ * OB / 256, UB = 8;
  static_assert(NE % UB == 0, "whole groups of UB elements per thread");
#pragma unroll
  for (int e0 = 0; e0 < NE; e0 += UB) {
    double v[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + (e0 + u) * 256, i = e % WQ, c = e / WQ, gi = r0 + i;
      v[u] = Vp[min(gi, mm - 1) + (size_t)min(c, ob - 1) * ldv];
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + (e0 + u) * 256, i = e % WQ, c = e / WQ, gi = r0 + i;
      const bool in = gi < mm && c < ob;
      const double keep = (in && gi > c) ? 1.0 : 0.0, one = (in && gi == c) ? 1.0 : 0.0;
      Vs[i][c] = v[u] * keep + one;
    }
  }
}

// W partials: Wp[((chunk * tiles + tile) * 4 + s) * 256 + m * 16 + n] =
// sum over the chunk's rows of V[i, 16 s + m] C[i, 16 tile + n].
__global__ void __launch_bounds__(256) k_qr_w64(const double* Vp, int ldv, size_t sV, int mm, int ob, const double* C,
                                                int nc, int ldc, size_t sC, double* Wp, size_t sW) {
  Vp += blockIdx.y * sV;
  C += blockIdx.y * sC;
  Wp += blockIdx.y * sW;
  __shared__ double Vs[WQ][OB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ch = blockIdx.x, r0 = ch * WQ;
  const int tiles = (nc + 15) / 16, ns = (ob + 15) / 16;
  stage_vpan(Vp, ldv, r0, mm, ob, Vs, tid);
  __syncthreads();
  for (int t = wv; t < tiles; t += 4) {
    const int c = t * 16 + li;
    const bool cok = c < nc;
    qdbl4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = qdbl4{0.0, 0.0, 0.0, 0.0};
    // the tile's 32 K-steps in two batches, the second loading while the
    // first multiplies
    constexpr int TB = WQ / 8;
    double b0[TB], b1[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int i = r0 + 4 * u + lk, i1 = i + 4 * TB;
      b0[u] = (i < mm && cok) ? C[i + (size_t)c * ldc] : 0.0;
      b1[u] = (i1 < mm && cok) ? C[i1 + (size_t)c * ldc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < ns) acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[4 * u + lk][16 * s + li], b0[u], acc[s], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < ns)
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[4 * (TB + u) + lk][16 * s + li], b1[u], acc[s], 0, 0, 0);
    // D[m][n] at lane (n = li, m = lk + 4 v)
    double* wp = Wp + ((size_t)ch * tiles + t) * 1024;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) wp[s * 256 + (lk + 4 * v) * 16 + li] = acc[s][v];
  }
}

// W2 = op(T) W for every tile (W: the chunk-0 slots, summed beforehand),
// into W2p[tile * 1024 + k * 16 + n] (k < 64), one workgroup per tile and block.
__global__ void __launch_bounds__(256) k_qr_w2(const double* T64, size_t s64, int trans, int ob, const double* Wp,
                                               size_t sW, double* W2p, size_t s2) {
  T64 += blockIdx.y * s64;
  Wp += blockIdx.y * sW + (size_t)blockIdx.x * 1024;
  W2p += blockIdx.y * s2 + (size_t)blockIdx.x * 1024;
  __shared__ double W[OB][17];
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 4; ++s) W[16 * s + (tid >> 4)][tid & 15] = Wp[s * 256 + tid];
  __syncthreads();
  for (int e = tid; e < OB * 16; e += 256) {
    const int i = e >> 4, n = e & 15;
    double sum = 0.0;
    if (i < ob)
      for (int k = 0; k < ob; ++k) sum += (trans ? T64[k + (size_t)i * OB] : T64[i + (size_t)k * OB]) * W[k][n];
    W2p[e] = sum;
  }
}

// C <- C - V W2 on one chunk of one block: V's chunk in LDS, the waves take
// the 16-column tiles in turn, per tile the chunk's 16-row tiles with
// ob / 4 MFMA steps each.
__global__ void __launch_bounds__(256) k_qr_c64(const double* Vp, int ldv, size_t sV, int mm, int ob, double* C,
                                                int nc, int ldc, size_t sC, const double* W2p, size_t s2) {
  Vp += blockIdx.y * sV;
  C += blockIdx.y * sC;
  W2p += blockIdx.y * s2;
  __shared__ double Vs[WQ][OB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ch = blockIdx.x, r0 = ch * WQ;
  const int tiles = (nc + 15) / 16, nst = (ob + 3) / 4;
  stage_vpan(Vp, ldv, r0, mm, ob, Vs, tid);
  __syncthreads();
  for (int t = wv; t < tiles; t += 4) {
    const int c = t * 16 + li;
    const bool cok = c < nc;
    // the tile's W2 rows and all of the chunk's C values load together
    double bw[16], cv[WQ / 16][4];
#pragma unroll
    for (int st = 0; st < 16; ++st) bw[st] = W2p[(size_t)t * 1024 + (4 * st + lk) * 16 + li];
#pragma unroll
    for (int h = 0; h < WQ / 16; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * h + lk + 4 * v;
        cv[h][v] = (row < mm && cok) ? C[row + (size_t)c * ldc] : 0.0;
      }
#pragma unroll
    for (int h = 0; h < WQ / 16; ++h) {
      qdbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < 16; ++st)
        if (st < nst) d = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * h + li][4 * st + lk], bw[st], d, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * h + lk + 4 * v;
        if (row < mm && cok) C[row + (size_t)c * ldc] = cv[h][v] - d[v];
      }
    }
  }
}

// (I - V op(T) V^T) C for the outer panel at Vp (mm rows, ob columns) on the
// nb blocks' C (nc columns, leading dimension ldc, block strides sV, s64,
// sC).  Wp holds the partials and W2 (at least nb * tiles * (ceil(mm /
// 128) + 1) * 1024 doubles).
void tsqr_update64(const double* Vp, int ldv, size_t sV, int mm, int ob, const double* T64, size_t s64, int trans,
                   double* C, int nc, int ldc, size_t sC, int nb, double* Wp, hipStream_t st) {
  const int tiles = (nc + 15) / 16;
  const int nch = (mm + WQ - 1) / WQ;
  const size_t sW = (size_t)tiles * (nch + 1) * 1024;   // the partials, then W2 at chunk slot nch
  double* W2p = Wp + (size_t)tiles * nch * 1024;
  hipLaunchKernelGGL(k_qr_w64, dim3(nch, nb), dim3(256), 0, st, Vp, ldv, sV, mm, ob, (const double*)C, nc, ldc, sC,
                     Wp, sW);
  hipLaunchKernelGGL(k_qr_apply_sum, dim3(tiles * 4, nb), dim3(256), 0, st, Wp, nch, tiles * 4, sW);
  hipLaunchKernelGGL(k_qr_w2, dim3(tiles, nb), dim3(256), 0, st, T64, s64, trans, ob, (const double*)Wp, sW, W2p, sW);
  hipLaunchKernelGGL(k_qr_c64, dim3(nch, nb), dim3(256), 0, st, Vp, ldv, sV, mm, ob, C, nc, ldc, sC,
                     (const double*)W2p, sW);
}

// (I - V op(T) V^T) on the nb blocks' C: one k_qr_apply per block for
// mm <= 4 QRC, else the row-chunked pair with each block's partials at
// Wp + b sW (at most 16 chunks, summed by k_qr_apply_c in chunk order).
void tsqr_update(const double* V, int mm, int jb, const double* T, int trans, double* C, int nc, int lda, int nb,
                 size_t sV, size_t sT, size_t sC, double* Wp, size_t sW, hipStream_t st) {
  const int tiles = (nc + 15) / 16;
  if (mm <= 4 * QRC) {
    hipLaunchKernelGGL(k_qr_apply, dim3(tiles, nb), dim3(QAW * 64), 0, st, V, mm, jb, T, trans, C, nc, lda, sV, sT,
                       sC);
    return;
  }
  // rows per chunk: QRC, or 4 QRC when that still leaves at least 16 blocks
  // per CU (many blocks of the batch: fewer, larger blocks schedule faster)
  const bool big = (int64_t)nb * tiles * ((mm + 4 * QRC - 1) / (4 * QRC)) >= 16 * 256;
  const int rc = big ? 4 * QRC : QRC;
  const int nch = (mm + rc - 1) / rc;
  if (big)
    hipLaunchKernelGGL(k_qr_apply_w<4 * QRC>, dim3(tiles, nch, nb), dim3(QSW * 64), 0, st, V, mm, jb,
                       (const double*)C, nc, lda, Wp, sV, sC, sW);
  else
    hipLaunchKernelGGL(k_qr_apply_w<QRC>, dim3(tiles, nch, nb), dim3(QSW * 64), 0, st, V, mm, jb, (const double*)C,
                       nc, lda, Wp, sV, sC, sW);
  // the partials summed once per tile (in chunk order, as k_qr_apply_c
  // would), so that the nch chunks of a tile each read one 16 x 16 sum
  // instead of all nch partials
  hipLaunchKernelGGL(k_qr_apply_sum, dim3(tiles, nb), dim3(256), 0, st, Wp, nch, tiles, sW);
  if (big)
    hipLaunchKernelGGL(k_qr_apply_c<4 * QRC>, dim3(tiles, nch, nb), dim3(QSW * 64), 0, st, V, mm, jb, T, trans, C,
                       nc, lda, (const double*)Wp, 1, sV, sT, sC, sW);
  else
    hipLaunchKernelGGL(k_qr_apply_c<QRC>, dim3(tiles, nch, nb), dim3(QSW * 64), 0, st, V, mm, jb, T, trans, C, nc,
                       lda, (const double*)Wp, 1, sV, sT, sC, sW);
}

// LDS of the strided copies: TR (c + 1) doubles, with the attribute raised once past 48 KB.
template <class F>
bool tsqr_lds(F kern, size_t sh) {
  static size_t attr = 48 * 1024;
  if (sh <= attr) return true;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) !=
      hipSuccess)
    return false;
  attr = sh;
  return true;
}

}  // namespace

// R factors of `count` square n x n matrices at once (matrix b at A + b sA,
// overwritten by its reflectors; R_b at R + b sR, ld ldr): the register
// panels and the trailing updates of the tall-skinny QR, batched over the
// matrices.  work: qr_r_batched_work(n, count) doubles.
size_t qr_r_batched_work(int n, int count) {
  constexpr int NB = 16;
  const size_t npan = (size_t)(n + NB - 1) / NB;
  return (size_t)count * ((size_t)n + (size_t)n * NB + npan * NB * NB);
}

__global__ void k_extract_r_batched(const double* A, int n, int lda, size_t sA, double* R, int ldr, size_t sR) {
  A += blockIdx.y * sA;
  R += blockIdx.y * sR;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    R[i + (size_t)c * ldr] = (i <= c) ? A[i + (size_t)c * lda] : 0.0;
  }
}

tt_status qr_r_batched(double* A, int n, int lda, size_t sA, double* R, int ldr, size_t sR, double* work, int count,
                       hipStream_t st) {
  constexpr int NB = 16;
  if (n < 1 || n > 4 * QRC || count < 1 || count > 65535)
    return fail(TTK_ERR_UNSUPPORTED, "batched QR of %d matrices of order %d", count, n);
  const int npan = (n + NB - 1) / NB;
  double* tau = work;
  double* V = tau + (size_t)count * n;
  double* T = V + (size_t)count * n * NB;
  for (int p = 0; p < npan; ++p) {
    const int j0 = p * NB, jb = std::min(NB, n - j0), mm = n - j0;
    if (!qr_panel_reg(A + j0 + (size_t)j0 * lda, mm, jb, lda, tau + j0, V, T + (size_t)p * NB * NB, st, count, sA,
                      (size_t)n, (size_t)n * NB, (size_t)npan * NB * NB))
      return fail(TTK_ERR_UNSUPPORTED, "batched QR: panel of %d rows", mm);
    const int nc = n - j0 - jb;
    if (nc > 0)
      tsqr_update(V, mm, jb, T + (size_t)p * NB * NB, 1, A + j0 + (size_t)(j0 + jb) * lda, nc, lda, count,
                  (size_t)n * NB, (size_t)npan * NB * NB, sA, nullptr, 0, st);
  }
  hipLaunchKernelGGL(k_extract_r_batched, dim3(tsqr_grid((int64_t)n * n), count), dim3(256), 0, st,
                     (const double*)A, n, lda, sA, R, ldr, sR);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tsqr_factor(int dtype, const void* A, int64_t sp, int64_t sc, int64_t N, int r, TsqrState* ts, double* R,
                      int ldr, hipStream_t st) {
  constexpr int NB = 16;
  if (r < 1 || r > 512) return fail(TTK_ERR_UNSUPPORTED, "tsqr: r = %d outside 1..512", r);
  if (N < r) return fail(TTK_ERR_UNSUPPORTED, "tsqr: %lld rows for %d columns", (long long)N, r);
  const int H = tsqr_h(r);
  ts->r = r;
  ts->N = N;
  ts->H = H;
  const int npan = (r + NB - 1) / NB;
  const int tiles_max = (r + 15) / 16;
  const int nch_max = (H + QRC - 1) / QRC;
  int64_t rows = N;
  int l = 0;
  for (;; ++l) {
    if (l >= TSQR_MAXLEV) return fail(TTK_ERR_UNSUPPORTED, "tsqr: too many levels");
    const int64_t nb64 = (rows + H - 1) / H;
    if (nb64 > 65535) return fail(TTK_ERR_UNSUPPORTED, "tsqr: %lld row blocks (at most 65535)", (long long)nb64);
    const int nb = (int)nb64;
    ts->nb[l] = nb;
    ts->rows[l] = rows;
    TTK_TRY(ts->A[l].alloc((size_t)nb * H * r * sizeof(double)));
    TTK_TRY(ts->tau[l].alloc((size_t)nb * r * sizeof(double)));
    TTK_TRY(ts->T[l].alloc((size_t)nb * npan * NB * NB * sizeof(double)));
    double* Al = ts->A[l].as<double>();
    if (l == 0) {
      const int TR = tsqr_tr(r);
      const size_t sh = (size_t)TR * (r + 1) * sizeof(double);
      const unsigned g = (unsigned)((N + TR - 1) / TR);
      fill_zero(Al, (size_t)nb * H * r * sizeof(double), st);   // the last block's tail
      bool ok;
      if (dtype == TTK_FP32) {
        ok = tsqr_lds(&k_tsqr_load<float>, sh);
        if (ok)
          hipLaunchKernelGGL(k_tsqr_load<float>, dim3(g), dim3(256), sh, st, static_cast<const float*>(A), sp, sc, N,
                             r, H, TR, Al);
      } else {
        ok = tsqr_lds(&k_tsqr_load<double>, sh);
        if (ok)
          hipLaunchKernelGGL(k_tsqr_load<double>, dim3(g), dim3(256), sh, st, static_cast<const double*>(A), sp, sc,
                             N, r, H, TR, Al);
      }
      if (!ok) return fail(TTK_ERR_HIP, "tsqr: LDS of %zu bytes refused", sh);
    } else {
      hipLaunchKernelGGL(k_tsqr_stack, dim3(tsqr_grid((int64_t)nb * H * r)), dim3(256), 0, st,
                         (const double*)ts->A[l - 1].as<double>(), r, H, rows, nb, Al);
    }
    TTK_TRY(ts->V.alloc((size_t)nb * H * NB * sizeof(double)));
    // many 2048-row blocks: outer panels of OB columns, each applied to the
    // columns right of it as one block reflector (partials: 4 x 256 per tile
    // and chunk); otherwise the whole matrix is one outer panel (a level of
    // few blocks gives the chunked 16-column updates more workgroups)
    const bool wide = H > 4 * QRC && nb >= 16;
    ts->wide[l] = wide;
    const int nout = (r + OB - 1) / OB;
    // partials of the chunked updates of 2048-row blocks, 16-column (256 per
    // tile and chunk) or 64-column (1024, plus W2)
    if (H > 4 * QRC) TTK_TRY(ts->Wp.alloc((size_t)nb * tiles_max * (nch_max + 1) * 1024 * sizeof(double)));
    if (wide) TTK_TRY(ts->T64[l].alloc((size_t)nb * nout * OB * OB * sizeof(double)));
    double* V = ts->V.as<double>();
    double* tau = ts->tau[l].as<double>();
    double* T = ts->T[l].as<double>();
    const int OW = wide ? OB : r;
    for (int c0 = 0; c0 < r; c0 += OW) {
      const int ob = std::min(OW, r - c0);
      for (int p = c0 / NB; p * NB < c0 + ob; ++p) {
        const int j0 = p * NB, jb = std::min(NB, r - j0), mm = H - j0;
        if (!qr_panel_reg(Al + j0 + (size_t)j0 * H, mm, jb, H, tau + j0, V, T + (size_t)p * NB * NB, st, nb,
                          (size_t)H * r, (size_t)r, (size_t)H * NB, (size_t)npan * NB * NB))
          return fail(TTK_ERR_UNSUPPORTED, "tsqr: panel of %d rows", mm);
        const int nc = c0 + ob - j0 - jb;   // the outer panel's columns right of this panel
        if (nc > 0)
          tsqr_update(V, mm, jb, T + (size_t)p * NB * NB, 1, Al + j0 + (size_t)(j0 + jb) * H, nc, H, nb,
                      (size_t)H * NB, (size_t)npan * NB * NB, (size_t)H * r,
                      H > 4 * QRC ? ts->Wp.as<double>() : nullptr,
                      (size_t)tiles_max * nch_max * 256, st);
      }
      if (wide) {
        double* T64 = ts->T64[l].as<double>() + (size_t)(c0 / OB) * OB * OB;
        const double* Vp = Al + c0 + (size_t)c0 * H;
        hipLaunchKernelGGL(k_qr_t64, dim3(nb), dim3(256), 0, st, Vp, H, (size_t)H * r, H - c0, ob,
                           (const double*)T, (size_t)npan * NB * NB, c0 / NB, T64, (size_t)nout * OB * OB);
        const int nc = r - c0 - ob;
        if (nc > 0)
          tsqr_update64(Vp, H, (size_t)H * r, H - c0, ob, T64, (size_t)nout * OB * OB, 1,
                        Al + c0 + (size_t)(c0 + ob) * H, nc, H, (size_t)H * r, nb, ts->Wp.as<double>(), st);
      }
    }
    if (nb == 1) break;
    rows = (int64_t)nb * r;
  }
  ts->nlev = l + 1;
  hipLaunchKernelGGL(k_extract_r, dim3((r * r + 255) / 256), dim3(256), 0, st,
                     (const double*)ts->A[l].as<double>(), r, H, R, ldr);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tsqr_apply(TsqrState* ts, const double* C, int ldc, int c, int out_dtype, void* Y, int64_t sp, int64_t sc,
                     hipStream_t st) {
  constexpr int NB = 16;
  if (c < 1 || c > 512) return fail(TTK_ERR_UNSUPPORTED, "tsqr: %d columns to apply Q to (1..512)", c);
  const int r = ts->r, H = ts->H, npan = (r + NB - 1) / NB;
  const int tiles = (c + 15) / 16, nch = (H + QRC - 1) / QRC;
  DBuf* D = ts->D;
  for (int l = ts->nlev - 1; l >= 0; --l) {
    const int nb = ts->nb[l];
    DBuf& Dl = D[l & 1];
    TTK_TRY(Dl.alloc((size_t)nb * H * c * sizeof(double)));
    if (l == ts->nlev - 1)
      hipLaunchKernelGGL(k_tsqr_top, dim3(tsqr_grid((int64_t)H * c)), dim3(256), 0, st, C, ldc, r, c, H,
                         Dl.as<double>());
    else
      hipLaunchKernelGGL(k_tsqr_down, dim3(tsqr_grid((int64_t)nb * H * c)), dim3(256), 0, st,
                         (const double*)D[(l + 1) & 1].as<double>(), c, nb, r, H, Dl.as<double>());
    const double* Al = ts->A[l].as<double>();
    if (H > 4 * QRC) TTK_TRY(ts->Wp.alloc((size_t)nb * tiles * (nch + 1) * 1024 * sizeof(double)));
    if (ts->wide[l]) {   // the outer panels' block reflectors, last to first
      const int nout = (r + OB - 1) / OB;
      for (int P = nout - 1; P >= 0; --P) {
        const int c0 = P * OB, ob = std::min(OB, r - c0);
        tsqr_update64(Al + c0 + (size_t)c0 * H, H, (size_t)H * r, H - c0, ob,
                      ts->T64[l].as<double>() + (size_t)P * OB * OB, (size_t)nout * OB * OB, 0,
                      Dl.as<double>() + c0, c, H, (size_t)H * c, nb, ts->Wp.as<double>(), st);
      }
      continue;
    }
    TTK_TRY(ts->V.alloc((size_t)nb * H * NB * sizeof(double)));
    double* V = ts->V.as<double>();
    const double* T = ts->T[l].as<double>();
    for (int p = npan - 1; p >= 0; --p) {   // Q [C; 0] = H_0 (H_1 (... [C; 0])), panels last to first
      const int j0 = p * NB, jb = std::min(NB, r - j0), mm = H - j0;
      hipLaunchKernelGGL(k_build_v, dim3((unsigned)(((int64_t)mm * jb + 255) / 256), nb), dim3(256), 0, st,
                         Al + j0 + (size_t)j0 * H, mm, jb, H, V, (size_t)H * r, (size_t)H * NB);
      tsqr_update(V, mm, jb, T + (size_t)p * NB * NB, 0, Dl.as<double>() + j0, c, H, nb, (size_t)H * NB,
                  (size_t)npan * NB * NB, (size_t)H * c, H > 4 * QRC ? ts->Wp.as<double>() : nullptr,
                  (size_t)tiles * nch * 256, st);
    }
  }
  const int TR = tsqr_tr(c);
  const size_t sh = (size_t)TR * (c + 1) * sizeof(double);
  const unsigned g = (unsigned)((ts->N + TR - 1) / TR);
  bool ok;
  if (out_dtype == TTK_FP32) {
    ok = tsqr_lds(&k_tsqr_store<float>, sh);
    if (ok)
      hipLaunchKernelGGL(k_tsqr_store<float>, dim3(g), dim3(256), sh, st, (const double*)D[0].as<double>(), ts->N, c,
                         H, TR, static_cast<float*>(Y), sp, sc);
  } else {
    ok = tsqr_lds(&k_tsqr_store<double>, sh);
    if (ok)
      hipLaunchKernelGGL(k_tsqr_store<double>, dim3(g), dim3(256), sh, st, (const double*)D[0].as<double>(), ts->N, c,
                         H, TR, static_cast<double*>(Y), sp, sc);
  }
  if (!ok) return fail(TTK_ERR_HIP, "tsqr: LDS of %zu bytes refused", sh);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

size_t qr_blocked_work(int m, int n) {
  constexpr int NB = 16;
  return (size_t)n + (size_t)NB * m + (size_t)NB * NB * ((n + NB - 1) / NB) + 2 * (size_t)NB * n + 64 +
         (size_t)256 * ((n + NB - 1) / NB) * (((size_t)m + QRC - 1) / QRC);
}

namespace {

// Launch the LDS form of the Jacobi SVD if the matrix fits; false if it does not.
template <int G, int E>
bool jacobi_lds_launch_e(double* A, int n, int lda, double* V, int ldv, double* sigma, size_t sh, int lds_limit,
                         hipStream_t st) {
  static size_t attr = 48 * 1024;   // dynamic LDS the instantiation is allowed so far
  if (sh > attr) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_lds<G, E>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    attr = sh;
  }
  hipLaunchKernelGGL((k_jacobi_lds<G, E>), dim3(1), dim3(BS), sh, st, A, n, lda, V, ldv, sigma, V ? 1 : 0);
  if (hipGetLastError() == hipSuccess) return true;
  (void)hipGetLastError();
  return false;
}

bool jacobi_lds_launch(double* A, int n, int lda, double* V, int ldv, double* sigma, hipStream_t st) {
  static int lds_limit = -1;
  if (lds_limit < 0) {
    int dev = 0, v = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      lds_limit = v;
    else
      lds_limit = 64 * 1024;
    (void)hipGetLastError();
  }
  const int np = (n + 1) & ~1;
  const size_t sh = (size_t)n * n * sizeof(double) + (size_t)(np / 2) * (2 * sizeof(double) + 2 * sizeof(int));
  if (n < 2 || sh + 64 > (size_t)lds_limit) return false;
  // 16 lanes per pair (64 pairs per round at once), E = ceil(n / 16) <= 9
  // entries per lane: the clamped entries past n are loaded and stored again,
  // so E is not rounded up further
  switch ((n + 15) / 16) {
    case 1:
    case 2: return jacobi_lds_launch_e<16, 2>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 3: return jacobi_lds_launch_e<16, 3>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 4: return jacobi_lds_launch_e<16, 4>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 5: return jacobi_lds_launch_e<16, 5>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 6: return jacobi_lds_launch_e<16, 6>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 7: return jacobi_lds_launch_e<16, 7>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 8: return jacobi_lds_launch_e<16, 8>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    case 9: return jacobi_lds_launch_e<16, 9>(A, n, lda, V, ldv, sigma, sh, lds_limit, st);
    default: return false;
  }
}

template <int E>
void jacobi_block_round(double* A, int n, int lda, int nbp, int rnd, double* aux, int count, size_t sA, size_t sS,
                        hipStream_t st) {
  static size_t attr = 48 * 1024;   // dynamic LDS the instantiation is allowed so far
  const size_t sh = (size_t)2 * JB_W * JB_L * E * sizeof(double);   // the columns padded to JB_L E rows
  if (sh > attr) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_block<E>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
      return;   // (the launch then fails and the error is reported by the caller's next check)
    attr = sh;
  }
  hipLaunchKernelGGL((k_jacobi_block<E>), dim3(nbp / 2, count), dim3(JB_T), sh, st, A, n, lda, nbp, rnd, aux, sA,
                     sS);
}

// The block iteration on `count` matrices at once (matrix b at A + b sA,
// its sigma and workspace at sigma + b sS): sweeps queued in batches, the
// host reading the convergence flags between batches (launches queued past a
// matrix's convergence return at once for it).
bool jacobi_block_left_n(double* A, int n, int lda, size_t sA, double* sigma, size_t sS, int count, hipStream_t st) {
  if (n < 2 || n > JB_L * 16 || count < 1 || count > 65535) return false;   // E <= 16: 128 KB of LDS at most
  const int nb = (n + JB_W - 1) / JB_W, nbp = nb + (nb & 1);
  double* aux = sigma + (size_t)n * n + 3 * (size_t)n + 2;
  hipLaunchKernelGGL(k_jb_init, dim3(count), dim3(BS), 0, st, (const double*)A, n, lda, aux, sA, sS);
  const int E = (n + JB_L - 1) / JB_L;
  int sweeps = 0;
  for (int batch = 6; sweeps < 60; batch = 2) {
    for (int b = 0; b < batch && sweeps < 60; ++b, ++sweeps) {
      for (int rnd = 0; rnd < nbp - 1; ++rnd) {
        if (E <= 2) jacobi_block_round<2>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
        else if (E <= 4) jacobi_block_round<4>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
        else if (E <= 6) jacobi_block_round<6>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
        else if (E <= 8) jacobi_block_round<8>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
        else if (E <= 12) jacobi_block_round<12>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
        else jacobi_block_round<16>(A, n, lda, nbp, rnd, aux, count, sA, sS, st);
      }
      hipLaunchKernelGGL(k_jb_check, dim3(count), dim3(64), 0, st, aux, sS);
    }
    // every matrix's done flag, folded on the device into one word
    hipLaunchKernelGGL(k_jb_all_done, dim3(1), dim3(BS), 0, st, aux, sS, count);
    int32_t all = 0;
    if (hipMemcpyAsync(&all, aux + 3, sizeof(all), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      break;   // (the error stays pending for the caller's next check)
    if (all) break;
  }
  hipLaunchKernelGGL(k_jb_finish, dim3(count), dim3(BS), 0, st, A, n, lda, sigma, sA, sS);
  return true;
}

bool jacobi_block_left(double* A, int n, int lda, double* sigma, hipStream_t st) {
  return jacobi_block_left_n(A, n, lda, 0, sigma, 0, 1, st);
}

}  // namespace

void jacobi_svd(double* A, int n, int lda, double* V, int ldv, double* sigma, hipStream_t st) {
  // work: n*n + n doubles followed by n int32 (caller-sized through sigma's buffer)
  if (jacobi_lds_launch(A, n, lda, V, ldv, sigma, st)) return;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(BS), 0, st, A, n, lda, V, ldv, sigma, (size_t)0, (size_t)0,
                     (size_t)0);
}

bool jacobi_svd_left(double* A, int n, int lda, double* sigma, hipStream_t st) {
  if (jacobi_lds_launch(A, n, lda, nullptr, 0, sigma, st)) return true;
  return jacobi_block_left(A, n, lda, sigma, st);
}

bool jacobi_svd_left_batched(double* A, int n, int lda, size_t sA, double* sigma, size_t sS, int count,
                             hipStream_t st) {
  return jacobi_block_left_n(A, n, lda, sA, sigma, sS, count, st);
}

void jacobi_svd_batched(double* A, int n, int lda, size_t sA, double* V, int ldv, size_t sV, double* sigma,
                        size_t sS, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_jacobi, dim3(count), dim3(BS), 0, st, A, n, lda, V, ldv, sigma, sA, sV, sS);
}

size_t jacobi_sigma_doubles(int n) { return (size_t)n * n + 3 * (size_t)n + 8; }

void gemm64(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B,
            int ldb, double beta, double* C, int ldc, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  constexpr int T = 16;
  hipLaunchKernelGGL(k_gemm64<T>, dim3((m + T - 1) / T, (n + T - 1) / T), dim3(T, T), 0, st, ta, tb, m, n,
                     k, alpha, A, lda, B, ldb, beta, C, ldc);
}

void nrm2(const double* x, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_nrm2, dim3(1), dim3(BS), 0, st, x, n, out);
}

}  // namespace ttk
