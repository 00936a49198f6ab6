// Small dense double-precision linear algebra for the cross and the rounding
// of the cores: LU with partial pivoting (solves with the intersection
// matrices of the cross), Householder QR (thin QR of the TT-Round sweeps and
// of the interpolation formula), one-sided Jacobi SVD (truncated SVD of
// TT-Round) and a small tiled GEMM.  Matrices are column-major.  The
// factorisations run in one workgroup: they are sequential in the column
// index and their sizes (<= 8192 x 256) keep them in L2.
#include "ttk_internal.h"

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
  __shared__ double sv[BS];
  __shared__ int si[BS];
  const int tid = threadIdx.x;
  if (tid == 0) *info = 0;
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < n; i += BS) {
      const double v = fabs(A[i + (size_t)j * lda]);
      if (v > best) { best = v; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double a = sv[tid], b = sv[tid + s];
        if (b > a || (b == a && si[tid + s] < si[tid])) { sv[tid] = b; si[tid] = si[tid + s]; }
      }
      __syncthreads();
    }
    const int p = si[0];
    const double pv = sv[0];
    __syncthreads();
    if (tid == 0) {
      piv[j] = p;
      if (pv == 0.0 && *info == 0) *info = j + 1;
    }
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
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += BS) {
      const int i = j + 1 + e % m, c = j + 1 + e / m;
      A[i + (size_t)c * lda] -= A[i + (size_t)j * lda] * A[j + (size_t)c * lda];
    }
    __syncthreads();
  }
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

// ------------------------------------------------------------ Jacobi SVD
// One-sided (Hestenes) Jacobi on the columns of A (n x n): A V = U Sigma.
// Pairs follow a round-robin tournament so each round's rotations are
// disjoint; one wave per pair.
__global__ void __launch_bounds__(BS) k_jacobi(double* A, int n, int lda, double* V, int ldv,
                                               double* sigma, double* work, int32_t* order) {
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < n * n; e += BS) V[e % n + (size_t)(e / n) * ldv] = (e % n == e / n) ? 1.0 : 0.0;
  const int np = (n + 1) & ~1;    // players, one dummy when n is odd
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
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
        if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
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
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // singular values, normalised left vectors
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
  for (int e = tid; e < n * n; e += BS) tmp[e] = V[e % n + (size_t)order[e / n] * ldv];
  __syncthreads();
  for (int e = tid; e < n * n; e += BS) V[e % n + (size_t)(e / n) * ldv] = tmp[e];
  for (int c = tid; c < n; c += BS) tmp[n * n + c] = sigma[order[c]];
  __syncthreads();
  for (int c = tid; c < n; c += BS) sigma[c] = tmp[n * n + c];
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
  hipLaunchKernelGGL(k_lu, dim3(1), dim3(BS), 0, st, A, n, lda, piv, info);
}

void lu_solve(const double* LU, int n, int lda, const int32_t* piv, int trans, double* B, int ldb,
              int nrhs, hipStream_t st) {
  if (nrhs <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_lu_solve, dim3((nrhs + 63) / 64), dim3(64), 0, st, LU, n, lda, piv, trans, B, ldb,
                     nrhs);
}

void qr_thin(double* A, int m, int n, int lda, double* R, int ldr, double* work, hipStream_t st) {
  hipLaunchKernelGGL(k_qr, dim3(1), dim3(BS), 0, st, A, m, n, lda, R, ldr, work);
}

void jacobi_svd(double* A, int n, int lda, double* V, int ldv, double* sigma, hipStream_t st) {
  // work: n*n + n doubles followed by n int32 (caller-sized through sigma's buffer)
  double* work = sigma + n;
  int32_t* order = reinterpret_cast<int32_t*>(work + (size_t)n * n + n);
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(BS), 0, st, A, n, lda, V, ldv, sigma, work, order);
}

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
