// PTTK-Global-1 (Algorithm 4, Section 3.5) for the symmetric case X = Y.
//
// Offline: thin QR of A = [U V] (N x k, k = r_s + r_t) in double precision by
// the tall-skinny Householder QR (k <= 512; blocked Householder on the whole
// matrix above that).  For one point set the source and target factors span
// nearly the same subspace (for d = 2, n = 8 and ranks n^d they span exactly
// the same 64-dimensional space), so [U V] is numerically rank deficient;
// Householder reflections keep Q orthonormal regardless, which a
// Gram-matrix (Cholesky QR) route cannot.
//
// Online: with Hhat = [[0, M/2], [M^T/2, 0]] (the symmetric-part identity of
// Section 3.5), W = U Lambda_+ U^T for R Hhat R^T = U Lambda U^T.  The
// non-negative spectral part is formed as (Mh + |Mh|) / 2 with |Mh| = V Sigma
// V^T from a one-sided Jacobi SVD Mh = U' Sigma V^T (for symmetric Mh the
// singular vectors are eigenvectors up to sign and Sigma = |Lambda|).
//
// PTTK-Global-2 (Algorithm 4 with Compress) keeps, for one theta, only the
// leading positive eigenpairs (Uhat, Lambdahat) and returns Z = Q Uhat.  The
// positive eigenpairs of Mh are the eigenpairs of the PSD matrix W_+ above
// with non-zero eigenvalue, so they are taken from a second one-sided
// Jacobi, on W_+: for a PSD matrix the left singular vectors are the
// eigenvectors and Sigma = Lambda, already sorted, and a pair of eigenvalues
// +-lambda of Mh (which a singular value decomposition of Mh itself cannot
// separate) never meets in W_+.
#include <cmath>
#include <vector>

#include "ttk_internal.h"

namespace ttk {

namespace {

// A (N x k column-major, FP64) = [U V].
template <class T>
__global__ void k_concat_cm(const T* U, int ldu, int rs, const T* V, int ldv, int rt, int64_t N, double* A) {
  const int k = rs + rt;
  const int64_t total = N * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % N;
    const int c = (int)(e / N);
    A[e] = c < rs ? (double)U[p * ldu + c] : (double)V[p * ldv + (c - rs)];
  }
}

// I (k x k, FP64) = the identity.
__global__ void k_identity(int k, double* I) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * k;
       e += (int64_t)gridDim.x * blockDim.x)
    I[e] = (e % k == e / k) ? 1.0 : 0.0;
}

// out (N x k row-major, dtype) = Q (N x k column-major, FP64).
template <class T>
__global__ void k_q_rowmajor(const double* Q, int64_t N, int k, T* out) {
  const int64_t total = N * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / k;
    const int c = (int)(e % k);
    out[e] = (T)Q[p + (int64_t)c * N];
  }
}

// Mh_b <- Mh_b + Mh_b^T (in place, k x k, one block per b) and copies to Jb
// (the Jacobi input, overwritten by the SVD).
// B_b = A_b^T for square k x k matrices, b = blockIdx.y (stride s)
__global__ void k_transpose_batched(const double* A, int k, size_t s, double* B) {
  A += blockIdx.y * s;
  B += blockIdx.y * s;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % k), j = (int)(e / k);
    B[j + (size_t)i * k] = A[i + (size_t)j * k];
  }
}

__global__ void k_sym_copy(double* Mh, double* J, int k, size_t stride) {
  double* M = Mh + blockIdx.x * stride;
  double* Jb = J + blockIdx.x * stride;
  const int64_t total = (int64_t)k * k;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e % k), j = (int)(e / k);
    if (i < j) {
      const double s = M[i + (size_t)j * k] + M[j + (size_t)i * k];
      M[i + (size_t)j * k] = s;
      M[j + (size_t)i * k] = s;
    } else if (i == j) {
      M[e] *= 2.0;
    }
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) Jb[e] = M[e];
}

// VS_b = V_b diag(sigma_b); the sigma buffer of matrix b starts at sig + b sS.
__global__ void k_scale_cols(const double* V, const double* sig, size_t sS, int k, size_t stride, double* VS) {
  const double* Vb = V + blockIdx.x * stride;
  const double* sb = sig + blockIdx.x * sS;
  double* out = VS + blockIdx.x * stride;
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) out[e] = Vb[e] * sb[e / k];
}

// out[e] = C[e] in the output precision
template <class T>
__global__ void k_store(const double* C, int64_t n, T* out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (T)C[e];
}

inline unsigned nblocks(int64_t n, int64_t cap = 8192) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

}  // namespace

tt_status global_qr(int dtype, const void* U, int ldu, int rs, const void* V, int ldv, int rt, int64_t N, void* Q,
                    double* R, hipStream_t st) {
  const int k = rs + rt;
  if (k <= 0) return fail(TTK_ERR_ARG, "Global-1 needs r_s + r_t > 0");
  if (N < k)
    return fail(TTK_ERR_UNSUPPORTED, "Global-1 QR needs at least r_s + r_t = %d points (got %lld)", k, (long long)N);
  if (N > INT32_MAX) return fail(TTK_ERR_UNSUPPORTED, "Global-1 QR supports at most 2^31 - 1 points");
  DBuf A, work;
  TTK_TRY(A.alloc((size_t)N * k * sizeof(double)));
  if (k > 512) TTK_TRY(work.alloc(qr_blocked_work((int)N, k) * sizeof(double)));
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_concat_cm<float>, dim3(nblocks(N * k)), dim3(256), 0, st, static_cast<const float*>(U), ldu,
                       rs, static_cast<const float*>(V), ldv, rt, N, A.as<double>());
  else
    hipLaunchKernelGGL(k_concat_cm<double>, dim3(nblocks(N * k)), dim3(256), 0, st, static_cast<const double*>(U),
                       ldu, rs, static_cast<const double*>(V), ldv, rt, N, A.as<double>());
  TTK_HIP(hipGetLastError());
  if (k <= 512) {
    // tall-skinny QR: R, then Q = Q [I; 0] written row-major in the dtype
    TsqrState ts;
    TTK_TRY(tsqr_factor(TTK_FP64, A.as<double>(), 1, N, N, k, &ts, R, k, st));
    DBuf I;
    TTK_TRY(I.alloc((size_t)k * k * sizeof(double)));
    hipLaunchKernelGGL(k_identity, dim3(nblocks((int64_t)k * k)), dim3(256), 0, st, k, I.as<double>());
    TTK_TRY(tsqr_apply(&ts, I.as<double>(), k, k, dtype, Q, k, 1, st));
    TTK_HIP(hipGetLastError());
    TTK_HIP(hipStreamSynchronize(st));   // the local buffers are freed on return
    return TTK_OK;
  }
  TTK_TRY(qr_blocked(A.as<double>(), (int)N, k, (int)N, R, k, work.as<double>(), st));
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_q_rowmajor<float>, dim3(nblocks(N * k)), dim3(256), 0, st, A.as<double>(), N, k,
                       static_cast<float*>(Q));
  else
    hipLaunchKernelGGL(k_q_rowmajor<double>, dim3(nblocks(N * k)), dim3(256), 0, st, A.as<double>(), N, k,
                       static_cast<double*>(Q));
  TTK_HIP(hipGetLastError());
  TTK_HIP(hipStreamSynchronize(st));   // the local buffers are freed on return
  return TTK_OK;
}

size_t global_online_work(int rs, int rt, int B) {
  const size_t k = (size_t)rs + rt;
  // per theta: P (k x rt), Mh, J (Jacobi input), V, VS (k x k each), sigma + SVD workspace
  return (size_t)B * (k * rt + 4 * k * k + jacobi_sigma_doubles((int)k)) + 16;
}

void global_online(const double* R, int rs, int rt, const double* M, int B, int out_dtype, void* W, double* work,
                   hipStream_t st) {
  if (B <= 0) return;
  const int k = rs + rt;
  const size_t kk = (size_t)k * k;
  double* P = work;
  double* Mh = P + (size_t)B * k * rt;
  double* J = Mh + (size_t)B * kk;
  double* V = J + (size_t)B * kk;
  double* VS = V + (size_t)B * kk;
  double* sig = VS + (size_t)B * kk;
  const size_t sS = jacobi_sigma_doubles(k);
  const double* R1 = R;                    // R[:, :rs]
  const double* R2 = R + (size_t)rs * k;   // R[:, rs:]
  for (int b = 0; b < B; ++b) {
    // P = R1 M_b / 2 (k x rt); Mh_b = P R2^T, symmetrised below: R Hhat R^T = P R2^T + R2 P^T
    gemm64(0, 0, k, rt, rs, 0.5, R1, k, M + (size_t)b * rs * rt, rs, 0.0, P + (size_t)b * k * rt, k, st);
    gemm64(0, 1, k, k, rt, 1.0, P + (size_t)b * k * rt, k, R2, k, 0.0, Mh + (size_t)b * kk, k, st);
  }
  hipLaunchKernelGGL(k_sym_copy, dim3(B), dim3(256), 0, st, Mh, J, k, kk);
  // |Mh| = V Sigma V^T from the right singular vectors; equally U Sigma U^T
  // from the left ones, since for a symmetric matrix the left and right
  // singular subspaces of every singular value coincide (also where +lambda
  // and -lambda share it).  Small k: all thetas at once, one workgroup each,
  // with V.  Large k (past one workgroup's LDS): per theta, the left vectors
  // by the block iteration over many workgroups.
  const double* Vuse = V;
  if (k <= 141) {
    jacobi_svd_batched(J, k, k, kk, V, k, kk, sig, sS, B, st);
  } else {
    // The block iteration runs on L_b = R2_b^T from J_b = Q2_b R2_b: J_b is
    // symmetric, so J_b = L_b Q2_b^T and L_b has its singular values and left
    // vectors, and one QR step leaves L_b's columns far closer to orthogonal
    // (fewer sweeps).  R2_b goes to V_b (unused on this path), the QR's
    // workspace to VS (used only after the iteration).
    if (qr_r_batched_work(k, B) <= (size_t)B * kk &&
        qr_r_batched(J, k, k, kk, V, k, kk, VS, B, st) == TTK_OK)
      hipLaunchKernelGGL(k_transpose_batched, dim3(nblocks((int64_t)k * k), B), dim3(256), 0, st, (const double*)V,
                         k, kk, J);
    if (!jacobi_svd_left_batched(J, k, k, kk, sig, sS, B, st))
      jacobi_svd_batched(J, k, k, kk, V, k, kk, sig, sS, B, st);   // (k above 512)
    Vuse = J;   // normalised left vectors on either path
  }
  hipLaunchKernelGGL(k_scale_cols, dim3(B), dim3(256), 0, st, Vuse, sig, sS, k, kk, VS);
  // W_b = (Mh_b + VS_b Vuse_b^T) / 2, one product per theta into whichever
  // of J and V does not hold the vectors, then in the output precision
  double* C = Vuse == J ? V : J;
  (void)hipMemcpyAsync(C, Mh, (size_t)B * kk * sizeof(double), hipMemcpyDeviceToDevice, st);
  for (int b = 0; b < B; ++b)
    gemm64(0, 1, k, k, k, 0.5, VS + (size_t)b * kk, k, Vuse + (size_t)b * kk, k, 0.5, C + (size_t)b * kk, k, st);
  if (out_dtype == TTK_FP32)
    hipLaunchKernelGGL(k_store<float>, dim3(nblocks((int64_t)B * kk)), dim3(256), 0, st, (const double*)C,
                       (int64_t)B * kk, static_cast<float*>(W));
  else
    hipLaunchKernelGGL(k_store<double>, dim3(nblocks((int64_t)B * kk)), dim3(256), 0, st, (const double*)C,
                       (int64_t)B * kk, static_cast<double*>(W));
}

size_t global2_work(int rs, int rt) {
  const size_t k = (size_t)rs + rt;
  return global_online_work(rs, rt, 1) + 2 * k * k + jacobi_sigma_doubles((int)k) + 64 + k * k +
         qr_r_batched_work((int)k, 1);
}

tt_status global2_online(const double* R, int rs, int rt, const double* M, double eps, double* work, double** Uhat,
                         double** lam, int* rc, hipStream_t st) {
  const int k = rs + rt;
  const size_t kk = (size_t)k * k;
  double* gw = work;                                    // global_online's workspace (B = 1)
  double* Wp = gw + global_online_work(rs, rt, 1);      // W_+ (k x k), FP64
  double* J = Wp + kk;                                  // its Jacobi input, then the eigenvectors
  double* sig = J + kk;                                 // eigenvalues, then the SVD workspace
  global_online(R, rs, rt, M, 1, TTK_FP64, Wp, gw, st);
  const double* Mh = gw + (size_t)k * rt;               // R Hhat R^T, symmetrised (global_online's layout)
  double* nrm = sig + jacobi_sigma_doubles(k);          // ||Mh||_F
  double* R2 = nrm + 64;                                // QR preconditioning: R2, then the QR's workspace
  nrm2(Mh, (int64_t)kk, nrm, st);
  TTK_HIP(hipMemcpyAsync(J, Wp, kk * sizeof(double), hipMemcpyDeviceToDevice, st));
  // as in global_online: the iteration on L = R2^T from W_+ = Q2 R2 (W_+ symmetric)
  if (k > 141 && qr_r_batched(J, k, k, kk, R2, k, kk, R2 + kk, 1, st) == TTK_OK)
    hipLaunchKernelGGL(k_transpose_batched, dim3(nblocks((int64_t)k * k), 1), dim3(256), 0, st, (const double*)R2, k,
                       kk, J);
  if (!jacobi_svd_left(J, k, k, sig, st)) {   // (k above 512: the single-workgroup form, with V, of W_+ itself)
    TTK_HIP(hipMemcpyAsync(J, Wp, kk * sizeof(double), hipMemcpyDeviceToDevice, st));
    DBuf V;
    TTK_TRY(V.alloc(kk * sizeof(double)));
    jacobi_svd(J, k, k, V.as<double>(), k, sig, st);
    TTK_HIP(hipStreamSynchronize(st));        // V is released on return
  }
  TTK_HIP(hipGetLastError());
  std::vector<double> ev(k + 1);
  TTK_HIP(hipMemcpyAsync(ev.data(), sig, (size_t)k * sizeof(double), hipMemcpyDeviceToHost, st));
  TTK_HIP(hipMemcpyAsync(ev.data() + k, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
  TTK_HIP(hipStreamSynchronize(st));
  // the smallest r whose discarded tail sqrt(sum_{i > r} lambda_i^2) is within
  // eps ||Mh||_F (eigenvalues already in decreasing order); k if none is
  const double bound = eps * ev[k];
  std::vector<double> tail(k + 1, 0.0);
  for (int i = k - 1; i >= 0; --i) tail[i] = tail[i + 1] + ev[i] * ev[i];
  int r = k;
  for (int q = 1; q <= k; ++q)
    if (std::sqrt(tail[q]) <= bound) { r = q; break; }
  if (!(ev[0] > 0.0)) r = 0;   // no positive eigenvalue
  *rc = r;
  *Uhat = J;
  *lam = sig;
  return TTK_OK;
}

}  // namespace ttk
