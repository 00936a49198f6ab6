// The apply y_b = S H(theta_b) T^T x_b of the low-rank form (Section 1) and
// its backward pass, split into tall contractions over the points
//     reduce:  W = F^T X   (r x B, F = S or T, N x r row-major, X N x B)
//     expand:  Y = F Z     (N x B)
// and small per-theta products done by batched_matvec / batched_bilinear.
// Plain (B = 1): a GEMV pair, bound by reading F once.  Batched: register-
// tiled GEMMs that read F once for all B columns.  Products are formed in
// the working precision and summed in double over point tiles (a float32
// running sum over 10^5 points loses digits); partial sums of the reduce over
// point chunks are combined with atomics (order not fixed).
#include "ttk_internal.h"

namespace ttk {

namespace {

template <class T>
__global__ void k_fill(T* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

// Widest factor the apply kernels take: U, V (r <= MAXR) and the Global-1 Q
// (k = r_s + r_t <= 2 MAXR).
constexpr int MAXF = 2 * MAXR;

// w[c] += sum_p F[p, c] x[p]; one row per wave at a time, lanes over columns.
template <class T>
__global__ void __launch_bounds__(256) k_reduce_plain(const T* F, int ldf, int64_t N, int r, const T* x, T* w) {
  __shared__ T red[4][MAXF];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // products in T, sums in double: a long reduction over points must not
  // accumulate the rounding of a float32 running sum
  double acc[MAXF / 64];
#pragma unroll
  for (int q = 0; q < MAXF / 64; ++q) acc[q] = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 4 + wv; p < N; p += (int64_t)gridDim.x * 4) {
    const T xv = x[p];
    const T* row = F + p * ldf;
#pragma unroll
    for (int q = 0; q < MAXF / 64; ++q) {
      const int c = lane + 64 * q;
      if (c < r) acc[q] += (double)(row[c] * xv);
    }
  }
#pragma unroll
  for (int q = 0; q < MAXF / 64; ++q) {
    const int c = lane + 64 * q;
    if (c < r) red[wv][c] = (T)acc[q];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += 256) atomicAdd(&w[c], red[0][c] + red[1][c] + red[2][c] + red[3][c]);
}

// y[p] = sum_c F[p, c] z[c]; 16 lanes per row, reduced by shuffles.
template <class T>
__global__ void __launch_bounds__(256) k_expand_plain(const T* F, int ldf, int64_t N, int r, const T* z, T* y) {
  __shared__ T zs[MAXF];
  for (int c = threadIdx.x; c < r; c += 256) zs[c] = z[c];
  __syncthreads();
  const int sub = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;   // 16 rows per block iteration
  for (int64_t p = (int64_t)blockIdx.x * 16 + grp; p < N; p += (int64_t)gridDim.x * 16) {
    const T* row = F + p * ldf;
    T s = (T)0;
    for (int c = sub; c < r; c += 16) s += row[c] * zs[c];
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    if (sub == 0) y[p] = s;
  }
}

// W (r x B) += F^T X over the rows of one chunk; tile 64 (r) x 64 (b).
template <class T>
__global__ void __launch_bounds__(256) k_reduce_tiled(const T* F, int ldf, int64_t N, int r, const T* X,
                                                      int64_t ldx, int B, int64_t chunk, T* W) {
  __shared__ T Fs[16][64 + 1];
  __shared__ T Xs[16][64 + 1];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
  const int64_t pbeg = (int64_t)blockIdx.z * chunk;
  const int64_t pend = (pbeg + chunk < N) ? pbeg + chunk : N;
  const int tr = tid / 16, tb = tid % 16;
  // each 16-row tile is summed in T, the tiles in double
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, c = e % 64;
      const int64_t p = p0 + kk;
      Fs[kk][c] = (p < pend && r0 + c < r) ? F[p * ldf + r0 + c] : (T)0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e % 16, j = e / 16;
      const int64_t p = p0 + kk;
      Xs[kk][j] = (p < pend && b0 + j < B) ? X[p + (int64_t)(b0 + j) * ldx] : (T)0;
    }
    __syncthreads();
    T t[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) t[i][j] = (T)0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Fs[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Xs[kk][tb * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[i][j] += a[i] * b[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += (double)t[i][j];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = r0 + tr * 4 + i, bb = b0 + tb * 4 + j;
      if (rr < r && bb < B) atomicAdd(&W[rr + (int64_t)bb * r], (T)acc[i][j]);
    }
}

// Y (N x B) = F Z, tile 64 rows x 64 columns; threads sweep rows fastest so
// the column-major stores coalesce.
template <class T>
__global__ void __launch_bounds__(256) k_expand_tiled(const T* F, int ldf, int64_t N, int r, const T* Z, int B,
                                                      T* Y, int64_t ldy) {
  __shared__ T Fs[64][16 + 1];
  __shared__ T Zs[16][64 + 1];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int b0 = blockIdx.y * 64;
  const int tp = tid % 16, tb = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < r; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int pl = e / 16, kk = e % 16;
      const int64_t p = p0 + pl;
      Fs[pl][kk] = (p < N && k0 + kk < r) ? F[p * ldf + k0 + kk] : (T)0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e % 16, j = e / 16;
      Zs[kk][j] = (k0 + kk < r && b0 + j < B) ? Z[(k0 + kk) + (int64_t)(b0 + j) * r] : (T)0;
    }
    __syncthreads();
    T t[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) t[i][j] = (T)0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Fs[tp + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Zs[kk][tb * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[i][j] += a[i] * b[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += (double)t[i][j];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int bb = b0 + tb * 4 + j;
    if (bb >= B) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = p0 + tp + 16 * i;
      if (p < N) Y[p + (int64_t)bb * ldy] = (T)acc[i][j];
    }
  }
}

// y_b = op(M_b) x_b, M_b rows x cols column-major at M + b rows cols.
template <class T>
__global__ void __launch_bounds__(256) k_bmatvec(const T* M, int rows, int cols, int trans, const T* x, int B,
                                                 T* y) {
  __shared__ T xs[MAXF];
  const int nin = trans ? rows : cols, nout = trans ? cols : rows;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const T* Mb = M + (size_t)b * rows * cols;
    __syncthreads();
    for (int i = threadIdx.x; i < nin; i += 256) xs[i] = x[(size_t)b * nin + i];
    __syncthreads();
    for (int o = threadIdx.x; o < nout; o += 256) {
      double s = 0.0;
      if (!trans)
        for (int c = 0; c < cols; ++c) s += (double)Mb[o + (size_t)c * rows] * (double)xs[c];
      else
        for (int i = 0; i < rows; ++i) s += (double)Mb[i + (size_t)o * rows] * (double)xs[i];
      y[(size_t)b * nout + o] = (T)s;
    }
  }
}

// dtheta[b, j] = a_b^T dM_{b,j} w_b.
template <class T>
__global__ void __launch_bounds__(256) k_bilinear(const T* A, const T* dM, const T* W, int rs, int rt, int B,
                                                  int dt, T* dth) {
  __shared__ T as[MAXR];
  __shared__ double red[256];
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    __syncthreads();
    for (int i = threadIdx.x; i < rs; i += 256) as[i] = A[(size_t)b * rs + i];
    __syncthreads();
    for (int j = 0; j < dt; ++j) {
      const T* D = dM + ((size_t)b * dt + j) * rs * rt;
      double s = 0.0;
      for (int c = threadIdx.x; c < rt; c += 256) {
        double t = 0.0;
        for (int i = 0; i < rs; ++i) t += (double)as[i] * (double)D[i + (size_t)c * rs];
        s += t * (double)W[(size_t)b * rt + c];
      }
      red[threadIdx.x] = s;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x == 0) dth[(size_t)b * dt + j] = (T)red[0];
      __syncthreads();
    }
  }
}

inline unsigned grid_cap(int64_t want, int64_t cap) { return (unsigned)std::max<int64_t>(1, std::min(want, cap)); }

}  // namespace

void fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (!n) return;
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_cap((int64_t)(n + 255) / 256, 4096)), dim3(256), 0, st,
                     static_cast<float*>(p), n);
}

void apply_reduce(int dtype, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx, int B, void* W,
                  hipStream_t st) {
  const size_t es = dtype == TTK_FP32 ? 4 : 8;
  fill_zero(W, (size_t)r * B * es, st);
  if (N <= 0) return;
  if (B == 1) {
    const unsigned g = grid_cap((N + 63) / 64, 4096);
    if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_reduce_plain<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(X), static_cast<float*>(W));
    else
      hipLaunchKernelGGL(k_reduce_plain<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(X), static_cast<double*>(W));
    return;
  }
  const int rt = (r + 63) / 64, bt = (B + 63) / 64;
  int64_t nch = std::max<int64_t>(1, std::min<int64_t>((N + 511) / 512, (4096 + rt * bt - 1) / (rt * bt)));
  int64_t chunk = (N + nch - 1) / nch;
  chunk = (chunk + 15) / 16 * 16;
  nch = (N + chunk - 1) / chunk;
  dim3 grid(rt, bt, (unsigned)nch);
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_reduce_tiled<float>, grid, dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                       static_cast<const float*>(X), ldx, B, chunk, static_cast<float*>(W));
  else
    hipLaunchKernelGGL(k_reduce_tiled<double>, grid, dim3(256), 0, st, static_cast<const double*>(F), ldf, N, r,
                       static_cast<const double*>(X), ldx, B, chunk, static_cast<double*>(W));
}

void apply_expand(int dtype, const void* F, int ldf, int64_t N, int r, const void* Z, int B, void* Y, int64_t ldy,
                  hipStream_t st) {
  if (N <= 0) return;
  if (B == 1) {
    const unsigned g = grid_cap((N + 15) / 16, 8192);
    if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_expand_plain<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(Z), static_cast<float*>(Y));
    else
      hipLaunchKernelGGL(k_expand_plain<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(Z), static_cast<double*>(Y));
    return;
  }
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((B + 63) / 64));
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_expand_tiled<float>, grid, dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                       static_cast<const float*>(Z), B, static_cast<float*>(Y), ldy);
  else
    hipLaunchKernelGGL(k_expand_tiled<double>, grid, dim3(256), 0, st, static_cast<const double*>(F), ldf, N, r,
                       static_cast<const double*>(Z), B, static_cast<double*>(Y), ldy);
}

void batched_matvec(int dtype, const void* M, int rows, int cols, int trans, const void* x, int B, void* y,
                    hipStream_t st) {
  if (B <= 0) return;
  const unsigned g = grid_cap(B, 2048);
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_bmatvec<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(M), rows, cols, trans,
                       static_cast<const float*>(x), B, static_cast<float*>(y));
  else
    hipLaunchKernelGGL(k_bmatvec<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(M), rows, cols,
                       trans, static_cast<const double*>(x), B, static_cast<double*>(y));
}

void batched_bilinear(int dtype, const void* A, const void* dM, const void* W, int rs, int rt, int B, int dt,
                      void* dtheta, hipStream_t st) {
  if (B <= 0 || dt <= 0) return;
  const unsigned g = grid_cap(B, 2048);
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_bilinear<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(A),
                       static_cast<const float*>(dM), static_cast<const float*>(W), rs, rt, B, dt,
                       static_cast<float*>(dtheta));
  else
    hipLaunchKernelGGL(k_bilinear<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(A),
                       static_cast<const double*>(dM), static_cast<const double*>(W), rs, rt, B, dt,
                       static_cast<double*>(dtheta));
}

}  // namespace ttk
