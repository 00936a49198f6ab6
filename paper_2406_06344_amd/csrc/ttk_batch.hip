// Apply and backward over an interaction list of box pairs (the FMM /
// H-matrix use of Section 1):
//     y[S_p, b] += U_p M_c(p)(theta_b) V_p^T x[T_p, b]     for every pair p,
// with the backward pass of L = sum_b <g_b, y_b>.  Each pair has its own
// factor blocks U_p, V_p (rows of its sources / targets) and shares the core
// M_c of its class.  Every tall contraction over points runs as ONE launch
// over a work list of (pair, row chunk, rank tile, theta tile) items, so the
// uneven pair sizes (about 1k to 64k points) balance across the chip.
//   reduce:  W_p = F_p^T X[rows of p]   (r_p x B per pair, atomics over chunks)
//   small:   Z_p[:, b] = M_c(theta_b) W_p[:, b]  (or M_c^T)
//   expand:  Y[rows of p] += F_p Z_p   (atomics: pairs may share rows)
//   bilinear: dtheta[b, j] = sum_p a_pb^T dM_c,bj w_pb  (per-pair partials, then a fixed-order sum)
#include "ttk_internal.h"

namespace ttk {

namespace {

constexpr int BT = 64;    // rank / theta tile
constexpr int BK = 16;    // rows per LDS step

template <class T>
__global__ void __launch_bounds__(256) k_batch_reduce(const T* F, const BatchSide* sides, const BatchItem* items,
                                                      const T* X, int64_t ldx, int B, T* W) {
  __shared__ T Fs[BK][BT + 1];
  __shared__ T Xs[BK][BT + 1];
  const BatchItem it = items[blockIdx.x];
  const BatchSide sd = sides[it.side];
  const int r = sd.r;
  const T* Fp = F + sd.foff;
  const int tid = threadIdx.x;
  const int tr = tid / 16, tb = tid % 16;
  double acc[4][4];   // tiles of BK rows summed in T, the tiles in double
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int64_t pend = it.row0 + it.nrows;
  for (int64_t p0 = it.row0; p0 < pend; p0 += BK) {
    for (int e = tid; e < BK * BT; e += 256) {
      const int kk = e / BT, c = e % BT;
      const int64_t p = p0 + kk;
      Fs[kk][c] = (p < pend && it.r0 + c < r) ? Fp[p * r + it.r0 + c] : (T)0;
    }
    for (int e = tid; e < BK * BT; e += 256) {
      const int kk = e % BK, j = e / BK;
      const int64_t p = p0 + kk;
      Xs[kk][j] = (p < pend && it.b0 + j < B) ? X[sd.roff + p + (int64_t)(it.b0 + j) * ldx] : (T)0;
    }
    __syncthreads();
    T t[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) t[i][j] = (T)0;
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
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
  T* Wp = W + sd.woff;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = it.r0 + tr * 4 + i, bb = it.b0 + tb * 4 + j;
      if (rr < r && bb < B) atomicAdd(&Wp[rr + (int64_t)bb * r], (T)acc[i][j]);
    }
}

// Y[roff + p, b] += sum_c F_p[p, c] Z_p[c, b] for 64 rows x 64 thetas.
template <class T>
__global__ void __launch_bounds__(256) k_batch_expand(const T* F, const BatchSide* sides, const BatchItem* items,
                                                      const T* Z, int B, T* Y, int64_t ldy) {
  __shared__ T Fs[BT][BK + 1];
  __shared__ T Zs[BK][BT + 1];
  const BatchItem it = items[blockIdx.x];
  const BatchSide sd = sides[it.side];
  const int r = sd.r;
  const T* Fp = F + sd.foff;
  const T* Zp = Z + sd.woff;
  const int tid = threadIdx.x;
  const int tp = tid % 16, tb = tid / 16;
  const int64_t pend = it.row0 + it.nrows;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  for (int k0 = 0; k0 < r; k0 += BK) {
    for (int e = tid; e < BT * BK; e += 256) {
      const int pl = e / BK, kk = e % BK;
      const int64_t p = it.row0 + pl;
      Fs[pl][kk] = (p < pend && k0 + kk < r) ? Fp[p * r + k0 + kk] : (T)0;
    }
    for (int e = tid; e < BK * BT; e += 256) {
      const int kk = e % BK, j = e / BK;
      Zs[kk][j] = (k0 + kk < r && it.b0 + j < B) ? Zp[(k0 + kk) + (int64_t)(it.b0 + j) * r] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Fs[tp + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Zs[kk][tb * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int bb = it.b0 + tb * 4 + j;
    if (bb >= B) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = it.row0 + tp + 16 * i;
      if (p < pend) atomicAdd(&Y[sd.roff + p + (int64_t)bb * ldy], acc[i][j]);
    }
  }
}

// One workgroup per pair: Zout_p[:, b] = op(M_c(theta_b)) Win_p[:, b], with
// M_c(theta_b) r_s x r_t column-major at M + moff[p] + b r_s r_t.
template <class T>
__global__ void __launch_bounds__(256) k_batch_small(const T* M, const int64_t* moff, const BatchSide* in_s,
                                                     const BatchSide* out_s, int trans, const T* Win, T* Zout,
                                                     int B) {
  const int p = blockIdx.x;
  const BatchSide si = in_s[p], so = out_s[p];
  const int rin = si.r, rout = so.r;
  const int rs = trans ? rin : rout;     // rows of M_c
  const T* Mp = M + moff[p];
  const T* w = Win + si.woff;
  T* z = Zout + so.woff;
  const int64_t total = (int64_t)rout * B;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e % rout), b = (int)(e / rout);
    const T* Mb = Mp + (int64_t)b * rin * rout;
    const T* wb = w + (int64_t)b * rin;
    double s = 0.0;
    if (!trans)
      for (int j = 0; j < rin; ++j) s += (double)Mb[i + (int64_t)j * rs] * (double)wb[j];
    else
      for (int j = 0; j < rin; ++j) s += (double)Mb[j + (int64_t)i * rs] * (double)wb[j];
    z[i + (int64_t)b * rout] = (T)s;
  }
}

// part[(b dt + j) npairs + p] = a_pb^T dM_c,bj w_pb; dM of pair p at dM + dmoff[p],
// matrix (b, j) at + (b dt + j) r_s r_t.
template <class T>
__global__ void __launch_bounds__(256) k_batch_bilinear(const T* A, const BatchSide* s_side, const T* dM,
                                                        const int64_t* dmoff, const T* W, const BatchSide* t_side,
                                                        int B, int dt, int npairs, double* part) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  const BatchSide ss = s_side[p], ts = t_side[p];
  const int rs = ss.r, rt = ts.r;
  const T* Ap = A + ss.woff;
  const T* Wp = W + ts.woff;
  const T* D = dM + dmoff[p];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int bj = 0; bj < B * dt; ++bj) {
    const int b = bj / dt;
    const T* Db = D + (int64_t)bj * rs * rt;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)rs * rt; e += blockDim.x) {
      const int i = (int)(e % rs), c = (int)(e / rs);
      s += (double)Ap[i + (int64_t)b * rs] * (double)Db[e] * (double)Wp[c + (int64_t)b * rt];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)bj * npairs + p] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

template <class T>
__global__ void k_batch_sum(const double* part, int npairs, int count, T* out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < npairs; ++p) s += part[(int64_t)e * npairs + p];
    out[e] = (T)s;
  }
}

// Y[i + b ldy] = 0 for i < rows, b < B.
template <class T>
__global__ void k_fill_cols(T* Y, int64_t rows, int B, int64_t ldy) {
  const int64_t total = rows * B;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    Y[e % rows + (e / rows) * ldy] = (T)0;
}

inline unsigned gridn(int64_t n, int64_t cap = 8192) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

}  // namespace

void batch_reduce(int dtype, const void* F, const BatchSide* sides, const BatchItem* items, int64_t nitems,
                  const void* X, int64_t ldx, int B, void* W, hipStream_t st) {
  if (nitems <= 0) return;
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_batch_reduce<float>, dim3((unsigned)nitems), dim3(256), 0, st, static_cast<const float*>(F),
                       sides, items, static_cast<const float*>(X), ldx, B, static_cast<float*>(W));
  else
    hipLaunchKernelGGL(k_batch_reduce<double>, dim3((unsigned)nitems), dim3(256), 0, st,
                       static_cast<const double*>(F), sides, items, static_cast<const double*>(X), ldx, B,
                       static_cast<double*>(W));
}

void batch_expand(int dtype, const void* F, const BatchSide* sides, const BatchItem* items, int64_t nitems,
                  const void* Z, int B, void* Y, int64_t ldy, hipStream_t st) {
  if (nitems <= 0) return;
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_batch_expand<float>, dim3((unsigned)nitems), dim3(256), 0, st, static_cast<const float*>(F),
                       sides, items, static_cast<const float*>(Z), B, static_cast<float*>(Y), ldy);
  else
    hipLaunchKernelGGL(k_batch_expand<double>, dim3((unsigned)nitems), dim3(256), 0, st,
                       static_cast<const double*>(F), sides, items, static_cast<const double*>(Z), B,
                       static_cast<double*>(Y), ldy);
}

void batch_small(int dtype, const void* M, const int64_t* moff, const BatchSide* in_s, const BatchSide* out_s,
                 int trans, const void* Win, void* Zout, int B, int npairs, hipStream_t st) {
  if (npairs <= 0) return;
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_batch_small<float>, dim3(npairs), dim3(256), 0, st, static_cast<const float*>(M), moff, in_s,
                       out_s, trans, static_cast<const float*>(Win), static_cast<float*>(Zout), B);
  else
    hipLaunchKernelGGL(k_batch_small<double>, dim3(npairs), dim3(256), 0, st, static_cast<const double*>(M), moff,
                       in_s, out_s, trans, static_cast<const double*>(Win), static_cast<double*>(Zout), B);
}

void batch_dtheta(int dtype, const void* A, const BatchSide* s_side, const void* dM, const int64_t* dmoff,
                  const void* W, const BatchSide* t_side, int B, int dt, int npairs, double* part, void* dtheta,
                  hipStream_t st) {
  if (npairs <= 0 || B <= 0 || dt <= 0) return;
  const int count = B * dt;
  if (dtype == TTK_FP32) {
    hipLaunchKernelGGL(k_batch_bilinear<float>, dim3(npairs), dim3(256), 0, st, static_cast<const float*>(A), s_side,
                       static_cast<const float*>(dM), dmoff, static_cast<const float*>(W), t_side, B, dt, npairs,
                       part);
    hipLaunchKernelGGL(k_batch_sum<float>, dim3(gridn(count)), dim3(256), 0, st, part, npairs, count,
                       static_cast<float*>(dtheta));
  } else {
    hipLaunchKernelGGL(k_batch_bilinear<double>, dim3(npairs), dim3(256), 0, st, static_cast<const double*>(A),
                       s_side, static_cast<const double*>(dM), dmoff, static_cast<const double*>(W), t_side, B, dt,
                       npairs, part);
    hipLaunchKernelGGL(k_batch_sum<double>, dim3(gridn(count)), dim3(256), 0, st, part, npairs, count,
                       static_cast<double*>(dtheta));
  }
}

void fill_cols(int dtype, void* Y, int64_t rows, int B, int64_t ldy, hipStream_t st) {
  if (rows <= 0 || B <= 0) return;
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_fill_cols<float>, dim3(gridn(rows * B)), dim3(256), 0, st, static_cast<float*>(Y), rows, B,
                       ldy);
  else
    hipLaunchKernelGGL(k_fill_cols<double>, dim3(gridn(rows * B)), dim3(256), 0, st, static_cast<double*>(Y), rows,
                       B, ldy);
}

}  // namespace ttk
