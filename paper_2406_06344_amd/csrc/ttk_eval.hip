// Kernel evaluation on the Chebyshev grid: the entries of the grid tensor
// m_{i_1..i_D} = f_kappa(eta) with eta_j the node i_j of dimension j, in the
// variable order (x, theta, y) (Section 1, "Our approach"; Section 2.4,
// "Multivariate approximation").  The cross algorithm addresses entries
// through its index sets, so multi-indices are assembled here on the device
// from (left set row, middle node indices, right set row) and never shipped
// from the host.  All evaluation is double precision.
#include "ttk_eval_dev.h"
#include "ttk_wave.h"

namespace ttk {

namespace {

constexpr int EB = 256;   // threads per evaluation block

// Block-wide max of |value| folded into amax[b mod AMAX_SLOTS] for block b
// with one atomic per block (non-negative doubles order like their bit
// patterns, so an integer atomic max is exact).
__device__ inline void fold_amax(double v, double* amax) {
  __shared__ double red[EB / 64];
  v = wave64_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    atomicMax(reinterpret_cast<unsigned long long*>(amax + (blockIdx.x % AMAX_SLOTS)),
              (unsigned long long)__double_as_longlong(v));
  }
}

// out[i + j*nr] (or out[j + i*nc] when trans_out) = A(rows[i], cols[j])
template <int d, int dt, bool G>
__global__ void __launch_bounds__(EB) k_eval_product(KSpec ks, Addr a, const int32_t* rows, int nr,
                                                     const int32_t* cols, int nc, int trans_out, double* out,
                                                     double* amax) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN];
  stage_nodes<D>(ks.nodes, sn);
  const int64_t total = (int64_t)nr * nc;
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int i, jj;
    if (trans_out) { jj = (int)(e % nc); i = (int)(e / nc); }
    else { i = (int)(e % nr); jj = (int)(e / nr); }
    const int row = rows ? rows[i] : i;
    const int col = cols ? cols[jj] : jj;
    double c[D];
    addr_coords<D>(a, sn, row, col, c);
    const double v = kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
    out[e] = v;
    m = fmax(m, fabs(v));
  }
  if (amax) fold_amax(m, amax);
}

template <int d, int dt, bool G>
__global__ void __launch_bounds__(EB) k_eval_list(KSpec ks, Addr a, const int32_t* rows, const int32_t* cols,
                                                  int np, double* out, double* amax) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN];
  stage_nodes<D>(ks.nodes, sn);
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    double c[D];
    addr_coords<D>(a, sn, rows[i], cols[i], c);
    const double v = kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
    out[i] = v;
    m = fmax(m, fabs(v));
  }
  if (amax) fold_amax(m, amax);
}

// Up to three blocks of entries in one launch (see EvalSeg).
template <int d, int dt, bool G>
__global__ void __launch_bounds__(EB) k_eval_segs(KSpec ks, Addr a, EvalSeg s0, EvalSeg s1, EvalSeg s2, int nseg,
                                                  double* amax) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN];
  stage_nodes<D>(ks.nodes, sn);
  const int64_t n0 = (int64_t)s0.nr * s0.nc;
  const int64_t n1 = nseg > 1 ? (int64_t)s1.nr * s1.nc : 0;
  const int64_t n2 = nseg > 2 ? (int64_t)s2.nr * s2.nc : 0;
  const int64_t total = n0 + n1 + n2;
  double m = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const bool in0 = g < n0, in1 = !in0 && g < n0 + n1;
    const EvalSeg sg = in0 ? s0 : (in1 ? s1 : s2);
    const int64_t e = in0 ? g : (in1 ? g - n0 : g - n0 - n1);
    int row, col;
    if (sg.mode == 2) {                   // list of (row, col) pairs, nc == 1
      row = sg.rows[e];
      col = sg.cols[e];
    } else {
      int i, jj;
      if (sg.mode == 1) { jj = (int)(e % sg.nc); i = (int)(e / sg.nc); }
      else { i = (int)(e % sg.nr); jj = (int)(e / sg.nr); }
      row = sg.rows ? sg.rows[i] : i;
      col = sg.cols ? sg.cols[jj] : jj;
    }
    double c[D];
    addr_coords<D>(a, sn, row, col, c);
    const double v = kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
    sg.out[e] = v;
    m = fmax(m, fabs(v));
  }
  if (amax) fold_amax(m, amax);
}

template <class I, int d, int dt, bool G>
__global__ void __launch_bounds__(EB) k_eval_multi(KSpec ks, const I* idx, int64_t P, double* out) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN];
  stage_nodes<D>(ks.nodes, sn);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    double c[D];
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = sn[j * MAXN + (int)idx[i * D + j]];
    out[i] = kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
  }
}

// Dense block: one thread per (i, j), i fastest so stores to column-major K coalesce.
template <class T, int d, int dt, bool G>
__global__ void __launch_bounds__(EB) k_eval_dense(KSpec ks, const T* X, int64_t nx, const T* Y, int64_t ny,
                                                   double th0, double th1, T* K, int64_t ldk) {
  const int64_t total = nx * ny;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % nx, j = e / nx;
    double c[2 * d + dt];
#pragma unroll
    for (int q = 0; q < d; ++q) c[q] = (double)X[q * nx + i];
    if (dt > 0) c[d] = th0;
    if (dt > 1) c[d + (dt > 1 ? 1 : 0)] = th1;
#pragma unroll
    for (int q = 0; q < d; ++q) c[d + dt + q] = (double)Y[q * ny + j];
    K[i + j * ldk] = (T)kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
  }
}

inline int blocks_for(int64_t n, int bs = EB, int cap = 16384) {
  int64_t b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

}  // namespace

void eval_product(const KSpec& ks, const Addr& a, const int32_t* rows, int nr, const int32_t* cols,
                  int nc, double* out, hipStream_t st, double* amax, bool trans_out) {
  if (nr <= 0 || nc <= 0) return;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_product<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
                       dim3(blocks_for((int64_t)nr * nc)), dim3(EB), 0, st, ks, a, rows, nr, cols, nc,
                       trans_out ? 1 : 0, out, amax);
  });
}

void eval_list(const KSpec& ks, const Addr& a, const int32_t* rows, const int32_t* cols, int np,
               double* out, hipStream_t st, double* amax) {
  if (np <= 0) return;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_list<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>), dim3(blocks_for(np)), dim3(EB),
                       0, st, ks, a, rows, cols, np, out, amax);
  });
}

void eval_segs(const KSpec& ks, const Addr& a, const EvalSeg* segs, int nseg, hipStream_t st, double* amax) {
  int64_t total = 0;
  for (int i = 0; i < nseg; ++i) total += (int64_t)segs[i].nr * segs[i].nc;
  if (total <= 0) return;
  const EvalSeg z{};
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_segs<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>), dim3(blocks_for(total)), dim3(EB),
                       0, st, ks, a, segs[0], nseg > 1 ? segs[1] : z, nseg > 2 ? segs[2] : z, nseg, amax);
  });
}

void eval_multi16(const KSpec& ks, const int16_t* idx, int64_t P, double* out, hipStream_t st) {
  if (P <= 0) return;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_multi<int16_t, decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>), dim3(blocks_for(P)),
                       dim3(EB), 0, st, ks, idx, P, out);
  });
}

void eval_multi32(const KSpec& ks, const int32_t* idx, int64_t P, double* out, hipStream_t st) {
  if (P <= 0) return;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_multi<int32_t, decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>), dim3(blocks_for(P)),
                       dim3(EB), 0, st, ks, idx, P, out);
  });
}

void eval_dense_f32(const KSpec& ks, const float* X, int64_t nx, const float* Y, int64_t ny,
                    const double* theta, float* K, int64_t ldk, hipStream_t st) {
  if (nx <= 0 || ny <= 0) return;
  const double t0 = ks.dt > 0 ? theta[0] : 0.0, t1 = ks.dt > 1 ? theta[1] : 0.0;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_dense<float, decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
                       dim3(blocks_for(nx * ny)), dim3(EB), 0, st, ks, X, nx, Y, ny, t0, t1, K, ldk);
  });
}

void eval_dense_f64(const KSpec& ks, const double* X, int64_t nx, const double* Y, int64_t ny,
                    const double* theta, double* K, int64_t ldk, hipStream_t st) {
  if (nx <= 0 || ny <= 0) return;
  const double t0 = ks.dt > 0 ? theta[0] : 0.0, t1 = ks.dt > 1 ? theta[1] : 0.0;
  with_dims(ks, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_eval_dense<double, decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
                       dim3(blocks_for(nx * ny)), dim3(EB), 0, st, ks, X, nx, Y, ny, t0, t1, K, ldk);
  });
}

}  // namespace ttk
