// The apply y_b = S H(theta_b) T^T x_b of the low-rank form (Section 1) and
// its backward pass, split into tall contractions over the points
//     reduce:  W = F^T X   (r x B, F = S or T, N x r row-major, X N x B)
//     expand:  Y = F Z     (N x B)
// and small per-theta products done by batched_matvec / batched_bilinear.
// Plain (B = 1): a GEMV pair, bound by reading F once.  Batched: GEMMs that
// read F once for all B columns: for B <= 16 the float32 skinny matrix-core
// kernels of ttk_apply_mfma.hip (aligned rows of F) or the skinny kernels
// here, for wider batches (r <= 128) the float32 matrix-core kernels of
// ttk_apply_mfma.hip, register-tiled VALU kernels otherwise (float64).  Products are formed in
// the working precision and summed in double over point tiles (a float32
// running sum over 10^5 points loses digits).  The plain and skinny reduces
// write one double partial sum per workgroup and a second launch adds them
// in a fixed order (thousands of same-address atomics serialise); the wide
// tiled reduce, with few workgroups per entry, combines its chunks by atomics
// (order not fixed).
#include "ttk_internal.h"
#include "ttk_wave.h"

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
__global__ void __launch_bounds__(256) k_reduce_plain(const T* F, int ldf, int64_t N, int r, const T* x,
                                                      double* part) {
  __shared__ double red[4][MAXF];
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
    if (c < r) red[wv][c] = acc[q];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += 256)
    part[(size_t)c * gridDim.x + blockIdx.x] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// out[e] = sum over workgroups w of part[e nw + w] (each entry's partials
// contiguous), e < count, in a fixed order: one wave per entry, eight
// interleaved sums per lane, then the wave's DPP sum.
template <class T>
__global__ void __launch_bounds__(256) k_sum_partials(const double* part, int nw, int count, T* out) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= count) return;   // (whole waves)
  const double* pe = part + (size_t)e * nw;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int w = lane;
  for (; w + 7 * 64 < nw; w += 8 * 64)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += pe[w + 64 * u];
  for (; w < nw; w += 64) a[0] += pe[w];
  const double s = wave64_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
  if (lane == 0) out[e] = (T)s;
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

// Skinny batches (2 <= B <= SB, r <= SR): the point dimension is long and the
// rest is small, so both contractions are bound by reading F once.
constexpr int SB = 16, SR = 128, ST = 64;   // batch, rank and point-tile limits

// W (r x B) += F^T X over one chunk of points.  Thread (g, c), c = t % 128,
// g = t / 128, owns column c of F and the rows g, g + 2, ... of every 64-row
// tile: it loads those 32 values at once (the next tile's while the current
// one is used) and multiplies them with the tile of X staged in LDS, summing
// the tile in T and the tiles in double; the two row groups meet in LDS and
// the chunk's sums go to part[blockIdx.x r B + c + b r] (contiguous per
// workgroup; k_sum_ranges and k_sum_final add them up).
template <class T>
__global__ void __launch_bounds__(256) k_reduce_skinny(const T* F, int ldf, int64_t N, int r, const T* X,
                                                       int64_t ldx, int B, int64_t chunk, double* part) {
  __shared__ T Xs[ST][SB + 1];
  __shared__ double red[SR][SB + 1];
  const int tid = threadIdx.x, c = tid & (SR - 1), g = tid >> 7;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = pbeg + chunk < N ? pbeg + chunk : N;
  const bool cok = c < r;
  double acc[SB];
#pragma unroll
  for (int b = 0; b < SB; ++b) acc[b] = 0.0;
  T f[ST / 2];
  auto load_f = [&](int64_t p0) {
#pragma unroll
    for (int u = 0; u < ST / 2; ++u) {
      const int64_t p = p0 + g + 2 * u;
      f[u] = (cok && p < pend) ? F[p * ldf + c] : (T)0;
    }
  };
  load_f(pbeg);
  for (int64_t p0 = pbeg; p0 < pend; p0 += ST) {
    __syncthreads();   // the previous tile of X is consumed
    for (int e = tid; e < ST * SB; e += 256) {
      const int row = e % ST, b = e / ST;
      const int64_t p = p0 + row;
      Xs[row][b] = (p < pend && b < B) ? X[p + (int64_t)b * ldx] : (T)0;
    }
    __syncthreads();
    T cur[ST / 2];
#pragma unroll
    for (int u = 0; u < ST / 2; ++u) cur[u] = f[u];
    if (p0 + ST < pend) load_f(p0 + ST);
    T t[SB];
#pragma unroll
    for (int b = 0; b < SB; ++b) t[b] = (T)0;
#pragma unroll
    for (int u = 0; u < ST / 2; ++u) {
      const T* xr = Xs[g + 2 * u];
#pragma unroll
      for (int b = 0; b < SB; ++b) t[b] += cur[u] * xr[b];
    }
#pragma unroll
    for (int b = 0; b < SB; ++b) acc[b] += (double)t[b];
  }
  if (g == 1)
#pragma unroll
    for (int b = 0; b < SB; ++b) red[c][b] = acc[b];
  __syncthreads();
  if (g == 0 && cok)
    for (int b = 0; b < B; ++b) part[(size_t)blockIdx.x * r * B + c + (size_t)b * r] = acc[b] + red[c][b];
}

// First level of the skinny reduce's sum: for 64 outputs per block (lanes,
// reads contiguous across them) and one of NRANGE ranges of workgroups
// (blockIdx.y), the four waves take every fourth workgroup of the range;
// the range's sum goes to sums[range count + e].
constexpr int NRANGE = 8;
__global__ void __launch_bounds__(256) k_sum_ranges(const double* part, int nw, int count, double* sums) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int per = (nw + NRANGE - 1) / NRANGE;
  const int w0 = blockIdx.y * per, w1 = min(nw, w0 + per);
  double a0 = 0.0, a1 = 0.0;
  if (e < count) {
    int w = w0 + wv;
    for (; w + 4 < w1; w += 8) {
      a0 += part[(size_t)w * count + e];
      a1 += part[(size_t)(w + 4) * count + e];
    }
    for (; w < w1; w += 4) a0 += part[(size_t)w * count + e];
  }
  red[wv][lane] = a0 + a1;
  __syncthreads();
  if (wv == 0 && e < count)
    sums[(size_t)blockIdx.y * count + e] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// out[e] = the NRANGE range sums of entry e, in order.
template <class T>
__global__ void k_sum_final(const double* sums, int count, T* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int k = 0; k < NRANGE; ++k) s += sums[(size_t)k * count + e];
  out[e] = (T)s;
}

// Y (N x B) = F Z for 64 points per block: the F tile (64 x r) is staged in
// LDS with row-contiguous loads, Z (r x B) beside it; thread (q, i) computes
// outputs 4 q .. 4 q + 3 of point i, summed in double.
template <class T>
__global__ void __launch_bounds__(256) k_expand_skinny(const T* F, int ldf, int64_t N, int r, const T* Z, int B,
                                                       T* Y, int64_t ldy) {
  __shared__ T Fs[ST][SR + 1];
  __shared__ T Zs[SR][SB];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * ST;
  for (int e = tid; e < r * SB; e += 256) {
    const int k = e / SB, b = e % SB;
    Zs[k][b] = b < B ? Z[k + (int64_t)b * r] : (T)0;
  }
  for (int e = tid; e < ST * r; e += 256) {
    const int i = e / r, k = e - i * r;
    const int64_t p = p0 + i;
    Fs[i][k] = p < N ? F[p * ldf + k] : (T)0;
  }
  __syncthreads();
  const int i = tid & (ST - 1), q = tid >> 6;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int k = 0; k < r; ++k) {
    const T fv = Fs[i][k];
    a0 += (double)(fv * Zs[k][4 * q]);
    a1 += (double)(fv * Zs[k][4 * q + 1]);
    a2 += (double)(fv * Zs[k][4 * q + 2]);
    a3 += (double)(fv * Zs[k][4 * q + 3]);
  }
  const int64_t p = p0 + i;
  if (p < N) {
    const double av[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * q + j < B) Y[p + (int64_t)(4 * q + j) * ldy] = (T)av[j];
  }
}

// y_b = op(M_b) x_b, M_b rows x cols column-major at M + b rows cols, one
// workgroup per b.  M x: 64 outputs per pass, the columns split over the four
// waves (coalesced loads down each column, four sums per lane), the waves'
// sums added in LDS.  M^T x: a wave per output, lanes down its column of M,
// a DPP wave sum.
template <class T>
__global__ void __launch_bounds__(256) k_bmatvec(const T* M, int rows, int cols, int trans, const T* x, int B,
                                                 T* y) {
  __shared__ double xs[MAXF];
  __shared__ double red[4][64];
  const int nin = trans ? rows : cols, nout = trans ? cols : rows;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const T* Mb = M + (size_t)b * rows * cols;
    __syncthreads();
    for (int i = tid; i < nin; i += 256) xs[i] = (double)x[(size_t)b * nin + i];
    __syncthreads();
    if (!trans) {
      for (int o0 = 0; o0 < rows; o0 += 64) {
        const int o = o0 + lane;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (o < rows) {
          int c = wv;
          for (; c + 12 < cols; c += 16) {
            s0 += (double)Mb[o + (size_t)c * rows] * xs[c];
            s1 += (double)Mb[o + (size_t)(c + 4) * rows] * xs[c + 4];
            s2 += (double)Mb[o + (size_t)(c + 8) * rows] * xs[c + 8];
            s3 += (double)Mb[o + (size_t)(c + 12) * rows] * xs[c + 12];
          }
          for (; c < cols; c += 4) s0 += (double)Mb[o + (size_t)c * rows] * xs[c];
        }
        red[wv][lane] = (s0 + s1) + (s2 + s3);
        __syncthreads();
        if (wv == 0 && o < rows) y[(size_t)b * nout + o] = (T)((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
        __syncthreads();
      }
    } else {
      for (int o = wv; o < cols; o += 4) {
        const T* mc = Mb + (size_t)o * rows;
        double s = 0.0;
        for (int i = lane; i < rows; i += 64) s += (double)mc[i] * xs[i];
        s = wave64_sum(s);
        if (lane == 0) y[(size_t)b * nout + o] = (T)s;
      }
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

// Small per-theta products whose matrix fits in LDS (SMALL_LDS_BYTES): the
// workgroup copies its matrix by direct global->LDS loads (every load in
// flight at once, one round trip to memory) and multiplies from LDS, sums
// in double.  Lane l of a wave's copy instruction writes dword base + l.
constexpr int SMALL_LDS_BYTES = 48 * 1024;
__device__ inline void copy_to_lds(const void* src, int ndw, float* dst, int lane, int wv) {
  const float* s = static_cast<const float*>(src);
  for (int j = wv; 64 * j < ndw; j += 4)
    if (64 * j + lane < ndw) __builtin_amdgcn_global_load_lds(s + 64 * j + lane, dst + 64 * j, 4, 0, 0);
}

// sum_i col[i] x[i] over i < n, the walk starting at `start` and wrapping
// (lanes with consecutive starts read consecutive LDS banks), in four
// interleaved partial sums so the loads and FMAs of successive terms
// overlap.
template <class T>
__device__ inline double dot_rotated(const T* col, const double* x, int n, int start) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + 3 < n; k += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int i = start + k + q;
      i -= i >= n ? n : 0;
      s[q] += (double)col[i] * x[i];
    }
  }
  for (; k < n; ++k) {
    int i = start + k;
    i -= i >= n ? n : 0;
    s[0] += (double)col[i] * x[i];
  }
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// y_b = op(M_b) x_b, one workgroup per b (grid-stride).  With `sums`, x_b is
// first formed as the fixed-order sum of the NRANGE range sums of the skinny
// reduce (entry i of x_b at sums[k count + b nin + i]) and also written to
// xout.  op = transpose: output o reads column o of M_b, the start of its
// walk down the column rotated by o so the lanes' LDS reads spread over
// the banks.  With dM (op = transpose, x_b = a_b): also
// dth[b, j] = a_b^T dM_{b,j} w_b for j < dt, each dM_{b,j} copied over M_b
// in LDS in turn, w_b = Wv[b cols ..].
template <class T>
__global__ void __launch_bounds__(256) k_bmatvec_lds(const T* M, int rows, int cols, int trans, const T* x,
                                                     const double* sums, int64_t count, T* xout, int B, T* y,
                                                     const T* dM, const T* Wv, int dt, T* dth) {
  extern __shared__ float smem[];
  const int nin = trans ? rows : cols, nout = trans ? cols : rows, nmax = rows > cols ? rows : cols;
  const int ndw = (int)((size_t)rows * cols * sizeof(T) / 4);
  const T* ms = reinterpret_cast<const T*>(smem);
  double* xs = reinterpret_cast<double*>(smem + ((ndw + 1) & ~1));
  double* ws = xs + nmax;
  double* red = ws + nmax;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    __syncthreads();                             // the previous b is consumed
    copy_to_lds(M + (size_t)b * rows * cols, ndw, smem, lane, wv);
    for (int i = tid; i < nin; i += 256) {
      double v;
      if (sums) {
        v = 0.0;
        for (int k = 0; k < NRANGE; ++k) v += sums[(size_t)k * count + (size_t)b * nin + i];
        xout[(size_t)b * nin + i] = (T)v;
      } else {
        v = (double)x[(size_t)b * nin + i];
      }
      xs[i] = v;
    }
    if (dM)
      for (int c = tid; c < cols; c += 256) ws[c] = (double)Wv[(size_t)b * cols + c];
    __builtin_amdgcn_s_waitcnt(0);               // this wave's copies have landed
    __syncthreads();                             // and everyone's
    asm volatile("" ::: "memory");
    for (int o = tid; o < nout; o += 256) {
      double s0 = 0.0, s1 = 0.0;
      if (!trans) {
        double s2 = 0.0, s3 = 0.0;
        int c = 0;
        for (; c + 3 < cols; c += 4) {
          s0 += (double)ms[o + (size_t)c * rows] * xs[c];
          s1 += (double)ms[o + (size_t)(c + 1) * rows] * xs[c + 1];
          s2 += (double)ms[o + (size_t)(c + 2) * rows] * xs[c + 2];
          s3 += (double)ms[o + (size_t)(c + 3) * rows] * xs[c + 3];
        }
        for (; c < cols; ++c) s0 += (double)ms[o + (size_t)c * rows] * xs[c];
        s0 += s2;
        s1 += s3;
      } else {
        s0 = dot_rotated(ms + (size_t)o * rows, xs, rows, o % rows);
      }
      y[(size_t)b * nout + o] = (T)(s0 + s1);
    }
    if (!dM) continue;
    for (int j = 0; j < dt; ++j) {
      __syncthreads();                           // M_b (or the last dM) is consumed
      copy_to_lds(dM + ((size_t)b * dt + j) * rows * cols, ndw, smem, lane, wv);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      asm volatile("" ::: "memory");
      double sb = 0.0;
      for (int c = tid; c < cols; c += 256) sb += dot_rotated(ms + (size_t)c * rows, xs, rows, c % rows) * ws[c];
      sb = wave64_sum(sb);
      if (lane == 0) red[wv] = sb;
      __syncthreads();
      if (tid == 0) dth[(size_t)b * dt + j] = (T)((red[0] + red[1]) + (red[2] + red[3]));
    }
  }
}

// dtheta[b, j] = a_b^T dM_{b,j} w_b, one workgroup per (b, j) (grid-stride):
// dM_{b,j} copied to LDS as above; thread c forms (a_b^T dM)[c] (rotated
// walk down column c) times w_b[c]; a block sum.
template <class T>
__global__ void __launch_bounds__(256) k_bilinear_lds(const T* A, const T* dM, const T* W, int rs, int rt, int B,
                                                      int dt, T* dth) {
  extern __shared__ float smem[];
  const int ndw = (int)((size_t)rs * rt * sizeof(T) / 4);
  const T* ds = reinterpret_cast<const T*>(smem);
  double* as = reinterpret_cast<double*>(smem + ((ndw + 1) & ~1));
  double* red = as + rs;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int q = blockIdx.x; q < B * dt; q += gridDim.x) {
    const int b = q / dt;
    __syncthreads();
    copy_to_lds(dM + (size_t)q * rs * rt, ndw, smem, lane, wv);
    for (int i = tid; i < rs; i += 256) as[i] = (double)A[(size_t)b * rs + i];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    asm volatile("" ::: "memory");
    double s = 0.0;
    for (int c = tid; c < rt; c += 256) s += dot_rotated(ds + (size_t)c * rs, as, rs, c % rs) * (double)W[(size_t)b * rt + c];
    s = wave64_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (tid == 0) dth[q] = (T)((red[0] + red[1]) + (red[2] + red[3]));
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

namespace {
constexpr int64_t SKINNY_CHUNK = 4 * ST;   // points per workgroup of the skinny reduce
unsigned plain_groups(int64_t N) { return grid_cap((N + 63) / 64, 4096); }
unsigned skinny_groups(int64_t N) { return (unsigned)((N + SKINNY_CHUNK - 1) / SKINNY_CHUNK); }
bool skinny(int r, int B) { return B >= 2 && B <= SB && r <= SR; }
}  // namespace

size_t apply_reduce_work(int64_t N, int r, int B) {
  if (N <= 0) return 0;
  if (B == 1) return (size_t)plain_groups(N) * r * sizeof(double);
  if (skinny(r, B)) return ((size_t)skinny_groups(N) + NRANGE) * r * B * sizeof(double);
  return apply_mfma_ok(r, B) ? apply_reduce_mfma_work(N, r, B) : 0;   // (float32 only; float64 needs none)
}

tt_status apply_reduce(int dtype, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx, int B,
                       void* W, void* work, hipStream_t st) {
  const size_t es = dtype == TTK_FP32 ? 4 : 8;
  if (N <= 0) {
    fill_zero(W, (size_t)r * B * es, st);
    return TTK_OK;
  }
  double* part = static_cast<double*>(work);
  if (B == 1) {
    const unsigned g = plain_groups(N);
    if (dtype == TTK_FP32) {
      hipLaunchKernelGGL(k_reduce_plain<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(X), part);
      hipLaunchKernelGGL(k_sum_partials<float>, dim3((r + 3) / 4), dim3(256), 0, st, (const double*)part, (int)g, r,
                         static_cast<float*>(W));
    } else {
      hipLaunchKernelGGL(k_reduce_plain<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(X), part);
      hipLaunchKernelGGL(k_sum_partials<double>, dim3((r + 3) / 4), dim3(256), 0, st, (const double*)part, (int)g, r,
                         static_cast<double*>(W));
    }
    return TTK_OK;
  }
  if (skinny(r, B)) {
    const unsigned g = skinny_groups(N);
    const int count = r * B;
    double* sums = part + (size_t)g * count;
    if (dtype == TTK_FP32 && skinny_mfma_ok(F, ldf, r, B))
      TTK_TRY(reduce_skinny_mfma(static_cast<const float*>(F), ldf, N, r, static_cast<const float*>(X), ldx, B,
                                 part, g, st));
    else if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_reduce_skinny<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(X), ldx, B, SKINNY_CHUNK, part);
    else
      hipLaunchKernelGGL(k_reduce_skinny<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(X), ldx, B, SKINNY_CHUNK, part);
    hipLaunchKernelGGL(k_sum_ranges, dim3((count + 63) / 64, NRANGE), dim3(256), 0, st, (const double*)part, (int)g,
                       count, sums);
    if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_sum_final<float>, dim3((count + 255) / 256), dim3(256), 0, st, (const double*)sums, count,
                         static_cast<float*>(W));
    else
      hipLaunchKernelGGL(k_sum_final<double>, dim3((count + 255) / 256), dim3(256), 0, st, (const double*)sums,
                         count, static_cast<double*>(W));
    return TTK_OK;
  }
  if (dtype == TTK_FP32 && apply_mfma_ok(r, B))
    return apply_reduce_mfma(static_cast<const float*>(F), ldf, N, r, static_cast<const float*>(X), ldx, B,
                             static_cast<float*>(W), part, st);
  fill_zero(W, (size_t)r * B * es, st);
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
  return TTK_OK;
}

tt_status apply_expand(int dtype, const void* F, int ldf, int64_t N, int r, const void* Z, int B, void* Y,
                       int64_t ldy, hipStream_t st) {
  if (N <= 0) return TTK_OK;
  if (B == 1) {
    const unsigned g = grid_cap((N + 15) / 16, 8192);
    if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_expand_plain<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(Z), static_cast<float*>(Y));
    else
      hipLaunchKernelGGL(k_expand_plain<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(Z), static_cast<double*>(Y));
    return TTK_OK;
  }
  if (B <= SB && r <= SR) {
    if (dtype == TTK_FP32 && skinny_expand_mfma_ok(F, ldf, r, B))
      return expand_skinny_mfma(static_cast<const float*>(F), ldf, N, r, static_cast<const float*>(Z), B,
                                static_cast<float*>(Y), ldy, st);
    const unsigned g = (unsigned)((N + ST - 1) / ST);
    if (dtype == TTK_FP32)
      hipLaunchKernelGGL(k_expand_skinny<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                         static_cast<const float*>(Z), B, static_cast<float*>(Y), ldy);
    else
      hipLaunchKernelGGL(k_expand_skinny<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N,
                         r, static_cast<const double*>(Z), B, static_cast<double*>(Y), ldy);
    return TTK_OK;
  }
  if (dtype == TTK_FP32 && apply_mfma_ok(r, B))
    return apply_expand_mfma(static_cast<const float*>(F), ldf, N, r, static_cast<const float*>(Z), B,
                             static_cast<float*>(Y), ldy, st);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((B + 63) / 64));
  if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_expand_tiled<float>, grid, dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                       static_cast<const float*>(Z), B, static_cast<float*>(Y), ldy);
  else
    hipLaunchKernelGGL(k_expand_tiled<double>, grid, dim3(256), 0, st, static_cast<const double*>(F), ldf, N, r,
                       static_cast<const double*>(Z), B, static_cast<double*>(Y), ldy);
  return TTK_OK;
}

namespace {
size_t matvec_lds_bytes(int rows, int cols, size_t es) {
  const size_t ndw = (size_t)rows * cols * es / 4;
  return ((ndw + 1) & ~(size_t)1) * 4 + ((size_t)2 * std::max(rows, cols) + 4) * sizeof(double);
}
bool matvec_lds_ok(int rows, int cols, size_t es) { return matvec_lds_bytes(rows, cols, es) <= SMALL_LDS_BYTES; }

template <class T>
void launch_bmatvec(const T* M, int rows, int cols, int trans, const T* x, const double* sums, int64_t count, T* xout,
                    int B, T* y, hipStream_t st, const T* dM = nullptr, const T* Wv = nullptr, int dt = 0,
                    T* dth = nullptr) {
  const unsigned g = grid_cap(B, 2048);
  if (matvec_lds_ok(rows, cols, sizeof(T)))
    hipLaunchKernelGGL(k_bmatvec_lds<T>, dim3(g), dim3(256), matvec_lds_bytes(rows, cols, sizeof(T)), st, M, rows,
                       cols, trans, x, sums, count, xout, B, y, dM, Wv, dt, dth);
  else
    hipLaunchKernelGGL(k_bmatvec<T>, dim3(g), dim3(256), 0, st, M, rows, cols, trans, x, B, y);
}
}  // namespace

void batched_matvec(int dtype, const void* M, int rows, int cols, int trans, const void* x, int B, void* y,
                    hipStream_t st) {
  if (B <= 0) return;
  if (dtype == TTK_FP32)
    launch_bmatvec(static_cast<const float*>(M), rows, cols, trans, static_cast<const float*>(x), nullptr, 0,
                   static_cast<float*>(nullptr), B, static_cast<float*>(y), st);
  else
    launch_bmatvec(static_cast<const double*>(M), rows, cols, trans, static_cast<const double*>(x), nullptr, 0,
                   static_cast<double*>(nullptr), B, static_cast<double*>(y), st);
}

tt_status apply_reduce_matvec(int dtype, const void* F, int ldf, int64_t N, int r, const void* X, int64_t ldx, int B,
                              void* W, const void* M, int rows, int cols, int trans, void* Z, void* work,
                              hipStream_t st, const void* dM, const void* Wv, int dt, void* dtheta) {
  if (B <= 0) return TTK_OK;
  if ((trans ? rows : cols) != r)
    return fail(TTK_ERR_ARG, "reduce_matvec: op(M) takes %d inputs, W has %d", trans ? rows : cols, r);
  const bool bil = dM && dt > 0;
  if (bil && (!trans || !Wv || !dtheta)) return fail(TTK_ERR_ARG, "reduce_matvec: bad bilinear arguments");
  const size_t es = dtype == TTK_FP32 ? 4 : 8;
  if (N <= 0 || !skinny(r, B) || !matvec_lds_ok(rows, cols, es)) {
    TTK_TRY(apply_reduce(dtype, F, ldf, N, r, X, ldx, B, W, work, st));
    batched_matvec(dtype, M, rows, cols, trans, W, B, Z, st);
    if (bil) batched_bilinear(dtype, W, dM, Wv, rows, cols, B, dt, dtheta, st);
    return TTK_OK;
  }
  // the skinny reduce's partials and range sums, then one launch that adds
  // the ranges (writing W) and multiplies
  const unsigned g = skinny_groups(N);
  const int count = r * B;
  double* part = static_cast<double*>(work);
  double* sums = part + (size_t)g * count;
  if (dtype == TTK_FP32 && skinny_mfma_ok(F, ldf, r, B))
    TTK_TRY(reduce_skinny_mfma(static_cast<const float*>(F), ldf, N, r, static_cast<const float*>(X), ldx, B, part,
                               g, st));
  else if (dtype == TTK_FP32)
    hipLaunchKernelGGL(k_reduce_skinny<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(F), ldf, N, r,
                       static_cast<const float*>(X), ldx, B, SKINNY_CHUNK, part);
  else
    hipLaunchKernelGGL(k_reduce_skinny<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(F), ldf, N, r,
                       static_cast<const double*>(X), ldx, B, SKINNY_CHUNK, part);
  hipLaunchKernelGGL(k_sum_ranges, dim3((count + 63) / 64, NRANGE), dim3(256), 0, st, (const double*)part, (int)g,
                     count, sums);
  if (dtype == TTK_FP32)
    launch_bmatvec(static_cast<const float*>(M), rows, cols, trans, static_cast<const float*>(nullptr), sums, count,
                   static_cast<float*>(W), B, static_cast<float*>(Z), st, static_cast<const float*>(bil ? dM : nullptr),
                   static_cast<const float*>(Wv), dt, static_cast<float*>(dtheta));
  else
    launch_bmatvec(static_cast<const double*>(M), rows, cols, trans, static_cast<const double*>(nullptr), sums,
                   count, static_cast<double*>(W), B, static_cast<double*>(Z), st,
                   static_cast<const double*>(bil ? dM : nullptr), static_cast<const double*>(Wv), dt,
                   static_cast<double*>(dtheta));
  return TTK_OK;
}

namespace {
template <class T>
void launch_bilinear(const T* A, const T* dM, const T* W, int rs, int rt, int B, int dt, T* dth, hipStream_t st) {
  const size_t ndw = (size_t)rs * rt * sizeof(T) / 4;
  const size_t sh = ((ndw + 1) & ~(size_t)1) * 4 + (size_t)(rs + 4) * sizeof(double);
  if (sh <= SMALL_LDS_BYTES)
    hipLaunchKernelGGL(k_bilinear_lds<T>, dim3(grid_cap((int64_t)B * dt, 4096)), dim3(256), sh, st, A, dM, W, rs, rt,
                       B, dt, dth);
  else
    hipLaunchKernelGGL(k_bilinear<T>, dim3(grid_cap(B, 2048)), dim3(256), 0, st, A, dM, W, rs, rt, B, dt, dth);
}
}  // namespace

void batched_bilinear(int dtype, const void* A, const void* dM, const void* W, int rs, int rt, int B, int dt,
                      void* dtheta, hipStream_t st) {
  if (B <= 0 || dt <= 0) return;
  if (dtype == TTK_FP32)
    launch_bilinear(static_cast<const float*>(A), static_cast<const float*>(dM), static_cast<const float*>(W), rs, rt,
                    B, dt, static_cast<float*>(dtheta), st);
  else
    launch_bilinear(static_cast<const double*>(A), static_cast<const double*>(dM), static_cast<const double*>(W), rs,
                    rt, B, dt, static_cast<double*>(dtheta), st);
}

}  // namespace ttk
