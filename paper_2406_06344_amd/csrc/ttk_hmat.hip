// A parametric hierarchical matrix for K(X, X; theta): the use the paper
// names for its low-rank blocks (the admissible blocks of fast multipole and
// hierarchical-matrix methods, Section 1; hierarchical parametric
// approximations as future work, Conclusions).  The root box is refined
// uniformly to level L; at every level k >= 2 the admissible blocks are the
// standard interaction lists (cells whose parents are neighbours, the cells
// themselves not), each a pair of separated boxes whose block is the PTTK
// low-rank form U_p M(theta) V_p^T (the pair batch: one TT per geometry class,
// Phase 3 for every pair in one launch, the apply as one captured graph); the
// blocks between neighbouring leaves are summed directly on the device.
//
// Points are sorted by the Morton code of their leaf, so every cell of every
// level is one contiguous range of the sorted points (the pair batch takes
// point ranges).  The sort is a device radix sort; the tree and the lists
// are built on the host from the sorted leaf codes.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "ttk_eval_dev.h"
#include "ttk_internal.h"

struct tt_kernel_hmat {
  tt_kernel_params P{};
  int d = 0, L = 0, dtype = TTK_FP32;
  size_t es = 4;
  int64_t N = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  ttk::DBuf perm;          // int32: sorted position -> input index
  ttk::DBuf Xs;            // sorted points, SoA d x N, dtype
  ttk::DBuf leaf_start;    // int64, 2^{L d} + 1 (Morton order)
  ttk::DBuf near_rows;     // int32: the non-empty leaves
  ttk::DBuf near_off;      // int32: CSR offsets per non-empty leaf
  ttk::DBuf near_cells;    // int32: neighbouring non-empty leaves
  ttk::DBuf xs, ys;        // apply work: sorted X and Y
  std::vector<int32_t> far_list, near_list;   // 7 / 6 ints per pair
  std::vector<int32_t> perm_host;
  tt_kernel_batch_t far = nullptr;
  int num_rows = 0;
  int singular = 0;        // kernel unbounded at r = 0: self terms are left out
  tt_kernel_hmat_info info{};
  ttk::KSpec ks{};
};

namespace ttk {

namespace {

// Morton code of integer coordinates i_0..i_{d-1} (L bits each): bit b of
// coordinate j at position b d + j.
__host__ __device__ inline uint32_t morton(const int* i, int d, int L) {
  uint32_t m = 0;
  for (int b = 0; b < L; ++b)
    for (int j = 0; j < d; ++j) m |= (uint32_t)((i[j] >> b) & 1) << (b * d + j);
  return m;
}
inline void unmorton(uint32_t m, int d, int L, int* i) {
  for (int j = 0; j < d; ++j) i[j] = 0;
  for (int b = 0; b < L; ++b)
    for (int j = 0; j < d; ++j) i[j] |= (int)((m >> (b * d + j)) & 1) << b;
}

struct BoxArg {
  double lo[3], hi[3];
};

// Leaf cell of every point: i_j = floor((x_j - lo_j) / (hi_j - lo_j) 2^L),
// clamped to [0, 2^L - 1] (points on the upper face); key = its Morton code.
template <class T>
__global__ void k_hm_keys(const T* X, int64_t N, int d, int L, BoxArg b, uint32_t* keys, int32_t* idx) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    int i[3] = {0, 0, 0};
    const int side = 1 << L;
    for (int j = 0; j < d; ++j) {
      const double u = ((double)X[(int64_t)j * N + p] - b.lo[j]) / (b.hi[j] - b.lo[j]) * (double)side;
      int v = (int)floor(u);
      i[j] = v < 0 ? 0 : (v >= side ? side - 1 : v);
    }
    keys[p] = morton(i, d, L);
    idx[p] = (int32_t)p;
  }
}

// Xs[j N + q] = X[j N + perm[q]]
template <class T>
__global__ void k_hm_gather_points(const T* X, int64_t N, int d, const int32_t* perm, T* Xs) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * d; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / N, q = e - j * N;
    Xs[e] = X[j * N + perm[q]];
  }
}

// xs[q + b N] = X[perm[q] + b ldx]  (dir 0); Y[perm[q] + b ldy] = ys[q + b N]  (dir 1)
template <class T>
__global__ void k_hm_permute(const T* in, int64_t ldin, T* out, int64_t ldout, int64_t N, int B, const int32_t* perm,
                             int dir) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * B; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / N, q = e - b * N;
    if (dir == 0) out[q + b * ldout] = in[perm[q] + b * ldin];
    else out[perm[q] + b * ldout] = in[q + b * ldin];
  }
}

// The near field: ys[i, b] += sum over the neighbouring leaves' points j of
// K(x_i, x_j; theta_b) x[j, b], one workgroup per (non-empty leaf, theta);
// the neighbours' coordinates and inputs pass through LDS in chunks of 256.
// Accumulated in double precision.  Each sorted row belongs to one leaf, so
// no two workgroups write the same entry.
constexpr int HN = 256;
template <class T, int d, int dt, bool G>
__global__ void __launch_bounds__(HN) k_hm_near(KSpec ks, const T* Xs, int64_t N, const int64_t* leaf_start,
                                                const int32_t* rows, const int32_t* noff, const int32_t* ncell,
                                                const T* theta, const T* xs, T* ys, int singular) {
  __shared__ double cs[HN][d + 1];
  const int c = rows[blockIdx.x];
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  double th[2] = {0.0, 0.0};
  for (int q = 0; q < dt; ++q) th[q] = (double)theta[(int64_t)b * dt + q];
  const int64_t s0 = leaf_start[c], s1 = leaf_start[c + 1];
  const T* xb = xs + (int64_t)b * N;
  for (int64_t i0 = s0; i0 < s1; i0 += HN) {
    const int64_t i = i0 + tid;
    double ci[2 * d + dt];
    if (i < s1) {
#pragma unroll
      for (int q = 0; q < d; ++q) ci[q] = (double)Xs[(int64_t)q * N + i];
    } else {
#pragma unroll
      for (int q = 0; q < d; ++q) ci[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < dt; ++q) ci[d + q] = th[q];
    double acc = 0.0;
    for (int e = noff[blockIdx.x]; e < noff[blockIdx.x + 1]; ++e) {
      const int cn = ncell[e];
      const int64_t t0 = leaf_start[cn], t1 = leaf_start[cn + 1];
      for (int64_t j0 = t0; j0 < t1; j0 += HN) {
        const int64_t j = j0 + tid;
        __syncthreads();   // the previous chunk is consumed
        if (j < t1) {
#pragma unroll
          for (int q = 0; q < d; ++q) cs[tid][q] = (double)Xs[(int64_t)q * N + j];
          cs[tid][d] = (double)xb[j];
        }
        __syncthreads();
        const int nj = (int)min<int64_t>(HN, t1 - j0);
        if (i < s1)
          for (int u = 0; u < nj; ++u) {
            if (singular && j0 + u == i) continue;
#pragma unroll
            for (int q = 0; q < d; ++q) ci[d + dt + q] = cs[u][q];
            acc += kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], ci) * cs[u][d];
          }
      }
    }
    if (i < s1) ys[i + (int64_t)b * N] = (T)((double)ys[i + (int64_t)b * N] + acc);
  }
}

inline unsigned hm_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace ttk

using namespace ttk;

tt_status tt_kernel_hmat_build(const tt_kernel_params* p, const void* X, int64_t N, int leaf_points, void* stream,
                               tt_kernel_hmat_t* out) {
  if (!p || !out) return fail(TTK_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (N < 1 || !X) return fail(TTK_ERR_ARG, "no points");
  if (N > INT32_MAX) return fail(TTK_ERR_UNSUPPORTED, "at most 2^31 - 1 points");
  if (leaf_points < 1) return fail(TTK_ERR_ARG, "leaf_points must be positive");
  // the kernel and grid are checked by the pair batch; the root box is box_s
  tt_kernel_params P = *p;
  for (int j = 0; j < 2 * P.d && j < 6; ++j) P.box_t[j] = P.box_s[j];
  P.symmetric_psd = 0;
  if (P.d < 1 || P.d > 3) return fail(TTK_ERR_ARG, "d must be 1..3");
  for (int j = 0; j < P.d; ++j)
    if (!(P.box_s[2 * j + 1] > P.box_s[2 * j])) return fail(TTK_ERR_ARG, "empty root box in dimension %d", j);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<tt_kernel_hmat> h(new (std::nothrow) tt_kernel_hmat());
  if (!h) return fail(TTK_ERR_OOM, "handle allocation failed");
  h->P = P;
  h->d = P.d;
  h->N = N;
  h->dtype = P.dtype;
  h->es = P.dtype == TTK_FP32 ? 4 : 8;
  const int d = P.d;
  tt_status warn = TTK_OK;
  // the leaf level: the smallest L with N / 2^{L d} <= leaf_points (Morton codes in 30 bits)
  int L = 0;
  while ((double)N / std::ldexp(1.0, L * d) > leaf_points && (L + 1) * d <= 30) ++L;
  h->L = L;
  BoxArg box{};
  for (int j = 0; j < 3; ++j) {
    box.lo[j] = j < d ? P.box_s[2 * j] : 0.0;
    box.hi[j] = j < d ? P.box_s[2 * j + 1] : 1.0;
    h->lo[j] = box.lo[j];
    h->hi[j] = box.hi[j];
  }
  h->singular = (P.kind == TTK_LAPLACE3D || P.kind == TTK_LAPLACE2D || P.kind == TTK_BIHARMONIC ||
                 P.kind == TTK_THINPLATE) ? 1 : 0;
  // leaf codes, sorted with the point indices
  {
    DBuf keys, keys2, idx;
    TTK_TRY(keys.alloc((size_t)N * 4));
    TTK_TRY(keys2.alloc((size_t)N * 4));
    TTK_TRY(idx.alloc((size_t)N * 4));
    TTK_TRY(h->perm.alloc((size_t)N * 4));
    if (P.dtype == TTK_FP32)
      hipLaunchKernelGGL(k_hm_keys<float>, dim3(hm_grid(N)), dim3(256), 0, st, static_cast<const float*>(X), N, d, L,
                         box, keys.as<uint32_t>(), idx.as<int32_t>());
    else
      hipLaunchKernelGGL(k_hm_keys<double>, dim3(hm_grid(N)), dim3(256), 0, st, static_cast<const double*>(X), N, d,
                         L, box, keys.as<uint32_t>(), idx.as<int32_t>());
    TTK_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    TTK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys.as<uint32_t>(), keys2.as<uint32_t>(),
                                               idx.as<int32_t>(), h->perm.as<int32_t>(), (int)N, 0,
                                               std::max(1, L * d), st));
    DBuf tmp;
    TTK_TRY(tmp.alloc(std::max<size_t>(tmp_bytes, 16)));
    TTK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, keys.as<uint32_t>(), keys2.as<uint32_t>(),
                                               idx.as<int32_t>(), h->perm.as<int32_t>(), (int)N, 0,
                                               std::max(1, L * d), st));
    std::vector<uint32_t> hk((size_t)N);
    h->perm_host.resize((size_t)N);
    TTK_HIP(hipMemcpyAsync(hk.data(), keys2.p, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    TTK_HIP(hipMemcpyAsync(h->perm_host.data(), h->perm.p, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    TTK_HIP(hipStreamSynchronize(st));
    // leaf_start over all 2^{L d} leaves (Morton order)
    const int64_t nleaf = (int64_t)1 << (L * d);
    std::vector<int64_t> ls((size_t)nleaf + 1, 0);
    for (int64_t q = 0; q < N; ++q) ls[(size_t)hk[(size_t)q] + 1]++;
    for (int64_t c = 0; c < nleaf; ++c) ls[(size_t)c + 1] += ls[(size_t)c];
    TTK_TRY(h->leaf_start.alloc(ls.size() * sizeof(int64_t)));
    TTK_HIP(hipMemcpyAsync(h->leaf_start.p, ls.data(), ls.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    TTK_TRY(h->Xs.alloc((size_t)N * d * h->es));
    if (P.dtype == TTK_FP32)
      hipLaunchKernelGGL(k_hm_gather_points<float>, dim3(hm_grid(N * d)), dim3(256), 0, st,
                         static_cast<const float*>(X), N, d, (const int32_t*)h->perm.as<int32_t>(), h->Xs.as<float>());
    else
      hipLaunchKernelGGL(k_hm_gather_points<double>, dim3(hm_grid(N * d)), dim3(256), 0, st,
                         static_cast<const double*>(X), N, d, (const int32_t*)h->perm.as<int32_t>(),
                         h->Xs.as<double>());
    TTK_HIP(hipGetLastError());
    // the point range of cell (level k, coordinates i): its leaves are a
    // contiguous run of Morton codes at level L
    auto range = [&](int k, const int* i, int64_t* a, int64_t* b) {
      const uint32_t m = morton(i, d, k);
      const int64_t f = (int64_t)m << ((L - k) * d), lcount = (int64_t)1 << ((L - k) * d);
      *a = ls[(size_t)f];
      *b = ls[(size_t)(f + lcount)];
    };
    // interaction lists (k >= 2) and the near field (leaves)
    std::vector<tt_kernel_pair> pairs;
    for (int k = 2; k <= L; ++k) {
      const int side = 1 << k;
      const int64_t ncell = (int64_t)1 << (k * d);
      for (int64_t m = 0; m < ncell; ++m) {
        int ic[3] = {0, 0, 0};
        unmorton((uint32_t)m, d, k, ic);
        int64_t a0, a1;
        range(k, ic, &a0, &a1);
        if (a1 == a0) continue;
        int pc[3] = {ic[0] >> 1, ic[1] >> 1, ic[2] >> 1};
        // neighbours of the parent (itself included), then their children
        int lo3[3], hi3[3];
        for (int j = 0; j < 3; ++j) {
          lo3[j] = j < d ? std::max(0, 2 * (pc[j] - 1)) : 0;
          hi3[j] = j < d ? std::min(side - 1, 2 * (pc[j] + 1) + 1) : 0;
        }
        for (int z = lo3[2]; z <= hi3[2]; ++z)
          for (int y = lo3[1]; y <= hi3[1]; ++y)
            for (int x = lo3[0]; x <= hi3[0]; ++x) {
              const int it[3] = {x, y, z};
              int far = 0;
              for (int j = 0; j < d; ++j) far |= std::abs(it[j] - ic[j]) >= 2;
              if (!far) continue;
              int64_t b0, b1;
              range(k, it, &b0, &b1);
              if (b1 == b0) continue;
              tt_kernel_pair pr{};
              const double w = 1.0 / side;
              for (int j = 0; j < d; ++j) {
                const double ext = box.hi[j] - box.lo[j];
                pr.box_s[2 * j] = box.lo[j] + ext * (ic[j] * w);
                pr.box_s[2 * j + 1] = box.lo[j] + ext * ((ic[j] + 1) * w);
                pr.box_t[2 * j] = box.lo[j] + ext * (it[j] * w);
                pr.box_t[2 * j + 1] = box.lo[j] + ext * ((it[j] + 1) * w);
              }
              pr.src_off = a0;
              pr.n_src = a1 - a0;
              pr.tgt_off = b0;
              pr.n_tgt = b1 - b0;
              pairs.push_back(pr);
              const int32_t rec[7] = {k, ic[0], ic[1], ic[2], it[0], it[1], it[2]};
              h->far_list.insert(h->far_list.end(), rec, rec + 7);
            }
      }
    }
    // near field: neighbouring non-empty leaves (self included)
    std::vector<int32_t> rows, off(1, 0), cells;
    {
      const int side = 1 << L;
      for (int64_t m = 0; m < nleaf; ++m) {
        if (ls[(size_t)m + 1] == ls[(size_t)m]) continue;
        int ic[3] = {0, 0, 0};
        unmorton((uint32_t)m, d, L, ic);
        rows.push_back((int32_t)m);
        int lo3[3], hi3[3];
        for (int j = 0; j < 3; ++j) {
          lo3[j] = j < d ? std::max(0, ic[j] - 1) : 0;
          hi3[j] = j < d ? std::min(side - 1, ic[j] + 1) : 0;
        }
        for (int z = lo3[2]; z <= hi3[2]; ++z)
          for (int y = lo3[1]; y <= hi3[1]; ++y)
            for (int x = lo3[0]; x <= hi3[0]; ++x) {
              const int it[3] = {x, y, z};
              const uint32_t mn = morton(it, d, L);
              if (ls[(size_t)mn + 1] == ls[(size_t)mn]) continue;
              cells.push_back((int32_t)mn);
              const int32_t rec[6] = {ic[0], ic[1], ic[2], it[0], it[1], it[2]};
              h->near_list.insert(h->near_list.end(), rec, rec + 6);
            }
        off.push_back((int32_t)cells.size());
      }
    }
    h->num_rows = (int)rows.size();
    TTK_TRY(h->near_rows.alloc(std::max<size_t>(rows.size(), 1) * 4));
    TTK_TRY(h->near_off.alloc(off.size() * 4));
    TTK_TRY(h->near_cells.alloc(std::max<size_t>(cells.size(), 1) * 4));
    TTK_HIP(hipMemcpyAsync(h->near_rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, st));
    TTK_HIP(hipMemcpyAsync(h->near_off.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, st));
    if (!cells.empty())
      TTK_HIP(hipMemcpyAsync(h->near_cells.p, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, st));
    TTK_HIP(hipStreamSynchronize(st));   // the host vectors and the sort buffers are released below
    h->info.levels = L;
    h->info.leaves = nleaf;
    h->info.nonempty_leaves = (int64_t)rows.size();
    h->info.far_pairs = (int64_t)pairs.size();
    h->info.near_pairs = (int64_t)cells.size();
    h->info.t_tree_ms = ms_since(t0);
    auto t1 = std::chrono::steady_clock::now();
    if (!pairs.empty()) {
      const tt_status s = tt_kernel_batch_build(&P, pairs.data(), (int)pairs.size(), h->Xs.p, N, h->Xs.p, N, stream,
                                                &h->far);
      if (s < 0) return s;
      if (s == TTK_WARN_NOT_CONVERGED) warn = s;   // (a class's cross stopped above tol: kept, and reported)
      tt_kernel_batch_info bi{};
      TTK_TRY(tt_kernel_batch_get_info(h->far, &bi, nullptr, nullptr));
      h->info.num_classes = bi.num_classes;
      h->info.kernel_evals = bi.kernel_evals;
    }
    h->info.t_build_ms = ms_since(t1);
  }
  Grid g;
  TTK_TRY(make_grid(&P, &g));
  h->ks = KSpec{P.kind, P.d, P.d_theta, g.D, P.kernel_const, nullptr, {P.theta_fixed[0], P.theta_fixed[1]}};
  *out = h.release();
  if (warn != TTK_OK) set_error("the cross of at least one geometry class stopped above tol");
  return warn;
}

tt_status tt_kernel_hmat_apply(tt_kernel_hmat_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, void* stream) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (B < 0) return fail(TTK_ERR_ARG, "B < 0");
  if (B == 0) return TTK_OK;
  if (!X || !Y || (h->P.d_theta > 0 && !theta)) return fail(TTK_ERR_ARG, "NULL argument");
  if (ldx < h->N || ldy < h->N) return fail(TTK_ERR_ARG, "leading dimension below N");
  if ((int64_t)B > 65535) return fail(TTK_ERR_ARG, "B above 65535");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t N = h->N;
  TTK_TRY(h->xs.alloc((size_t)N * B * h->es));
  TTK_TRY(h->ys.alloc((size_t)N * B * h->es));
  const int32_t* perm = h->perm.as<int32_t>();
  if (h->dtype == TTK_FP32)
    hipLaunchKernelGGL(k_hm_permute<float>, dim3(hm_grid(N * B)), dim3(256), 0, st, static_cast<const float*>(X), ldx,
                       h->xs.as<float>(), N, N, B, perm, 0);
  else
    hipLaunchKernelGGL(k_hm_permute<double>, dim3(hm_grid(N * B)), dim3(256), 0, st, static_cast<const double*>(X),
                       ldx, h->xs.as<double>(), N, N, B, perm, 0);
  TTK_HIP(hipGetLastError());
  if (h->far)
    TTK_TRY(tt_kernel_batch_apply(h->far, theta, B, h->xs.p, N, h->ys.p, N, nullptr, 0, nullptr, 0, nullptr, stream));
  else
    fill_zero(h->ys.p, (size_t)N * B * h->es, st);
  if (h->num_rows > 0) {
    const dim3 grid((unsigned)h->num_rows, (unsigned)B);
    const KSpec ks = h->ks;
    const int64_t* ls = h->leaf_start.as<int64_t>();
    const int32_t *rows = h->near_rows.as<int32_t>(), *off = h->near_off.as<int32_t>(),
                  *cells = h->near_cells.as<int32_t>();
    with_dims(ks, [&](auto dd, auto tt, auto gg) {
      constexpr int D_ = decltype(dd)::value, T_ = decltype(tt)::value;
      constexpr bool G_ = decltype(gg)::value;
      if (h->dtype == TTK_FP32)
        hipLaunchKernelGGL((k_hm_near<float, D_, T_, G_>), grid, dim3(HN), 0, st, ks, (const float*)h->Xs.p, N, ls,
                           rows, off, cells, static_cast<const float*>(theta), (const float*)h->xs.p, h->ys.as<float>(),
                           h->singular);
      else
        hipLaunchKernelGGL((k_hm_near<double, D_, T_, G_>), grid, dim3(HN), 0, st, ks, (const double*)h->Xs.p, N, ls,
                           rows, off, cells, static_cast<const double*>(theta), (const double*)h->xs.p,
                           h->ys.as<double>(), h->singular);
    });
    TTK_HIP(hipGetLastError());
  }
  if (h->dtype == TTK_FP32)
    hipLaunchKernelGGL(k_hm_permute<float>, dim3(hm_grid(N * B)), dim3(256), 0, st, (const float*)h->ys.p, N,
                       static_cast<float*>(Y), ldy, N, B, perm, 1);
  else
    hipLaunchKernelGGL(k_hm_permute<double>, dim3(hm_grid(N * B)), dim3(256), 0, st, (const double*)h->ys.p, N,
                       static_cast<double*>(Y), ldy, N, B, perm, 1);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

tt_status tt_kernel_hmat_get_info(tt_kernel_hmat_t h, tt_kernel_hmat_info* info) {
  if (!h || !info) return fail(TTK_ERR_ARG, "NULL argument");
  *info = h->info;
  return TTK_OK;
}

tt_status tt_kernel_hmat_get_lists(tt_kernel_hmat_t h, int32_t* far, int32_t* near, int32_t* perm) {
  if (!h) return fail(TTK_ERR_ARG, "NULL handle");
  if (far && !h->far_list.empty()) std::copy(h->far_list.begin(), h->far_list.end(), far);
  if (near && !h->near_list.empty()) std::copy(h->near_list.begin(), h->near_list.end(), near);
  if (perm) std::copy(h->perm_host.begin(), h->perm_host.end(), perm);
  return TTK_OK;
}

tt_status tt_kernel_hmat_get_batch(tt_kernel_hmat_t h, tt_kernel_batch_t* b) {
  if (!h || !b) return fail(TTK_ERR_ARG, "NULL argument");
  *b = h->far;
  return TTK_OK;
}

tt_status tt_kernel_hmat_destroy(tt_kernel_hmat_t h) {
  if (!h) return TTK_OK;
  if (h->far) (void)tt_kernel_batch_destroy(h->far);
  (void)hipDeviceSynchronize();   // queued work may still read the buffers
  delete h;
  return TTK_OK;
}
