// Device helpers shared by the kernels that evaluate entries of the grid
// tensor m_{i_1..i_D} = f_kappa(eta) (Section 2.4, multivariate
// approximation; variable order (x, theta, y)): the node table staged in LDS,
// the multi-index of a super-core or fibre position and the compile-time
// dispatch over (d, d_theta) that keeps coordinates in registers.
#pragma once

#include <type_traits>

#include "ttk_internal.h"
#include "ttk_kappa.h"

namespace ttk {

// The node table (D x MAXN doubles, 2 KB at most) staged in LDS by every block.
template <int D>
__device__ inline void stage_nodes(const double* nodes, double* sn) {
  for (int i = threadIdx.x; i < D * MAXN; i += blockDim.x) sn[i] = nodes[i];
  __syncthreads();
}

// Multi-index of super-core / fibre position (row, col) -> coordinates.  Every
// position j is resolved with constant indexing so that c stays in registers:
// j < lk from the left set, then the middle node(s), then the right set.
template <int D>
__device__ inline void addr_coords(const Addr& a, const double* sn, int row, int col, double (&c)[D]) {
  const int s = row % a.rl;
  const int i0 = row / a.rl;
  int i1 = 0, t = col;
  if (a.nmid == 2) { i1 = col % a.nm1; t = col / a.nm1; }
  const int16_t* L = a.left + (int64_t)s * a.lk;
  const int roff = t * a.lr - a.lk - a.nmid;   // right[roff + j] for trailing positions j
#pragma unroll
  for (int j = 0; j < D; ++j) {
    int node;
    if (j < a.lk) node = L[j];
    else if (j == a.lk) node = i0;
    else if (a.nmid == 2 && j == a.lk + 1) node = i1;
    else node = a.right[roff + j];
    c[j] = sn[j * MAXN + node];
  }
}

// The two halves of addr_coords: positions 0..lk come from the row (left set,
// then i_k), positions lk+1..D-1 from the column (i_{k+1} of a super-core,
// then the right set).  Each fills only its own positions of c.
template <int D>
__device__ inline void addr_row_part(const Addr& a, const double* sn, int row, double (&c)[D]) {
  const int s = row % a.rl;
  const int i0 = row / a.rl;
  const int16_t* L = a.left + (int64_t)s * a.lk;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (j < a.lk) c[j] = sn[j * MAXN + L[j]];
    else if (j == a.lk) c[j] = sn[j * MAXN + i0];
  }
}
template <int D>
__device__ inline void addr_col_part(const Addr& a, const double* sn, int col, double (&c)[D]) {
  int i1 = 0, t = col;
  if (a.nmid == 2) { i1 = col % a.nm1; t = col / a.nm1; }
  const int roff = t * a.lr - a.lk - a.nmid;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (j <= a.lk) continue;
    if (a.nmid == 2 && j == a.lk + 1) c[j] = sn[j * MAXN + i1];
    else c[j] = sn[j * MAXN + a.right[roff + j]];
  }
}

// Node indices of the same halves (positions 0..lk from the row, lk+1..D-1
// from the column): the global loads of addr_row_part / addr_col_part
// without the node table, so they can be issued before the table is staged.
template <int D>
__device__ inline void addr_row_nodes(const Addr& a, int row, int (&nd)[D]) {
  const int s = row % a.rl;
  const int i0 = row / a.rl;
  const int16_t* L = a.left + (int64_t)s * a.lk;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (j < a.lk) nd[j] = L[j];
    else if (j == a.lk) nd[j] = i0;
  }
}
template <int D>
__device__ inline void addr_col_nodes(const Addr& a, int col, int (&nd)[D]) {
  int i1 = 0, t = col;
  if (a.nmid == 2) { i1 = col % a.nm1; t = col / a.nm1; }
  const int roff = t * a.lr - a.lk - a.nmid;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (j <= a.lk) continue;
    if (a.nmid == 2 && j == a.lk + 1) nd[j] = i1;
    else nd[j] = a.right[roff + j];
  }
}

// Entry (row, col) of the super-core / fibre addressed by a.
template <int d, int dt, bool G>
__device__ inline double addr_eval(const KSpec& ks, const Addr& a, const double* sn, int row, int col) {
  double c[2 * d + dt];
  addr_coords<2 * d + dt>(a, sn, row, col, c);
  return kappa_eval<d, dt, G>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c);
}
// The same entry evaluated by the 16 lanes of a DPP row together (every lane
// of the row with the same row and col; l16 = the lane in the row).
template <int d, int dt, bool G>
__device__ inline double addr_eval_row16(const KSpec& ks, const Addr& a, const double* sn, int row, int col, int l16) {
  double c[2 * d + dt];
  addr_coords<2 * d + dt>(a, sn, row, col, c);
  return kappa_eval<d, dt, G, true>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c, l16);
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<d>, IC<dt>, IC<G>) for the spatial dimension d in 1..3, the
// parameter dimension dt in 0..2 (the ranges the parameter check admits) and
// G = 1 for the general Matern kinds.
template <class F>
void with_dims(const KSpec& ks, F&& f) {
  const bool g = ks.kind == TTK_MATERN || ks.kind == TTK_MATERN_NU;
  auto pick = [&](auto dd, auto tt) {
    if (g) f(dd, tt, IC<1>{});
    else f(dd, tt, IC<0>{});
  };
  switch ((ks.d - 1) * 3 + ks.dt) {
    case 0: pick(IC<1>{}, IC<0>{}); break;
    case 1: pick(IC<1>{}, IC<1>{}); break;
    case 2: pick(IC<1>{}, IC<2>{}); break;
    case 3: pick(IC<2>{}, IC<0>{}); break;
    case 4: pick(IC<2>{}, IC<1>{}); break;
    case 5: pick(IC<2>{}, IC<2>{}); break;
    case 6: pick(IC<3>{}, IC<0>{}); break;
    case 7: pick(IC<3>{}, IC<1>{}); break;
    case 8: pick(IC<3>{}, IC<2>{}); break;
    default: break;
  }
}

}  // namespace ttk
