// TT greedy-cross on the grid tensor of f_kappa (Appendices A and B):
// index initialisation (Algorithm 7), update cross steps (Algorithm 5) swept
// left to right (Algorithm 6), the sampled stopping test and the
// interpolation formula for the cores.
//
// Split of the work.  The host keeps the (small, integer) index sets and the
// counter-based random stream and decides where pivots go; every kernel
// entry, every residual, every argmax and every FP64 factorisation runs on
// the device.  One update step costs one host round trip (the pivot it
// chose); the stopping test one more per sweep.
//
// Readings shared with the oracle: residual R = A(:,J) A(I,J)^{-1} A(I,:) - A;
// max{rows, cols} samples by Floyd's algorithm from the splitmix64 stream
// keyed (seed, 2, sweep, k), then the bit; argmax ties (within 1e-10 x the
// largest |entry| evaluated so far in the step) go to the lowest position;
// a pivot is added only if |R| exceeds that band, is new, and the rank is
// below the cap.  Stopping: max |X - X^| / max |X| over n_test fixed
// multi-indices (stream (seed, 3)), with cores C_k = F_k P_k^{-1} (LU solve);
// the cores returned are those of the last stopping test.
//
// Each intersection matrix P_k = X(I^{<=k}, I^{>k}) is kept factored in the
// order the cross added its pivots: P = L D U with L unit lower, U unit upper
// and D the pivots (the residuals at which they were added).  The device
// holds Li = L^{-1} and W = U^{-1} D^{-1}, so that P^{-1} = W Li and every
// solve of the cross is two products: the residuals of the sampled entries
// and of the searched fibre, and the cores C_k = F_k P_k^{-1} of the stopping
// test.  The ill-conditioning of P (pivots from about 1 down to the
// tolerance) sits in D alone, which enters as a scaling; L and U have
// entries bounded by the pivot rule (each pivot is the largest residual of
// its row or column), so products with their inverses stay as accurate as
// substitution.  When step k adds (l, t), P grows by a border:
// b = X(I, t), c = X(l, J), d = X(l, t);  u = Li b, g^T = c^T W,
// s = d - g^T u (minus the residual at the pivot), and
//     Li' = [[Li, 0], [-g^T Li, 1]],   W' = [[W, -W u / s], [0, 1 / s]],
// an O(r^2) update on the device.  The first (rank <= 2) matrices are
// factored with the larger diagonal entry first (a symmetric permutation that
// only Li and W carry).
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ttk_eval_dev.h"
#include "ttk_internal.h"
#include "ttk_rng.h"
#include "ttk_wave.h"

namespace ttk {

namespace {

constexpr double TIE_REL = 1e-10;

// Result of one update step, written on the device, read back once.
struct StepRes {
  int32_t s_pos, l, t, q_pos;
  int32_t pivot_row, pivot_col, added, info;
  double s_max, s_margin, s_scale, s_tau;
  double q_max, q_margin, q_scale, q_tau;
  double pivot_abs, pad;
  int32_t pad2, pad3;
  // running max |entry| of the step's evaluations, spread over AMAX_SLOTS
  // slots (block b folds into slot b mod AMAX_SLOTS) to avoid one contended
  // address; cleared at the end of every step
  double s_slot[AMAX_SLOTS], q_slot[AMAX_SLOTS];
};

// The inputs of one update step in one of its two variants: variant v holds
// what the step uses when the previous step of the sweep added (v = 1) or did
// not add (v = 0) a pivot, which changes the left rank r_{k-1}, hence the
// super-core rows, the sample draw, the row positions of P_k's pivots and the
// left index set (whose extra row the previous step's finishing kernel
// writes).  The step's kernels read desc[*sel], with *sel written by that
// finishing kernel, so the host can enqueue a step before the previous one
// has decided.
struct StepDesc {
  Addr a;                 // super-core k: left set (with a spare row), right set
  const int32_t* I;       // row positions of P_k's pivots (r_k)
  const int32_t* J;       // column positions (r_k)
  const int32_t* srow;    // samples, generation order (ns)
  const int32_t* scol;
  int rows, cols, ns, bit;
};

// The fibre cache.  Every value a step reads besides its own samples and
// its searched fibre is an entry of a fibre core
//   F_k(a, i, b) = X(I^{<=k-1}[a], i, I^{>k}[b]),   a < r_{k-1}, i < n_k, b < r_k:
// A(s, J_q) of super-core k is F_k(s, i_k, q) and A(I_q, s) is
// F_{k+1}(q, i_{k+1}, t) for a position s = (row s + i_k r_{k-1}, column
// i_{k+1} + t n_{k+1}); the intersection matrix P_k is F_k at its pivot rows,
// and F_k is the fibre of the interpolation formula.  The index sets only
// grow at their ends, so F_k only gains rows (when step k - 1 adds a pivot:
// the row of super-core k - 1 through that pivot) and columns (when step k
// adds one: the column of super-core k through it).  Each F_k is kept on the
// device twice, with capacity MAXR in both ranks:
//   FL_k[(i MAXR + a) MAXR + b]   (rows of the unfolding contiguous in b), and
//   FR_k[(i MAXR + b) MAXR + a]   (contiguous in a),
// so that the gathers of either side of a super-core read contiguous runs.
// A step writes the fibre it searched into the slot a pivot would occupy
// (row r_k of F_{k+1} or column r_k of F_k) before it knows whether the pivot
// is added: the slot lies past every extent read until an addition makes it
// part of the core.  The entries are the same numbers a fresh evaluation
// gives, so the cache changes no decision, only the count of evaluations
// (the O(D n r^2) of the interpolation itself, plus the samples and the
// searched fibres).
__device__ inline int64_t fibre_left_row(int a, int i) { return ((int64_t)i * MAXR + a) * MAXR; }
__device__ inline int64_t fibre_right_col(int i, int b) { return ((int64_t)i * MAXR + b) * MAXR; }

__device__ inline double wsum(double v) { return wave64_sum(v); }

// Largest |value| over up to four buffers, combined with *base (if non-NULL).
__global__ void k_absmax(const double* a, int na, const double* b, int nb, const double* c, int nc,
                         const double* d, int nd, const double* base, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < na; i += blockDim.x) m = fmax(m, fabs(a[i]));
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, fabs(b[i]));
  for (int i = threadIdx.x; i < nc; i += blockDim.x) m = fmax(m, fabs(c[i]));
  for (int i = threadIdx.x; i < nd; i += blockDim.x) m = fmax(m, fabs(d[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = base ? fmax(*base, red[0]) : red[0];
}

// 2-norm condition number of the 2x2 probe e = j1 n + j2 of the index
// initialisation.  F (2-row-set fibre, (rl*n) x rr col-major) holds
// phi(left_s, j, right_t).
// mode 0 (left-to-right): M = [[F(a,j1,c), F(a,j1,c')], [F(b,j2,c), F(b,j2,c')]]
// mode 1 (right-to-left): M = [[F(a,j1,c), F(a,j2,c')], [F(b,j1,c), F(b,j2,c')]]
__device__ inline double init_cond_at(const double* F, int rl, int rr, int n, int mode, int excl_diag, int e) {
  const int j1 = e / n, j2 = e % n;   // linear position j1 * n + j2
  const int m = rl * n;
  const int sa = 0, sb = rl > 1 ? 1 : 0;
  const int ca = 0, cb = rr > 1 ? 1 : 0;
  double a, b, c, d;
  if (mode == 0) {
    a = F[sa + j1 * rl + ca * m]; b = F[sa + j1 * rl + cb * m];
    c = F[sb + j2 * rl + ca * m]; d = F[sb + j2 * rl + cb * m];
  } else {
    a = F[sa + j1 * rl + ca * m]; b = F[sa + j2 * rl + cb * m];
    c = F[sb + j1 * rl + ca * m]; d = F[sb + j2 * rl + cb * m];
  }
  // singular values of [[a, b], [c, d]]: (p +- q)/2 with
  // p = |(a + d, c - b)|, q = |(a - d, b + c)|
  const double p = hypot(a + d, c - b), q = hypot(a - d, b + c);
  const double s1 = 0.5 * (p + q), s2 = 0.5 * fabs(p - q);
  double cv = (s2 > 0.0) ? s1 / s2 : INFINITY;
  if (!(cv == cv)) cv = INFINITY;
  if (excl_diag && j1 == j2) cv = INFINITY;
  return cv;
}

// P[a + b*r] = F[rows[a] + b*ldf]  (rows of F at the given positions)
__global__ void k_gather_rows(const double* F, int ldf, const int32_t* rows, int r, int c, double* P) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * c) return;
  const int a = e % r, b = e / r;
  P[a + b * r] = F[rows[a] + (int64_t)b * ldf];
}

// P[a + b r] = F_k(s_a, i_a, b) for the pivot rows I[a] = s_a + i_a rl of
// super-core k (a, b < r <= 4): the intersection matrix from the fibre cache.
__global__ void k_gather_pivots(const double* FL, const int32_t* I, int rl, int r, double* P) {
  const int e = threadIdx.x;
  if (e >= r * r) return;
  const int a = e % r, b = e / r;
  P[e] = FL[fibre_left_row(I[a] % rl, I[a] / rl) + b];
}

// B (n x m) = A^T for A (m x n)
__global__ void k_transpose(const double* A, int m, int n, int lda, double* B, int ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  B[j + (int64_t)i * ldb] = A[i + (int64_t)j * lda];
}

// The index initialisation in one block: max_it passes of 2-row probes,
// left to right (k = 1..N-1, the new rows of I^{<=k}) then right to left
// (k = N..2, the new rows of I^{>k-1}), each probe evaluating its fibre,
// the condition numbers of all n^2 candidate 2x2 submatrices and the lowest
// position within a relative band 1e-12 of the smallest (positions with
// j1 = j2 excluded where one side has a single row; if every candidate is
// +inf, the lowest allowed one).  The sets live in LDS (int16, row-major
// like the upload arena), and after every pass they and the pass's largest
// chosen condition number go to snapshot slot 2 it + pass:
//   snap[slot * INIT_SNAP + k * 2 MAXD + e]            rows of I^{<=k} (2 k entries),
//   snap[slot * INIT_SNAP + (MAXD + k) * 2 MAXD + e]   rows of I^{>k} (2 (N - k) entries).
struct InitArgs {
  int N, max_it;
  int n[MAXD];
  int32_t q1[MAXD], q2[MAXD];   // the two random points the right sets start from
};
constexpr int INIT_SNAP = 4 * MAXD * MAXD;
template <int d, int dt, bool G>
__global__ void __launch_bounds__(1024) k_init_sets(KSpec ks, InitArgs ia, int32_t* snap, double* snap_mc) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN], F[2 * MAXN * 2], sv[1024], wmin[16];
  __shared__ int wpos[16];
  __shared__ int16_t Ls[MAXD][2 * MAXD], Rs[MAXD + 1][2 * MAXD];
  const int tid = threadIdx.x, N = ia.N;
  stage_nodes<D>(ks.nodes, sn);   // (synchronises the block)
  if (tid == 0)
    for (int k = 1; k < N; ++k) {
      const int len = N - k;
      for (int j = 0; j < len; ++j) {
        Rs[k][j] = (int16_t)ia.q1[k + j];
        Rs[k][len + j] = (int16_t)ia.q2[k + j];
      }
    }
  __syncthreads();
  // one probe: kl = k - 1 left rows, kr = k right rows; the chosen (j1, j2) and its condition number
  auto probe = [&](int k, int mode, int* j1, int* j2, double* cv) {
    const int n = ia.n[k - 1];
    Addr a{};
    a.left = Ls[k - 1];
    a.right = Rs[k];
    a.rl = (k - 1 == 0) ? 1 : 2;
    a.lk = k - 1;
    a.rr = (k == N) ? 1 : 2;
    a.lr = N - k;
    a.nmid = 1;
    a.nm0 = n;
    a.nm1 = 1;
    const int m = a.rl * n;
    for (int e = tid >> 4; e < m * a.rr; e += 64) {   // one entry per row of 16 lanes
      const double v = addr_eval_row16<d, dt, G>(ks, a, sn, e % m, e / m, tid & 15);
      if ((tid & 15) == 0) F[e] = v;
    }
    __syncthreads();
    const int excl = (mode == 0) ? (k == 1) : (k == N);
    const int nn = n * n;   // <= 1024: one candidate per thread
    const double v = tid < nn ? init_cond_at(F, a.rl, a.rr, n, mode, excl, tid) : INFINITY;
    sv[tid] = v;
    // the smallest condition number: per wave, then over the 16 waves
    const double wm = -wave64_max(-v);
    if ((tid & 63) == 0) wmin[tid >> 6] = wm;
    __syncthreads();
    double mn = wmin[0];
#pragma unroll
    for (int w = 1; w < 16; ++w) mn = fmin(mn, wmin[w]);
    // the lowest allowed position within the band (every allowed one if all are +inf)
    int pos = 0x7fffffff;
    if (tid < nn && !(excl && tid / n == tid % n) && (isinf(mn) || v <= mn * (1.0 + 1e-12))) pos = tid;
    pos = wave64_min_i(pos);
    if ((tid & 63) == 0) wpos[tid >> 6] = pos;
    __syncthreads();
    int p = wpos[0];
#pragma unroll
    for (int w = 1; w < 16; ++w) p = min(p, wpos[w]);
    if (p == 0x7fffffff) p = 0;   // (n >= 2 always leaves an allowed position)
    *j1 = p / n;
    *j2 = p % n;
    *cv = sv[p];
    __syncthreads();   // sv, the wave slots and F are reused by the next probe
  };
  auto snapshot = [&](int slot, double mc) {
    int32_t* o = snap + (size_t)slot * INIT_SNAP;
    for (int e = tid; e < MAXD * 2 * MAXD; e += 1024) {
      const int k = e / (2 * MAXD), j = e % (2 * MAXD);
      o[e] = (k >= 1 && k < N && j < 2 * k) ? Ls[k][j] : 0;
      o[MAXD * 2 * MAXD + e] = (k >= 1 && k < N && j < 2 * (N - k)) ? Rs[k][j] : 0;
    }
    if (tid == 0) snap_mc[slot] = mc;
  };
  for (int it = 0; it < ia.max_it; ++it) {
    double mc = 0.0;
    for (int k = 1; k < N; ++k) {   // left to right: I^{<=k} = (I^{<=k-1} row 0, j1), (row 1, j2)
      int j1, j2;
      double cv;
      probe(k, 0, &j1, &j2, &cv);
      mc = fmax(mc, cv);
      if (tid == 0) {
        const int len = k - 1;
        for (int j = 0; j < len; ++j) {
          Ls[k][j] = Ls[k - 1][j];
          Ls[k][k + j] = Ls[k - 1][len + j];
        }
        Ls[k][len] = (int16_t)j1;
        Ls[k][k + len] = (int16_t)j2;
      }
      __syncthreads();
    }
    snapshot(2 * it, mc);
    mc = 0.0;
    for (int k = N; k >= 2; --k) {   // right to left: I^{>k-1} = (j1, I^{>k} row 0), (j2, row 1)
      int j1, j2;
      double cv;
      probe(k, 1, &j1, &j2, &cv);
      mc = fmax(mc, cv);
      if (tid == 0) {
        const int len = N - k;
        Rs[k - 1][0] = (int16_t)j1;
        Rs[k - 1][len + 1] = (int16_t)j2;
        for (int j = 0; j < len; ++j) {
          Rs[k - 1][1 + j] = Rs[k][j];
          Rs[k - 1][len + 2 + j] = Rs[k][len + j];
        }
      }
      __syncthreads();
    }
    snapshot(2 * it + 1, mc);
  }
}

// The stopping test's TT values at the fixed test multi-indices, one core at
// a time: the running row vectors of the P test points (P x r_{k-1}) times
// the slice C_k[:, i_p, :] of each point's index.  The points are grouped
// by their index at core k once for the whole cross (the test points never
// change), so every group is one product (rows: its points, K = r_{k-1},
// N = r_k) whose slice is read once per 16 points instead of once per
// point.  A block takes 16 points of one group and every column: their rows
// of V go to LDS, then each wave forms 16 x 16 output tiles with
// v_mfma_f64_16x16x4 (A at [l % 16][l / 16], B at [l / 16][l % 16], D row
// l / 16 + 4 v, column l % 16 in lane l, slot v).  C_k is column-major
// ((r_{k-1} n_k) x r_k): entry (s, i, t) at C[(s + i r_{k-1}) + t m].
constexpr int TEST_SLOTS = 64;
typedef double dbl4 __attribute__((ext_vector_type(4)));
struct TTTile {
  int32_t i, start, count, pad;   // the group's index, first position in perm, points (<= 16)
};
constexpr int TTW = 16;  // waves per block of k_tt_core (one 16-column tile each up to r = 256)
constexpr int TTB = 8;   // MFMA steps whose B operands are loaded together
__global__ void __launch_bounds__(TTW * 64) k_tt_core(const double* C, int r0, int r1, int m, const double* Vin,
                                                      int ldin, double* Vout, int ldout, const int32_t* perm,
                                                      const TTTile* tiles) {
  __shared__ double As[16][MAXR + 1];
  const TTTile t = tiles[blockIdx.x];
  // (wv through readfirstlane: the tile loop and the step guards below are
  // then known to be wave-uniform, scalar branches)
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nst = (r0 + 3) / 4;
  {   // the 16 points' rows of V: each thread's (at most 4 at 16 waves) point
      // indices first, then their rows, so the two rounds of loads issue together
    constexpr int ST = TTW * 64, NU = (16 * MAXR + ST - 1) / ST;
    int pidx[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * ST, row = e / r0;
      pidx[u] = (e < 16 * r0 && row < t.count) ? perm[t.start + row] : -1;
    }
    double v[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * ST, row = e / r0, kk = e - row * r0;
      v[u] = pidx[u] >= 0 ? Vin[(int64_t)pidx[u] * ldin + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * ST, row = e / r0, kk = e - row * r0;
      if (e < 16 * r0) As[row][kk] = v[u];
    }
    // zeros in the columns r0 .. 4 nst - 1 of the last MFMA step, so the A
    // operand reads need no guard
    if (tid < 64 && r0 + (tid & 3) < 4 * nst) As[tid >> 2][r0 + (tid & 3)] = 0.0;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  const double* Ci = C + (int64_t)t.i * r0;
  for (int ct = wv; ct < (r1 + 15) / 16; ct += TTW) {
    const int col = ct * 16 + li;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    // batches of TTB steps; the B operands of the next batch are loaded
    // while the current batch's products issue (two register sets).  Every
    // load reads a clamped, valid entry of the slice and nothing is masked:
    // past r0 the A operand is zero, and columns past r1 are not stored (a
    // guarded or selected load makes the compiler wait for every outstanding
    // load at once, the next batch's included)
    const int cc = min(col, r1 - 1);
    auto loadb = [&](int s0, double (&b)[TTB]) {
#pragma unroll
      for (int u = 0; u < TTB; ++u) b[u] = Ci[min(4 * (s0 + u) + lk, r0 - 1) + (int64_t)cc * m];
    };
    auto mma = [&](int s0, const double (&b)[TTB]) {
#pragma unroll
      for (int u = 0; u < TTB; ++u) {
        const int kk = 4 * (s0 + u) + lk;
        if (s0 + u < nst) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[li][kk], b[u], acc, 0, 0, 0);
      }
    };
    const int nbat = (nst + TTB - 1) / TTB;
    double bA[TTB], bB[TTB];
    loadb(0, bA);
    int bi = 0;
    for (; bi + 1 < nbat; bi += 2) {
      loadb((bi + 1) * TTB, bB);
      mma(bi * TTB, bA);
      if (bi + 2 < nbat) loadb((bi + 2) * TTB, bA);
      mma((bi + 1) * TTB, bB);
    }
    if (bi < nbat) mma(bi * TTB, bA);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = lk + 4 * v;
      if (row < t.count && col < r1) Vout[(int64_t)perm[t.start + row] * ldout + col] = acc[v];
    }
  }
}

// |vals[p] - V[p]| (the TT value after the last core) folded into
// err[p mod TEST_SLOTS] (cleared beforehand; non-negative doubles order like
// their bit patterns, so an integer atomic max is exact); the host takes the
// max of the slots.
__global__ void k_tt_err(const double* V, int ldv, const double* vals, int P, double* err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  atomicMax(reinterpret_cast<unsigned long long*>(err + p % TEST_SLOTS),
            (unsigned long long)__double_as_longlong(fabs(vals[p] - V[(int64_t)p * ldv])));
}

__global__ void k_fill1(double* p, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 1.0;
}

__global__ void k_zero1(double* p) {
  if (threadIdx.x == 0) *p = 0.0;
}

// Li^T and W^T, kept beside Li and W (second half of each factor buffer) so
// that every product of the cross reads its factor along rows.
constexpr int64_t FT = (int64_t)MAXR * MAXR;

// Copies of the leading r x r blocks of Li and W into their transposes.
__device__ inline void store_transposes(double* Li, double* W, int r) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      Li[FT + j + i * MAXR] = Li[i + j * MAXR];
      W[FT + j + i * MAXR] = W[i + j * MAXR];
    }
}

// Factors of the initial intersection matrix (r <= 2), written with leading
// dimension MAXR: Li (pivot x row), W (column x pivot), and their
// transposes; amax = max |entry|, info = 1 if no diagonal entry can lead.
__global__ void k_ldu_init(const double* P, int r, double* Li, double* W, double* amax, int32_t* info) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int i = 0; i < r * r; ++i) m = fmax(m, fabs(P[i]));
  *amax = m;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      Li[i + j * MAXR] = 0.0;
      W[i + j * MAXR] = 0.0;
    }
  if (r == 1) {
    *info = !(P[0] != 0.0) || !isfinite(P[0]);
    Li[0] = 1.0;
    W[0] = 1.0 / P[0];
    store_transposes(Li, W, 1);
    return;
  }
  const int f = fabs(P[3]) > fabs(P[0]) ? 1 : 0, g = 1 - f;   // first pivot: the larger diagonal entry
  const double d1 = P[f + f * r];
  // second pivot (g, g): b = P(:, g), c = P(g, :)
  const double u = P[f + g * r];          // Li row 0 = e_f, so u = b_f
  const double gl = P[g + f * r] / d1;    // W col 0 = e_f / d1, so g = c_f / d1
  const double sv = P[g + g * r] - gl * u;
  *info = !(d1 != 0.0) || !(sv != 0.0) || !isfinite(sv) || !isfinite(d1);
  Li[0 + f * MAXR] = 1.0;                 // pivot 0 reads row f
  Li[1 + g * MAXR] = 1.0;                 // pivot 1: e_g - gl e_f
  Li[1 + f * MAXR] = -gl;
  W[f + 0 * MAXR] = 1.0 / d1;             // column f of P^{-1}'s factor for pivot 0
  W[g + 1 * MAXR] = 1.0 / sv;             // pivot 1: (e_g - e_f u / d1) / s
  W[f + 1 * MAXR] = -(u / d1) / sv;
  store_transposes(Li, W, 2);
}


// Which entries of a factor can be non-zero: M(t, q) with q <= t (TRI_LO:
// Li and W^T), q >= t (TRI_UP: W and Li^T), or all (TRI_ALL), except that
// the leading 2 x 2 block is full (the initial factors put the larger
// diagonal entry first, which permutes their first two pivots; every later
// pivot borders them triangularly).  The entries outside are zeros by
// construction, so they are neither loaded nor added (their products would
// add exact zeros).
constexpr int TRI_ALL = 0, TRI_LO = 1, TRI_UP = 2;
__device__ inline int tri_qmax(int t) { return t > 1 ? t : 1; }   // TRI_LO: q <= tri_qmax(t)
__device__ inline int tri_qmin(int t) { return t > 1 ? t : 0; }   // TRI_UP: q >= tri_qmin(t)
__device__ inline bool tri_in(int tri, int t, int q) {
  return tri == TRI_LO ? q <= tri_qmax(t) : (tri == TRI_UP ? q >= tri_qmin(t) : true);
}

// out[t] = sum_q M(t, q) v[q] for t < r (row t of M, leading dimension
// MAXR, so a wave's loads are contiguous).  With r rounded up to 64 as ru,
// min(8, BS / ru) threads share a row, each over a contiguous range of q in
// batches of 16 loads issued together (the callers run 1024 threads, whose
// register budget holds no more without spilling); the partial sums meet in
// scratch (BS doubles).  TRI: the triangle of M that holds its non-zeros.  Every thread
// of the block calls it; out is visible to all on return.
template <int BS, int TRI>
__device__ __forceinline__ void row_dots(const double* M, const double* v, int r, double* out, double* scratch) {
  constexpr int RB = 16;
  const int ru = (r + 63) & ~63;
  const int S = min(8, BS / ru);
  const int tid = threadIdx.x, t = tid % ru, h = tid / ru;
  double acc = 0.0;
  if (h < S && t < r) {
    const int chunk = (r + S - 1) / S;
    const int q0 = h * chunk, q1 = min(r, q0 + chunk);
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q = q0; q < q1; q += RB) {
      if (TRI == TRI_LO && q > tri_qmax(t)) break;             // the rest of the row is zero
      if (TRI == TRI_UP && q + RB <= tri_qmin(t)) continue;    // this batch is zero
      double mv[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u)
        mv[u] = (q + u < q1 && tri_in(TRI, t, q + u)) ? M[t + (int64_t)(q + u) * MAXR] : 0.0;
      if (q + RB <= q1) {   // a whole batch: no guard, so the LDS reads of v issue together
#pragma unroll
        for (int u = 0; u < RB; ++u) a[u & 7] += mv[u] * v[q + u];
      } else {
#pragma unroll
        for (int u = 0; u < RB; ++u) a[u & 7] += q + u < q1 ? mv[u] * v[q + u] : 0.0;
      }
    }
    acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  scratch[tid] = acc;
  __syncthreads();
  if (tid < r) {
    double sum = scratch[tid];
    for (int k = 1; k < S; ++k) sum += scratch[tid + k * ru];
    out[tid] = sum;
  }
  __syncthreads();
}

// Robust argmax of |R| over the whole block (lowest key within tau of the
// max) and the relative top-2 margin; stage 0 = sample stage (also records
// row/col of the chosen sample), stage 1 = search stage.  The sample list is
// in generation order, so its key is the linear position row * cols + col;
// the searched fibre is in natural order.  |R| is read once, C values per
// thread held in registers (n <= BS C), then wave shuffles and one LDS stage
// per pass.  Returns the chosen position in every thread, its key and its
// |R|.
template <int BS, int C>
__device__ int select_block(const double* R, int n, const int32_t* srow, const int32_t* scol, int cols, int stage,
                            double scale, StepRes* res, int* key_out, double* val_out) {
  constexpr int NWV = BS / 64;
  __shared__ double sv[NWV];
  __shared__ int sk[NWV], si[NWV];
  __shared__ double s_mx, s_pa;
  __shared__ int s_p, s_key;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double tau = TIE_REL * scale;
  double av[C];
  double m = -1.0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = tid + c * BS;
    av[c] = i < n ? fabs(R[i]) : -1.0;
    m = fmax(m, av[c]);
  }
  m = wave64_max(m);
  if (lane == 0) sv[w] = m;
  __syncthreads();
  if (tid == 0) {
    double x = sv[0];
    for (int k = 1; k < NWV; ++k) x = fmax(x, sv[k]);
    s_mx = x;
  }
  __syncthreads();
  const double mx = s_mx;
  int best = 0x7fffffff, bi = 0x7fffffff;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = tid + c * BS;
    if (i < n && av[c] >= mx - tau) {
      const int key = stage == 0 ? srow[i] * cols + scol[i] : i;
      if (key < best) { best = key; bi = i; }
    }
  }
  {   // keys are distinct, so the lowest key names one entry
    const int kmin = wave64_min_i(best);
    bi = wave64_min_i(best == kmin ? bi : 0x7fffffff);
    best = kmin;
  }
  if (lane == 0) { sk[w] = best; si[w] = bi; }
  __syncthreads();
  if (tid == 0) {
    int b = sk[0], ii = si[0];
    for (int k = 1; k < NWV; ++k)
      if (sk[k] < b) { b = sk[k]; ii = si[k]; }
    const bool found = ii < n;   // (no candidate compares, e.g. all residuals NaN: the first)
    s_p = found ? ii : 0;
    s_key = found ? b : (stage == 0 ? srow[0] * cols + scol[0] : 0);
  }
  __syncthreads();
  const int p = s_p;
  double sec = 0.0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = tid + c * BS;
    if (i < n && i != p) sec = fmax(sec, av[c]);
    if (i == p) s_pa = av[c];
  }
  sec = wave64_max(sec);
  if (lane == 0) sv[w] = sec;
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < NWV; ++k) sec = fmax(sec, sv[k]);
    sec = fmax(sec, sv[0]);
    const double margin = mx > 0.0 ? (mx - sec) / mx : 0.0;
    if (stage == 0) {
      res->s_pos = p; res->s_max = mx; res->s_margin = margin; res->s_tau = tau;
      res->l = s_key / cols; res->t = s_key % cols;
      res->s_scale = scale;
      res->q_scale = scale;             // the search stage widens this scale
    } else {
      res->q_pos = p; res->q_max = mx; res->q_margin = margin; res->q_tau = tau;
      res->q_scale = scale;
      res->pivot_abs = s_pa;
    }
  }
  *key_out = s_key;
  *val_out = s_pa;
  return p;
}

// max of the AMAX_SLOTS slots of a fold
__device__ inline double slots_max(const double* sl) {
  double m = 0.0;
  for (int i = 0; i < AMAX_SLOTS; ++i) m = fmax(m, sl[i]);
  return m;
}

// Sample stage: residuals R_i = A(s_i, J) P^{-1} A(I, s_i) - A(s_i) of the
// sampled entries, written as the row-wise dot product of G = A(s, J) W and
// T = (Li A(I, s))^T, both formed with FP64 MFMA on 16-row tiles of 16
// samples (v_mfma_f64_16x16x4: A at [l % 16][l / 16], B at [l / 16][l % 16],
// D row l / 16 + 4 v, column l % 16 in lane l, slot v).  A(s_i, J_q) and
// A(I_q, s_i) are entries of the fibre cores F_k and F_{k+1} (the fibre
// cache), gathered straight into LDS in MFMA lane order; only A(s_i) itself
// is evaluated, by a row of 16 lanes per sample.  The max |.| of all of them folds into the
// sample-stage slots.  Each wave owns one 16-column tile of G and T at a
// time; the B operands of its first tile (rows of W^T and Li) are loaded into
// registers before the gathers.
constexpr int SW = 8;    // waves per block
constexpr int SPB = 16;  // samples per block: one full MFMA row tile
constexpr int SB = 32;   // MFMA steps of B operands held in registers (r <= 128: one batch)

// The it-th 16-column tile of wave wv among nw waves, in snake order (wv,
// 2 nw - 1 - wv, 2 nw + wv, ...): the products with a triangular factor cost
// more for later tiles, and the snake spreads them evenly over the waves.
__device__ inline int snake_tile(int it, int wv, int nw) {
  return (it & 1) ? (it + 1) * nw - 1 - wv : it * nw + wv;
}
template <int d, int dt, bool G>
__global__ void __launch_bounds__(SW * 64) k_sample_resid(KSpec ks, const StepDesc* desc, const int32_t* sel, int r,
                                                          const double* Li, const double* W, const double* FLk,
                                                          const double* FRk1, double* R, double* slots) {
  constexpr int D = 2 * d + dt;
  const StepDesc& sd = desc[*sel];
  const Addr ad = sd.a;
  const int32_t* srow = sd.srow;
  const int32_t* scol = sd.scol;
  const int ns = sd.ns;
  extern __shared__ double sa[];   // A operands (2 x 64 x nst)
  __shared__ double red[SW][16], sn[D * MAXN], sAs[16], redm[SW], S[SPB * D];
  __shared__ int64_t offL[SPB], offR[SPB];
  // (wv through readfirstlane: the tile index and the triangular step bound
  // below are then known to be wave-uniform, so the step guards are scalar
  // branches)
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int i0 = blockIdx.x * SPB;
  const int nv = min(SPB, ns - i0);   // samples of this block (none past the variant's extent)
  const int nst = (r + 3) / 4;
  const int ntile = (r + 15) / 16;
  const double* Wt = W + FT;
  // B operands in batches of HB steps, two register sets: the next batch
  // loads while the current one multiplies; the first tile's first batch
  // loads before the gathers.  Every load reads a clamped, valid address and
  // zeros what lies past r by a select (a guarded load compiles to a branch
  // per load, after which the compiler waits for all loads at every MFMA).
  constexpr int HB = SB / 2;
  double bgA[HB], btA[HB], bgB[HB], btB[HB];
  auto loadb = [&](int p, int s0, double (&bg)[HB], double (&bt)[HB]) {
    const int pc = min(p, MAXR - 1);
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const int q = 4 * (s0 + u) + lg;
      const bool ok = p < r && q < r;
      const int64_t e = pc + (int64_t)min(q, MAXR - 1) * MAXR;
      const double w = Wt[e], l = Li[e];
      bg[u] = ok ? w : 0.0;
      bt[u] = ok ? l : 0.0;
    }
  };
  loadb(wv * 16 + li, 0, bgA, btA);
  stage_nodes<D>(ks.nodes, sn);   // (synchronises the block)
  if (tid < SPB) {
    double c[D];
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = 0.0;
    int64_t oL = 0, oR = 0;
    if (tid < nv) {
      const int row = srow[i0 + tid], col = scol[i0 + tid];
      addr_row_part<D>(ad, sn, row, c);
      addr_col_part<D>(ad, sn, col, c);
      oL = fibre_left_row(row % ad.rl, row / ad.rl);
      oR = fibre_right_col(col % ad.nm1, col / ad.nm1);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) S[tid * D + j] = c[j];
    offL[tid] = oL;
    offR[tid] = oR;
  }
  for (int e = tid; e < 64 * nst; e += SW * 64) {   // operand rows without a sample or a q
    const int ii = e & 15, q = e >> 4;
    if (ii >= nv || q >= r) {
      const int slot = (q >> 2) * 64 + (q & 3) * 16 + ii;
      sa[slot] = 0.0;
      sa[64 * nst + slot] = 0.0;
    }
  }
  __syncthreads();
  double m = 0.0;
  for (int e = tid; e < nv * r; e += SW * 64) {   // q fastest: contiguous cache rows
    const int ii = e / r, q = e - ii * r;
    const double vg = FLk[offL[ii] + q];    // A(s_i, J_q) = F_k(s, i_k, q)
    const double vt = FRk1[offR[ii] + q];   // A(I_q, s_i) = F_{k+1}(q, i_{k+1}, t)
    const int slot = (q >> 2) * 64 + (q & 3) * 16 + ii;
    sa[slot] = vg;
    sa[64 * nst + slot] = vt;
    m = fmax(m, fmax(fabs(vg), fabs(vt)));
  }
  {   // A(s_i): one sample per row of 16 lanes, which share its evaluation
    const int g = tid >> 4, l16 = tid & 15;
    if (g < nv) {
      double c[D];
#pragma unroll
      for (int j = 0; j < D; ++j) c[j] = S[g * D + j];
      const double v = kappa_eval<d, dt, G, true>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c, l16);
      if (l16 == 0) sAs[g] = v;
      m = fmax(m, fabs(v));
    }
  }
  m = wave64_max(m);
  if (lane == 0) redm[wv] = m;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < SW; ++w) m = fmax(m, redm[w]);
    m = fmax(m, redm[0]);
    atomicMax(reinterpret_cast<unsigned long long*>(slots + blockIdx.x % AMAX_SLOTS),
              (unsigned long long)__double_as_longlong(m));
  }
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it * SW < ntile; ++it) {
    const int jt = snake_tile(it, wv, SW);
    if (jt >= ntile) continue;
    const int p = jt * 16 + li;
    // W (upper) and Li (lower) hold W(q, p) and Li(p, q) only for q <= p:
    // the tile's products end at the step holding its last column
    const int nst_t = min(nst, 4 * jt + 4);
    dbl4 g = {0.0, 0.0, 0.0, 0.0}, t = {0.0, 0.0, 0.0, 0.0};
    auto mma = [&](int s0, const double (&bg)[HB], const double (&bt)[HB]) {
#pragma unroll
      for (int u = 0; u < HB; ++u) {
        if (s0 + u < nst_t) {
          g = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[(s0 + u) * 64 + lane], bg[u], g, 0, 0, 0);
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[64 * nst + (s0 + u) * 64 + lane], bt[u], t, 0, 0, 0);
        }
      }
    };
    const int nbat = (nst_t + HB - 1) / HB;
    if (it != 0) loadb(p, 0, bgA, btA);   // (the first tile's first batch is loaded already)
    int bi = 0;
    for (; bi + 1 < nbat; bi += 2) {
      loadb(p, (bi + 1) * HB, bgB, btB);
      mma(bi * HB, bgA, btA);
      if (bi + 2 < nbat) loadb(p, (bi + 2) * HB, bgA, btA);
      mma((bi + 1) * HB, bgB, btB);
    }
    if (bi < nbat) mma(bi * HB, bgA, btA);
#pragma unroll
    for (int v = 0; v < 4; ++v) part[v] += g[v] * t[v];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    part[v] = row16_sum(part[v]);
  if (li == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv][lg + 4 * v] = part[v];
  __syncthreads();
  if (tid < nv) {
    double s = 0.0;
    for (int w = 0; w < SW; ++w) s += red[w][tid];
    R[i0 + tid] = s - sAs[tid];
  }
}

// dynamic LDS of k_sample_resid for rank r
inline size_t sample_lds(int r) { return (size_t)2 * 64 * ((r + 3) / 4) * sizeof(double); }

// Sample-stage selection over the residuals of k_sample_resid (one block),
// then the search stage's solve: u = A(l, J) for a row search (bit 1) or
// u = A(I, t) for a column search (bit 0), read from the fibre cache, and
// x = (u W) Li = Li^T (W^T u), or x = W (Li u), is written for k_search
// (P^{-1} applied to one vector, through the rows of the factors or of their
// transposes), followed at x + MAXR by the intermediate W^T u or Li u.  |u|
// folds into the search-stage scale.
template <int d, int dt, bool G>
__global__ void __launch_bounds__(1024) k_sample_select(KSpec ks, const StepDesc* desc, const int32_t* sel,
                                                        const double* R, const double* luamax, StepRes* res, int r,
                                                        const double* Li, const double* W, const double* FLk,
                                                        const double* FRk1, double* x) {
  const StepDesc& sdv = desc[*sel];
  const Addr a = sdv.a;
  const int32_t* srow = sdv.srow;
  const int32_t* scol = sdv.scol;
  const int ns = sdv.ns, cols = sdv.cols, bit = sdv.bit;
  __shared__ double su[MAXR], sy[MAXR], scr[1024], red[16];
  const int tid = threadIdx.x;
  int key;
  double val;
  select_block<1024, (MAXR * MAXN + 1023) / 1024>(R, ns, srow, scol, cols, 0,
                                                  fmax(slots_max(res->s_slot), *luamax), res, &key, &val);
  const int l = key / cols, t = key - l * cols;
  double m = 0.0;
  if (tid < r) {
    const double v = bit ? FLk[fibre_left_row(l % a.rl, l / a.rl) + tid]      // A(l, J_q)
                         : FRk1[fibre_right_col(t % a.nm1, t / a.nm1) + tid];  // A(I_q, t)
    su[tid] = v;
    m = fabs(v);
  }
  m = wave64_max(m);
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    m = fmax(m, red[0]);
    res->q_slot[0] = fmax(res->q_slot[0], m);
  }
  if (bit) {
    row_dots<1024, TRI_LO>(W + FT, su, r, sy, scr);    // W^T u
    row_dots<1024, TRI_UP>(Li + FT, sy, r, su, scr);   // Li^T (W^T u), into su (u is consumed)
  } else {
    row_dots<1024, TRI_LO>(Li, su, r, sy, scr);        // Li u
    row_dots<1024, TRI_UP>(W, sy, r, su, scr);         // W (Li u)
  }
  for (int q = tid; q < r; q += 1024) {
    x[q] = su[q];
    x[MAXR + q] = sy[q];   // the intermediate vector, which the border reuses
  }
}

// Search stage: the residual over the searched fibre,
//   R_i = sum_q A(I_q, i) x_q - A(l, i)   (row search, bit 1, i < cols), or
//   R_i = sum_q A(i, J_q) x_q - A(i, t)   (column search, bit 0, i < rows),
// with (l, t) the chosen sample and x = P^{-1} u from k_sample_select.
// A(I_q, i) = F_{k+1}(q, i_{k+1}, t_i) and A(i, J_q) = F_k(s_i, i_k, q) come
// from the fibre cache; the fibre entries A(l, i) or A(i, t) are evaluated
// (by the entry's 16 lanes together) and stored in the slot the pivot would
// occupy: row r of F_{k+1} (bit 1) or column r of F_k (bit 0), when r < MAXR.
// Sixteen fibre entries per block, one 16-lane row per entry with the q
// terms strided over its lanes (the fibre entry as term q = r, weight -1)
// and summed by DPP.  Every value's
// max |.| folds into the search-stage slots.
constexpr int QE = 16;   // fibre entries per block
template <int d, int dt, bool G>
__global__ void __launch_bounds__(256) k_search(KSpec ks, const StepDesc* desc, const int32_t* sel,
                                                const StepRes* res, const double* x, int r, double* FLk, double* FRk,
                                                double* FLk1, double* FRk1, double* R, double* slots) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN], sx[MAXR + 1], fc[D], redm[4];
  const StepDesc& sd = desc[*sel];
  const Addr a = sd.a;
  const int bit = sd.bit;
  const int n = bit ? sd.cols : sd.rows;
  const int tid = threadIdx.x;
  stage_nodes<D>(ks.nodes, sn);   // (synchronises the block)
  const int l = res->l, t = res->t;
  if (tid == 0) {   // the fixed half of the fibre: the row of l or the column of t
    double c[D];
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = 0.0;
    if (bit) addr_row_part<D>(a, sn, l, c);
    else addr_col_part<D>(a, sn, t, c);
#pragma unroll
    for (int j = 0; j < D; ++j) fc[j] = c[j];
  }
  for (int q = tid; q <= r; q += 256) sx[q] = q < r ? x[q] : -1.0;   // the fibre's own entry enters with weight -1
  __syncthreads();
  const int i = blockIdx.x * QE + (tid >> 4), lj = tid & 15;
  double acc = 0.0, m = 0.0;
  if (i < n) {
    // the entry's position in the cache: column (i_{k+1}, t_i) of F_{k+1}
    // (bit 1) or row (s_i, i_k) of F_k (bit 0)
    const int ia = bit ? i % a.nm1 : i % a.rl, ib = bit ? i / a.nm1 : i / a.rl;
    const double* crow = bit ? FRk1 + fibre_right_col(ia, ib) : FLk + fibre_left_row(ia, ib);
    double vf;   // the fibre entry, evaluated by the entry's 16 lanes together
    {
      double c[D], vc[D];
#pragma unroll
      for (int j = 0; j < D; ++j) vc[j] = 0.0;
      if (bit) addr_col_part<D>(a, sn, i, vc);
      else addr_row_part<D>(a, sn, i, vc);
#pragma unroll
      for (int j = 0; j < D; ++j) c[j] = ((j <= a.lk) == (bit != 0)) ? fc[j] : vc[j];
      vf = kappa_eval<d, dt, G, true>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c, lj);
    }
    if (lj == 0 && r < MAXR) {
      if (bit) {   // row r of F_{k+1}: F_{k+1}(r, i_{k+1}, t_i)
        FLk1[fibre_left_row(r, ia) + ib] = vf;
        FRk1[fibre_right_col(ia, ib) + r] = vf;
      } else {     // column r of F_k: F_k(s_i, i_k, r)
        FLk[fibre_left_row(ia, ib) + r] = vf;
        FRk[fibre_right_col(ib, r) + ia] = vf;
      }
    }
    // the lane's terms q = lj, lj + 16, ... in order; four at a time while
    // all four lie below r, so their loads issue together
    int q = lj;
    for (; q + 48 < r; q += 64) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = crow[q + 16 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc += v[u] * sx[q + 16 * u];
        m = fmax(m, fabs(v[u]));
      }
    }
    for (; q <= r; q += 16) {
      const double v = q < r ? crow[q] : vf;
      acc += v * sx[q];
      m = fmax(m, fabs(v));
    }
  }
  acc = row16_sum(acc);
  if (lj == 0 && i < n) R[i] = acc;
  m = wave64_max(m);
  if ((tid & 63) == 0) redm[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    m = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
    atomicMax(reinterpret_cast<unsigned long long*>(slots + blockIdx.x % AMAX_SLOTS),
              (unsigned long long)__double_as_longlong(m));
  }
}

// The border of P_k's factors for the pivot (row, col) added by step k:
// b = A(I, t), c = A(l, J) and d = A(l, t) are read from the fibre cache
// (d from the fibre the search stage stored), then
// u = Li b, g = W^T c, s = d - g^T u,
//   Li' = [[Li, 0], [-g^T Li, 1]],  W' = [[W, -W u / s], [0, 1 / s]]
// (leading dimension MAXR, transposes alongside).  One side is already at
// xs (k_sample_select): after a row search the pivot row's c was the solved
// vector, so g = xs[MAXR..] and Li^T g = xs[..]; after a column search b
// was, so u and W u are.  amax0 is the value of *amax read at the start of
// the kernel.  Every thread of the block calls it.
constexpr int FB = 1024;   // threads of the finishing kernel
__device__ void border_factors(const Addr& a, int bit, StepRes* res, int r, int row, int col, double* Li, double* W,
                               double* amax, double amax0, int32_t* info, const double* FLk, const double* FLk1,
                               const double* FRk1, const double* xs) {
  constexpr int NW = FB / 64;
  __shared__ double bv[MAXR], cv[MAXR], u[MAXR], gv[MAXR], nl[MAXR], nw[MAXR], scr[FB];
  __shared__ double s_d, s_s;
  const int tid = threadIdx.x;
  const int sl = row % a.rl, il = row / a.rl;     // the pivot row: (s, i_k)
  const int it = col % a.nm1, tt = col / a.nm1;   // the pivot column: (i_{k+1}, t)
  for (int e = tid; e <= 2 * r; e += FB) {
    if (e < r) bv[e] = FRk1[fibre_right_col(it, tt) + e];            // F_{k+1}(e, i_{k+1}, t)
    else if (e < 2 * r) cv[e - r] = FLk[fibre_left_row(sl, il) + (e - r)];   // F_k(s, i_k, e)
    else s_d = bit ? FLk1[fibre_left_row(r, it) + tt] : FLk[fibre_left_row(sl, il) + r];
  }
  for (int e = tid; e < r; e += FB) {
    if (bit) {
      gv[e] = xs[MAXR + e];
      nl[e] = xs[e];
    } else {
      u[e] = xs[MAXR + e];
      nw[e] = xs[e];
    }
  }
  __syncthreads();
  double* Lit = Li + FT;
  double* Wt = W + FT;
  if (bit) row_dots<FB, TRI_LO>(Li, bv, r, u, scr);    // Li b
  else row_dots<FB, TRI_LO>(Wt, cv, r, gv, scr);       // W^T c
  {
    double gu = 0.0, m = 0.0;
    for (int p = tid; p < r; p += FB) {
      gu += gv[p] * u[p];
      m = fmax(m, fmax(fabs(bv[p]), fabs(cv[p])));
    }
    gu = wsum(gu);
    m = wave64_max(m);
    if ((tid & 63) == 0) { scr[tid >> 6] = gu; scr[NW + (tid >> 6)] = m; }   // (nl or nw holds x)
    __syncthreads();
    if (tid == 0) {
      gu = 0.0;
      m = 0.0;
      for (int w = 0; w < NW; ++w) {
        gu += scr[w];
        m = fmax(m, scr[NW + w]);
      }
      s_s = s_d - gu;
      *amax = fmax(fmax(amax0, m), fabs(s_d));
      if (!(s_s != 0.0) || !isfinite(s_s)) {
        *info = 1;
        res->info = 1;
      }
    }
    __syncthreads();
  }
  const double is = 1.0 / s_s;
  if (bit) row_dots<FB, TRI_UP>(W, u, r, nw, scr);     // W u
  else row_dots<FB, TRI_UP>(Lit, gv, r, nl, scr);      // Li^T g (i.e. g^T Li, old factors)
  for (int e = tid; e <= 2 * r + 1; e += FB) {
    if (e < r) {
      Li[r + (int64_t)e * MAXR] = -nl[e];    // row r, column e
      Lit[e + (int64_t)r * MAXR] = -nl[e];
      Li[e + (int64_t)r * MAXR] = 0.0;       // column r above the diagonal
      Lit[r + (int64_t)e * MAXR] = 0.0;
    } else if (e < 2 * r) {
      const int j = e - r;
      W[j + (int64_t)r * MAXR] = -nw[j] * is;    // column r
      Wt[r + (int64_t)j * MAXR] = -nw[j] * is;
      W[r + (int64_t)j * MAXR] = 0.0;            // row r left of the diagonal
      Wt[j + (int64_t)r * MAXR] = 0.0;
    } else if (e == 2 * r) {
      Li[r + (int64_t)r * MAXR] = 1.0;
      Lit[r + (int64_t)r * MAXR] = 1.0;
    } else {
      W[r + (int64_t)r * MAXR] = is;
      Wt[r + (int64_t)r * MAXR] = is;
    }
  }
}

// End of a step, one block: the search stage's selection, then the pivot
// (l, t) from the two stages; it is added
// if its residual exceeds the tie band, it is not yet in I or J and the rank
// is below the cap.  Then, if added, the border of P_k (border_factors).
// Clears the fold slots for the next step and publishes the result to the
// host mailbox.
static_assert(MAXR <= FB, "k_finish_step holds one pivot per thread");
__global__ void __launch_bounds__(FB) k_finish_step(const StepDesc* desc, const int32_t* sel, const double* R,
                                                     StepRes* res, int r, int max_rank, double* Li, double* W,
                                                     double* amax, int32_t* info, StepRes* mail, uint32_t* mail_seq,
                                                     uint32_t seq, int32_t* sel_next, int16_t* next_left,
                                                     int next_row, const double* FLk, const double* FLk1,
                                                     const double* FRk1, const double* xs) {
  const StepDesc& sd = desc[*sel];
  const Addr a = sd.a;
  const int bit = sd.bit;
  __shared__ int s_added;
  const int tid = threadIdx.x;
  // loads that do not depend on the selection, issued before it
  int32_t iq = -1, jq = -1;
  if (tid < r) {
    iq = sd.I[tid];
    jq = sd.J[tid];
  }
  const int l0 = res->l, t0 = res->t;
  const double amax0 = *amax;
  const int32_t info0 = *info;
  const double scale = fmax(res->q_scale, slots_max(res->q_slot));
  // the search stage's selection over R (written by k_search)
  int key;
  double pabs;
  const int qp = select_block<FB, (MAXR * MAXN + FB - 1) / FB>(R, bit ? sd.cols : sd.rows, nullptr, nullptr,
                                                               sd.cols, 1, scale, res, &key, &pabs);
  const int row = bit ? l0 : qp, col = bit ? qp : t0;
  // the pivot's left row, for the next step's left set: loaded now, stored
  // at the end if the pivot is added
  int16_t lv = 0;
  if (next_left && tid <= a.lk) {
    const int s = row % a.rl;
    lv = tid < a.lk ? a.left[(size_t)s * a.lk + tid] : (int16_t)(row / a.rl);
  }
  const int stale = __syncthreads_or(tid < r && (iq == row || jq == col));
  if (tid == 0) {
    const int added = (pabs > TIE_REL * scale && !stale && r < max_rank) ? 1 : 0;
    res->pivot_row = row;
    res->pivot_col = col;
    res->added = added;
    res->info = info0;   // status of the kept factors (non-zero after a singular border)
    s_added = added;
  }
  if (tid < AMAX_SLOTS) {   // the next step folds its maxima into cleared slots
    res->s_slot[tid] = 0.0;
    res->q_slot[tid] = 0.0;
  }
  __syncthreads();
  if (s_added) border_factors(a, bit, res, r, row, col, Li, W, amax, amax0, info, FLk, FLk1, FRk1, xs);
  // the next step of the sweep runs on variant s_added; if the pivot was
  // added, I^{<=k} gains the row (left row s of the pivot, node i_k), which
  // the next step's left set receives after its r_k current rows
  if (tid == 0 && sel_next) *sel_next = s_added;
  if (s_added && next_left && tid <= a.lk) next_left[(size_t)next_row * (a.lk + 1) + tid] = lv;
  // publish the step's result to the host mailbox: the fields up to the
  // fold slots, one 8-byte word per thread so that the copies to host memory
  // overlap (a single thread's copy loop waited for every store), then, after
  // a system-scope fence, the sequence number the host waits for
  constexpr int MAIL_WORDS = (int)(offsetof(StepRes, s_slot) / 8);
  static_assert(MAIL_WORDS <= 64, "the copying threads are those of wave 0, as is the fencing one");
  __syncthreads();
  if (tid < MAIL_WORDS)
    reinterpret_cast<uint64_t*>(mail)[tid] = reinterpret_cast<const uint64_t*>(res)[tid];
  __syncthreads();
  if (tid == 0) {
    __threadfence_system();
    __hip_atomic_store(mail_seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// After a step that added its pivot (l, t): the fibre the search stage did
// not evaluate goes into the fibre cache, the column of super-core k through
// t as column r of F_k (after a row search, bit 1) or its row through l as
// row r of F_{k+1} (after a column search, bit 0), 16 entries per block, one
// per row of 16 lanes.  Nothing happens when the pivot was not added (the
// flag is read by every block alike).
template <int d, int dt, bool G>
__global__ void __launch_bounds__(256) k_add_fibre(KSpec ks, const StepDesc* desc, const int32_t* sel,
                                                   const StepRes* res, int r, double* FLk, double* FRk, double* FLk1,
                                                   double* FRk1) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN], fc[D];
  if (!res->added) return;
  const StepDesc& sd = desc[*sel];
  const Addr a = sd.a;
  const int bit = sd.bit;
  const int n = bit ? sd.rows : sd.cols;
  if ((int)blockIdx.x * 16 >= n) return;
  stage_nodes<D>(ks.nodes, sn);   // (synchronises the block)
  const int row = res->pivot_row, col = res->pivot_col;
  const int tid = threadIdx.x, l16 = tid & 15;
  if (tid == 0) {   // the fixed half: the pivot's column (bit 1) or row (bit 0)
    double c[D];
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = 0.0;
    if (bit) addr_col_part<D>(a, sn, col, c);
    else addr_row_part<D>(a, sn, row, c);
#pragma unroll
    for (int j = 0; j < D; ++j) fc[j] = c[j];
  }
  __syncthreads();
  const int i = blockIdx.x * 16 + (tid >> 4);   // one entry per row of 16 lanes
  if (i >= n) return;
  double c[D], vc[D];
#pragma unroll
  for (int j = 0; j < D; ++j) vc[j] = 0.0;
  if (bit) addr_row_part<D>(a, sn, i, vc);
  else addr_col_part<D>(a, sn, i, vc);
#pragma unroll
  for (int j = 0; j < D; ++j) c[j] = ((j <= a.lk) == (bit != 0)) ? vc[j] : fc[j];
  const double v = kappa_eval<d, dt, G, true>(ks.kind, ks.kconst, ks.thfix[0], ks.thfix[1], c, l16);
  if (l16 != 0) return;
  if (bit) {   // F_k(s_i, i_k, r)
    const int sa = i % a.rl, ia = i / a.rl;
    FLk[fibre_left_row(sa, ia) + r] = v;
    FRk[fibre_right_col(ia, r) + sa] = v;
  } else {     // F_{k+1}(r, i_{k+1}, t_i)
    const int ia = i % a.nm1, tb = i / a.nm1;
    FLk1[fibre_left_row(r, ia) + tb] = v;
    FRk1[fibre_right_col(ia, tb) + r] = v;
  }
}

// The fibre cores of the initial index sets (ranks <= 2) into the cache:
// F_k(a, i, b) for the fibre address of core k (rows a + i r_{k-1}, columns b).
template <int d, int dt, bool G>
__global__ void __launch_bounds__(256) k_fill_fibre(KSpec ks, Addr a, int rows, int rk, double* FL, double* FR) {
  constexpr int D = 2 * d + dt;
  __shared__ double sn[D * MAXN];
  stage_nodes<D>(ks.nodes, sn);   // (synchronises the block)
  const int e = blockIdx.x * 16 + (threadIdx.x >> 4);   // one entry per row of 16 lanes
  if (e >= rows * rk) return;
  const int row = e % rows, b = e / rows;
  const double v = addr_eval_row16<d, dt, G>(ks, a, sn, row, b, threadIdx.x & 15);
  if ((threadIdx.x & 15) != 0) return;
  const int sa = row % a.rl, ia = row / a.rl;
  FL[fibre_left_row(sa, ia) + b] = v;
  FR[fibre_right_col(ia, b) + sa] = v;
}

// The stopping test's result, published to a mailbox slot: the largest of
// the error slots (one per lane) and the OR of the factor status flags of
// P_1 .. P_{N-1}.
__global__ void __launch_bounds__(64) k_test_publish(const double* err, const int32_t* info, int N, StepRes* mail,
                                                     uint32_t* mail_seq, uint32_t seq) {
  const int lane = threadIdx.x;
  const double m = wave64_max(lane < TEST_SLOTS ? err[lane] : 0.0);
  int flag = 0;
  for (int k = 1; k < N; ++k) flag |= info[k];
  if (lane == 0) {
    mail->s_max = m;
    mail->info = flag;
    __threadfence_system();
    __hip_atomic_store(mail_seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The fibres F_k = X(I^{<=k-1}, i_k, I^{>k}) ((r_{k-1} n_k) x r_k,
// column-major) of the stopping test: the cache they are read from (FL_k),
// the column-major copies written, and their sizes.
struct CoreEval {
  const double* FL[MAXD];
  double* out[MAXD];
  int nr[MAXD], rl[MAXD];
  int64_t size[MAXD];
  int n;
};

// One 16 x 16 output tile of A B with FP64 MFMA: A (16 rows x 4 nst) in LDS in
// lane order (step s, lane l at s * 64 + l), B(q, p) = Bt[p + q MAXR] for this
// lane's column p, over the steps [sb, se) (B is zero outside them); the B
// loads of the next SB / 2 steps are in flight while the current ones
// multiply.  The A rows past r must be zero in LDS and the output columns
// past r are not stored, so the B loads read clamped entries of the r x r
// factor unmasked (a masked load makes the compiler wait for every
// outstanding load before each MFMA, the next batch's included).
__device__ __attribute__((always_inline)) inline dbl4 mfma_tile_lds(const double* sa, int sb, int se, const double* Bt, int p,
                                                                  int r, int lane) {
  constexpr int HB = SB / 2;   // steps per batch: the next batch loads while this one multiplies
  const int lk = lane >> 4;
  const double* Bp = Bt + min(p, r - 1);
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  auto loadb = [&](int s0, double (&b)[HB]) {
#pragma unroll
    for (int u = 0; u < HB; ++u) b[u] = Bp[(int64_t)min(4 * (s0 + u) + lk, r - 1) * MAXR];
  };
  auto mma = [&](int s0, const double (&b)[HB]) {
#pragma unroll
    for (int u = 0; u < HB; ++u)
      if (s0 + u < se) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[(s0 + u) * 64 + lane], b[u], acc, 0, 0, 0);
  };
  if (se <= sb) return acc;
  const int nbat = (se - sb + HB - 1) / HB;
  double bA[HB], bB[HB];
  loadb(sb, bA);
  int bi = 0;
  for (; bi + 1 < nbat; bi += 2) {
    loadb(sb + (bi + 1) * HB, bB);
    mma(sb + bi * HB, bA);
    if (bi + 2 < nbat) loadb(sb + (bi + 2) * HB, bA);
    mma(sb + (bi + 1) * HB, bB);
  }
  if (bi < nbat) mma(sb + bi * HB, bA);
  return acc;
}

// Cores of the interpolation formula C_k = F_k P_k^{-1} = (F_k W) Li for
// every k < D: one block per 16 rows of one core (tile ranges
// tile[j] .. tile[j + 1]); F rows and then T = F W are held in LDS in lane
// order (dynamic, 2 x 64 x ceil(r / 4) doubles), W and Li read through their
// transposes.
struct CoreSolve {
  const double* F[MAXD];
  double* C[MAXD];
  const double* Li[MAXD];
  const double* W[MAXD];
  int m[MAXD], r[MAXD];
  int tile[MAXD + 1];
  int n;
};
constexpr int CW = 4;   // waves per block of the solve

// dynamic LDS of the core solve (k_eval_solve) for rank r
inline size_t solve_lds(int r) { return (size_t)2 * 64 * ((r + 3) / 4) * sizeof(double); }

// The stopping test's fibres and cores in one launch: the solve tiles read
// their 16 rows of F_k from the fibre cache (straight into the lane order of
// the first product, and into the column-major F_k in memory, which the
// refinement of the returned cores reads), then blocks past the tiles copy
// the last fibre F_D (C_D = F_D, no solve), 256 entries each.  Block 0 also
// clears the test's error slots.
__global__ void __launch_bounds__(CW * 64) k_eval_solve(CoreEval ce, CoreSolve cs, double* clear) {
  extern __shared__ double lds[];
  if (blockIdx.x == 0 && threadIdx.x < TEST_SLOTS) clear[threadIdx.x] = 0.0;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= cs.tile[cs.n]) {   // the last fibre
    const int j = ce.n - 1;
    const int64_t e = (int64_t)((int)blockIdx.x - cs.tile[cs.n]) * (CW * 64) + tid;
    if (e < ce.size[j]) {
      const int row = (int)(e % ce.nr[j]), b = (int)(e / ce.nr[j]);
      ce.out[j][e] = ce.FL[j][fibre_left_row(row % ce.rl[j], row / ce.rl[j]) + b];
    }
    return;
  }
  int j = 0;
  while (j + 1 < cs.n && (int)blockIdx.x >= cs.tile[j + 1]) ++j;
  const int m = cs.m[j], r = cs.r[j], rl = ce.rl[j];
  const int row0 = ((int)blockIdx.x - cs.tile[j]) * 16;
  const int nst = (r + 3) / 4;
  const int lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* sa = lds;
  double* sb = lds + 64 * nst;
  double* F = ce.out[j];
  const double* FL = ce.FL[j];
  for (int e = tid; e < 64 * nst; e += CW * 64) {
    const int ii = e & 15, q = e >> 4;
    const int i = row0 + ii;
    double v = 0.0;
    if (i < m && q < r) {
      v = FL[fibre_left_row(i % rl, i / rl) + q];
      F[i + (int64_t)q * m] = v;
    }
    sa[(q >> 2) * 64 + (q & 3) * 16 + ii] = v;
    sb[e] = 0.0;
  }
  __syncthreads();
  const int ntile = (r + 15) / 16;
  for (int it = 0; it * CW < ntile; ++it) {   // T = F W (W upper: rows q <= p of column p)
    const int jt = snake_tile(it, wv, CW);
    if (jt >= ntile) continue;
    const int p = jt * 16 + li;
    const dbl4 t = mfma_tile_lds(sa, 0, min(nst, 4 * jt + 4), cs.W[j] + FT, p, r, lane);
    if (p < r)
#pragma unroll
      for (int v = 0; v < 4; ++v) sb[(p >> 2) * 64 + (p & 3) * 16 + lk + 4 * v] = t[v];
  }
  __syncthreads();
  double* C = cs.C[j];
  for (int it = 0; it * CW < ntile; ++it) {   // C = T Li (Li lower: rows q >= p of column p)
    const int jt = snake_tile(it, wv, CW);
    if (jt >= ntile) continue;
    const int p = jt * 16 + li;
    const dbl4 c = mfma_tile_lds(sb, 4 * jt, nst, cs.Li[j] + FT, p, r, lane);
    if (p < r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + lk + 4 * v;
        if (row < m) C[row + (int64_t)p * m] = c[v];
      }
  }
}

inline int nblk(int64_t n, int bs) { return (int)std::max<int64_t>(1, (n + bs - 1) / bs); }

// A few host threads for the update steps' sample draws (Floyd's algorithm
// over millions of positions, the host's largest cost per step), which run
// for all staged steps and both variants at once.  run(n, f) calls f(i) for
// i < n on the workers and the calling thread and returns when all are
// done.  Workers spin briefly for the next batch (batches come every few
// hundred microseconds during a cross), then sleep.  One batch at a time.
class DrawPool {
 public:
  static DrawPool& get() {
    static DrawPool pool;
    return pool;
  }
  template <class F>
  void run(int n, F&& f) {
    if (n <= 1 || th_.empty()) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    std::lock_guard<std::mutex> one(batch_);
    Task t{[](void* c, int i) { (*static_cast<F*>(c))(i); }, &f, n, 0};
    done_.store(0, std::memory_order_relaxed);
    {
      std::lock_guard<std::mutex> g(m_);
      t.gen = (uint32_t)(gen_.load(std::memory_order_relaxed) + 1);
      ticket_.store((uint64_t)t.gen << 32, std::memory_order_relaxed);
      task_ = t;
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work(t);
    while (done_.load(std::memory_order_acquire) < n) std::this_thread::yield();
  }
  ~DrawPool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }

 private:
  struct Task {
    void (*call)(void*, int) = nullptr;
    void* ctx = nullptr;
    int n = 0;
    uint32_t gen = 0;
  };
  DrawPool() {
    const unsigned hw = std::thread::hardware_concurrency();
    const int nw = (int)std::min<unsigned>(hw > 1 ? hw - 1 : 0, 7);
    for (int i = 0; i < nw; ++i) th_.emplace_back([this] { loop(); });
  }
  // takes indices of batch t.gen while any are left: the ticket holds the
  // batch's generation (high half) and its next index (low half), and an
  // index is taken only by a compare-exchange that sees t's generation, so a
  // worker late for a finished batch takes nothing from the next one
  void work(const Task& t) {
    for (;;) {
      uint64_t cur = ticket_.load(std::memory_order_acquire);
      if ((uint32_t)(cur >> 32) != t.gen || (int)(uint32_t)cur >= t.n) return;
      if (!ticket_.compare_exchange_weak(cur, cur + 1, std::memory_order_acq_rel)) continue;
      t.call(t.ctx, (int)(uint32_t)cur);
      done_.fetch_add(1, std::memory_order_acq_rel);
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      // spin for about a millisecond for the next batch, then sleep
      const auto t0 = std::chrono::steady_clock::now();
      while (gen_.load(std::memory_order_acquire) == seen &&
             std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(1))
        std::this_thread::yield();
      Task t;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return gen_.load(std::memory_order_acquire) != seen; });
        seen = gen_.load(std::memory_order_acquire);
        if (stop_) return;
        t = task_;
      }
      work(t);
    }
  }
  std::vector<std::thread> th_;
  std::mutex m_, batch_;
  std::condition_variable cv_;
  std::atomic<uint64_t> gen_{0}, ticket_{0};
  std::atomic<int> done_{0};
  Task task_;
  bool stop_ = false;
};


// Key of a multi-index (node indices < 32, at most 8 dims: 5 bits each).
inline uint64_t mkey(const int32_t* e, int len) {
  uint64_t k = (uint64_t)len;
  for (int i = 0; i < len; ++i) k = (k << 5) | (uint64_t)e[i];
  return k;
}

// Host mailbox of the update steps: mapped, coherent pinned memory that the
// finishing kernel writes (the step's result, then its sequence number) and
// the host polls, so a step costs no copy and no stream synchronisation.
// Mapped, coherent pinned host memory the finishing kernels publish to: one
// result slot and one sequence word per super-core k, so a whole sweep can
// be queued and its results read in order.
struct HostMail {
  StepRes* res = nullptr;        // host addresses, MAXD slots each
  uint32_t* seq = nullptr;
  StepRes* dres = nullptr;       // device addresses of the same memory
  uint32_t* dseq = nullptr;
  void* p = nullptr;
  HostMail() = default;
  HostMail(const HostMail&) = delete;
  HostMail& operator=(const HostMail&) = delete;
  ~HostMail() { if (p) (void)hipHostFree(p); }
  tt_status alloc() {
    if (p) return TTK_OK;
    const size_t bytes = MAXD * sizeof(StepRes) + MAXD * sizeof(uint32_t) + 64;
    if (hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(TTK_ERR_OOM, "pinned host allocation of %zu bytes failed", bytes);
    }
    std::memset(p, 0, bytes);
    void* dp = nullptr;
    TTK_HIP(hipHostGetDevicePointer(&dp, p, 0));
    res = static_cast<StepRes*>(p);
    seq = reinterpret_cast<uint32_t*>(static_cast<char*>(p) + MAXD * sizeof(StepRes));
    dres = static_cast<StepRes*>(dp);
    dseq = reinterpret_cast<uint32_t*>(static_cast<char*>(dp) + MAXD * sizeof(StepRes));
    return TTK_OK;
  }
};

class Cross {
 public:
  Cross(const tt_kernel_params* p, const Grid& g, const KSpec& ks, hipStream_t st)
      : P_(*p), g_(g), ks_(ks), st_(st), N_(g.D) {}

  tt_status run(CrossOut* out);

 private:
  // index sets: L_[k] = I^{<=k} (r_k rows of k ints), R_[k] = I^{>k} (rows of N-k ints)
  std::vector<std::vector<int32_t>> L_, R_;
  int rank(int k) const {
    if (k == 0 || k == N_) return 1;
    return (int)(L_[k].size() / (size_t)k);
  }

  tt_status upload_sets(int k_left, int k_right, int16_t* dl, int16_t* dr);
  tt_status init_sets();
  // One update step of a sweep (Alg 5) as the host prepares it.  Step k of a
  // sweep depends on the earlier steps only through whether step k - 1 added
  // a pivot, so every step is prepared at the start of the sweep in both of
  // its variants (v = 1: step k - 1 added) and the kernels read the variant
  // that step k - 1's finishing kernel selects; the whole sweep is queued in
  // one go and the host reads the results afterwards.
  struct HostStep {
    int k = 0, sweep = 0, rk = 0, nvar = 1, var = 0, cols = 0;
    int rows[2] = {0, 0}, ns[2] = {0, 0}, bit[2] = {0, 0};
    std::vector<int64_t> lin[2];        // samples (linear positions), generation order
    std::vector<int32_t> hi[2];         // the variant's pivot rows/columns and sample rows/columns
    const StepDesc* desc = nullptr;     // device, two entries
    const int32_t* sel = nullptr;       // device: the entry the kernels read
    int16_t* left = nullptr;            // device I^{<=k-1}, spare row after rank(k-1) rows
    uint32_t seq = 0;                   // mailbox sequence number of its finishing kernel
  };
  HostStep hs_[MAXD];
  DBuf d_sel_;   // int32 [MAXD + 1]: variant selector of step k at k (k >= 2); 0 stays 0
  int max_rank() const { return std::min(P_.max_rank > 0 ? P_.max_rank : MAXR, MAXR); }
  // An upper bound of r_j: the rank cap, and the number of distinct index
  // tuples on either side (I^{<=j} holds j-tuples, I^{>j} (N-j)-tuples).
  int rank_cap(int j) const {
    if (j == 0 || j == N_) return 1;
    int64_t a = 1, b = 1;
    for (int i = 0; i < j && a < MAXR; ++i) a *= g_.n[i];
    for (int i = j; i < N_ && b < MAXR; ++i) b *= g_.n[i];
    return (int)std::min<int64_t>({(int64_t)max_rank(), a, b});
  }
  tt_status reserve_buffers();
  tt_status prepare_step(HostStep& h, int k, int sweep, bool speculate);
  void draw_variant(HostStep& h, int v);   // the samples of variant v (thread-safe across steps and variants)
  tt_status upload_step(HostStep& h);
  tt_status enqueue_front(const HostStep& h);
  tt_status enqueue_finish(HostStep& h, const HostStep* next);
  tt_status collect(const HostStep& h, tt_kernel_decision* rec);
  tt_status stage_steps(int sweep, int k0, int k1);
  tt_status enqueue_first_half();
  tt_status run_sweep(int sweep, bool staged, bool queued, std::vector<tt_kernel_decision>* log, int* added,
                      bool* next_staged);
  int first_half() const { return N_ / 2; }   // steps 1..first_half() are staged first
  tt_status test_launch(int j0, int j1, bool last);
  bool test_queued_ = false;   // the sweep queued its stopping test already
  uint32_t test_seq_ = 0;      // mailbox sequence number of the queued test
  tt_status stage_core(int k);
  CoreEval ce_{};
  int ce_next_ = 1;   // stopping-test staging: the next core to stage
  tt_status refine_cores();
  tt_status init_inverses();
  void pivot_positions(int k, std::vector<int32_t>* I, std::vector<int32_t>* J);
  std::vector<int32_t> pls_[MAXD], pli_[MAXD], prf_[MAXD], prt_[MAXD];   // pivot (s, i_k), (i_{k+1}, t)
  tt_status solve_right(int k, int m, const double* F, double* C);
  tt_status sampled_error(double* err, bool queue_next = false);
  Addr fibre_addr(int k) const;   // F_k, k = 1..N
  Addr super_addr(int k) const;   // super-core k, k = 1..N-1
  // Working buffers that follow the growing ranks: grown by at least half
  // their size at a time, so that the (synchronising) reallocations are few.
  tt_status ensure(DBuf& b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return TTK_OK;
    return b.alloc(std::max(bytes, b.bytes + b.bytes / 2));
  }
  tt_status sync() { TTK_HIP(hipStreamSynchronize(st_)); return TTK_OK; }

  tt_kernel_params P_;
  const Grid& g_;
  KSpec ks_;
  hipStream_t st_;
  int N_;
  int64_t evals_ = 0;
  double min_margin_ = 1.0;

  // device buffers
  DBuf d_res_, d_R_, d_x_;
  DBuf d_test_idx_, d_test_val_, d_core_[MAXD], d_cint_[MAXD], d_P_, d_err_, d_ref_;
  // factors Li, W of P_k per k (MAXR x MAXR, leading dimension MAXR), max
  // |entry| of P_k and the factors' status
  DBuf d_li_[MAXD], d_w_[MAXD], d_luaux_, d_E_;
  // the fibre cache of core k (1-based): FL_k and FR_k, n_k x MAXR x MAXR each
  DBuf d_fl_[MAXD], d_fr_[MAXD];
  double* fl(int k) { return d_fl_[k - 1].as<double>(); }
  double* fr(int k) { return d_fr_[k - 1].as<double>(); }
  tt_status fill_fibres();
  double* luamax(int k) { return d_luaux_.as<double>() + k; }
  int32_t* luinfo(int k) { return reinterpret_cast<int32_t*>(d_luaux_.as<double>() + MAXD) + k; }
  HostMail mail_;
  uint32_t mail_seq_ = 0;
  tt_status wait_mail(int slot, uint32_t seq);
  // upload arenas: host pinned + device mirror, bump-allocated, flushed with
  // one copy before the kernels that read them.  Arenas 0 and 1 hold the
  // update steps of even and odd sweeps, arena 2 everything else, so a sweep
  // can be staged while the previous one and its stopping test still read
  // their own uploads.  An arena is reset only once its readers have drained.
  static constexpr int NAR = 3, AR_OTHER = 2;
  HBuf ar_h_[NAR];
  DBuf ar_d_[NAR];
  size_t ar_off_[NAR] = {0, 0, 0}, ar_flushed_[NAR] = {0, 0, 0}, ar_cap_ = 0;
  int ar_ = AR_OTHER;   // the arena in use
  const int16_t* cur_left_ = nullptr;
  const int16_t* cur_right_ = nullptr;
  tt_status arena_init(size_t bytes) {
    ar_cap_ = bytes;
    for (int i = 0; i < NAR; ++i) {
      TTK_TRY(ar_h_[i].alloc(bytes));
      TTK_TRY(ar_d_[i].alloc(bytes));
    }
    return TTK_OK;
  }
  void arena_reset() { ar_off_[ar_] = ar_flushed_[ar_] = 0; }   // once its readers have drained
  template <class T>
  tt_status arena_push(const T* src, size_t n, const T** dev) {
    const size_t at = (ar_off_[ar_] + 255) & ~(size_t)255;
    const size_t bytes = n * sizeof(T);
    if (at + bytes > ar_cap_) return fail(TTK_ERR_OOM, "cross upload arena too small (%zu bytes)", ar_cap_);
    if (bytes) std::memcpy(ar_h_[ar_].as<char>() + at, src, bytes);
    *dev = reinterpret_cast<const T*>(ar_d_[ar_].as<char>() + at);
    ar_off_[ar_] = at + bytes;
    return TTK_OK;
  }
  tt_status arena_flush() {
    const size_t off = ar_off_[ar_], done = ar_flushed_[ar_];
    if (off > done)
      TTK_HIP(hipMemcpyAsync(ar_d_[ar_].as<char>() + done, ar_h_[ar_].as<char>() + done, off - done,
                             hipMemcpyHostToDevice, st_));
    ar_flushed_[ar_] = off;
    return TTK_OK;
  }
  int n_test_ = 0;
  double test_max_ = 0.0;
  // the test points grouped by their index at each core: perm (N x n_test,
  // int32) and the 16-point tiles of every group (offsets per core)
  DBuf d_tperm_, d_ttiles_, d_tv_[2], d_ones_;
  int ttile_off_[MAXD + 1] = {0};
  double init_max_cond_ = 0.0;
};

Addr Cross::fibre_addr(int k) const {
  Addr a{};
  a.left = cur_left_;
  a.right = cur_right_;
  a.rl = rank(k - 1);
  a.lk = k - 1;
  a.rr = rank(k);
  a.lr = N_ - k;
  a.nmid = 1;
  a.nm0 = g_.n[k - 1];
  a.nm1 = 1;
  return a;
}

Addr Cross::super_addr(int k) const {
  Addr a{};
  a.left = cur_left_;
  a.right = cur_right_;
  a.rl = rank(k - 1);
  a.lk = k - 1;
  a.rr = rank(k + 1);
  a.lr = N_ - k - 1;
  a.nmid = 2;
  a.nm0 = g_.n[k - 1];
  a.nm1 = g_.n[k];
  return a;
}

// Stage I^{<=k_left} and I^{>k_right} (int16, row-major) in the upload arena;
// cur_left_ / cur_right_ point at their device copies after the next flush.
tt_status Cross::upload_sets(int k_left, int k_right, int16_t*, int16_t*) {
  const size_t nl = (k_left == 0) ? 0 : L_[k_left].size();
  const size_t nr = (k_right == N_) ? 0 : R_[k_right].size();
  std::vector<int16_t> tmp(nl + nr + 1);
  for (size_t i = 0; i < nl; ++i) tmp[i] = (int16_t)L_[k_left][i];
  for (size_t i = 0; i < nr; ++i) tmp[nl + i] = (int16_t)R_[k_right][i];
  TTK_TRY(arena_push(tmp.data(), nl + 1, &cur_left_));
  TTK_TRY(arena_push(tmp.data() + nl, nr + 1, &cur_right_));
  return TTK_OK;
}

tt_status Cross::init_sets() {
  const int N = N_;
  SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_INIT);
  L_.assign(N + 1, {});
  R_.assign(N + 1, {});
  if (P_.init_card == 1) {
    std::vector<int32_t> q(N);
    for (int j = 0; j < N; ++j) q[j] = (int32_t)g.below((uint64_t)g_.n[j]);
    for (int k = 1; k < N; ++k) {
      L_[k].assign(q.begin(), q.begin() + k);
      R_[k].assign(q.begin() + k, q.end());
    }
    return TTK_OK;
  }
  std::vector<int32_t> q1(N), q2(N);
  for (int j = 0; j < N; ++j) q1[j] = (int32_t)g.below((uint64_t)g_.n[j]);
  for (int j = 0; j < N; ++j) q2[j] = (int32_t)g.below((uint64_t)g_.n[j]);
  // the probes run in one launch (k_init_sets); the host reads the snapshots
  const int max_it = P_.init_max_it > 0 ? P_.init_max_it : 10;
  InitArgs ia{};
  ia.N = N;
  ia.max_it = max_it;
  for (int j = 0; j < N; ++j) {
    ia.n[j] = g_.n[j];
    ia.q1[j] = q1[j];
    ia.q2[j] = q2[j];
  }
  const int nsnap = 2 * max_it;
  DBuf d_snap;
  TTK_TRY(d_snap.alloc((size_t)nsnap * (INIT_SNAP * sizeof(int32_t) + sizeof(double))));
  int32_t* dsnap = d_snap.as<int32_t>();
  double* dmc = reinterpret_cast<double*>(dsnap + (size_t)nsnap * INIT_SNAP);
  with_dims(ks_, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_init_sets<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>), dim3(1),
                       dim3(1024), 0, st_, ks_, ia, dsnap, dmc);
  });
  TTK_HIP(hipGetLastError());
  std::vector<int32_t> hsnap((size_t)nsnap * INIT_SNAP);
  std::vector<double> hmc(nsnap);
  TTK_HIP(hipMemcpyAsync(hsnap.data(), dsnap, hsnap.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st_));
  TTK_HIP(hipMemcpyAsync(hmc.data(), dmc, hmc.size() * sizeof(double), hipMemcpyDeviceToHost, st_));
  TTK_TRY(sync());
  // the kernel entries the probes evaluated: (rows of I^{<=k-1}) n_k (rows of I^{>k}) each
  for (int it = 0; it < max_it; ++it) {
    for (int k = 1; k < N; ++k) evals_ += (int64_t)(k == 1 ? 1 : 2) * g_.n[k - 1] * 2;
    for (int k = N; k >= 2; --k) evals_ += (int64_t)2 * g_.n[k - 1] * (k == N ? 1 : 2);
  }
  struct Snap { std::vector<std::vector<int32_t>> L, R; double maxc; };
  std::vector<Snap> snaps(nsnap);
  for (int sI = 0; sI < nsnap; ++sI) {
    const int32_t* o = hsnap.data() + (size_t)sI * INIT_SNAP;
    Snap& sp = snaps[sI];
    sp.L.assign(N + 1, {});
    sp.R.assign(N + 1, {});
    for (int k = 1; k < N; ++k) {
      sp.L[k].assign(o + k * 2 * MAXD, o + k * 2 * MAXD + 2 * k);
      sp.R[k].assign(o + (MAXD + k) * 2 * MAXD, o + (MAXD + k) * 2 * MAXD + 2 * (N - k));
    }
    sp.maxc = hmc[sI];
  }
  // smallest maximum condition number, earliest within a relative band
  double best = INFINITY;
  for (auto& s : snaps) best = std::min(best, s.maxc);
  size_t pick = 0;
  for (size_t i = 0; i < snaps.size(); ++i) {
    if (std::isinf(best) ? std::isinf(snaps[i].maxc) : (snaps[i].maxc <= best * (1.0 + 1e-12))) {
      pick = i;
      break;
    }
  }
  L_ = snaps[pick].L;
  R_ = snaps[pick].R;
  init_max_cond_ = snaps[pick].maxc;
  return TTK_OK;
}


// Positions of the pivots (I^{<=k} as rows, I^{>k} as columns) in the
// unfolding of super-core k: row s + i_k r_{k-1}, column i_{k+1} + t n_{k+1}.
// Each pivot of core k is kept as (s, i_k) and (i_{k+1}, t) with s its row in
// I^{<=k-1} and t its row in I^{>k+1}; both sets only grow at the end, so the
// pairs stay valid and only the multipliers r_{k-1}, n_{k+1} enter the positions.
void Cross::pivot_positions(int k, std::vector<int32_t>* I, std::vector<int32_t>* J) {
  const int N = N_;
  const int rl = rank(k - 1), rr = rank(k + 1), rk = rank(k);
  const int nk1 = g_.n[k];
  if ((int)pls_[k].size() != rk) {   // first use: look the pivots up in the neighbouring sets
    std::unordered_map<uint64_t, int> lpos, rpos;
    for (int s = 0; s < rl; ++s) lpos[mkey(k > 1 ? &L_[k - 1][(size_t)s * (k - 1)] : nullptr, k - 1)] = s;
    for (int t = 0; t < rr; ++t)
      rpos[mkey(k + 1 < N ? &R_[k + 1][(size_t)t * (N - k - 1)] : nullptr, N - k - 1)] = t;
    pls_[k].resize(rk);
    pli_[k].resize(rk);
    prf_[k].resize(rk);
    prt_[k].resize(rk);
    for (int q = 0; q < rk; ++q) {
      const int32_t* e = &L_[k][(size_t)q * k];
      pls_[k][q] = lpos.at(mkey(e, k - 1));
      pli_[k][q] = e[k - 1];
      const int32_t* f = &R_[k][(size_t)q * (N - k)];
      prf_[k][q] = f[0];
      prt_[k][q] = rpos.at(mkey(f + 1, N - k - 1));
    }
  }
  I->resize(rk);
  J->resize(rk);
  for (int q = 0; q < rk; ++q) {
    (*I)[q] = pls_[k][q] + pli_[k][q] * rl;
    (*J)[q] = prf_[k][q] + prt_[k][q] * nk1;
  }
}

// P_k^{-1} of the initial index sets (ranks 1 or 2), with P_k gathered from
// the fibre cache (F_k at the pivot rows).
tt_status Cross::init_inverses() {
  TTK_TRY(d_P_.alloc(16 * sizeof(double)));
  // every core's pivot positions in one upload
  arena_reset();
  const int32_t* dIk[MAXD] = {nullptr};
  for (int k = 1; k < N_; ++k) {
    std::vector<int32_t> I, J;
    pivot_positions(k, &I, &J);
    TTK_TRY(arena_push(I.data(), I.size(), &dIk[k]));
  }
  TTK_TRY(arena_flush());
  for (int k = 1; k < N_; ++k) {
    const int rk = rank(k);
    TTK_TRY(d_li_[k].alloc((size_t)2 * MAXR * MAXR * sizeof(double)));   // Li, then Li^T
    TTK_TRY(d_w_[k].alloc((size_t)2 * MAXR * MAXR * sizeof(double)));    // W, then W^T
    hipLaunchKernelGGL(k_gather_pivots, dim3(1), dim3(64), 0, st_, (const double*)fl(k), dIk[k], rank(k - 1), rk,
                       d_P_.as<double>());
    hipLaunchKernelGGL(k_ldu_init, dim3(1), dim3(64), 0, st_, d_P_.as<double>(), rk, d_li_[k].as<double>(),
                       d_w_[k].as<double>(), luamax(k), luinfo(k));
  }
  TTK_HIP(hipGetLastError());
  return sync();   // the arena's host side is reused after this
}

// The fibre cores of the initial index sets into the fibre cache (every
// later entry is added by the update steps).
tt_status Cross::fill_fibres() {
  arena_reset();
  Addr ak[MAXD + 1];
  for (int k = 1; k <= N_; ++k) {
    TTK_TRY(upload_sets(k - 1, k, nullptr, nullptr));
    ak[k] = fibre_addr(k);
  }
  TTK_TRY(arena_flush());
  for (int k = 1; k <= N_; ++k) {
    const int rows = rank(k - 1) * g_.n[k - 1], rk = rank(k);
    with_dims(ks_, [&](auto dd, auto tt, auto gg) {
      hipLaunchKernelGGL((k_fill_fibre<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
                         dim3(nblk((int64_t)rows * rk, 16)), dim3(256), 0, st_, ks_, ak[k], rows, rk, fl(k), fr(k));
    });
    evals_ += (int64_t)rows * rk;
  }
  TTK_HIP(hipGetLastError());
  return sync();   // the arena's host side is reused after this
}

// The buffers whose size follows the ranks (the stopping test's fibres and
// cores, the products of solve_right and refine_cores), reserved once at the
// largest size the rank bounds allow: growing one later would reallocate it,
// and a reallocation waits for all queued work, which would drain a queued
// sweep.
tt_status Cross::reserve_buffers() {
  size_t cmax = 16;
  for (int k = 1; k <= N_; ++k) {
    const size_t c = (size_t)rank_cap(k - 1) * g_.n[k - 1] * rank_cap(k) * sizeof(double);
    TTK_TRY(ensure(d_core_[k - 1], c));
    if (k < N_) TTK_TRY(ensure(d_cint_[k - 1], c));
    cmax = std::max(cmax, c);
  }
  TTK_TRY(ensure(d_E_, cmax));
  TTK_TRY(ensure(d_ref_, 2 * cmax));
  for (int k = 1; k <= N_; ++k) {
    const size_t c = (size_t)g_.n[k - 1] * MAXR * MAXR * sizeof(double);
    TTK_TRY(ensure(d_fl_[k - 1], c));
    TTK_TRY(ensure(d_fr_[k - 1], c));
  }
  TTK_TRY(ensure(d_P_, (size_t)MAXR * MAXR * sizeof(double)));
  return TTK_OK;
}

// C = F P_k^{-1} = (F W) Li for F (m x r, leading dimension m).
tt_status Cross::solve_right(int k, int m, const double* F, double* C) {
  const int r = rank(k);
  TTK_TRY(ensure(d_E_, (size_t)m * r * sizeof(double)));
  double* T = d_E_.as<double>();
  gemm64(0, 0, m, r, r, 1.0, F, m, d_w_[k].as<double>(), MAXR, 0.0, T, m, st_);
  gemm64(0, 0, m, r, r, 1.0, T, m, d_li_[k].as<double>(), MAXR, 0.0, C, m, st_);
  return TTK_OK;
}

// Polls mailbox slot `slot` until its finishing kernel has published
// sequence number seq.  Every 1024 polls the stream is queried: an error is
// returned as such, and a stream that has drained without publishing is an
// error too (so a failed launch cannot leave the host polling forever).
tt_status Cross::wait_mail(int slot, uint32_t seq) {
  const uint32_t* w = mail_.seq + slot;
  for (uint64_t spin = 1;; ++spin) {
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return TTK_OK;
    if ((spin & 1023) == 0) {
      const hipError_t e = hipStreamQuery(st_);
      if (e == hipSuccess) {
        if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return TTK_OK;
        return fail(TTK_ERR_HIP, "cross: the step kernel finished without publishing its result");
      }
      if (e != hipErrorNotReady) return fail(TTK_ERR_HIP, "cross: %s", hipGetErrorString(e));
    }
  }
}

// Stages step k of the sweep in the upload arena: the left set I^{<=k-1}
// (with a spare row for the one step k - 1 may add, which its finishing
// kernel writes), the right set I^{>k+1}, and per variant the pivot
// positions, the samples (drawn from the step's own keyed stream, so both
// variants draw as the oracle does for its r_{k-1}) and the descriptor.
// Host set-up of step k before its draws: its shape and variant count (and
// the pivots' positions in the neighbouring sets, looked up on first use).
tt_status Cross::prepare_step(HostStep& h, int k, int sweep, bool speculate) {
  const int rl0 = rank(k - 1), rr = rank(k + 1), rk = rank(k);
  const int nk = g_.n[k - 1], nk1 = g_.n[k];
  if ((int)pls_[k].size() != rk) {
    std::vector<int32_t> I, J;
    pivot_positions(k, &I, &J);
  }
  h.k = k;
  h.sweep = sweep;
  h.rk = rk;
  h.var = 0;
  h.nvar = (speculate && rl0 < max_rank()) ? 2 : 1;
  h.cols = nk1 * rr;
  if ((int64_t)(rl0 + h.nvar - 1) * nk > (int64_t)MAXR * MAXN || h.cols > MAXR * MAXN)
    return fail(TTK_ERR_ARG, "cross: super-core %d unfolding exceeds %d rows or columns", k, MAXR * MAXN);
  return TTK_OK;
}

// The samples of variant v of step h (Floyd's algorithm on the step's keyed
// stream) and the rows and columns the step's kernels read: the pivots'
// (pivot row, pivot column) positions, then the samples' rows and columns.
// Reads only host sets that no step changes while the draws run.
void Cross::draw_variant(HostStep& h, int v) {
  const int k = h.k, rk = h.rk;
  const int rl = rank(k - 1) + v, rows = rl * g_.n[k - 1], nk1 = g_.n[k];
  SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_UPDATE, (uint64_t)h.sweep, (uint64_t)k);
  const int ns = std::max(rows, h.cols);
  h.lin[v] = g.floyd_unsorted((int64_t)rows * h.cols, ns);
  h.bit[v] = g.bit();
  h.rows[v] = rows;
  h.ns[v] = ns;
  std::vector<int32_t>& hi = h.hi[v];
  hi.resize((size_t)2 * rk + 2 * (size_t)ns);
  for (int q = 0; q < rk; ++q) {
    hi[q] = pls_[k][q] + pli_[k][q] * rl;
    hi[rk + q] = prf_[k][q] + prt_[k][q] * nk1;
  }
  for (int i = 0; i < ns; ++i) {
    hi[2 * rk + i] = (int32_t)(h.lin[v][i] / h.cols);
    hi[2 * rk + ns + i] = (int32_t)(h.lin[v][i] % h.cols);
  }
}

// Uploads step k's sets, samples and descriptors to the current arena.
tt_status Cross::upload_step(HostStep& h) {
  const int N = N_, k = h.k, rk = h.rk, rr = rank(k + 1), nk = g_.n[k - 1], nk1 = g_.n[k];
  {
    const size_t lk = (size_t)k - 1, nl = (k == 1) ? 0 : L_[k - 1].size();
    const size_t nr = (k + 1 == N) ? 0 : R_[k + 1].size();
    std::vector<int16_t> tmp(nl + lk + 1 + nr + 1, 0);
    for (size_t i = 0; i < nl; ++i) tmp[i] = (int16_t)L_[k - 1][i];
    for (size_t i = 0; i < nr; ++i) tmp[nl + lk + 1 + i] = (int16_t)R_[k + 1][i];
    const int16_t* dl = nullptr;
    TTK_TRY(arena_push(tmp.data(), nl + lk + 1, &dl));
    TTK_TRY(arena_push(tmp.data() + nl + lk + 1, nr + 1, &cur_right_));
    h.left = const_cast<int16_t*>(dl);
  }
  StepDesc hd[2];
  for (int v = 0; v < h.nvar; ++v) {
    const int ns = h.ns[v];
    const int32_t* dI = nullptr;
    TTK_TRY(arena_push(h.hi[v].data(), h.hi[v].size(), &dI));
    StepDesc& sd = hd[v];
    sd.a.left = h.left;
    sd.a.right = cur_right_;
    sd.a.rl = rank(k - 1) + v;
    sd.a.lk = k - 1;
    sd.a.rr = rr;
    sd.a.lr = N - k - 1;
    sd.a.nmid = 2;
    sd.a.nm0 = nk;
    sd.a.nm1 = nk1;
    sd.I = dI;
    sd.J = dI + rk;
    sd.srow = dI + 2 * rk;
    sd.scol = dI + 2 * rk + ns;
    sd.rows = h.rows[v];
    sd.cols = h.cols;
    sd.ns = ns;
    sd.bit = h.bit[v];
  }
  if (h.nvar == 1) hd[1] = hd[0];   // a selector of 1 cannot occur, but stays in bounds
  TTK_TRY(arena_push(hd, 2, &h.desc));
  h.sel = d_sel_.as<int32_t>() + (k > 1 ? k : 0);   // (steps after the first select their variant)
  return TTK_OK;
}

// The step's sample and search stages (four launches), sized for the larger
// variant; blocks past the selected variant's extent do no work.
tt_status Cross::enqueue_front(const HostStep& h) {
  const int k = h.k, rk = h.rk;
  int nsm = 0, nqm = 0;
  for (int v = 0; v < h.nvar; ++v) {
    nsm = std::max(nsm, h.ns[v]);
    nqm = std::max(nqm, h.bit[v] ? h.cols : h.rows[v]);
  }
  StepRes* dres = d_res_.as<StepRes>();
  const double* Li = d_li_[k].as<double>();
  const double* W = d_w_[k].as<double>();
  double* R = d_R_.as<double>();
  double* x = d_x_.as<double>();
  with_dims(ks_, [&](auto dd, auto tt, auto gg) {
    constexpr int D_ = decltype(dd)::value, T_ = decltype(tt)::value;
    constexpr bool G_ = decltype(gg)::value;
    hipLaunchKernelGGL((k_sample_resid<D_, T_, G_>), dim3(nblk(nsm, SPB)), dim3(SW * 64), sample_lds(rk), st_, ks_,
                       h.desc, h.sel, rk, Li, W, (const double*)fl(k), (const double*)fr(k + 1), R, dres->s_slot);
    hipLaunchKernelGGL((k_sample_select<D_, T_, G_>), dim3(1), dim3(1024), 0, st_, ks_, h.desc, h.sel,
                       (const double*)R, (const double*)luamax(k), dres, rk, Li, W, (const double*)fl(k),
                       (const double*)fr(k + 1), x);
    hipLaunchKernelGGL((k_search<D_, T_, G_>), dim3(nblk(nqm, QE)), dim3(256), 0, st_, ks_, h.desc, h.sel,
                       (const StepRes*)dres, (const double*)x, rk, fl(k), fr(k), fl(k + 1), fr(k + 1), R,
                       dres->q_slot);
  });
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// The step's decision, the border of P_k's factors, the next step's
// variant selector and spare left row, and the mailbox.
tt_status Cross::enqueue_finish(HostStep& h, const HostStep* next) {
  const int k = h.k;
  h.seq = ++mail_seq_;
  int32_t* sel_next = next ? const_cast<int32_t*>(next->sel) : nullptr;
  int16_t* next_left = (next && next->nvar == 2) ? next->left : nullptr;
  StepRes* dres = d_res_.as<StepRes>();
  hipLaunchKernelGGL(k_finish_step, dim3(1), dim3(FB), 0, st_, h.desc, h.sel, (const double*)d_R_.as<double>(), dres,
                     h.rk, max_rank(), d_li_[k].as<double>(), d_w_[k].as<double>(), luamax(k), luinfo(k),
                     mail_.dres + k, mail_.dseq + k, h.seq, sel_next, next_left, h.rk, (const double*)fl(k),
                     (const double*)fl(k + 1), (const double*)fr(k + 1), (const double*)d_x_.as<double>());
  // the fibre the search did not evaluate, when the pivot is added
  int nf = 0;
  for (int v = 0; v < h.nvar; ++v) nf = std::max(nf, h.bit[v] ? h.rows[v] : h.cols);
  with_dims(ks_, [&](auto dd, auto tt, auto gg) {
    hipLaunchKernelGGL((k_add_fibre<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
                       dim3(nblk(nf, 16)), dim3(256), 0, st_, ks_, h.desc, h.sel, (const StepRes*)dres, h.rk, fl(k),
                       fr(k), fl(k + 1), fr(k + 1));
  });
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// Waits for the step's result and applies it to the host index sets.
tt_status Cross::collect(const HostStep& h, tt_kernel_decision* rec) {
  const int N = N_, k = h.k, v = h.var, rk = h.rk;
  const int rl = rank(k - 1), nk = g_.n[k - 1], nk1 = g_.n[k];
  if (v >= h.nvar || rl * nk != h.rows[v] || rank(k) != rk)
    return fail(TTK_ERR_HIP, "cross: step %d ran on a variant its predecessor did not select", k);
  TTK_TRY(wait_mail(k, h.seq));
  StepRes r;
  std::memcpy(&r, mail_.res + k, offsetof(StepRes, s_slot));
  if (r.info != 0)
    return fail(TTK_ERR_SINGULAR_CROSS, "cross: intersection matrix of super-core %d singular (sweep %d)", k,
                h.sweep);
  const int rows = h.rows[v], cols = h.cols, ns = h.ns[v], bit = h.bit[v];
  evals_ += ns + (bit ? cols : rows);   // the samples and the searched fibre (the rest is cached)
  rec->sweep = h.sweep;
  rec->k = k;
  rec->rank_before = rk;
  rec->sample_pos = h.lin[v][r.s_pos];
  rec->bit = bit;
  rec->pivot_row = r.pivot_row;
  rec->pivot_col = r.pivot_col;
  rec->added = r.added;
  rec->sample_max = r.s_max;
  rec->sample_margin = r.s_margin;
  rec->pivot_abs = r.pivot_abs;
  rec->search_margin = r.q_margin;
  rec->tau = r.q_tau;
  if (r.s_max > 0) min_margin_ = std::min(min_margin_, r.s_margin);
  if (r.q_max > 0) min_margin_ = std::min(min_margin_, r.q_margin);
  if (r.added) {
    evals_ += bit ? rows : cols;                  // the other fibre through the pivot
    const int l = r.pivot_row, t = r.pivot_col;   // the factors of P_k are already bordered
    const int s = l % rl, ik = l / rl;
    pls_[k].push_back(s);
    pli_[k].push_back(ik);
    prf_[k].push_back(t % nk1);
    prt_[k].push_back(t / nk1);
    if (k > 1) L_[k].insert(L_[k].end(), L_[k - 1].begin() + (size_t)s * (k - 1),
                            L_[k - 1].begin() + (size_t)(s + 1) * (k - 1));
    L_[k].push_back(ik);
    const int i1 = t % nk1, tt = t / nk1;
    R_[k].push_back(i1);
    if (k + 1 < N)
      R_[k].insert(R_[k].end(), R_[k + 1].begin() + (size_t)tt * (N - k - 1),
                   R_[k + 1].begin() + (size_t)(tt + 1) * (N - k - 1));
  }
  return TTK_OK;
}

// Stages steps k0..k1-1 of a sweep in the sweep's arena (sweep & 1, reset
// at k0 = 1) and uploads them in one copy.
tt_status Cross::stage_steps(int sweep, int k0, int k1) {
  struct Use {   // the sweep's arena while staging, the other arena again on every return
    int& a;
    Use(int& x, int v) : a(x) { a = v; }
    ~Use() { a = AR_OTHER; }
  } use(ar_, sweep & 1);
  if (k0 == 1) arena_reset();   // its last readers, two sweeps back, have drained
  // the steps' shapes, then every step's and variant's draws at once on the
  // host pool, then the uploads in order
  int tk[2 * MAXD], tv[2 * MAXD], nt = 0;
  for (int k = k0; k < k1; ++k) {
    TTK_TRY(prepare_step(hs_[k], k, sweep, k > 1));
    for (int v = 0; v < hs_[k].nvar; ++v) {
      tk[nt] = k;
      tv[nt++] = v;
    }
  }
  DrawPool::get().run(nt, [&](int i) { draw_variant(hs_[tk[i]], tv[i]); });
  for (int k = k0; k < k1; ++k) TTK_TRY(upload_step(hs_[k]));
  return arena_flush();
}

// Queues the staged first half of a sweep (steps 1..h, without the finish
// of step h, whose successor is queued with the second half).
tt_status Cross::enqueue_first_half() {
  const int h = first_half();
  for (int k = 1; k <= h; ++k) {
    TTK_TRY(enqueue_front(hs_[k]));
    if (k < h) TTK_TRY(enqueue_finish(hs_[k], &hs_[k + 1]));
  }
  return TTK_OK;
}

// One sweep (Alg 6, k = 1..N-1).  Every step is staged already (while the
// previous sweep's stopping test ran) when `staged`; otherwise the first half
// is staged, queued, and the second half staged while it runs.  All steps
// are queued without waiting, then the results are read in order and applied
// to the host sets; the stopping test is queued in two parts behind them,
// and the whole next sweep is staged while it runs (*next_staged; discarded
// if the test ends the cross).  (`queued`: the first half is on the stream
// already, behind the previous sweep's stopping test.)
tt_status Cross::run_sweep(int sweep, bool staged, bool queued, std::vector<tt_kernel_decision>* log, int* added,
                           bool* next_staged) {
  const int N = N_, h = first_half();
  if (!queued) {
    if (!staged) TTK_TRY(stage_steps(sweep, 1, h + 1));
    TTK_TRY(enqueue_first_half());
  }
  if (!staged) TTK_TRY(stage_steps(sweep, h + 1, N));
  for (int k = h; k < N; ++k) {
    if (k > h) TTK_TRY(enqueue_front(hs_[k]));
    TTK_TRY(enqueue_finish(hs_[k], k + 1 < N ? &hs_[k + 1] : nullptr));
  }
  *added = 0;
  *next_staged = false;
  const int max_sweeps = P_.max_sweeps > 0 ? P_.max_sweeps : 200;
  for (int k = 1; k < N; ++k) {
    tt_kernel_decision rec{};
    TTK_TRY(collect(hs_[k], &rec));
    log->push_back(rec);
    *added += rec.added;
    if (k + 1 < N) hs_[k + 1].var = rec.added;
    TTK_TRY(stage_core(k));   // core k's sets are final for this sweep's test
    if (k + 1 == N) TTK_TRY(stage_core(N));
    // the stopping test, queued in two parts behind the steps still running
    if (k == N - 2) TTK_TRY(test_launch(0, N - 2, false));
    if (k == N - 1) {
      TTK_TRY(test_launch(N >= 3 ? N - 2 : 0, N - 1, true));
      test_queued_ = true;
      // the whole next sweep, staged while the test runs (every step of this
      // sweep is collected, so its records are free)
      if (sweep + 1 < max_sweeps) {
        TTK_TRY(stage_steps(sweep + 1, 1, N));
        *next_staged = true;
      }
    }
  }
  if (*added == 0) *next_staged = false;
  return TTK_OK;
}

// Cores of the cross interpolant, column-major C_k ((r_{k-1} n_k) x r_k):
// C_k = F_k P_k^{-1} with the kept factors, C_D = F_D.  One upload of the
// index sets, one launch for every fibre, one for every product.
// Stages the fibre of core k for the next stopping test (its index sets
// uploaded, its entry in the CoreEval table): cores are staged in order, and
// core k may be staged as soon as its sets are final (after step k of a
// sweep), so a sweep stages them while its last steps still run.
tt_status Cross::stage_core(int k) {
  if (k != ce_next_) return fail(TTK_ERR_HIP, "cross: core %d staged out of order", k);
  if (k == 1) {
    arena_reset();   // the other-uses arena: its last reader, the previous test, has drained
    ce_ = CoreEval{};
    ce_.n = N_;
  }
  const int r0 = rank(k - 1), r1 = rank(k), n = g_.n[k - 1];
  const int m = r0 * n;
  TTK_TRY(ensure(d_core_[k - 1], (size_t)m * r1 * sizeof(double)));
  ce_.FL[k - 1] = fl(k);
  ce_.out[k - 1] = d_core_[k - 1].as<double>();
  ce_.nr[k - 1] = m;
  ce_.rl[k - 1] = r0;
  ce_.size[k - 1] = (int64_t)m * r1;
  ce_next_ = k + 1;
  return TTK_OK;
}

// The stopping test for cores j0 + 1 .. j1 (C_{j+1} = F_{j+1} P_{j+1}^{-1}
// by k_eval_solve, then their grouped products with the running test rows,
// V_{j+1} = V_j C_{j+1}); with `last`, also the last core (C_D = F_D, copied
// by the same launch), the error fold and its publication to mailbox slot
// 0.  A sweep queues cores 1 .. N-2 as soon as its step N-2 is collected
// (their ranks and factors are final), while step N-1 still runs, and the
// rest after step N-1, so the device waits only for the last part's launch.
tt_status Cross::test_launch(int j0, int j1, bool last) {
  const int N = N_;
  for (int k = ce_next_; k <= (last ? N : j1); ++k) TTK_TRY(stage_core(k));
  if (last) ce_next_ = 1;   // the next test stages from core 1 again
  if (j0 == 0) TTK_TRY(arena_flush());
  CoreSolve cs{};
  CoreEval ce{};
  cs.n = j1 - j0;
  int nt = 0, rmax = 1;
  for (int j = j0; j < j1; ++j) {
    const int k = j + 1, q = j - j0;
    const int m = rank(k - 1) * g_.n[k - 1], r = rank(k);
    TTK_TRY(ensure(d_cint_[j], (size_t)m * r * sizeof(double)));
    cs.F[q] = d_core_[j].as<double>();
    cs.C[q] = d_cint_[j].as<double>();
    cs.Li[q] = d_li_[k].as<double>();
    cs.W[q] = d_w_[k].as<double>();
    cs.m[q] = m;
    cs.r[q] = r;
    cs.tile[q] = nt;
    nt += nblk(m, 16);
    rmax = std::max(rmax, r);
    ce.FL[q] = ce_.FL[j];
    ce.out[q] = ce_.out[j];
    ce.nr[q] = ce_.nr[j];
    ce.rl[q] = ce_.rl[j];
    ce.size[q] = ce_.size[j];
  }
  cs.tile[cs.n] = nt;
  ce.n = cs.n;
  int nlast = 0;
  if (last) {   // the last fibre, copied by the blocks past the solve tiles
    const int q = cs.n;
    ce.FL[q] = ce_.FL[N - 1];
    ce.out[q] = ce_.out[N - 1];
    ce.nr[q] = ce_.nr[N - 1];
    ce.rl[q] = ce_.rl[N - 1];
    ce.size[q] = ce_.size[N - 1];
    ce.n = q + 1;
    nlast = nblk(ce_.size[N - 1], CW * 64);
  }
  if (nt + nlast > 0)
    hipLaunchKernelGGL(k_eval_solve, dim3(nt + nlast), dim3(CW * 64), solve_lds(rmax), st_, ce, cs,
                       d_err_.as<double>());
  const TTTile* tiles = reinterpret_cast<const TTTile*>(d_ttiles_.as<int32_t>());
  const int jend = last ? N : j1;
  for (int j = j0; j < jend; ++j) {
    const double* vin = j == 0 ? d_ones_.as<double>() : d_tv_[(j - 1) & 1].as<double>();
    const double* C = j < N - 1 ? d_cint_[j].as<double>() : d_core_[N - 1].as<double>();
    const int nt_j = ttile_off_[j + 1] - ttile_off_[j];
    hipLaunchKernelGGL(k_tt_core, dim3(nt_j), dim3(TTW * 64), 0, st_, C, rank(j), rank(j + 1), rank(j) * g_.n[j], vin,
                       j == 0 ? 1 : MAXR, d_tv_[j & 1].as<double>(), MAXR,
                       (const int32_t*)d_tperm_.as<int32_t>() + (size_t)j * n_test_, tiles + ttile_off_[j]);
  }
  if (last) {
    hipLaunchKernelGGL(k_tt_err, dim3((n_test_ + 255) / 256), dim3(256), 0, st_,
                       (const double*)d_tv_[(N - 1) & 1].as<double>(), MAXR, (const double*)d_test_val_.as<double>(),
                       n_test_, d_err_.as<double>());
    test_seq_ = ++mail_seq_;
    hipLaunchKernelGGL(k_test_publish, dim3(1), dim3(64), 0, st_, (const double*)d_err_.as<double>(),
                       (const int32_t*)luinfo(0), N_, mail_.dres, mail_.dseq, test_seq_);
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

// One step of residual refinement of the returned cores C_k = F_k P_k^{-1}
// (k < D): with P_k = F_k(I, :) (the rows at the pivot positions),
// C_k <- C_k + (F_k - C_k P_k) W Li.  The factors are exact up to the growth
// of elimination in pivot order, which can amplify rounding where P_k is
// very ill-conditioned; the correction brings C_k to the accuracy of a
// pivoted solve at the cost of three products per core.
tt_status Cross::refine_cores() {
  const int N = N_;
  // every core's pivot rows in one upload
  arena_reset();
  const int32_t* dIk[MAXD] = {nullptr};
  for (int k = 1; k < N; ++k) {
    std::vector<int32_t> I, J;
    pivot_positions(k, &I, &J);
    TTK_TRY(arena_push(I.data(), I.size(), &dIk[k]));
  }
  TTK_TRY(arena_flush());
  for (int k = 1; k < N; ++k) {
    const int r0 = rank(k - 1), r = rank(k), n = g_.n[k - 1];
    const int m = r0 * n;
    const int32_t* dI = dIk[k];
    const double* F = d_core_[k - 1].as<double>();
    double* C = d_cint_[k - 1].as<double>();
    TTK_TRY(ensure(d_P_, (size_t)r * r * sizeof(double)));
    TTK_TRY(ensure(d_ref_, (size_t)2 * m * r * sizeof(double)));
    double* P = d_P_.as<double>();
    double* E = d_ref_.as<double>();
    double* T = E + (size_t)m * r;
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk((int64_t)r * r, 256)), dim3(256), 0, st_, F, m, dI, r, r, P);
    TTK_HIP(hipMemcpyAsync(E, F, (size_t)m * r * sizeof(double), hipMemcpyDeviceToDevice, st_));
    gemm64(0, 0, m, r, r, -1.0, C, m, P, r, 1.0, E, m, st_);
    gemm64(0, 0, m, r, r, 1.0, E, m, d_w_[k].as<double>(), MAXR, 0.0, T, m, st_);
    gemm64(0, 0, m, r, r, 1.0, T, m, d_li_[k].as<double>(), MAXR, 1.0, C, m, st_);
  }
  TTK_HIP(hipGetLastError());
  return sync();   // the arena's host side is reused after this
}

// The stopping test: the cores by the interpolation formula, the TT at the
// test points against the stored values, and the result read from mailbox
// slot 0 (the update steps use slots 1..N-1).  With `queue_next`, the next
// sweep's staged first half is queued behind the test before its result is
// read, so the device does not wait for the host's decision; if the test
// ends the cross those steps are never collected.  They change nothing the
// result depends on: the returned cores are the test's, and bordering P_k
// only appends a row and a column beyond the kept rank to its factors.
tt_status Cross::sampled_error(double* err, bool queue_next) {
  if (!test_queued_) TTK_TRY(test_launch(0, N_ - 1, true));
  test_queued_ = false;
  if (queue_next) TTK_TRY(enqueue_first_half());
  TTK_TRY(wait_mail(0, test_seq_));
  StepRes r;
  std::memcpy(&r, mail_.res, offsetof(StepRes, s_slot));
  if (r.info != 0) {
    // which P_k: read the flags (rare; a failure path)
    std::vector<int32_t> info(MAXD, 0);
    TTK_HIP(hipMemcpyAsync(info.data(), luinfo(0), MAXD * sizeof(int32_t), hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
    for (int k = 1; k < N_; ++k)
      if (info[k] != 0) return fail(TTK_ERR_SINGULAR_CROSS, "cross: P_%d singular in the interpolation formula", k);
    return fail(TTK_ERR_SINGULAR_CROSS, "cross: an intersection matrix is singular");
  }
  *err = test_max_ > 0 ? r.s_max / test_max_ : r.s_max;
  return TTK_OK;
}

tt_status Cross::run(CrossOut* out) {
  const int N = N_;
  TTK_TRY(arena_init((size_t)4 << 20));
  TTK_TRY(d_luaux_.alloc(MAXD * (sizeof(double) + sizeof(int32_t))));
  fill_zero(d_luaux_.p, MAXD * (sizeof(double) + sizeof(int32_t)), st_);
  TTK_TRY(init_sets());
  TTK_TRY(reserve_buffers());
  TTK_TRY(fill_fibres());
  TTK_TRY(init_inverses());
  // fixed test multi-indices of the stopping rule
  int nmax = 0;
  for (int j = 0; j < N; ++j) nmax = std::max(nmax, g_.n[j]);
  n_test_ = P_.n_test > 0 ? P_.n_test : std::max(1000, 20 * N * nmax);
  {
    SplitMix64 g = SplitMix64::keyed(P_.seed, RNG_TAG_TEST);
    std::vector<int16_t> idx((size_t)n_test_ * N);
    for (int p = 0; p < n_test_; ++p)
      for (int j = 0; j < N; ++j) idx[(size_t)p * N + j] = (int16_t)g.below((uint64_t)g_.n[j]);
    {   // the points grouped by their index at each core, in tiles of at most 16
      std::vector<int32_t> perm((size_t)N * n_test_);
      std::vector<TTTile> tl;
      for (int k = 0; k < N; ++k) {
        ttile_off_[k] = (int)tl.size();
        std::vector<int> cnt(g_.n[k] + 1, 0);
        for (int p = 0; p < n_test_; ++p) cnt[idx[(size_t)p * N + k] + 1]++;
        for (int i = 0; i < g_.n[k]; ++i) cnt[i + 1] += cnt[i];
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        for (int p = 0; p < n_test_; ++p) perm[(size_t)k * n_test_ + pos[idx[(size_t)p * N + k]]++] = p;
        for (int i = 0; i < g_.n[k]; ++i)
          for (int o = cnt[i]; o < cnt[i + 1]; o += 16) tl.push_back(TTTile{i, o, std::min(16, cnt[i + 1] - o), 0});
      }
      ttile_off_[N] = (int)tl.size();
      TTK_TRY(d_tperm_.alloc(perm.size() * sizeof(int32_t)));
      TTK_TRY(d_ttiles_.alloc(std::max<size_t>(tl.size(), 1) * sizeof(TTTile)));
      TTK_HIP(hipMemcpyAsync(d_tperm_.p, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, st_));
      TTK_HIP(hipMemcpyAsync(d_ttiles_.p, tl.data(), tl.size() * sizeof(TTTile), hipMemcpyHostToDevice, st_));
      for (int b = 0; b < 2; ++b) TTK_TRY(d_tv_[b].alloc((size_t)n_test_ * MAXR * sizeof(double)));
      TTK_TRY(d_ones_.alloc((size_t)n_test_ * sizeof(double)));
      hipLaunchKernelGGL(k_fill1, dim3((n_test_ + 255) / 256), dim3(256), 0, st_, d_ones_.as<double>(), n_test_);
      TTK_TRY(sync());   // (the host vectors are released at the end of this block)
    }
    TTK_TRY(d_test_idx_.alloc(idx.size() * sizeof(int16_t)));
    TTK_TRY(d_test_val_.alloc((size_t)n_test_ * sizeof(double)));
    TTK_TRY(d_err_.alloc(TEST_SLOTS * sizeof(double)));
    TTK_HIP(hipMemcpyAsync(d_test_idx_.p, idx.data(), idx.size() * sizeof(int16_t), hipMemcpyHostToDevice, st_));
    eval_multi16(ks_, d_test_idx_.as<int16_t>(), n_test_, d_test_val_.as<double>(), st_);
    evals_ += n_test_;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st_, d_test_val_.as<double>(), n_test_,
                       (const double*)nullptr, 0, (const double*)nullptr, 0, (const double*)nullptr, 0,
                       (const double*)nullptr, d_err_.as<double>());
    TTK_HIP(hipMemcpyAsync(&test_max_, d_err_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
    TTK_TRY(sync());
  }
  // the sample stage stages up to 2 x 64 x MAXR / 4 doubles of LDS per block
  if (sample_lds(MAXR) > 48 * 1024) {
    hipError_t e = hipSuccess;
    with_dims(ks_, [&](auto dd, auto tt, auto gg) {
      e = hipFuncSetAttribute(
          reinterpret_cast<const void*>(
              &k_sample_resid<decltype(dd)::value, decltype(tt)::value, (bool)decltype(gg)::value>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sample_lds(MAXR));
    });
    TTK_HIP(e);
  }
  if (solve_lds(MAXR) > 48 * 1024)
    TTK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval_solve),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)solve_lds(MAXR)));
  TTK_TRY(mail_.alloc());
  TTK_TRY(d_x_.alloc(2 * MAXR * sizeof(double)));   // the search stage's P^{-1} u and its intermediate
  // the residuals of either stage: at most max(rows, cols) <= MAXR x MAXN
  // entries, allocated once so that no queued step ever sees it move
  TTK_TRY(d_R_.alloc((size_t)MAXR * MAXN * sizeof(double)));
  TTK_TRY(d_sel_.alloc((MAXD + 1) * sizeof(int32_t)));
  fill_zero(d_sel_.p, (MAXD + 1) * sizeof(int32_t), st_);
  // step state: the fold slots and the sample-stage scale start at zero
  TTK_TRY(d_res_.alloc(sizeof(StepRes)));
  fill_zero(d_res_.p, sizeof(StepRes), st_);
  double err = 0.0;
  TTK_TRY(sampled_error(&err));
  int sweep = 0;
  const int max_sweeps = P_.max_sweeps > 0 ? P_.max_sweeps : 200;
  bool staged = false, queued = false;
  while (err > P_.tol && sweep < max_sweeps) {
    int added = 0;
    bool next = false;
    TTK_TRY(run_sweep(sweep, staged, queued, &out->log, &added, &next));
    ++sweep;
    staged = next;
    // the next sweep starts behind the test unless nothing more can run
    queued = staged && added > 0 && sweep < max_sweeps;
    TTK_TRY(sampled_error(&err, queued));
    if (added == 0) break;
  }
  // the cores of the last stopping test, refined, are the result (C_k in
  // d_cint_, C_D in d_core_)
  TTK_TRY(refine_cores());
  out->ranks.assign(N + 1, 1);
  for (int k = 0; k <= N; ++k) out->ranks[k] = rank(k);
  out->cores.clear();
  out->cores.resize(N);
  for (int k = 1; k <= N; ++k) {
    const int r0 = rank(k - 1), r1 = rank(k), n = g_.n[k - 1];
    const size_t cnt = (size_t)r0 * n * r1;
    // column-major C_k ((r0 n) x r1) is the little-endian core layout itself;
    // the cores stay on the device, in buffers of their own size
    TTK_TRY(out->cores[k - 1].alloc(std::max<size_t>(cnt, 1) * sizeof(double)));
    const DBuf& src = (k == N) ? d_core_[k - 1] : d_cint_[k - 1];
    TTK_HIP(hipMemcpyAsync(out->cores[k - 1].p, src.p, cnt * sizeof(double), hipMemcpyDeviceToDevice, st_));
  }
  TTK_TRY(sync());
  out->left.assign(N + 1, {});
  out->right.assign(N + 1, {});
  for (int k = 1; k < N; ++k) { out->left[k] = L_[k]; out->right[k] = R_[k]; }
  out->sweeps = sweep;
  out->error = err;
  out->converged = err <= P_.tol;
  out->init_max_cond = init_max_cond_;
  out->min_margin = min_margin_;
  out->evals = evals_;
  return TTK_OK;
}

}  // namespace

tt_status run_cross(const tt_kernel_params* p, const Grid& g, const KSpec& ks, hipStream_t st, CrossOut* out) {
  if (g.D < 2) return fail(TTK_ERR_ARG, "cross needs at least two dimensions");
  Cross c(p, g, ks, st);
  const tt_status s = c.run(out);
  // a failed run may leave update steps queued on the stream; they finish
  // before the buffers they use are released
  if (s != TTK_OK && s != TTK_WARN_NOT_CONVERGED) (void)hipStreamSynchronize(st);
  return s;
}

}  // namespace ttk
