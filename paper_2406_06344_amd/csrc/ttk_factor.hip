// Phase 3 of the offline stage (Algorithm 2): the factor matrices
//     S <- U_1 G_1^{2},   S <- (U_i face-split S) G_i^{2},  i = 2..d
// and the mirrored chain for T, evaluated point by point without forming
// U_i: row p of (U_i face-split S) times G_i^{2} is
//     out[p, b] = sum_{a, k} S[p, a] q_k(x_{p,i}) G_i[a, k, b].
// Here the cores are in the Chebyshev coefficient basis (a DCT along mode 2
// of the nodal cores, Section 2.4's regrouping of the basis sum), so q_k is
// T_k(t(x)), generated per point by the three-term recurrence in double
// precision and rounded once.
//
// Each stage is a GEMM whose left operand A[p, a + k r_in] = S[p, a] T_k(t_p)
// is produced on the fly: a workgroup owns TP points, keeps their running
// rows S in LDS, and forms the next rows 64 columns at a time with a 4 x 4
// register tile per thread.  Target cores are passed transposed so the
// target chain (which runs from G_D down to G_{d+dt+1}) uses the same code.
#include "ttk_internal.h"

namespace ttk {

namespace {

constexpr int FC_THREADS = 256;

struct StageArgs {
  const void* G2[3];
  int r_in[3], r_out[3], n[3], coord[3];
  double lo[3], hi[3];
  int nst;
  int rmax;   // max over stages of r_out (and r_in)
};

template <class T, int TP>
__global__ void __launch_bounds__(FC_THREADS) k_factor(StageArgs sa, const T* P, int64_t ldp, int64_t npts, T* out,
                                                       int ldo) {
  extern __shared__ unsigned char smem_raw[];
  T* sTk = reinterpret_cast<T*>(smem_raw);              // TP x MAXN
  T* s0 = sTk + TP * MAXN;                              // TP x rmax
  T* s1 = s0 + (size_t)TP * sa.rmax;                    // TP x rmax
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * TP;
  // micro-tile: 16 x 16 thread grid -> TP/16 points x 4 columns per thread
  constexpr int PPT = TP / 16;
  const int tp = tid / 16, tb = tid % 16;
  T* sin = s0;
  T* sout = s1;
  if (tid < TP) sin[tid * sa.rmax] = (T)1;   // r_0 = 1
  for (int st = 0; st < sa.nst; ++st) {
    const int rin = sa.r_in[st], rout = sa.r_out[st], n = sa.n[st];
    const T* G = static_cast<const T*>(sa.G2[st]);
    // Chebyshev values of this stage's coordinate
    if (tid < TP) {
      const int64_t p = p0 + tid;
      const double x = (p < npts) ? (double)P[(int64_t)sa.coord[st] * ldp + p] : 0.5 * (sa.lo[st] + sa.hi[st]);
      const double t = (2.0 * x - (sa.lo[st] + sa.hi[st])) / (sa.lo[st] - sa.hi[st]);
      double tkm = 1.0, tk = t;
      sTk[tid * MAXN + 0] = (T)1;
      if (n > 1) sTk[tid * MAXN + 1] = (T)t;
      for (int k = 2; k < n; ++k) {
        const double tn = 2.0 * t * tk - tkm;
        tkm = tk;
        tk = tn;
        sTk[tid * MAXN + k] = (T)tn;
      }
    }
    __syncthreads();
    const int K = rin * n;
    for (int b0 = 0; b0 < rout; b0 += 64) {
      T acc[PPT][4];
#pragma unroll
      for (int i = 0; i < PPT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
      const int bc = b0 + tb * 4;
      for (int kk = 0; kk < K; ++kk) {
        const int a = kk % rin, k = kk / rin;
        T bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = (bc + j < rout) ? G[(int64_t)kk * rout + bc + j] : (T)0;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          const int pl = tp * PPT + i;
          const T av = sin[pl * sa.rmax + a] * sTk[pl * MAXN + k];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += av * bv[j];
        }
      }
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int pl = tp * PPT + i;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (bc + j < rout) sout[pl * sa.rmax + bc + j] = acc[i][j];
      }
    }
    __syncthreads();
    T* tmp = sin;
    sin = sout;
    sout = tmp;
  }
  const int rfin = sa.r_out[sa.nst - 1];
  for (int e = tid; e < TP * rfin; e += FC_THREADS) {
    const int pl = e / rfin, b = e % rfin;
    const int64_t p = p0 + pl;
    if (p < npts) out[p * ldo + b] = sin[pl * sa.rmax + b];
  }
}

// ---------------------------------------------------------------- MFMA path
// The same contraction on the matrix cores (float32 in, float32 accumulate):
// v_mfma_f32_16x16x4f32, whose 64 lanes hold A[i][k] at lane i + 16 k,
// B[k][j] at lane j + 16 k and D[4 (l / 16) + v][l % 16] in register v.
// A workgroup of 4 waves owns 64 points (16 per wave) and walks the
// contraction index kk = a + k r_in in slabs of 64 rows of G^{2}, staged in
// LDS; the A operand s[p, a] T_k(t_p) is formed per lane from LDS.  Output
// columns go in passes of at most 128, each as wide as its stage needs
// (r_out rounded up to 16), so no MFMA work is spent on padding beyond that.
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int MF_P = 64;     // points per workgroup
constexpr int MF_KS = 64;    // rows of G^{2} per LDS slab
constexpr int MF_NC = 128;   // output columns per pass (8 tiles of 16)
// Slab row stride for running-row stride sld (> every rank): the widest pass
// rounded up to 32, plus 16, so it is 16 mod 32 banks and the two rows a
// half-wave reads in one K-step fall on disjoint banks.
__host__ __device__ inline int mfma_gld(int sld) {
  const int wc = min(MF_NC, 16 * ((sld - 1 + 15) / 16));
  return (wc + 31) / 32 * 32 + 16;
}
constexpr int MF_TLD = 33;   // row stride of the Chebyshev table

// The MFMA steps over one staged slab of G^{2} for NJ 16-column tiles.  The
// A operand of step s is s_in[p, a] T_k(t_p) at this lane's contraction index
// kk = kk0 + 4 s + kq = a + k r_in, zero past K (from clamped, always valid
// LDS indices, so no branch); the next step's A and B operands are read from
// LDS while the current step's MFMAs issue.
template <int NJ>
__device__ inline void slab_steps(const float* Gs, int gld, const float* srow, const float* trow, int lane, int kq,
                                  int kk0, int ck, int K, int rin, int n, f4 (&acc)[MF_NC / 16]) {
  const int nsteps = (ck + 3) >> 2;
  int kk = kk0 + kq;
  int a = kk % rin, k = kk / rin;
  const int da = 4 % rin, dk = 4 / rin;   // kk += 4 as (a, k) += (da, dk), then at most one wrap
  const float* g0 = Gs + kq * gld + (lane & 15);
  // operands of step s into (av, bv): A from the lane's point row and the
  // Chebyshev table (clamped indices, zero past K), B from the staged slab
  auto load = [&](int s, float& av, float (&bv)[NJ]) {
    const float x = srow[min(a, rin - 1)] * trow[min(k, n - 1)];
    av = kk < K ? x : 0.0f;
    const float* g = g0 + 4 * s * gld;
#pragma unroll
    for (int jb = 0; jb < NJ; ++jb) bv[jb] = g[16 * jb];
    kk += 4;
    a += da;
    k += dk;
    if (a >= rin) { a -= rin; ++k; }
  };
  auto issue = [&](float av, const float (&bv)[NJ]) {
#pragma unroll
    for (int jb = 0; jb < NJ; ++jb) acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[jb], acc[jb], 0, 0, 0);
  };
  // two operand sets in ping-pong: the loads of one step overlap the MFMAs of
  // the other, with no register copies
  float a0, a1, b0v[NJ], b1v[NJ];
  load(0, a0, b0v);
  int s = 0;
  for (; s + 1 < nsteps; s += 2) {
    load(s + 1, a1, b1v);
    issue(a0, b0v);
    if (s + 2 < nsteps) load(s + 2, a0, b0v);
    issue(a1, b1v);
  }
  if (s < nsteps) issue(a0, b0v);
}

// One tile of MF_P points of one chain.  P: coordinate j of point q at
// P[j * ldp + q]; points p0 .. p0 + MF_P - 1 of npts; rows written to out.
__device__ void mfma_tile(const StageArgs& sa, const float* P, int64_t ldp, int64_t npts, int64_t p0, float* out,
                          int ldo, int sld, float* smf) {
  float* sTk = smf;                                  // MF_P x MF_TLD
  float* s0 = sTk + MF_P * MF_TLD;                    // MF_P x sld
  float* s1 = s0 + MF_P * sld;                        // MF_P x sld
  float* Gs = s1 + MF_P * sld;                        // MF_KS x gld
  const int gld = mfma_gld(sld);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int pl = 16 * w + (lane & 15);                // this lane's point for the A operand
  const int kq = lane >> 4;                           // this lane's row within a K-step
  float* sin = s0;
  float* sout = s1;
  if (tid < MF_P) sin[tid * sld] = 1.0f;
  for (int st = 0; st < sa.nst; ++st) {
    const int rin = sa.r_in[st], rout = sa.r_out[st], n = sa.n[st];
    const float* G = static_cast<const float*>(sa.G2[st]);
    if (tid < MF_P) {
      const int64_t p = p0 + tid;
      const double x = (p < npts) ? (double)P[(int64_t)sa.coord[st] * ldp + p] : 0.5 * (sa.lo[st] + sa.hi[st]);
      const double t = (2.0 * x - (sa.lo[st] + sa.hi[st])) / (sa.lo[st] - sa.hi[st]);
      double tkm = 1.0, tk = t;
      sTk[tid * MF_TLD + 0] = 1.0f;
      if (n > 1) sTk[tid * MF_TLD + 1] = (float)t;
      for (int k = 2; k < n; ++k) {
        const double tn = 2.0 * t * tk - tkm;
        tkm = tk;
        tk = tn;
        sTk[tid * MF_TLD + k] = (float)tn;
      }
    }
    __syncthreads();
    const int K = rin * n;
    for (int b0 = 0; b0 < rout; b0 += MF_NC) {
      const int cb = min(MF_NC, rout - b0);
      const int nj = (cb + 15) >> 4;                 // 16-column tiles in this pass
      const int wc = nj * 16;                        // staged slab width
      f4 acc[MF_NC / 16];
#pragma unroll
      for (int jb = 0; jb < MF_NC / 16; ++jb) acc[jb] = f4{0.f, 0.f, 0.f, 0.f};
      // slab staging: thread t owns column t % 128 of rows t / 128 + 2 u; the
      // next slab is loaded into registers while the current one is used
      const int sc = tid & (MF_NC - 1), sr = tid >> 7;
      float pre[MF_KS / 2];
      auto load_slab = [&](int k0) {
        const int ckn = min(MF_KS, K - k0);
        const float* g = G + (size_t)(k0 + sr) * rout + b0 + sc;   // row k0 + sr of this pass
        const int stride = 2 * rout;
#pragma unroll
        for (int u = 0; u < MF_KS / 2; ++u)
          pre[u] = (sc < cb && sr + 2 * u < ckn) ? g[u * stride] : 0.0f;
      };
      load_slab(0);
      for (int kk0 = 0; kk0 < K; kk0 += MF_KS) {
        const int ck = min(MF_KS, K - kk0);
        __syncthreads();                               // the previous slab is consumed
        if (sc < wc)
#pragma unroll
          for (int u = 0; u < MF_KS / 2; ++u) Gs[(sr + 2 * u) * gld + sc] = pre[u];
        __syncthreads();
        if (kk0 + MF_KS < K) load_slab(kk0 + MF_KS);
        const float* srow = sin + pl * sld;
        const float* trow = sTk + pl * MF_TLD;
        switch (nj) {
          case 1: slab_steps<1>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 2: slab_steps<2>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 3: slab_steps<3>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 4: slab_steps<4>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 5: slab_steps<5>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 6: slab_steps<6>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          case 7: slab_steps<7>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
          default: slab_steps<8>(Gs, gld, srow, trow, lane, kq, kk0, ck, K, rin, n, acc); break;
        }
      }
      // D[4 (l / 16) + v][l % 16]: point 16 w + 4 (l / 16) + v, column b0 + 16 jb + l % 16
#pragma unroll
      for (int jb = 0; jb < MF_NC / 16; ++jb) {
        const int col = b0 + 16 * jb + (lane & 15);
        if (jb < nj && col < rout)
#pragma unroll
          for (int v = 0; v < 4; ++v) sout[(16 * w + 4 * kq + v) * sld + col] = acc[jb][v];
      }
    }
    __syncthreads();
    float* tmp = sin;
    sin = sout;
    sout = tmp;
  }
  const int rfin = sa.r_out[sa.nst - 1];
  for (int e = tid; e < MF_P * rfin; e += 256) {
    const int q = e / rfin, b = e % rfin;
    const int64_t p = p0 + q;
    if (p < npts) out[p * ldo + b] = sin[q * sld + b];
  }
  __syncthreads();                                     // LDS is reused by the next tile
}

__global__ void __launch_bounds__(256) k_factor_mfma(StageArgs sa, const float* P, int64_t npts, float* out, int ldo,
                                                     int sld) {
  extern __shared__ float smf[];
  mfma_tile(sa, P, npts, npts, (int64_t)blockIdx.x * MF_P, out, ldo, sld, smf);
}

// Phase 3 of many chains (one per box pair and side) in one persistent launch:
// tile t of the concatenated work list belongs to job j with
// prefix[j] <= t < prefix[j + 1]; workgroups stride over the tiles.
struct FacJob {
  StageArgs sa;
  const float* P;
  int64_t ldp, npts;
  float* out;
  int ldo;
};

__global__ void __launch_bounds__(256) k_factor_mfma_batch(const FacJob* jobs, const int64_t* prefix, int njobs,
                                                           int sld) {
  extern __shared__ float smf[];
  __shared__ FacJob job;
  __shared__ int cur;
  const int64_t total = prefix[njobs];
  if (threadIdx.x == 0) cur = -1;
  __syncthreads();
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    // job of tile t: the last j with prefix[j] <= t
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    if (lo != cur) {
      __syncthreads();
      if (threadIdx.x == 0) {
        job = jobs[lo];
        cur = lo;
      }
      __syncthreads();
    }
    mfma_tile(job.sa, job.P, job.ldp, job.npts, (t - prefix[lo]) * MF_P, job.out, job.ldo, sld, smf);
  }
}

// LDS row stride of the running rows: odd, so the 16 points a K-step reads
// fall on 16 distinct banks
inline int mfma_sld(int rmax) { return (rmax + 1) | 1; }

size_t mfma_lds_bytes(int rmax) {
  const int sld = mfma_sld(rmax);
  return sizeof(float) * ((size_t)MF_P * MF_TLD + 2 * (size_t)MF_P * sld + (size_t)MF_KS * mfma_gld(sld));
}

int lds_limit() {
  static int lim = -1;
  if (lim < 0) {
    int dev = 0, v = 64 * 1024;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 64 * 1024;
    (void)hipGetLastError();
    lim = v;
  }
  return lim;
}

tt_status launch_factor_mfma(const StageArgs& sa, const void* P, int64_t ldp, int64_t npts, void* out, int ldo,
                             hipStream_t st, bool* launched) {
  *launched = false;
  const size_t sh = mfma_lds_bytes(sa.rmax);
  if (sh > (size_t)lds_limit()) return TTK_OK;
  if (sh > 64 * 1024)
    TTK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_mfma),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  if (ldp == npts) {
    hipLaunchKernelGGL(k_factor_mfma, dim3((unsigned)((npts + MF_P - 1) / MF_P)), dim3(256), sh, st, sa,
                       static_cast<const float*>(P), npts, static_cast<float*>(out), ldo, mfma_sld(sa.rmax));
    TTK_HIP(hipGetLastError());
    *launched = true;
  }
  return TTK_OK;
}

template <class T, int TP>
tt_status launch_tile(const StageArgs& sa, const void* P, int64_t ldp, int64_t npts, void* out, int ldo, size_t sh,
                      hipStream_t st) {
  if (sh > 64 * 1024)
    TTK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor<T, TP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  hipLaunchKernelGGL((k_factor<T, TP>), dim3((unsigned)((npts + TP - 1) / TP)), dim3(FC_THREADS), sh, st, sa,
                     static_cast<const T*>(P), ldp, npts, static_cast<T*>(out), ldo);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

template <class T>
tt_status launch_factor(const StageArgs& sa, const void* P, int64_t ldp, int64_t npts, void* out, int ldo,
                        hipStream_t st) {
  const int lds = lds_limit();
  const size_t per_tp = (size_t)(MAXN + 2 * sa.rmax) * sizeof(T);
  // the largest point tile whose LDS footprint fits one workgroup
  if (per_tp * 64 <= (size_t)lds) return launch_tile<T, 64>(sa, P, ldp, npts, out, ldo, per_tp * 64, st);
  if (per_tp * 32 <= (size_t)lds) return launch_tile<T, 32>(sa, P, ldp, npts, out, ldo, per_tp * 32, st);
  if (per_tp * 16 <= (size_t)lds) return launch_tile<T, 16>(sa, P, ldp, npts, out, ldo, per_tp * 16, st);
  return fail(TTK_ERR_UNSUPPORTED, "Phase 3 tile for rank %d does not fit %d bytes of LDS", sa.rmax, lds);
}

StageArgs make_stage_args(const ChainStage* stages, int nstages) {
  StageArgs sa{};
  sa.nst = nstages;
  sa.rmax = 1;
  for (int i = 0; i < nstages; ++i) {
    sa.G2[i] = stages[i].G2;
    sa.r_in[i] = stages[i].r_in;
    sa.r_out[i] = stages[i].r_out;
    sa.n[i] = stages[i].n;
    sa.coord[i] = stages[i].coord;
    sa.lo[i] = stages[i].lo;
    sa.hi[i] = stages[i].hi;
    sa.rmax = std::max(sa.rmax, std::max(stages[i].r_in, stages[i].r_out));
  }
  return sa;
}

tt_status contract_one(int dtype, const StageArgs& sa, const void* P, int64_t ldp, int64_t npts, void* out, int ldo,
                       hipStream_t st) {
  if (npts <= 0) return TTK_OK;
  if (dtype == TTK_FP32) {
    // matrix cores when the LDS tiles fit the workgroup, register-tiled VALU otherwise
    bool launched = false;
    TTK_TRY(launch_factor_mfma(sa, P, ldp, npts, out, ldo, st, &launched));
    if (launched) return TTK_OK;
    return launch_factor<float>(sa, P, ldp, npts, out, ldo, st);
  }
  return launch_factor<double>(sa, P, ldp, npts, out, ldo, st);
}

}  // namespace

tt_status factor_contract(int dtype, const ChainStage* stages, int nstages, const void* P_soa, int64_t npts,
                          void* out, int ldo, hipStream_t st) {
  return contract_one(dtype, make_stage_args(stages, nstages), P_soa, npts, npts, out, ldo, st);
}

tt_status factor_contract_batch(int dtype, const FactorJob* jobs, int njobs, int grid, hipStream_t st,
                                FactorBatchPlan* plan) {
  if (njobs <= 0) return TTK_OK;
  int rmax = 1;
  for (int j = 0; j < njobs; ++j) {
    const StageArgs sa = make_stage_args(jobs[j].stages, jobs[j].nstages);
    rmax = std::max(rmax, sa.rmax);
  }
  const size_t sh = mfma_lds_bytes(rmax);
  if (dtype != TTK_FP32 || sh > (size_t)lds_limit()) {
    // one launch per job (double precision, or ranks beyond the MFMA tile)
    for (int j = 0; j < njobs; ++j)
      TTK_TRY(contract_one(dtype, make_stage_args(jobs[j].stages, jobs[j].nstages), jobs[j].P, jobs[j].ldp,
                           jobs[j].npts, jobs[j].out, jobs[j].ldo, st));
    plan->persistent = false;
    return TTK_OK;
  }
  // the work list: job descriptors and the prefix sum of their tile counts
  if (plan->njobs != njobs) {
    std::vector<FacJob> hj(njobs);
    std::vector<int64_t> pre(njobs + 1, 0);
    for (int j = 0; j < njobs; ++j) {
      hj[j].sa = make_stage_args(jobs[j].stages, jobs[j].nstages);
      hj[j].P = static_cast<const float*>(jobs[j].P);
      hj[j].ldp = jobs[j].ldp;
      hj[j].npts = jobs[j].npts;
      hj[j].out = static_cast<float*>(jobs[j].out);
      hj[j].ldo = jobs[j].ldo;
      pre[j + 1] = pre[j] + (jobs[j].npts + MF_P - 1) / MF_P;
    }
    TTK_TRY(plan->desc.alloc(sizeof(FacJob) * njobs));
    TTK_TRY(plan->prefix.alloc(sizeof(int64_t) * (njobs + 1)));
    TTK_HIP(hipMemcpyAsync(plan->desc.p, hj.data(), sizeof(FacJob) * njobs, hipMemcpyHostToDevice, st));
    TTK_HIP(hipMemcpyAsync(plan->prefix.p, pre.data(), sizeof(int64_t) * (njobs + 1), hipMemcpyHostToDevice, st));
    TTK_HIP(hipStreamSynchronize(st));   // host staging vectors go out of scope
    plan->njobs = njobs;
    plan->tiles = pre[njobs];
  }
  if (plan->tiles == 0) return TTK_OK;
  if (sh > 64 * 1024)
    TTK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_mfma_batch),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  const int64_t g = grid > 0 ? std::min<int64_t>(grid, plan->tiles) : plan->tiles;
  hipLaunchKernelGGL(k_factor_mfma_batch, dim3((unsigned)g), dim3(256), sh, st, plan->desc.as<const FacJob>(),
                     plan->prefix.as<const int64_t>(), njobs, mfma_sld(rmax));
  TTK_HIP(hipGetLastError());
  plan->persistent = true;
  return TTK_OK;
}

}  // namespace ttk
