// The two tall contractions of the batched apply and its backward pass
// (the low-rank form of Section 1, y_b = S H(theta_b) T^T x_b, and its
// adjoint) on the matrix cores, float32 in, float32 accumulate:
//     expand:  Y (N x B) = F Z,    F = S or T (N x r row-major), Z r x B
//     reduce:  W (r x B) = F^T X,  X N x B
// Both are dense (N x r) by (r x B) products with N ~ 10^6, r <= 128 and B
// in the thousands, so they are bound by the matrix cores (2 r flops per
// byte of X or Y).  v_mfma_f32_16x16x4f32: lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and D[4 (l / 16) + v][l % 16] in register v.
//
// expand: a wave owns 64 points and keeps their rows of F as A operands in
//   registers for the whole launch; the workgroup (4 waves, 256 points)
//   walks the thetas in blocks of 64, each block of Z fetched into LDS by
//   direct global->LDS loads while the previous block is multiplied, in two
//   halves of 32 thetas (half the accumulators live: three waves per SIMD).
//   Each K-step reads 2 B operands from LDS for 8 MFMAs.
//   Output: register v of a lane is 4 consecutive points of one column of
//   the column-major Y, stored as one 16-byte write.
// reduce: a workgroup owns 128 thetas and one chunk of the points; blocks of
//   64 points of X (column segments, 16-byte loads) and of F (contiguous
//   rows) go through LDS; each wave owns 32 thetas by all r.  The float32
//   MFMA sums of a 64-point block are folded into float64 accumulators, the
//   chunk's sums are written as float64 partials, and k_sum_chunks adds the
//   chunks in a fixed order (deterministic, no atomics).
#include "ttk_internal.h"

namespace ttk {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// ------------------------------------------------------------------ expand
constexpr int EX_PW = 64;             // points per wave
constexpr int EX_P = 4 * EX_PW;       // points per workgroup
constexpr int EX_TB = 64;             // thetas per staged block of Z

// LDS of the expand: two buffers of a Z block (EX_TB columns of r values, as
// they lie in memory) plus KP floats of padding, so K-step reads past r of
// the last column stay inside the buffer.
inline size_t expand_lds_floats(int r, int kp) { return (size_t)2 * (EX_TB * r + kp); }

// KS = K-steps = ceil(r / 4).  VEC: Y's columns are 16-byte aligned (ldy
// and the base a multiple of 4 floats), so a lane's 4 points go as one store.
// ACC: Y += F Z instead of Y = F Z (a K dimension above 128 in passes).
// Blocks of Z are fetched by direct global->LDS loads (4 bytes per lane,
// lane l to the wave's base + 4 l), double-buffered: the next block is in
// flight while this one is multiplied.  A operands past r are zero, so the
// padding reads (finite values: LDS starts zeroed, later blocks overwrite
// with Z) contribute nothing.
template <int KS, bool VEC, bool ACC>
__global__ void __launch_bounds__(256, 2) k_expand_mfma(const float* __restrict__ F, int ldf, int64_t N, int r,
                                                        const float* __restrict__ Z, int B, float* __restrict__ Y,
                                                        int64_t ldy, int bpw) {
  extern __shared__ float zsm[];
  constexpr int KP = 4 * KS;                     // r rounded up to 4
  const int stage = EX_TB * r + KP;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * EX_P + (int64_t)w * EX_PW;
  for (int e = tid; e < 2 * stage; e += 256) zsm[e] = 0.0f;
  // A operands: F[p0 + 16 s + i16, 4 t + kq], zero past N or r
  float af[4][KS];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t p = p0 + 16 * s + i16;
    const float* row = F + (p < N ? p : 0) * (int64_t)ldf;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int c = 4 * t + kq;
      af[s][t] = (p < N && c < r) ? row[c] : 0.0f;
    }
  }
  // this workgroup's theta blocks: bpw of them from blockIdx.y * bpw
  const int bfirst = blockIdx.y * bpw;
  const int nb = min(bpw, (B + EX_TB - 1) / EX_TB - bfirst);
  if (nb <= 0) return;                           // (whole workgroup: no barrier is skipped by part of it)
  auto issue = [&](int b0, float* buf) {
    const int total = min(EX_TB, B - b0) * r;    // the block's columns are contiguous in Z
    const float* zb = Z + (int64_t)b0 * r;
    for (int j = w; 64 * j < total; j += 4)
      if (64 * j + lane < total) __builtin_amdgcn_global_load_lds(zb + 64 * j + lane, buf + 64 * j, 4, 0, 0);
  };
  __syncthreads();                               // the zero fill is done before any load lands
  issue(bfirst * EX_TB, zsm);
  for (int ib = 0; ib < nb; ++ib) {
    const int b0 = (bfirst + ib) * EX_TB;
    const float* zs = zsm + (size_t)(ib & 1) * stage;
    __builtin_amdgcn_s_waitcnt(0);               // this wave's loads of block ib have landed
    __syncthreads();                             // everyone's; and block ib - 1 is consumed
    asm volatile("" ::: "memory");               // LDS reads below see the DMA writes
    if (ib + 1 < nb) issue(b0 + EX_TB, zsm + (size_t)((ib + 1) & 1) * stage);
    // the block's 64 thetas in two halves of 32 (half the accumulators live)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f4 acc[4][2];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[s][q] = f4{0.f, 0.f, 0.f, 0.f};
      // B[c][theta] = Z[c + (b0 + theta) r] = zs[theta r + c], read one
      // K-step ahead of its MFMAs (scheduling barriers keep the reads there)
      const float* zrow = zs + (32 * h + i16) * r + kq;
      float bz[2][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) bz[0][q] = zrow[16 * q * r];
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        if (t + 1 < KS)
#pragma unroll
          for (int q = 0; q < 2; ++q) bz[(t + 1) & 1][q] = zrow[16 * q * r + 4 * (t + 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int q = 0; q < 2; ++q) acc[s][q] = mfma4(af[s][t], bz[t & 1][q], acc[s][q]);
        __builtin_amdgcn_sched_barrier(0);
      }
      // D[4 kq + v][i16]: points p0 + 16 s + 4 kq + v, theta b0 + 32 h + 16 q + i16
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int th = b0 + 32 * h + 16 * q + i16;
        if (th >= B) continue;
        float* ycol = Y + (int64_t)th * ldy;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int64_t p = p0 + 16 * s + 4 * kq;
          if (VEC && p + 3 < N) {
            if (ACC) *reinterpret_cast<f4*>(ycol + p) += acc[s][q];
            else *reinterpret_cast<f4*>(ycol + p) = acc[s][q];
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (p + v < N) {
                if (ACC) ycol[p + v] += acc[s][q][v];
                else ycol[p + v] = acc[s][q][v];
              }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ reduce
constexpr int RD_P = 64;              // points per staged block
constexpr int RD_TB = 128;            // thetas per workgroup
constexpr int RD_XLD = RD_P + 4;      // LDS row stride of X (4 mod 32 banks): conflict-free B reads

// Row stride of the staged F block for CT 16-column tiles: 16 mod 32 banks,
// so the 4 rows of a K-step land on disjoint banks.
__host__ __device__ constexpr int rd_fld(int ct) { return (16 * ct) % 32 == 16 ? 16 * ct : 16 * ct + 16; }
template <int CT>
constexpr size_t reduce_lds_floats() { return (size_t)RD_TB * RD_XLD + (size_t)RD_P * rd_fld(CT); }

// part[chunk * r * B + b * r + c] = sum over the chunk's points p of
// F[p, c] X[p, b] for this workgroup's 128 thetas; r <= 16 CT.  VEC: X's
// columns are 16-byte aligned (ldx and the base a multiple of 4 floats).
template <int CT, bool VEC>
__global__ void __launch_bounds__(256, 2) k_reduce_mfma(const float* __restrict__ F, int ldf, int64_t N, int r,
                                                     const float* __restrict__ X, int64_t ldx, int B, int64_t chunk,
                                                     double* __restrict__ part) {
  extern __shared__ float rsm[];
  constexpr int FLD = rd_fld(CT);
  constexpr int FC = 16 * CT;                    // staged columns of F
  float* Xs = rsm;                               // [theta][point], RD_TB x RD_XLD
  float* Fs = rsm + RD_TB * RD_XLD;              // [point][column], RD_P x FLD
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int b0 = blockIdx.y * RD_TB;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = pbeg + chunk < N ? pbeg + chunk : N;
  double out[CT][2][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[ct][q][v] = 0.0;
  for (int64_t q0 = pbeg; q0 < pend; q0 += RD_P) {
    __syncthreads();                             // the previous block is consumed
    // X block: theta 16 u + tid / 16, points q0 + 4 (tid % 16) .. + 3
    {
      const int seg = tid & 15;
      const int64_t p = q0 + 4 * seg;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int th = 16 * u + (tid >> 4);
        const int bb = b0 + th;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (bb < B) {
          const float* xc = X + (int64_t)bb * ldx;
          if (VEC && p + 3 < pend) {
            v = *reinterpret_cast<const f4*>(xc + p);
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (p + k < pend) v[k] = xc[p + k];
          }
        }
        *reinterpret_cast<f4*>(Xs + th * RD_XLD + 4 * seg) = v;
      }
    }
    // F block: wave w takes rows w, w + 4, ..., lanes the columns
    {
#pragma unroll
      for (int u = 0; u < RD_P / 4; ++u) {
        const int pt = 4 * u + w;
        const int64_t p = q0 + pt;
        const float* row = F + (p < pend ? p : q0) * (int64_t)ldf;
#pragma unroll
        for (int h = 0; h < (FC + 63) / 64; ++h) {
          const int c = lane + 64 * h;
          if (c < FC) Fs[pt * FLD + c] = (p < pend && c < r) ? row[c] : 0.0f;
        }
      }
    }
    __syncthreads();
    f4 acc[CT][2];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct][0] = acc[ct][1] = f4{0.f, 0.f, 0.f, 0.f};
    // A[c][point] = Fs[point][c], B[point][theta] = Xs[theta][point]
    const float* xa = Xs + (32 * w + i16) * RD_XLD + kq;
    const float* fa = Fs + kq * FLD + i16;
#pragma unroll 4
    for (int t = 0; t < RD_P / 4; ++t) {
      const float bx0 = xa[4 * t], bx1 = xa[16 * RD_XLD + 4 * t];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const float a = fa[4 * t * FLD + 16 * ct];
        acc[ct][0] = mfma4(a, bx0, acc[ct][0]);
        acc[ct][1] = mfma4(a, bx1, acc[ct][1]);
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[ct][q][v] += (double)acc[ct][q][v];
  }
  // D[4 kq + v][i16]: column c = 16 ct + 4 kq + v, theta b0 + 32 w + 16 q + i16
  double* pc = part + (size_t)blockIdx.x * r * B;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int bb = b0 + 32 * w + 16 * q + i16;
    if (bb >= B) continue;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * ct + 4 * kq + v;
        if (c < r) pc[(size_t)bb * r + c] = out[ct][q][v];
      }
  }
}

// The same reduction with both staged blocks fetched by direct global->LDS
// loads (global_load_lds_dwordx4, no registers), double-buffered: the loads
// of block i + 1 are in flight while block i is multiplied.  A lane's 16
// bytes land at the wave's LDS base + 16 lane, so the layouts are:
//   X: row theta of 64 points, its 16-byte runs rotated by theta (run j of
//      row theta at slot (j - theta) mod 16), so the 16 thetas of a B operand
//      read fall on 16 different bank groups;
//   F: the 64 rows of the block copied as they lie in memory (row stride ldf,
//      which must be 16 mod 32 so the 4 rows of a K-step hit disjoint banks).
// Needs ldf % 32 == 16, ldx % 4 == 0 and 16-byte aligned F and X.  Only whole
// 64-point blocks go through the DMA; a chunk's ragged tail is staged by
// ordinary loads with zero fill.
// NH: 16-theta halves per wave; the workgroup takes TBD = 64 NH thetas.  With
// NH = 1 a stage is half as large, so two workgroups share a CU's LDS and
// one can multiply while the other waits at its barrier.
template <int CT, int NH>
__global__ void __launch_bounds__(256, 2) k_reduce_mfma_dma(const float* __restrict__ F, int ldf, int64_t N, int r,
                                                            const float* __restrict__ X, int64_t ldx, int B,
                                                            int64_t chunk, double* __restrict__ part) {
  constexpr int TBD = 64 * NH;                   // thetas per workgroup
  extern __shared__ float dsm[];
  const int stage = TBD * RD_P + RD_P * ldf;     // floats per buffer
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int b0 = blockIdx.y * TBD;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = pbeg + chunk < N ? pbeg + chunk : N;
  const int64_t nfull = (pend - pbeg) / RD_P;
  const int64_t nblk = nfull + ((pend - pbeg) % RD_P != 0);
  auto issue = [&](int64_t q0, float* buf) {
    float* xs = buf;
    float* fs = buf + TBD * RD_P;
#pragma unroll
    for (int u = 0; u < 4 * NH; ++u) {
      const int th = 16 * NH * w + 4 * u + kq;                 // row of this lane
      const int bb = min(b0 + th, B - 1);                       // rows past B: any valid column, discarded
      const int seg = (i16 + th) & 15;                          // the run stored at slot i16
      __builtin_amdgcn_global_load_lds(X + (int64_t)bb * ldx + q0 + 4 * seg, xs + (16 * NH * w + 4 * u) * RD_P, 16,
                                       0, 0);
    }
    const float* fb = F + q0 * ldf;
    for (int j = w; j < ldf / 4; j += 4)                        // 16 ldf bytes-runs = ldf / 4 wave loads
      __builtin_amdgcn_global_load_lds(fb + 4 * (64 * j + lane), fs + 256 * j, 16, 0, 0);
  };
  double out[CT][NH][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int q = 0; q < NH; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[ct][q][v] = 0.0;
  if (nfull > 0) issue(pbeg, dsm);
  for (int64_t i = 0; i < nblk; ++i) {
    float* cur = dsm + (size_t)(i & 1) * stage;
    const int64_t q0 = pbeg + i * RD_P;
    __builtin_amdgcn_s_waitcnt(0);                 // this wave's loads of block i have landed
    __syncthreads();                               // everyone's; and block i - 1 is consumed
    asm volatile("" ::: "memory");                 // LDS reads below see the DMA writes
    if (i >= nfull) {                              // the ragged tail: ordinary loads, zero fill
      for (int e = tid; e < TBD * RD_P; e += 256) {
        const int th = e / RD_P, k = e % RD_P;
        const int64_t p = q0 + k;
        const int bb = b0 + th;
        cur[th * RD_P + 4 * (((k >> 2) - th) & 15) + (k & 3)] =
            (p < pend && bb < B) ? X[(int64_t)bb * ldx + p] : 0.0f;
      }
      for (int e = tid; e < RD_P * ldf; e += 256) {
        const int pt = e / ldf, c = e % ldf;
        const int64_t p = q0 + pt;
        cur[TBD * RD_P + e] = (p < pend && c < r) ? F[p * ldf + c] : 0.0f;
      }
      __syncthreads();
    }
    if (i + 1 < nfull) issue(q0 + RD_P, dsm + (size_t)((i + 1) & 1) * stage);
    const float* xs = cur;
    const float* fa = cur + TBD * RD_P + kq * ldf + i16;
    f4 acc[CT][NH];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < NH; ++q) acc[ct][q] = f4{0.f, 0.f, 0.f, 0.f};
    // the K-steps' LDS operands one step ahead of their MFMAs (two register
    // sets), so the reads are in flight while the previous step multiplies
    auto ldop = [&](int t, float (&a)[CT], float (&b)[NH]) {
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        const int th = 16 * NH * w + 16 * q + i16;
        b[q] = xs[th * RD_P + 4 * ((t - th) & 15) + kq];
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) a[ct] = fa[4 * t * ldf + 16 * ct];
    };
    auto mm = [&](const float (&a)[CT], const float (&b)[NH]) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int q = 0; q < NH; ++q) acc[ct][q] = mfma4(a[ct], b[q], acc[ct][q]);
    };
    // (scheduling barriers keep the compiler from sinking each read next
    // to its MFMA, which would leave one read in flight at a time)
    float a0[CT], b0[NH], a1[CT], b1[NH];
    ldop(0, a0, b0);
#pragma unroll
    for (int t = 0; t < RD_P / 4; t += 2) {
      ldop(t + 1, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      mm(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      if (t + 2 < RD_P / 4) ldop(t + 2, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      mm(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[ct][q][v] += (double)acc[ct][q][v];
  }
  double* pc = part + (size_t)blockIdx.x * r * B;
#pragma unroll
  for (int q = 0; q < NH; ++q) {
    const int bb = b0 + 16 * NH * w + 16 * q + i16;
    if (bb >= B) continue;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * ct + 4 * kq + v;
        if (c < r) pc[(size_t)bb * r + c] = out[ct][q][v];
      }
  }
}

// W[e] = sum over chunks of part[chunk * count + e], in chunk order.
__global__ void __launch_bounds__(256) k_sum_chunks(const double* __restrict__ part, int nch, int64_t count,
                                                    float* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int k = 0; k < nch; ++k) s += part[(size_t)k * count + e];
    W[e] = (float)s;
  }
}

// ------------------------------------------------------------------ skinny
// Short batches (2 <= B <= 16 thetas, r <= 128) with F rows 16-byte aligned
// (ldf % 4 == 0): one 16 x 16 theta tile, so a wave keeps Z or X and its
// sums in registers (the expand stages its rows of F in LDS, the reduce
// loads them straight into registers).  Each lane reads 4 consecutive
// columns of a row of F (16 bytes) and the MFMA K index is permuted to
// match: within a 16-row step of the reduce, lane group kq = l / 16 takes
// rows 4 kq .. 4 kq + 3, the four MFMAs of the step one row each; in the
// expand, the four MFMAs of a 16-column step take one column each of the
// lane's 4-column load.  The permutation is the same on both operands, so
// the sums are those of the plain product.

// W (r x B) = F^T X over 256 rows per workgroup (64 per wave, in 16-row
// steps), float32 MFMA sums over the wave's rows, the four waves' sums added
// in float64 and written as the workgroup's partial
// part[blockIdx.x r B + c + theta r] (k_sum_ranges, then k_sum_final or
// k_bmatvec_lds, add them).
// Columns: G groups of 64 read as 16-byte loads (group g, element e of lane
// i16 is column 64 g + 4 i16 + e: four MFMA tiles per group, tile (g, e)
// holding the columns 64 g + 4 m + e, m < 16), then TT tiles of 16 columns
// read one float per lane (column 64 G + 16 t + i16).  VEC: X's columns are
// 16-byte aligned, so a lane's 4 rows of one theta are one load.
constexpr int SK_P = 256;   // rows per workgroup of the skinny reduce

template <int G, int TT, bool VEC>
__global__ void __launch_bounds__(256, 2) k_reduce_skinny_mfma(const float* __restrict__ F, int ldf, int64_t N,
                                                               int r, const float* __restrict__ X, int64_t ldx,
                                                               int B, double* __restrict__ part) {
  constexpr int NT = 4 * G + TT;
  __shared__ float red[3][NT][4][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * SK_P + (int64_t)w * 64;
  // operands of the wave's four 16-row steps: rows base + 16 st + 4 kq + j
  f4 xv[4];
  f4 fg[4][4][G > 0 ? G : 1];
  float ft[4][4][TT > 0 ? TT : 1];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int64_t p = base + 16 * st + 4 * kq;
    f4 x = f4{0.f, 0.f, 0.f, 0.f};
    if (i16 < B) {
      const float* xc = X + (int64_t)i16 * ldx;
      if (VEC && p + 3 < N) {
        x = *reinterpret_cast<const f4*>(xc + p);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (p + j < N) x[j] = xc[p + j];
      }
    }
    xv[st] = x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool pin = p + j < N;
      const float* row = F + (pin ? p + j : 0) * (int64_t)ldf;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int c = 64 * g + 4 * i16;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (pin && c < r) {
          v = *reinterpret_cast<const f4*>(row + c);
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c + e >= r) v[e] = 0.f;
        }
        fg[st][j][g < G ? g : 0] = v;
      }
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const int c = 64 * G + 16 * t + i16;
        ft[st][j][t < TT ? t : 0] = (pin && c < r) ? row[c] : 0.f;
      }
    }
  }
  f4 acc[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float b = xv[st][j];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[4 * g + e] = mfma4(fg[st][j][g < G ? g : 0][e], b, acc[4 * g + e]);
#pragma unroll
      for (int t = 0; t < TT; ++t) acc[4 * G + t] = mfma4(ft[st][j][t < TT ? t : 0], b, acc[4 * G + t]);
    }
  if (w > 0) {
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w - 1][k][v][lane] = acc[k][v];
  }
  __syncthreads();
  if (w > 0 || i16 >= B) return;
  const int64_t count = (int64_t)r * B;
  double* pw = part + (int64_t)blockIdx.x * count + (int64_t)i16 * r;
  // D[4 kq + v][i16] of tile k: column c below, theta i16
#pragma unroll
  for (int k = 0; k < NT; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = k < 4 * G ? 64 * (k / 4) + 16 * kq + 4 * v + (k % 4) : 64 * G + 16 * (k - 4 * G) + 4 * kq + v;
      if (c < r)
        pw[c] = (double)acc[k][v] + (double)red[0][k][v][lane] + (double)red[1][k][v][lane] +
                (double)red[2][k][v][lane];
    }
}

// Y (N x B) = F Z, one wave per workgroup, 64 points in four 16-point
// tiles.  The wave first copies its 64 rows of F (contiguous in memory, ldf
// apart) into LDS by 16-byte direct global->LDS loads, lane l to dword 4 l
// of each 1 KB piece, so every quarter-wave reads 256 contiguous bytes (the
// A operands loaded straight from memory would take 16 rows per
// quarter-wave); of the last row only the first ceil(r / 4) 16-byte pieces
// are copied.  Z (r x B, leading dimension r) is held in registers: lane
// (i16, kq) keeps Z[16 u + 4 kq + e][i16]; its A operand for step (u, e) is
// element e of its 16-byte LDS read F[p][16 u + 4 kq ..].  U = ceil(r / 16).
// VEC: Y's columns are 16-byte aligned, a lane's 4 consecutive points go as
// one store.  ldf <= SK_DMA_MAXLD (64 rows in LDS).
constexpr int SK_DMA_MAXLD = 160;
template <int U, bool VEC>
__global__ void __launch_bounds__(64) k_expand_skinny_dma(const float* __restrict__ F, int ldf, int64_t N, int r,
                                                          const float* __restrict__ Z, int B, float* __restrict__ Y,
                                                          int64_t ldy) {
  extern __shared__ __attribute__((aligned(16))) float fsm[];
  const int lane = threadIdx.x, i16 = lane & 15, kq = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int rows = (int)(N - p0 < 64 ? N - p0 : 64);
  const int ndw = (rows - 1) * ldf + ((r + 3) & ~3);
  const float* src = F + p0 * (int64_t)ldf;
  for (int j = 0; 256 * j < ndw; ++j)
    if (256 * j + 4 * lane < ndw) __builtin_amdgcn_global_load_lds(src + 256 * j + 4 * lane, fsm + 256 * j, 16, 0, 0);
  float zr[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = 16 * u + 4 * kq + e;
      zr[u][e] = (i16 < B && c < r) ? Z[c + (int64_t)i16 * r] : 0.f;
    }
  __builtin_amdgcn_s_waitcnt(0);                 // the wave's copies have landed (LDS is private to the wave)
  asm volatile("" ::: "memory");
  f4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < U; ++u) {
    f4 fv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int row = 16 * s + i16, c = 16 * u + 4 * kq;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (row < rows && c < r) {
        v = *reinterpret_cast<const f4*>(fsm + row * ldf + c);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (c + e >= r) v[e] = 0.f;
      }
      fv[s] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = mfma4(fv[s][e], zr[u][e], acc[s]);
  }
  if (i16 >= B) return;
  float* ycol = Y + (int64_t)i16 * ldy;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t p = p0 + 16 * s + 4 * kq;
    if (VEC && p + 3 < N) {
      *reinterpret_cast<f4*>(ycol + p) = acc[s];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (p + v < N) ycol[p + v] = acc[s][v];
    }
  }
}

// Chunking of the reduce: enough workgroups to fill the chip (RD_WG_TARGET
// over the theta blocks), every chunk a whole number of 64-point blocks.
constexpr int RD_WG_TARGET = 512;
void reduce_shape(int64_t N, int B, int64_t* chunk, int* nch, int tbd = RD_TB) {
  const int tb = (B + tbd - 1) / tbd;
  const int64_t blocks = (N + RD_P - 1) / RD_P;
  int64_t want = std::max<int64_t>(1, (RD_WG_TARGET + tb - 1) / tb);
  want = std::min<int64_t>(want, blocks);
  const int64_t per = (blocks + want - 1) / want;   // 64-point blocks per chunk
  *chunk = per * RD_P;
  *nch = (int)((N + *chunk - 1) / *chunk);
}

template <class K>
tt_status set_lds(K kern, size_t bytes) {
  static_assert(sizeof(K) > 0, "");
  if (bytes > 64 * 1024)
    TTK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
  return TTK_OK;
}

// Workgroups over the points; when those are few (a short, wide product such
// as the online core's) the theta blocks are split over grid.y as well, so
// about EX_WG_TARGET workgroups run.
constexpr int EX_WG_TARGET = 512;

template <int KS>
tt_status launch_expand(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y, int64_t ldy,
                        bool acc, hipStream_t st) {
  const size_t sh = expand_lds_floats(r, 4 * KS) * sizeof(float);
  const bool vec = (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
  const int64_t gx = (N + EX_P - 1) / EX_P;
  const int nb = (B + EX_TB - 1) / EX_TB;
  const int gy_want = (int)std::min<int64_t>(nb, std::max<int64_t>(1, (EX_WG_TARGET + gx - 1) / gx));
  const int bpw = (nb + gy_want - 1) / gy_want;
  const dim3 grid((unsigned)gx, (unsigned)((nb + bpw - 1) / bpw));
  if (acc) {
    TTK_TRY(set_lds(&k_expand_mfma<KS, false, true>, sh));
    hipLaunchKernelGGL((k_expand_mfma<KS, false, true>), grid, dim3(256), sh, st, F, ldf, N, r, Z, B, Y, ldy, bpw);
  } else if (vec) {
    TTK_TRY(set_lds(&k_expand_mfma<KS, true, false>, sh));
    hipLaunchKernelGGL((k_expand_mfma<KS, true, false>), grid, dim3(256), sh, st, F, ldf, N, r, Z, B, Y, ldy, bpw);
  } else {
    TTK_TRY(set_lds(&k_expand_mfma<KS, false, false>, sh));
    hipLaunchKernelGGL((k_expand_mfma<KS, false, false>), grid, dim3(256), sh, st, F, ldf, N, r, Z, B, Y, ldy, bpw);
  }
  return TTK_OK;
}

template <int CT>
tt_status launch_reduce(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B, float* W,
                        double* part, hipStream_t st) {
  int64_t chunk;
  int nch;
  reduce_shape(N, B, &chunk, &nch);
  const dim3 grid((unsigned)nch, (unsigned)((B + RD_TB - 1) / RD_TB));
  const bool xal = (ldx % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
  const bool dma = xal && ldf % 32 == 16 && ldf >= 16 * CT && reinterpret_cast<uintptr_t>(F) % 16 == 0;
  if (dma) {
    // 64 thetas per workgroup: two workgroups per CU (half the LDS each)
    int64_t chunk1;
    int nch1;
    reduce_shape(N, B, &chunk1, &nch1, 64);
    if (nch1 > nch) return fail(TTK_ERR_ARG, "reduce: chunk partials exceed the workspace");
    const dim3 grid1((unsigned)nch1, (unsigned)((B + 63) / 64));
    const size_t sh = (size_t)2 * (64 * RD_P + RD_P * ldf) * sizeof(float);
    TTK_TRY(set_lds(&k_reduce_mfma_dma<CT, 1>, sh));
    hipLaunchKernelGGL((k_reduce_mfma_dma<CT, 1>), grid1, dim3(256), sh, st, F, ldf, N, r, X, ldx, B, chunk1, part);
    nch = nch1;
  } else {
    const size_t sh = reduce_lds_floats<CT>() * sizeof(float);
    if (xal) {
      TTK_TRY(set_lds(&k_reduce_mfma<CT, true>, sh));
      hipLaunchKernelGGL((k_reduce_mfma<CT, true>), grid, dim3(256), sh, st, F, ldf, N, r, X, ldx, B, chunk, part);
    } else {
      TTK_TRY(set_lds(&k_reduce_mfma<CT, false>, sh));
      hipLaunchKernelGGL((k_reduce_mfma<CT, false>), grid, dim3(256), sh, st, F, ldf, N, r, X, ldx, B, chunk,
                         part);
    }
  }
  const int64_t count = (int64_t)r * B;
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 4096)), dim3(256), 0, st,
                     (const double*)part, nch, count, W);
  return TTK_OK;
}


template <int G, int TT>
void launch_reduce_skinny(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B,
                          double* part, unsigned groups, hipStream_t st) {
  if ((ldx % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0))
    hipLaunchKernelGGL((k_reduce_skinny_mfma<G, TT, true>), dim3(groups), dim3(256), 0, st, F, ldf, N, r, X, ldx, B,
                       part);
  else
    hipLaunchKernelGGL((k_reduce_skinny_mfma<G, TT, false>), dim3(groups), dim3(256), 0, st, F, ldf, N, r, X, ldx,
                       B, part);
}

template <int U>
void launch_expand_skinny(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y, int64_t ldy,
                          hipStream_t st) {
  const bool vec = (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
  const dim3 grid((unsigned)((N + 63) / 64));
  const size_t sh = (size_t)64 * ldf * sizeof(float);
  if (vec)
    hipLaunchKernelGGL((k_expand_skinny_dma<U, true>), grid, dim3(64), sh, st, F, ldf, N, r, Z, B, Y, ldy);
  else
    hipLaunchKernelGGL((k_expand_skinny_dma<U, false>), grid, dim3(64), sh, st, F, ldf, N, r, Z, B, Y, ldy);
}
}  // namespace

bool apply_mfma_ok(int r, int B) { return r >= 1 && r <= MFMA_APPLY_MAXR && B > 16; }

int mfma_ld(int r) {
  int ld = r < 16 ? 16 : r;
  while (ld % 32 != 16) ++ld;
  return ld;
}

size_t apply_reduce_mfma_work(int64_t N, int r, int B) {
  if (N <= 0) return 0;
  int64_t chunk;
  int nch;
  reduce_shape(N, B, &chunk, &nch);
  return (size_t)nch * r * B * sizeof(double);
}

tt_status apply_reduce_mfma(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B, float* W,
                            double* part, hipStream_t st) {
  switch ((r + 15) / 16) {
    case 1: return launch_reduce<1>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 2: return launch_reduce<2>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 3: return launch_reduce<3>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 4: return launch_reduce<4>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 5: return launch_reduce<5>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 6: return launch_reduce<6>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 7: return launch_reduce<7>(F, ldf, N, r, X, ldx, B, W, part, st);
    case 8: return launch_reduce<8>(F, ldf, N, r, X, ldx, B, W, part, st);
    default: return fail(TTK_ERR_UNSUPPORTED, "MFMA reduce: rank %d > %d", r, MFMA_APPLY_MAXR);
  }
}

bool skinny_mfma_ok(const void* F, int ldf, int r, int B) {
  return B >= 2 && B <= 16 && r >= 1 && r <= MFMA_APPLY_MAXR && ldf >= r && ldf % 4 == 0 &&
         reinterpret_cast<uintptr_t>(F) % 16 == 0;
}

tt_status reduce_skinny_mfma(const float* F, int ldf, int64_t N, int r, const float* X, int64_t ldx, int B,
                             double* part, unsigned groups, hipStream_t st) {
  if (N <= 0) return TTK_OK;
  if (!skinny_mfma_ok(F, ldf, r, B) || (int64_t)groups * SK_P < N)
    return fail(TTK_ERR_ARG, "skinny MFMA reduce: unsupported shape (r %d, ldf %d, B %d)", r, ldf, B);
  // G 64-column groups of 16-byte loads, then TT 16-column tiles
  int G = r / 64, rem = r - 64 * G, TT = (rem + 15) / 16;
  if (rem > 48) ++G, TT = 0;
  switch (4 * G + TT) {
    case 1: launch_reduce_skinny<0, 1>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 2: launch_reduce_skinny<0, 2>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 3: launch_reduce_skinny<0, 3>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 4: launch_reduce_skinny<1, 0>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 5: launch_reduce_skinny<1, 1>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 6: launch_reduce_skinny<1, 2>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 7: launch_reduce_skinny<1, 3>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    case 8: launch_reduce_skinny<2, 0>(F, ldf, N, r, X, ldx, B, part, groups, st); break;
    default: return fail(TTK_ERR_UNSUPPORTED, "skinny MFMA reduce: rank %d", r);
  }
  return TTK_OK;
}

bool skinny_expand_mfma_ok(const void* F, int ldf, int r, int B) {
  return skinny_mfma_ok(F, ldf, r, B) && ldf <= SK_DMA_MAXLD;
}

tt_status expand_skinny_mfma(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y,
                             int64_t ldy, hipStream_t st) {
  if (N <= 0) return TTK_OK;
  if (!skinny_expand_mfma_ok(F, ldf, r, B))
    return fail(TTK_ERR_ARG, "skinny MFMA expand: unsupported shape (r %d, ldf %d, B %d)", r, ldf, B);
  switch ((r + 15) / 16) {
    case 1: launch_expand_skinny<1>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 2: launch_expand_skinny<2>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 3: launch_expand_skinny<3>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 4: launch_expand_skinny<4>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 5: launch_expand_skinny<5>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 6: launch_expand_skinny<6>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 7: launch_expand_skinny<7>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    case 8: launch_expand_skinny<8>(F, ldf, N, r, Z, B, Y, ldy, st); break;
    default: return fail(TTK_ERR_UNSUPPORTED, "skinny MFMA expand: rank %d", r);
  }
  return TTK_OK;
}

tt_status apply_expand_mfma(const float* F, int ldf, int64_t N, int r, const float* Z, int B, float* Y, int64_t ldy,
                            hipStream_t st, bool accumulate) {
  switch ((r + 3) / 4) {
#define TTK_EXPAND_CASE(k) \
  case k: return launch_expand<k>(F, ldf, N, r, Z, B, Y, ldy, accumulate, st);
    TTK_EXPAND_CASE(1) TTK_EXPAND_CASE(2) TTK_EXPAND_CASE(3) TTK_EXPAND_CASE(4) TTK_EXPAND_CASE(5)
    TTK_EXPAND_CASE(6) TTK_EXPAND_CASE(7) TTK_EXPAND_CASE(8) TTK_EXPAND_CASE(9) TTK_EXPAND_CASE(10)
    TTK_EXPAND_CASE(11) TTK_EXPAND_CASE(12) TTK_EXPAND_CASE(13) TTK_EXPAND_CASE(14) TTK_EXPAND_CASE(15)
    TTK_EXPAND_CASE(16) TTK_EXPAND_CASE(17) TTK_EXPAND_CASE(18) TTK_EXPAND_CASE(19) TTK_EXPAND_CASE(20)
    TTK_EXPAND_CASE(21) TTK_EXPAND_CASE(22) TTK_EXPAND_CASE(23) TTK_EXPAND_CASE(24) TTK_EXPAND_CASE(25)
    TTK_EXPAND_CASE(26) TTK_EXPAND_CASE(27) TTK_EXPAND_CASE(28) TTK_EXPAND_CASE(29) TTK_EXPAND_CASE(30)
    TTK_EXPAND_CASE(31) TTK_EXPAND_CASE(32)
#undef TTK_EXPAND_CASE
    default: return fail(TTK_ERR_UNSUPPORTED, "MFMA expand: rank %d > %d", r, MFMA_APPLY_MAXR);
  }
}

}  // namespace ttk
