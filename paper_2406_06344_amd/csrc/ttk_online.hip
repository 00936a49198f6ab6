// Online stage (Algorithm 3): M(theta) = H_1(theta_1) ... H_dt(theta_dt) with
// H_j = G_{d+j} x_2 q^p_j(theta_j), batched over theta samples, and its
// derivative dM/dtheta_j, obtained by replacing q^p_j with d q^p_j / d theta_j.
// The parameter cores are held in the Chebyshev coefficient basis, so
// q_k = T_k(t(theta)) and dq_k/dtheta = T_k'(t) dt/dtheta, with T_k' from the
// differentiated three-term recurrence T'_{k+1} = 2 T_k + 2 t T'_k - T'_{k-1}.
// Work is O(dt (n r^2 + r^3)) per theta, independent of N (Section 3.2).
//
// Two grid-parallel launches: every entry of every factor H_j(theta_b) (and
// its derivative, from the same loads of the core) gets its own thread, which
// runs the recurrence for its theta in registers; for d_theta = 2 a second
// launch forms the products H_1 H_2, dH_1 H_2 and H_1 dH_2, one thread per
// entry.  Everything is accumulated in double precision and rounded once on
// store.
#include <algorithm>

#include "ttk_internal.h"

namespace ttk {

namespace {

struct OnlineArgs {
  const double* G[2];
  int r0[2], n[2], r1[2];
  double lo[2], hi[2];
  int dt;
};

// Factor entries: blockIdx.y = theta, blockIdx.z = parameter dimension j.
// For d_theta = 1 the factor is M itself and is stored in the output type;
// for d_theta = 2 the factors go to the double workspace.
template <class TT, class T>
__global__ void __launch_bounds__(256) k_online_factor(OnlineArgs oa, const TT* theta, T* M, T* dM, double* H,
                                                       double* dH, size_t hstride, int want_d) {
  const int b = blockIdx.y, j = blockIdx.z;
  const int n = oa.n[j], r0 = oa.r0[j], r1 = oa.r1[j];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r0 * r1) return;
  const double th = (double)theta[(int64_t)b * oa.dt + j];
  const double lo = oa.lo[j], hi = oa.hi[j];
  const double t = (2.0 * th - (lo + hi)) / (lo - hi);
  const double dtdth = 2.0 / (lo - hi);
  const int a = e % r0, c = e / r0;
  const double* G = oa.G[j] + a + (int64_t)c * r0 * n;
  // T_0 = 1, T_1 = t; T'_0 = 0, T'_1 = 1.  The coefficients are loaded in
  // chunks of OCH, all of a chunk's loads in flight before its terms.
  constexpr int OCH = 8;
  double tm = 1.0, tc = t, dm = 0.0, dc = 1.0;
  double s = 0.0, ds = 0.0;
  for (int k0 = 0; k0 < n; k0 += OCH) {
    double g[OCH];
#pragma unroll
    for (int q = 0; q < OCH; ++q) g[q] = k0 + q < n ? G[(int64_t)(k0 + q) * r0] : 0.0;
#pragma unroll
    for (int q = 0; q < OCH; ++q) {
      const int k = k0 + q;
      if (k >= n) break;
      if (k == 0) {
        s = g[q];
      } else if (k == 1) {
        s += t * g[q];
        ds += g[q];
      } else {
        const double tn = 2.0 * t * tc - tm;
        const double dn = 2.0 * tc + 2.0 * t * dc - dm;
        tm = tc; tc = tn; dm = dc; dc = dn;
        s += tn * g[q];
        ds += dn * g[q];
      }
    }
  }
  ds *= dtdth;
  if (oa.dt == 1) {
    const size_t msz = (size_t)r0 * r1;
    M[(size_t)b * msz + e] = (T)s;
    if (want_d) dM[(size_t)b * msz + e] = (T)ds;
  } else {
    // workspace per theta: H_1 (r0 x rm), H_2 (rm x r1), then their derivatives
    double* hb = H + (size_t)b * hstride + (j == 0 ? 0 : (size_t)oa.r0[0] * oa.r1[0]);
    hb[e] = s;
    if (want_d) {
      double* db = dH + (size_t)b * hstride + (j == 0 ? 0 : (size_t)oa.r0[0] * oa.r1[0]);
      db[e] = ds;
    }
  }
}

// d_theta = 2: blockIdx.y = theta, blockIdx.z = product (0: H1 H2 -> M,
// 1: dH1 H2 -> dM[., 0], 2: H1 dH2 -> dM[., 1]).
template <class T>
__global__ void __launch_bounds__(256) k_online_product(OnlineArgs oa, const double* H, const double* dH,
                                                        size_t hstride, T* M, T* dM) {
  const int b = blockIdx.y, which = blockIdx.z;
  const int rs = oa.r0[0], rm = oa.r1[0], rt = oa.r1[1];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rs * rt) return;
  const int i = e % rs, c = e / rs;
  const double* h1 = (which == 1 ? dH : H) + (size_t)b * hstride;
  const double* h2 = (which == 2 ? dH : H) + (size_t)b * hstride + (size_t)rs * rm;
  double s = 0.0;
  for (int m = 0; m < rm; ++m) s += h1[i + (int64_t)m * rs] * h2[m + (int64_t)c * rm];
  const size_t msz = (size_t)rs * rt;
  if (which == 0) M[(size_t)b * msz + e] = (T)s;
  else dM[((size_t)b * 2 + (which - 1)) * msz + e] = (T)s;
}

OnlineArgs make_args(const ParamCore* pc, int dt) {
  OnlineArgs oa{};
  oa.dt = dt;
  for (int j = 0; j < dt; ++j) {
    oa.G[j] = pc[j].Ghat;
    oa.r0[j] = pc[j].r0;
    oa.n[j] = pc[j].n;
    oa.r1[j] = pc[j].r1;
    oa.lo[j] = pc[j].lo;
    oa.hi[j] = pc[j].hi;
  }
  return oa;
}

// per-theta workspace (d_theta = 2): H_1 and H_2
size_t online_stride(const ParamCore* pc, int dt) {
  if (dt < 2) return 0;
  return (size_t)pc[0].r0 * pc[0].r1 + (size_t)pc[1].r0 * pc[1].r1;
}

template <class TT, class T>
void launch_online(const OnlineArgs& oa, const TT* theta, int B, T* M, T* dM, double* work, hipStream_t st) {
  int maxe = 0;
  for (int j = 0; j < oa.dt; ++j) maxe = std::max(maxe, oa.r0[j] * oa.r1[j]);
  const size_t stride = oa.dt == 2 ? (size_t)oa.r0[0] * oa.r1[0] + (size_t)oa.r0[1] * oa.r1[1] : 0;
  const size_t msz = (size_t)oa.r0[0] * oa.r1[oa.dt - 1];
  double* H = work;
  double* dH = work + stride * B;
  const int want_d = dM != nullptr;
  constexpr int BMAX = 65535;   // grid.y limit
  for (int b0 = 0; b0 < B; b0 += BMAX) {
    const int nb = std::min(BMAX, B - b0);
    const TT* th = theta + (size_t)b0 * oa.dt;
    T* Mb = M + (size_t)b0 * msz;
    T* dMb = want_d ? dM + (size_t)b0 * oa.dt * msz : nullptr;
    double* Hb = H + (size_t)b0 * stride;
    double* dHb = dH + (size_t)b0 * stride;
    hipLaunchKernelGGL((k_online_factor<TT, T>), dim3((maxe + 255) / 256, nb, oa.dt), dim3(256), 0, st, oa, th, Mb,
                       dMb, Hb, dHb, stride, want_d);
    if (oa.dt == 2) {
      const int rs = oa.r0[0], rt = oa.r1[1];
      hipLaunchKernelGGL(k_online_product<T>, dim3((rs * rt + 255) / 256, nb, want_d ? 3 : 1), dim3(256), 0, st, oa,
                         Hb, dHb, stride, Mb, dMb);
    }
  }
}

// C[e, k1 n2 + k2] = sum_m Ghat_1[a, k1, m] Ghat_2[m, k2, c], e = a + c rs,
// accumulated in double, stored as float; one thread per entry.
__global__ void __launch_bounds__(256) k_online_cprod(const double* G1, const double* G2, int rs, int n1, int rm,
                                                      int n2, int rt, float* C) {
  const int nk = n1 * n2;
  const int64_t total = (int64_t)rs * rt * nk;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int kk = (int)(idx % nk);
    const int64_t e = idx / nk;
    const int a = (int)(e % rs), c = (int)(e / rs);
    const int k1 = kk / n2, k2 = kk % n2;
    const double* g1 = G1 + a + (int64_t)k1 * rs;            // stride rs n1 over m
    const double* g2 = G2 + (int64_t)k2 * rm + (int64_t)c * rm * n2;
    double s = 0.0;
    for (int m = 0; m < rm; ++m) s += g1[(int64_t)m * rs * n1] * g2[m];
    C[idx] = (float)s;
  }
}

// Coefficients of one theta: column b of coefM holds T_k1(t_1) T_k2(t_2) at
// row k1 n2 + k2; columns 2 b + j of coefD the products with T_kj replaced by
// dT_kj/dtheta_j.  Rows are split in passes of 128 (pass p, row kk at
// p * 128 * cols + b * 128 + kk % 128) so every pass is a contiguous 128 x cols
// block.  One thread per (b, kk).
__global__ void __launch_bounds__(256) k_online_coef(const float* theta, int B, int n1, int n2, double lo1,
                                                     double hi1, double lo2, double hi2, int want_d, float* coefM,
                                                     float* coefD) {
  const int nk = n1 * n2;
  const int64_t total = (int64_t)B * nk;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int kk = (int)(idx % nk);
    const int b = (int)(idx / nk);
    const int k1 = kk / n2, k2 = kk % n2;
    double v[2], dv[2];
    const int kj[2] = {k1, k2};
    const double lo[2] = {lo1, lo2}, hi[2] = {hi1, hi2};
    for (int j = 0; j < 2; ++j) {
      const double t = (2.0 * (double)theta[2 * (int64_t)b + j] - (lo[j] + hi[j])) / (lo[j] - hi[j]);
      double tm = 1.0, tc = t, dm = 0.0, dc = 1.0;   // T_0, T_1 and their derivatives
      double tk = 1.0, dk = 0.0;
      if (kj[j] == 1) { tk = t; dk = 1.0; }
      for (int k = 2; k <= kj[j]; ++k) {
        const double tn = 2.0 * t * tc - tm;
        const double dn = 2.0 * tc + 2.0 * t * dc - dm;
        tm = tc; tc = tn; dm = dc; dc = dn;
        tk = tn; dk = dn;
      }
      v[j] = tk;
      dv[j] = dk * 2.0 / (lo[j] - hi[j]);
    }
    const int p = kk / 128, kr = kk % 128;
    const int prow = min(128, nk - 128 * p);
    coefM[(size_t)p * 128 * B + (size_t)b * prow + kr] = (float)(v[0] * v[1]);
    if (want_d) {
      float* cd = coefD + (size_t)p * 128 * 2 * B;
      cd[(size_t)(2 * b) * prow + kr] = (float)(dv[0] * v[1]);
      cd[(size_t)(2 * b + 1) * prow + kr] = (float)(v[0] * dv[1]);
    }
  }
}

}  // namespace

void online_core_mixed(int theta_dtype, int out_dtype, const ParamCore* pc, int dt, const void* theta, int B,
                       void* M, void* dM, double* work, hipStream_t st) {
  if (B <= 0 || dt <= 0) return;
  const OnlineArgs oa = make_args(pc, dt);
  const bool tf = theta_dtype == TTK_FP32, of = out_dtype == TTK_FP32;
  if (tf && of)
    launch_online(oa, static_cast<const float*>(theta), B, static_cast<float*>(M), static_cast<float*>(dM), work, st);
  else if (tf)
    launch_online(oa, static_cast<const float*>(theta), B, static_cast<double*>(M), static_cast<double*>(dM), work,
                  st);
  else if (of)
    launch_online(oa, static_cast<const double*>(theta), B, static_cast<float*>(M), static_cast<float*>(dM), work,
                  st);
  else
    launch_online(oa, static_cast<const double*>(theta), B, static_cast<double*>(M), static_cast<double*>(dM), work,
                  st);
}

void online_core(int dtype, const ParamCore* pc, int dt, const void* theta, int B, void* M, void* dM,
                 double* work, hipStream_t st) {
  online_core_mixed(dtype, dtype, pc, dt, theta, B, M, dM, work, st);
}

tt_status online_gemm_prepare(const ParamCore* pc, float* C, hipStream_t st) {
  const int rs = pc[0].r0, n1 = pc[0].n, rm = pc[0].r1, n2 = pc[1].n, rt = pc[1].r1;
  if (pc[1].r0 != rm) return fail(TTK_ERR_ARG, "parameter cores do not chain");
  const int64_t total = (int64_t)rs * rt * n1 * n2;
  hipLaunchKernelGGL(k_online_cprod, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0, st,
                     pc[0].Ghat, pc[1].Ghat, rs, n1, rm, n2, rt, C);
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

size_t online_gemm_work_floats(const OnlineGemm& og, int B, bool want_d) {
  const size_t passes = (size_t)(og.nk + 127) / 128;
  return passes * 128 * (size_t)B * (want_d ? 3 : 1);
}

tt_status online_core_gemm(const ParamCore* pc, const OnlineGemm& og, const float* theta, int B, float* M, float* dM,
                           float* work, hipStream_t st) {
  if (B <= 0) return TTK_OK;
  const int nk = og.nk, n1 = pc[0].n, n2 = pc[1].n;
  const size_t passes = (size_t)(nk + 127) / 128;
  float* coefM = work;
  float* coefD = work + passes * 128 * (size_t)B;
  const int64_t total = (int64_t)B * nk;
  hipLaunchKernelGGL(k_online_coef, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0, st,
                     theta, B, n1, n2, pc[0].lo, pc[0].hi, pc[1].lo, pc[1].hi, dM != nullptr ? 1 : 0, coefM, coefD);
  const int64_t ne = (int64_t)og.rs * og.rt;
  for (size_t p = 0; p < passes; ++p) {
    const int kr = std::min(128, nk - (int)(128 * p));
    const float* Cp = og.C + 128 * p;
    TTK_TRY(apply_expand_mfma(Cp, nk, ne, kr, coefM + p * 128 * (size_t)B, B, M, ne, st, p > 0));
    if (dM)
      TTK_TRY(apply_expand_mfma(Cp, nk, ne, kr, coefD + p * 128 * 2 * (size_t)B, 2 * B, dM, ne, st, p > 0));
  }
  TTK_HIP(hipGetLastError());
  return TTK_OK;
}

size_t online_work_doubles(const ParamCore* pc, int dt, int B) {
  // H_1, H_2 and their derivatives for every theta (d_theta = 2 only)
  return 2 * online_stride(pc, dt) * (size_t)std::max(B, 1) + 16;
}

}  // namespace ttk
