"""Benchmark of the offline U/V build and the batched, differentiated apply.

One step = the whole hot path on one batch of synthetic input:
  offline stage (cross on the Chebyshev grid with device kernel evaluation,
  rounding of the cores, Phase 3 for all sources and targets), the online
  core for B theta samples, the batched apply y_b = U M(theta_b) V^T x_b and
  its backward pass (dX, dtheta).
Workload (default, matern_batched): d = 3, 1M + 1M points uniform in
separated unit cubes (target cube offset by 2 along axis 1), Matern in
theta = (l, nu), l in [0.5, 2], nu in [0.5, 2.5], 16 nodes per dimension,
tol 7e-7, B = 4096 theta samples each with its own x_b and cotangent g_b,
float32 bulk with float64 cross / factorisations.  Inputs are resident in HBM
before the timed steps.

Prints one JSON line.  value = whole-step offline U/V rows per second,
(N_s + N_t) / seconds per step.  Extra fields report Phase 3 alone, the
apply + gradient against the plain per-theta apply, kernel evaluations,
accuracy against dense float64 K and the roofline of the projection kernel
(timed with HIP events on the stream it runs on).  Other workloads:
--workload matern32_d3 | se_d2_fp64 | matern_global | uneven_pairs | ttk_e1.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "offline U/V rows/s + batched apply+grad GB/s vs plain apply, at ≤1e-5 rel err"
HBM_PEAK_GBPS = 8000.0
# HBM bytes per launch of k_factor_mfma on matern32_d3 (the roofline of that
# workload's line): None, the kernel's output rows are padded since the
# counters in profiles/ were taken.
TRAFFIC = None
FP32_PEAK_TFLOPS = 157.3
# HBM bytes per launch of the projection kernel k_reduce_mfma_dma<5, 1> on
# the 1M-point workload from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE,
# separate runs): (2.000 x 8426797.5 + 1.000 x 19840.8) KiB, averaged over its
# two launches, with the scales 2.000 and 1.000 read off the same counters on
# a plain 1 GiB copy.  None whenever the kernel has changed since.
PROJECT_TRAFFIC = 17278398259
PROJECT_TRAFFIC_NOTE = ("HBM bytes per launch: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (scales from a plain 1 GiB "
                        "copy), average of the two launches; algorithmic 16.72 GB (X, F, float64 chunk partials)")


def phase3_flops_per_point(ranks, n):
    """Algorithmic flops of one point's chain: sum_j 2 n r_{j-1} r_j."""
    return sum(2 * n * ranks[j] * ranks[j + 1] for j in range(len(ranks) - 1))


def time_events(fn, reps, torch):
    """Average duration (ms) of fn() over reps launches, HIP events on the current stream."""
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(w, X, Y, thetas, n_pts):
    """The oracle, as it stands, on a bounded sample of the workload."""
    import threadpoolctl

    from oracle import driver as odriver
    from oracle import kernels as okernels
    from oracle import pttk as opttk

    P = okernels.Problem(w.kind, w.d, w.box_s, w.box_t, w.box_theta, w.n_spatial, w.n_param, w.const or None)
    Xs, Ys = X[:n_pts], Y[:n_pts]
    xb = synth.rhs(n_pts, len(thetas), seed=2)
    gb = synth.rhs(n_pts, len(thetas), seed=3)
    t0 = time.perf_counter()
    out = odriver.offline(P, Xs, Ys, w.tol, seed=0)
    Hs = [opttk.online_H(out["param"], th, P.box_theta, w.n_param) for th in thetas]
    dHs = [opttk.online_dH(out["param"], th, P.box_theta, w.n_param) for th in thetas]
    opttk.apply_batched(out["S"], Hs, out["T"], xb)
    opttk.backward_batched(out["S"], Hs, dHs, out["T"], xb, gb)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    return {"value": round(2 * n_pts / dt, 3), "unit": "rows/s", "cores": int(threads), "kind": "oracle",
            "sample": f"full offline stage (cross, rounding, Phase 3) + apply and backward at "
                      f"{len(thetas)} theta on {n_pts} + {n_pts} points of the same workload "
                      f"(the cross does not depend on N); {dt:.1f} s",
            "host_cpus": len(os.sched_getaffinity(0))}


def time_wall(fn, reps, torch):
    """Average wall time (ms) of fn() over reps calls, device synchronised on both sides."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps


def base_result(w, args, value, unit, ms_per_step, B, extra_cfg=None):
    cfg = {"workload": w.name, "kernel": w.kind, "d": w.d, "d_theta": w.d_theta, "N_s": w.n_src, "N_t": w.n_tgt,
           "n_spatial": w.n_spatial, "n_param": w.n_param, "tol": w.tol, "n_theta": B,
           "parallelism": "single GPU"}
    cfg.update(extra_cfg or {})
    return {"metric": METRIC, "value": round(value, 1), "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if w.fp64 else "f32", "data": "synthetic",
            "config": cfg}


def bench_global(args, torch, pkg):
    """Symmetric PSD variant (Algorithm 4, Global-1): X = Y, N points in the unit cube."""
    w = synth.WORKLOADS["matern_global"]
    X, _ = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    B = th.shape[0]
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    xb = torch.tensor(synth.rhs(w.n_src, B, seed=2).T.copy(), dtype=torch.float32, device="cuda")
    kw = dict(kind=w.kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta, n_spatial=w.n_spatial,
              n_param=w.n_param, tol=w.tol, dtype=torch.float32, seed=0, symmetric_psd=True)

    def step():
        kern = pkg.TTKernel.build_offline(Xd, None, **kw)
        y = kern.global_apply(xb, theta=thd)
        return kern, y

    for i in range(args.warmup):
        kern, _ = step()
        print(f"warmup {i} done: ranks {kern.info()['ranks']}", file=sys.stderr, flush=True)
    ms = time_wall(step, args.steps, torch)
    kern, _ = step()
    inf = kern.info()
    Q, R = kern.global_factors()
    k = Q.shape[1]
    ms_online = time_events(lambda: kern.global_online(thd), 5, torch)
    W = kern.global_online(thd)
    ms_apply = time_events(lambda: kern.global_apply(xb, W=W), 10, torch)
    bytes_apply = 2 * 4 * w.n_src * k + 2 * 4 * B * w.n_src
    # accuracy against dense float64 K(X, X) on a 4000-point subsample
    rng = np.random.default_rng(11)
    si = np.sort(rng.choice(w.n_src, 4000, replace=False))
    Qs = Q[si].double()
    errs = []
    for b in range(B):
        K = pkg.eval_dense(torch.tensor(X[si]), torch.tensor(X[si]), th[b], w.kind, w.d, dtype=torch.float64)
        Kh = Qs @ W[b].double() @ Qs.t()
        errs.append((torch.linalg.norm(K - Kh) / torch.linalg.norm(K)).item())
    # Global-2 (Compress, eps = the build's tolerance) for the first theta:
    # the eigen-truncation and Z = Q Uhat, then its apply
    ms_g2 = time_wall(lambda: kern.global2_online(thd[0], w.tol), 3, torch)
    Z, lam = kern.global2_online(thd[0], w.tol)
    ms_g2_apply = time_events(lambda: kern.global2_apply(Z, lam, xb), 10, torch)
    K0 = pkg.eval_dense(torch.tensor(X[si]), torch.tensor(X[si]), th[0], w.kind, w.d, dtype=torch.float64)
    Zs = Z[si].double()
    err_g2 = (torch.linalg.norm(K0 - (Zs * lam.double()) @ Zs.t()) / torch.linalg.norm(K0)).item()
    hm = bench_hmatrix(w, X, th, si, torch, pkg)
    rows = 2 * w.n_src
    res = base_result(w, args, rows / (ms / 1000.0), "rows/s", ms, B, {"variant": "Global-1", "X=Y": True})
    res.update({"ranks": inf["ranks"], "cross_ranks": inf["cross_ranks"], "cross_sweeps": inf["sweeps"],
                "k": k, "kernel_evals": inf["kernel_evals"], "t_cross_ms": round(inf["t_cross_ms"], 2),
                "t_round_ms": round(inf["t_round_ms"], 2), "t_factor_and_qr_ms": round(inf["t_factor_ms"], 2),
                "online_ms_per_theta": round(ms_online / B, 4), "global_apply_ms": round(ms_apply, 4),
                "global_apply_GBps": round(bytes_apply / (ms_apply * 1e-3) / 1e9, 1),
                "max_rel_err_vs_dense_fp64": float(f"{max(errs):.3e}"), "status": kern.status,
                "global2": {"eps": w.tol, "r_c": int(lam.shape[0]), "online_ms": round(ms_g2, 3),
                            "apply_ms": round(ms_g2_apply, 4), "rel_err_vs_dense_fp64": float(f"{err_g2:.3e}"),
                            "note": "Global-2 for the first theta: eigen-truncation of R Hhat R^T and Z = Q Uhat "
                                    "(online, host-synchronised), then y = Z diag(lam) Z^T x for all right-hand "
                                    "sides"},
                "accuracy_note": "Q W Q^T against dense float64 K(X, X) on a 4000-point subsample, worst theta",
                "hmatrix": hm})
    res["roofline"] = {"kernel": "Global-1 apply (Q^T x, W, Q z)", "bound": "hbm",
                       "achieved": res["global_apply_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(res["global_apply_GBps"] / HBM_PEAK_GBPS, 4), "traffic": None}
    return res


def bench_hmatrix(w, X, th, si, torch, pkg, n_theta=4, leaf=400, tol=1e-6):
    """The X = Y problem through the hierarchical form of Section 5: the far
    blocks of a uniform tree over the unit cube (interaction lists of every
    level >= 2) as PTTK low-rank blocks, one TT per geometry class, the near
    blocks (neighbouring leaves) summed directly.  Build time, apply time for
    n_theta thetas at once, and the error of H(theta) x against dense float64
    K(X, X) x on the subsampled rows si (K's rows summed over all N columns
    in chunks)."""
    N = X.shape[0]
    Xt = torch.tensor(X, dtype=torch.float32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = pkg.HMatrix.build(Xt, w.kind, w.d, w.box_s, w.box_theta, leaf_points=leaf, n_spatial=w.n_spatial,
                          n_param=w.n_param, tol=tol, dtype=torch.float32, max_sweeps=400)
    torch.cuda.synchronize()
    ms_build = (time.perf_counter() - t0) * 1000.0
    inf = H.info()
    print(f"hmatrix built: {inf['far_pairs']} far pairs, {inf['num_classes']} classes, {ms_build:.0f} ms",
          file=sys.stderr, flush=True)
    thb = torch.tensor(th[:n_theta], dtype=torch.float32, device="cuda")
    xs = synth.rhs(N, n_theta, seed=4).T.copy()
    xd = torch.tensor(xs, dtype=torch.float32, device="cuda")
    ms_apply = time_events(lambda: H.apply(thb, xd), 3, torch)
    Y = H.apply(thb, xd).double()
    Xs = torch.tensor(X[si])
    errs = []
    for b in range(n_theta):
        ref = torch.zeros(len(si), dtype=torch.float64, device="cuda")
        xb = torch.tensor(xs[b], dtype=torch.float64, device="cuda")
        for c0 in range(0, N, 25000):
            K = pkg.eval_dense(Xs, torch.tensor(X[c0:c0 + 25000]), th[b], w.kind, w.d, dtype=torch.float64)
            ref += K @ xb[c0:c0 + 25000]
        got = Y[b][torch.tensor(si, device="cuda")]
        errs.append((torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item())
    return {"levels": inf["levels"], "classes": inf["num_classes"], "far_pairs": inf["far_pairs"],
            "near_pairs": inf["near_pairs"], "leaf_points": leaf, "tol": tol, "build_ms": round(ms_build, 1),
            "apply_ms_per_theta": round(ms_apply / n_theta, 3), "thetas": n_theta, "status": H.status,
            "max_rel_err_vs_dense_fp64": float(f"{max(errs):.3e}"),
            "note": "H(theta) x against dense float64 K(X, X) x, rows of the 4000-point subsample summed over all "
                    "N columns; far blocks PTTK (float32 bulk), near blocks direct"}


def oracle_baseline(w, ranks, n_pts, n_theta, threads_note=True):
    """The oracle, as it stands, on a bounded sample of the workload: Phase 3
    (Algorithm 2) for n_pts sources and n_pts targets, and the batched apply +
    backward (the low-rank form and its adjoint) for n_theta thetas on those
    points.  Its timings depend only on the shapes, so the cores are random
    with the ranks of the GPU build; the oracle's own cross for this workload
    (N-independent, minutes of CPU) is not part of the sample."""
    import threadpoolctl

    from oracle import pttk as opttk

    rng = np.random.default_rng(21)
    n = [w.n_spatial] * w.d + [w.n_param] * w.d_theta + [w.n_spatial] * w.d
    cores = [rng.standard_normal((ranks[k], n[k], ranks[k + 1])) / np.sqrt(ranks[k] * n[k]) for k in range(len(n))]
    bs, bt, bth = (np.asarray(b, float) for b in (w.box_s, w.box_t, w.box_theta))
    X = rng.uniform(bs[:, 0], bs[:, 1], (n_pts, w.d))
    Y = rng.uniform(bt[:, 0], bt[:, 1], (n_pts, w.d))
    d, dt = w.d, w.d_theta
    t0 = time.perf_counter()
    S = opttk.phase3_source(opttk.factor_values(X, bs, w.n_spatial), cores[:d])
    T = opttk.phase3_target(opttk.factor_values(Y, bt, w.n_spatial), cores[d + dt:])
    t_p3 = time.perf_counter() - t0
    th = rng.uniform(bth[:, 0], bth[:, 1], (n_theta, dt))
    xb = rng.standard_normal((n_pts, n_theta))
    gb = rng.standard_normal((n_pts, n_theta))
    t0 = time.perf_counter()
    Hs = [opttk.online_H(cores[d:d + dt], t, bth, w.n_param) for t in th]
    dHs = [opttk.online_dH(cores[d:d + dt], t, bth, w.n_param) for t in th]
    opttk.apply_batched(S, Hs, T, xb)
    opttk.backward_batched(S, Hs, dHs, T, xb, gb)
    t_ag = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    # scaled to the workload: Phase 3 linear in N, the apply + backward in N * B
    t_p3_full = t_p3 * (w.n_src + w.n_tgt) / (2 * n_pts)
    t_ag_full = t_ag * (w.n_src / n_pts) * (w.n_theta / n_theta)
    return {"value": round((w.n_src + w.n_tgt) / (t_p3_full + t_ag_full), 3), "unit": "rows/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"oracle Phase 3 on {n_pts} + {n_pts} points ({t_p3:.1f} s) and batched apply + backward "
                      f"for {n_theta} thetas on them ({t_ag:.1f} s), float64 NumPy, cores random with the GPU "
                      f"build's ranks {list(ranks)}; scaled linearly to {w.n_src} + {w.n_tgt} points and "
                      f"{w.n_theta} thetas.  Excludes the N-independent cross (the GPU step includes it).",
            "phase3_rows_per_s": round(2 * n_pts / t_p3, 1),
            "apply_grad_theta_per_s": round(n_theta * (n_pts / w.n_src) / t_ag, 4),
            "host_cpus": len(os.sched_getaffinity(0))}


def bench_batched(args, torch, pkg):
    """The whole hot path at 1M + 1M points and B = 4096 theta samples."""
    w = synth.WORKLOADS["matern_batched"]
    X, Y = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    B = th.shape[0]
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    xb = torch.randn((B, w.n_tgt), generator=gen, device="cuda", dtype=torch.float32)
    gb = torch.randn((B, w.n_src), generator=gen, device="cuda", dtype=torch.float32)
    kw = dict(kind=w.kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta, n_spatial=w.n_spatial,
              n_param=w.n_param, tol=w.tol, dtype=torch.float32, seed=0, max_sweeps=w.extra["max_sweeps"])

    def step():
        kern = pkg.TTKernel.build_offline(Xd, Yd, **kw)
        Yo, Wv = kern.apply(thd, xb, save_w=True)
        kern.apply_backward(thd, gb, W=Wv)
        return kern

    for i in range(args.warmup):
        kern = step()
        print(f"warmup {i} done: status {kern.status} ranks {kern.info()['ranks']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        kern = step()
        print(f"step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    inf = kern.info()
    rs, rt = kern.r_s, kern.r_t
    res = base_result(w, args, (w.n_src + w.n_tgt) / (ms / 1000.0), "rows/s", ms, B,
                      {"max_sweeps": w.extra["max_sweeps"]})
    res.update({"build_status": "converged" if kern.status == 0 else "not converged (sweep or rank cap)",
                "ranks": inf["ranks"], "cross_ranks": inf["cross_ranks"], "cross_sweeps": inf["sweeps"],
                "sampled_error": float(f"{inf['sampled_error']:.3e}"), "kernel_evals": inf["kernel_evals"],
                "kernel_evals_per_s": round(inf["kernel_evals"] / (inf["t_cross_ms"] * 1e-3), 1),
                "t_cross_ms": round(inf["t_cross_ms"], 2), "t_round_ms": round(inf["t_round_ms"], 2)})
    if args.steps_only:
        return res
    print("timing the phases", file=sys.stderr, flush=True)
    # ---- Phase 3 alone (one launch per side), HIP events on the current stream
    Xs, Ys = Xd.t().contiguous(), Yd.t().contiguous()
    U_out = torch.empty((w.n_src, rs), dtype=torch.float32, device="cuda")
    V_out = torch.empty((w.n_tgt, rt), dtype=torch.float32, device="cuda")
    ms_u = time_events(lambda: kern.factor_rows_soa(Xs, 0, U_out), 10, torch)
    ms_v = time_events(lambda: kern.factor_rows_soa(Ys, 1, V_out), 10, torch)
    r = inf["ranks"]
    d, dth = w.d, w.d_theta
    fl_u = w.n_src * phase3_flops_per_point(r[:d + 1], w.n_spatial)
    fl_v = w.n_tgt * phase3_flops_per_point(r[d + dth:][::-1], w.n_spatial)
    # ---- the projection W = F^T X (the roofline kernel), one launch per call
    Wv = torch.empty((B, rt), dtype=torch.float32, device="cuda")
    Av = torch.empty((B, rs), dtype=torch.float32, device="cuda")
    ms_pv = time_events(lambda: kern.project(xb, side=1, out=Wv), 5, torch)
    ms_pu = time_events(lambda: kern.project(gb, side=0, out=Av), 5, torch)
    fl_proj = 2.0 * B * (w.n_tgt * rt + w.n_src * rs) / 2          # average of the two launches
    ms_proj = (ms_pv + ms_pu) / 2
    # ---- batched apply + backward, and the plain per-theta apply
    def fwd_bwd():
        Yo, W_ = kern.apply(thd, xb, save_w=True)
        kern.apply_backward(thd, gb, W=W_)
    ms_ag = time_events(fwd_bwd, 5, torch)
    bytes_ag = 2 * 4 * (w.n_src * rs + w.n_tgt * rt) + 2 * 4 * B * (w.n_src + w.n_tgt)
    flops_ag = 4 * B * (w.n_src * rs + w.n_tgt * rt)        # four tall products, 2 N r B each
    nplain = 64
    ms_plain = time_events(lambda: kern.apply_plain(thd[:nplain], xb[:nplain]), 2, torch)
    bytes_plain = nplain * 4 * (w.n_tgt * (rt + 1) + w.n_src * (rs + 1))
    # ---- accuracy against dense float64 K: 64 thetas x a 4000 x 4000 subsample
    print("accuracy against dense K", file=sys.stderr, flush=True)
    rng = np.random.default_rng(11)
    si = np.sort(rng.choice(w.n_src, 4000, replace=False))
    ti = np.sort(rng.choice(w.n_tgt, 4000, replace=False))
    cols = np.linspace(0, B - 1, 64).astype(int)
    U, V = kern.factors()
    M = kern.online_core(thd[torch.tensor(cols, device="cuda")])
    Us, Vs = U[si].double(), V[ti].double()
    Xsub, Ysub = torch.tensor(X[si]), torch.tensor(Y[ti])
    errs = []
    for j, b in enumerate(cols):
        K = pkg.eval_dense(Xsub, Ysub, th[b], w.kind, w.d, dtype=torch.float64)
        errs.append((torch.linalg.norm(K - Us @ M[j].double() @ Vs.t()) / torch.linalg.norm(K)).item())
    errs = np.array(errs)
    res.update({
        "phase3_rows_per_s": round((w.n_src + w.n_tgt) / ((ms_u + ms_v) * 1e-3), 1),
        "phase3_ms": {"sources": round(ms_u, 4), "targets": round(ms_v, 4)},
        "phase3_tflops": round((fl_u + fl_v) / ((ms_u + ms_v) * 1e-3) / 1e12, 2),
        "apply_grad_ms": round(ms_ag, 3), "apply_grad_GBps": round(bytes_ag / (ms_ag * 1e-3) / 1e9, 1),
        "apply_grad_TFLOPs": round(flops_ag / (ms_ag * 1e-3) / 1e12, 2),
        "apply_grad_frac_fp32_mfma": round(flops_ag / (ms_ag * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
        "plain_apply_GBps": round(bytes_plain / (ms_plain * 1e-3) / 1e9, 1),
        "batched_vs_plain_theta_per_s": round((B / ms_ag) / (nplain / ms_plain), 3),
        "plain_note": f"plain per-theta forward apply timed on {nplain} of the {B} thetas; the batched figure "
                      "is forward + backward",
        "max_rel_err_vs_dense_fp64": float(f"{errs.max():.3e}"),
        "median_rel_err_vs_dense_fp64": float(f"{np.median(errs):.3e}"),
        "accuracy_note": "relative Frobenius error of U M(theta) V^T against dense float64 K on a 4000 x 4000 "
                         "subsample, for 64 of the thetas (evenly spaced in the sample)",
    })
    achieved = fl_proj / (ms_proj * 1e-3) / 1e12
    res["roofline"] = {
        "kernel": "k_reduce_mfma_dma<5, 1> (tt_kernel_project: W = V^T X and A = U^T G, float32 MFMA)",
        "bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": PROJECT_TRAFFIC,
        "avg_launch_ms": round(ms_proj, 4),
        "algorithmic": f"2 N r B flops per launch: N = {w.n_tgt} points, B = {B}, r = {rt} (W = V^T X) and "
                       f"r = {rs} (A = U^T G), averaged; each call also runs a {B * max(rs, rt)}-entry "
                       "fixed-order sum of the chunk partials (about 0.1% of its time), inside the timing",
        "traffic_note": PROJECT_TRAFFIC_NOTE,
    }
    # ---- the paper's Phase 4 (TT-Round through S and T, on a tall-skinny QR)
    # on the same kernel handle, after every other measurement (it replaces U, V and the
    # parameter cores of the handle)
    print("phase 4", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    kern.phase4_round(w.tol)
    torch.cuda.synchronize()
    ms4 = (time.perf_counter() - t4) * 1000.0
    inf4 = kern.info()
    U4, V4 = kern.factors()
    M4 = kern.online_core(thd[torch.tensor(cols, device="cuda")])
    U4s, V4s = U4[si].double(), V4[ti].double()
    errs4 = []
    for j, b in enumerate(cols):
        K = pkg.eval_dense(Xsub, Ysub, th[b], w.kind, w.d, dtype=torch.float64)
        errs4.append((torch.linalg.norm(K - U4s @ M4[j].double() @ V4s.t()) / torch.linalg.norm(K)).item())
    res["phase4"] = {
        "ms": round(ms4, 2), "ranks": inf4["ranks"][w.d:w.d + w.d_theta + 1],
        "ranks_before": r[w.d:w.d + w.d_theta + 1],
        "max_rel_err_vs_dense_fp64": float(f"{max(errs4):.3e}"),
        "note": "Phase 4 of Algorithm 2 at eps = tol on the final build: tall-skinny QR of U and V (1M rows "
                "each), TT-Round of the small TT, U' = Q_S A_S and V' = Q_T A_T^T; error on the same subsample "
                "and thetas as above; not part of the timed step"}
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = oracle_baseline(w, inf["ranks"], args.cpu_points or 200_000, 256)
    return res


def bench_ttk_e1(args, torch, pkg):
    """The non-parametric TTK experiment (Section 4.1): every kernel of Table 1
    at fixed l = 1 on 10^4 + 10^4 points in [0,1]^3 and [2,3]^3, n = 27,
    tol 1e-9, float64.  Per kernel: the compression rank, the offline build
    time, the 2-norm relative error of U V^T against dense K (power
    iteration) and, for context, the error of the truncated SVD at the same
    rank (sigma_{r+1} / sigma_1 from a randomized range finder)."""
    w = synth.WORKLOADS["ttk_e1"]
    X, Y = synth.points(w, seed=0)
    Xd, Yd = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(3)
    rows, total_ms = [], 0.0
    for kind, tf in w.extra["kernels"]:
        kw = dict(kind=kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=[], n_spatial=w.n_spatial, tol=w.tol,
                  dtype=torch.float64, seed=0, theta_fixed=tf)
        for _ in range(args.warmup):
            pkg.TTKernel.build_offline(Xd, Yd, **kw)
        ms = time_wall(lambda: pkg.TTKernel.build_offline(Xd, Yd, **kw), max(args.steps, 1), torch)
        kern = pkg.TTKernel.build_offline(Xd, Yd, **kw)
        total_ms += ms
        inf = kern.info()
        U, V = kern.factors()
        K = pkg.eval_dense(Xd, Yd, tf if tf is not None else [], kind, w.d, dtype=torch.float64)
        E = K - U @ V.t()

        def norm2(A, its=40):
            v = torch.randn((A.shape[1],), generator=gen, device="cuda", dtype=torch.float64)
            s = 0.0
            for _ in range(its):
                u = A @ v
                v = A.t() @ u
                s = torch.linalg.norm(v).sqrt().item()
                v = v / torch.linalg.norm(v)
            return s
        r = kern.r_s
        Om = torch.randn((K.shape[1], r + 20), generator=gen, device="cuda", dtype=torch.float64)
        Q, _ = torch.linalg.qr(K @ Om)
        for _ in range(2):
            Q, _ = torch.linalg.qr(K @ (K.t() @ Q))
        sv = torch.linalg.svdvals(Q.t() @ K)
        rows.append({"kernel": kind, "theta": tf, "rank": r, "ranks": inf["ranks"], "build_ms": round(ms, 2),
                     "tt_error_2norm": float(f"{norm2(E) / norm2(K):.3e}"),
                     "svd_error_2norm_same_rank": float(f"{(sv[r] / sv[0]).item():.3e}"),
                     "kernel_evals": inf["kernel_evals"], "status": kern.status})
        print(f"{kind}: rank {r} build {ms:.1f} ms error {rows[-1]['tt_error_2norm']:.2e}", file=sys.stderr,
              flush=True)
        del K, E
    n_k = len(rows)
    res = base_result(w, args, n_k * (w.n_src + w.n_tgt) / (total_ms / 1000.0), "rows/s", total_ms / n_k, 1,
                      {"variant": "TTK (d_theta = 0)", "kernels": n_k})
    res["note"] = ("value: offline U/V rows per second, (N_s + N_t) per kernel over the mean build time of the "
                   f"{n_k} kernels; ms_per_step is that mean")
    res["per_kernel"] = rows
    return res


def bench_pairs(args, torch, pkg):
    """Uneven batch: 512 box pairs of an FMM-like interaction list, 256 thetas."""
    base = synth.WORKLOADS["matern_batched"]
    pairs = synth.uneven_pairs()
    rng = np.random.default_rng(0)
    xs, ys = [], []
    so = to = 0
    for p in pairs:
        bs, bt = np.asarray(p["box_s"]), np.asarray(p["box_t"])
        xs.append(np.clip(rng.uniform(bs[:, 0], bs[:, 1], (p["n_src"], 3)).astype(np.float32), bs[:, 0], bs[:, 1]))
        ys.append(np.clip(rng.uniform(bt[:, 0], bt[:, 1], (p["n_tgt"], 3)).astype(np.float32), bt[:, 0], bt[:, 1]))
        p["src_off"], p["tgt_off"] = so, to
        so += p["n_src"]
        to += p["n_tgt"]
    # (np.clip against the float64 box bounds returns float64: the points are
    # handed over in the batch's float32, as its Phase 3 entry point expects)
    Xd = torch.tensor(np.vstack(xs), dtype=torch.float32, device="cuda")
    Yd = torch.tensor(np.vstack(ys), dtype=torch.float32, device="cuda")
    B = 256
    th = synth.thetas(base, count=B, seed=1)
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    xb = torch.randn((B, to), generator=gen, device="cuda")
    gb = torch.randn((B, so), generator=gen, device="cuda")
    out = (torch.empty((B, so), device="cuda"), torch.empty((B, to), device="cuda"),
           torch.empty((B, 2), device="cuda"))
    kw = dict(kind="matern", d=3, box_theta=base.box_theta, n_spatial=14, n_param=14, tol=1e-6,
              dtype=torch.float32, seed=0)

    def step():
        bt = pkg.TTBatch.build(pairs, Xd, Yd, **kw)
        bt.apply(thd, xb, G=gb, out=out)
        return bt

    for i in range(args.warmup):
        bt = step()
        print(f"warmup {i} done: {bt.info()['num_classes']} classes", file=sys.stderr, flush=True)
    ms = time_wall(step, args.steps, torch)
    bt = step()
    inf = bt.info()
    Xs, Ys = Xd.t().contiguous(), Yd.t().contiguous()
    ms_p3 = time_events(lambda: bt.refactor_soa(Xs, Ys), 5, torch)
    ms_ag = time_events(lambda: bt.apply(thd, xb, G=gb, out=out), 5, torch)
    rs_rows = sum(p["n_src"] * inf["class_ranks"][c][3] for p, c in zip(pairs, inf["class_of_pair"]))
    rt_rows = sum(p["n_tgt"] * inf["class_ranks"][c][5] for p, c in zip(pairs, inf["class_of_pair"]))
    bytes_ag = 2 * 4 * (rs_rows + rt_rows) + 2 * 4 * B * (so + to)
    gbps = bytes_ag / (ms_ag * 1e-3) / 1e9
    res = {"metric": METRIC, "value": round((so + to) / (ms / 1000.0), 1), "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uneven_pairs", "kernel": "matern", "d": 3, "d_theta": 2, "pairs": len(pairs),
                      "N_s": so, "N_t": to, "n_spatial": 14, "n_param": 14, "tol": 1e-6, "n_theta": B,
                      "parallelism": "single GPU"},
           "classes": inf["num_classes"], "kernel_evals": inf["kernel_evals"],
           "t_cross_ms": round(inf["t_cross_ms"], 1), "t_round_ms": round(inf["t_round_ms"], 1),
           "phase3_all_pairs_ms": round(ms_p3, 3), "phase3_rows_per_s": round((so + to) / (ms_p3 * 1e-3), 1),
           "factor_grid": inf["factor_grid"], "reduce_rows": inf["reduce_rows"], "graph": inf["graph"],
           "apply_grad_ms": round(ms_ag, 3), "apply_grad_GBps": round(gbps, 1)}
    res["roofline"] = {"kernel": "batched apply + backward over all pairs", "bound": "hbm", "achieved": round(gbps, 1),
                       "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                       "traffic": None}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="matern_batched",
                    help="matern_batched (default), matern32_d3, se_d2_fp64, matern_global, uneven_pairs, ttk_e1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--steps-only", action="store_true", help="time the steps only (profiling runs)")
    ap.add_argument("--cpu-points", type=int, default=None,
                    help="points per side of the oracle's sample (default: 200000 for matern_batched, 2000 "
                         "otherwise)")
    ap.add_argument("--tol", type=float, default=None, help="override the workload's tolerance")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the path would shard by rows of U and V, with one small "
              "all-reduce per apply direction, but runs on more than one GPU are not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2406_06344_amd as pkg

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = 1 << 28                                   # 2^28 floats = 1 GiB read + 1 GiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 3}), flush=True)
        return
    other = {"matern_global": bench_global, "matern_batched": bench_batched, "uneven_pairs": bench_pairs,
             "ttk_e1": bench_ttk_e1}
    if args.workload in other:
        print(json.dumps(other[args.workload](args, torch, pkg)), flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    if args.tol is not None:
        w = synth.small(w, w.n_src, w.n_tgt, tol=args.tol)
    X, Y = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    B = th.shape[0]
    dtype = torch.float64 if w.fp64 else torch.float32
    Xd = torch.tensor(X, dtype=dtype, device="cuda")
    Yd = torch.tensor(Y, dtype=dtype, device="cuda")
    thd = torch.tensor(th, dtype=dtype, device="cuda")
    xb = torch.tensor(synth.rhs(w.n_tgt, B, seed=2, fp64=w.fp64).T.copy(), dtype=dtype, device="cuda")
    gb = torch.tensor(synth.rhs(w.n_src, B, seed=3, fp64=w.fp64).T.copy(), dtype=dtype, device="cuda")
    build_kw = dict(kind=w.kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta,
                    n_spatial=w.n_spatial, n_param=w.n_param, tol=w.tol, dtype=dtype, seed=0,
                    kernel_const=w.const)

    def step():
        kern = pkg.TTKernel.build_offline(Xd, Yd, **build_kw)
        Yo, W = kern.apply(thd, xb, save_w=True)
        dX, dth = kern.apply_backward(thd, gb, W=W)
        return kern, Yo, dX, dth

    for i in range(args.warmup):
        kern, *_ = step()
        print(f"warmup {i} done: ranks {kern.info()['ranks']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        kern, Yo, dX, dth = step()
        print(f"step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    rows = w.n_src + w.n_tgt
    value = rows / (ms_per_step / 1000.0)
    inf = kern.info()
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.fp64 else "f32", "data": "synthetic",
        "config": {"workload": w.name, "kernel": w.kind, "d": w.d, "d_theta": w.d_theta,
                   "N_s": w.n_src, "N_t": w.n_tgt, "n_spatial": w.n_spatial, "n_param": w.n_param,
                   "tol": w.tol, "n_theta": B, "parallelism": "single GPU"},
        "ranks": inf["ranks"], "cross_ranks": inf["cross_ranks"], "cross_sweeps": inf["sweeps"],
        "kernel_evals": inf["kernel_evals"], "t_cross_ms": round(inf["t_cross_ms"], 2),
        "t_round_ms": round(inf["t_round_ms"], 2), "t_factor_ms": round(inf["t_factor_ms"], 3),
    }
    if args.steps_only:
        print(json.dumps(result), flush=True)
        return

    # ---- Phase 3 alone (one kernel launch per side), HIP events on the current stream
    Xs = Xd.t().contiguous()
    Ys = Yd.t().contiguous()
    U_out = torch.empty((w.n_src, kern.r_s), dtype=dtype, device="cuda")
    V_out = torch.empty((w.n_tgt, kern.r_t), dtype=dtype, device="cuda")
    reps = 20
    ms_u = time_events(lambda: kern.factor_rows_soa(Xs, 0, U_out), reps, torch)
    ms_v = time_events(lambda: kern.factor_rows_soa(Ys, 1, V_out), reps, torch)
    d, dt = w.d, w.d_theta
    r = inf["ranks"]
    fl_u = w.n_src * phase3_flops_per_point(r[:d + 1], w.n_spatial)
    fl_v = w.n_tgt * phase3_flops_per_point(r[d + dt:][::-1], w.n_spatial)
    tf_u = fl_u / (ms_u * 1e-3) / 1e12
    tf_v = fl_v / (ms_v * 1e-3) / 1e12
    phase3_rows = rows / ((ms_u + ms_v) * 1e-3)

    # ---- apply: batched forward + backward vs plain per-theta forward
    es = 8 if w.fp64 else 4
    rs, rt = kern.r_s, kern.r_t
    ms_batched = time_events(lambda: kern.apply_backward(thd, gb, W=kern.apply(thd, xb, save_w=True)[1]), 10,
                             torch)
    ms_plain = time_events(lambda: kern.apply_plain(thd, xb), 10, torch)
    bytes_batched = 2 * es * (w.n_src * rs + w.n_tgt * rt) + 2 * es * B * (w.n_src + w.n_tgt)
    bytes_plain = B * es * (w.n_tgt * (rt + 1) + w.n_src * (rs + 1))
    gbps_batched = bytes_batched / (ms_batched * 1e-3) / 1e9
    gbps_plain = bytes_plain / (ms_plain * 1e-3) / 1e9
    # per theta: the batched form does forward AND backward
    thetas_per_s_batched = B / (ms_batched * 1e-3)
    thetas_per_s_plain = B / (ms_plain * 1e-3)

    # ---- accuracy against dense float64 K on a 4k x 4k subsample
    rng = np.random.default_rng(11)
    si = np.sort(rng.choice(w.n_src, 4000, replace=False))
    ti = np.sort(rng.choice(w.n_tgt, 4000, replace=False))
    U, V = kern.factors()
    M = kern.online_core(thd)
    errs = []
    for b in range(B):
        K = pkg.eval_dense(torch.tensor(X[si]), torch.tensor(Y[ti]), th[b], w.kind, w.d, dtype=torch.float64,
                           kernel_const=w.const)
        Kh = U[si].double() @ M[b].double() @ V[ti].double().t()
        errs.append((torch.linalg.norm(K - Kh) / torch.linalg.norm(K)).item())

    result.update({
        "phase3_rows_per_s": round(phase3_rows, 1),
        "phase3_ms": {"sources": round(ms_u, 4), "targets": round(ms_v, 4)},
        "phase3_tflops": {"sources": round(tf_u, 2), "targets": round(tf_v, 2)},
        "apply_grad_GBps": round(gbps_batched, 1), "plain_apply_GBps": round(gbps_plain, 1),
        "apply_grad_ms": round(ms_batched, 4), "plain_apply_ms": round(ms_plain, 4),
        "batched_vs_plain_theta_per_s": round(thetas_per_s_batched / thetas_per_s_plain, 3),
        "max_rel_err_vs_dense_fp64": float(f"{max(errs):.3e}"),
        "accuracy_note": "relative Frobenius error of U M V^T against dense float64 K on a 4000 x 4000 "
                         "subsample, worst of the theta samples",
    })
    # the dominant N-dependent kernel: Phase 3 (k_factor_mfma), one launch per side;
    # achieved = algorithmic flops of both launches / their summed durations
    tf_both = (fl_u + fl_v) / ((ms_u + ms_v) * 1e-3) / 1e12
    # algorithmic HBM bytes per launch (average): d float32 coordinates in and
    # r float32 entries out per point (the cores stay in L2)
    rk = inf["ranks"]
    r_u, r_v = rk[w.d], rk[w.d + w.d_theta]
    alg_bytes = (w.n_src * 4 * (w.d + r_u) + w.n_tgt * 4 * (w.d + r_v)) / 2
    result["roofline"] = {
        "kernel": "k_factor_mfma (Phase 3, source and target launches)", "bound": "mfma",
        "achieved": round(tf_both, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(tf_both / FP32_PEAK_TFLOPS, 4), "traffic": TRAFFIC,
        "avg_launch_ms": round((ms_u + ms_v) / 2, 4),
        "traffic_note": "HBM bytes per launch: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (scales from a plain "
                        "1 GiB copy), average of the two launches; algorithmic "
                        f"{alg_bytes / 1e6:.2f} MB (points in, rows out, float32)",
        "algorithmic": f"{fl_u / w.n_src:.0f} (source) and {fl_v / w.n_tgt:.0f} (target) flop per point, "
                       f"{w.n_src} and {w.n_tgt} points per launch",
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, X, Y, th, args.cpu_points or 2000)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
