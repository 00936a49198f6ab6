"""Full-size GPU checks, in the launch configurations bench.py times.

- matern32_d3 (the benchmark workload, 100k + 100k points, float32): the
  oracle replays the GPU's cross decisions (each must lie in the oracle's own
  tie band) and reaches the same index sets, ranks and stopping error; the
  free-running oracle's decision log, stored in tests/golden (written by
  tests/golden/make_oracle_offline.py from oracle/ alone), must agree up to
  the first step that is a tie within rounding.  Sampled rows of U and V, and
  the apply and backward on inputs supported on sampled points, are compared
  with the oracle computing those entries one by one from the replay's cores.
- se_d2_fp64 (2000 + 2000 points, float64): everything against a live oracle
  run, including U M V^T on the full 2000 x 2000 block.
- matern_batched (1M + 1M points, 4096 thetas, the default benchmark):
  against the stored free-running oracle (decisions up to the first tie,
  sampled TT entries, U M V^T, apply, dX and dtheta on sampled rows), the
  error against dense K, the adjoint identity and batched = plain apply.
- The Global-1 (200k points) and uneven-pair (512 pairs, 15M points, 256
  thetas) workloads: properties that hold at any size (orthonormal Q,
  Q R = [U V], PSD W, the adjoint identity of the backward), since the
  oracle's cross for them takes far longer than a test.  Their oracle parity
  is checked at reduced sizes in test_gpu_global.py and test_gpu_batch.py.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import synth
from oracle import dense as odense
from oracle import driver as odriver
from oracle import kernels as okernels
from oracle import pttk as opttk
from oracle import tt as ott

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return odense.rel_fro(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


def mx(a, b):
    """largest entry error over the largest entry of the reference"""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def adjoint_gap(dX, x, g, y, chunk=256):
    """max over b of |<dX_b, x_b> - <g_b, y_b>| / (|g_b| |y_b|), in float64, by chunks of thetas."""
    worst = 0.0
    for b0 in range(0, x.shape[0], chunk):
        sl = slice(b0, b0 + chunk)
        lhs = (dX[sl].double() * x[sl].double()).sum(dim=1)
        rhs = (g[sl].double() * y[sl].double()).sum(dim=1)
        scale = g[sl].double().norm(dim=1) * y[sl].double().norm(dim=1)
        worst = max(worst, ((lhs - rhs).abs() / scale).max().item())
    return worst


def test_benchmark_workload_full_size_matches_oracle():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    from oracle import cross as ocross
    w = synth.WORKLOADS["matern32_d3"]
    say(f"[full] {w.name}: build on {w.n_src} + {w.n_tgt} points")
    g = np.load(os.path.join(GOLDEN, "matern32_d3_oracle.npz"))
    X, Y = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    B = th.shape[0]
    kern = pkg.TTKernel.build_offline(torch.tensor(X, dtype=torch.float32), torch.tensor(Y, dtype=torch.float32),
                                      kind=w.kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta,
                                      n_spatial=w.n_spatial, n_param=w.n_param, tol=w.tol, dtype=torch.float32,
                                      seed=0)
    inf = kern.info()
    say(f"  ranks {inf['ranks']} cross {inf['cross_ranks']} sweeps {inf['sweeps']} min margin {inf['min_margin']:.2e}")
    L, R, log = kern.cross_record()
    D = inf["D"]
    d, dt = w.d, w.d_theta
    P = okernels.Problem(w.kind, w.d, w.box_s, w.box_t, w.box_theta, w.n_spatial, w.n_param)
    # 1. against the free-running oracle (stored): identical decisions up to
    #    the first step whose top-2 margin is a tie within rounding (R6); when
    #    the whole sequence agrees, the index sets, ranks and sweep count are
    #    the stored ones too
    lp, lm = g["log_pivot"], g["log_margin"]
    n_same = 0
    for a, r in zip(lp, log):
        if (int(a[0]), int(a[1]), int(a[2])) != (r["pivot_row"], r["pivot_col"], int(r["added"])):
            assert lm[n_same] < 1e-9, (n_same, lm[n_same])
            break
        n_same += 1
    say(f"  decisions {len(log)}, identical to the free-running oracle for the first {n_same} "
        f"(free-running: {len(lp)} decisions, cross ranks {list(g['cross_ranks'])})")
    if n_same == len(lp) == len(log):
        assert inf["cross_ranks"] == list(g["cross_ranks"]) and inf["sweeps"] == int(g["sweeps"])
        for k in range(1, D):
            assert np.array_equal(L[k], g[f"left{k}"]), k
            assert np.array_equal(R[k], g[f"right{k}"]), k
        say("  index sets identical to the free-running oracle's")
    # 2. the oracle replays the GPU's choices (no GPU residual value enters):
    #    each lies in the oracle's own tie band, widened only by the rounding
    #    noise the oracle measures on its own residuals, and the replay
    #    reaches the same index sets, ranks, sweep count and stopping error
    forced = [{"sample_pos": r["sample_pos"], "pivot_row": r["pivot_row"], "pivot_col": r["pivot_col"],
               "added": r["added"]} for r in log]
    cross_cores, rep = ocross.greedy_cross(ocross.Entries(P.entries, P.n), w.tol, seed=0, forced=forced)
    bad = [i for i, r in enumerate(rep["log"])
           if not (r["replay_sample_ok"] and r["replay_search_ok"] and r["replay_add_ok"])]
    assert not bad, bad[:5]
    assert inf["cross_ranks"] == rep["ranks"] and inf["sweeps"] == rep["sweeps"]
    for k in range(1, D):
        assert np.array_equal(L[k], rep["L"][k]), k
        assert np.array_equal(R[k], rep["R"][k]), k
    say(f"  stopping error: gpu {inf['sampled_error']:.6e} oracle replay {rep['error']:.6e}")
    assert abs(inf["sampled_error"] - rep["error"]) <= 1e-4 * rep["error"]
    # rounded cores from the replay's cross: same ranks, and the two TTs agree
    # at sampled multi-indices
    Go = opttk.round_and_gauge(cross_cores, w.tol, d, dt)
    assert inf["ranks"] == [1] + [c.shape[2] for c in Go]
    Gg = kern.cores()
    rng = np.random.default_rng(21)
    idx = np.stack([rng.integers(0, nj, 20000) for nj in P.n], axis=1)
    vo = ott.evaluate(Go, idx)
    assert np.abs(ott.evaluate(Gg, idx) - vo).max() <= 1e-10 * np.abs(vo).max()
    # sampled rows of U and V against the oracle's Phase 3 at those points
    si = np.sort(rng.choice(w.n_src, 2000, replace=False))
    ti = np.sort(rng.choice(w.n_tgt, 2000, replace=False))
    S = opttk.phase3_source(opttk.factor_values(X[si], P.box_s, w.n_spatial), Go[:d])
    T = opttk.phase3_target(opttk.factor_values(Y[ti], P.box_t, w.n_spatial), Go[d + dt:])
    U, V = kern.factors()
    Ug, Vg = U[si].double().cpu().numpy(), V[ti].double().cpu().numpy()
    eu, ev = rel(Ug, S), rel(Vg, T)
    mu, mv = mx(Ug, S), mx(Vg, T)
    say(f"  sampled rows: U {eu:.2e} (max entry {mu:.2e}) V {ev:.2e} (max entry {mv:.2e})")
    assert max(eu, ev, mu, mv) <= 1e-5
    # apply + backward in the benchmark's configuration, inputs supported on the samples
    xs = synth.rhs(2000, B, seed=2)
    gs = synth.rhs(2000, B, seed=3)
    xb = torch.zeros((B, w.n_tgt), dtype=torch.float32, device="cuda")
    gb = torch.zeros((B, w.n_src), dtype=torch.float32, device="cuda")
    xb[:, torch.tensor(ti)] = torch.tensor(xs.T, dtype=torch.float32, device="cuda")
    gb[:, torch.tensor(si)] = torch.tensor(gs.T, dtype=torch.float32, device="cuda")
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    Yo, Wv = kern.apply(thd, xb, save_w=True)
    dX, dth = kern.apply_backward(thd, gb, W=Wv)
    Hs = [opttk.online_H(Go[d:d + dt], t, P.box_theta, w.n_param) for t in th]
    dHs = [opttk.online_dH(Go[d:d + dt], t, P.box_theta, w.n_param) for t in th]
    y_o = np.stack([S @ (Hs[b] @ (T.T @ xs[:, b])) for b in range(B)])
    dx_o = np.stack([T @ (Hs[b].T @ (S.T @ gs[:, b])) for b in range(B)])
    dth_o = np.array([[(S.T @ gs[:, b]) @ dHs[b][j] @ (T.T @ xs[:, b]) for j in range(dt)] for b in range(B)])
    yg = Yo[:, torch.tensor(si)].double().cpu().numpy()
    xg = dX[:, torch.tensor(ti)].double().cpu().numpy()
    tg = dth.double().cpu().numpy()
    errs = [rel(yg, y_o), rel(xg, dx_o), rel(tg, dth_o), mx(yg, y_o), mx(xg, dx_o), mx(tg, dth_o)]
    say("  apply, dX, dtheta: rel Frobenius %.2e %.2e %.2e, max entry %.2e %.2e %.2e" % tuple(errs))
    assert max(errs) <= 1e-5


def test_fp64_workload_full_size_matches_oracle():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    w = synth.WORKLOADS["se_d2_fp64"]
    say(f"[full] {w.name}")
    X, Y = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    P = okernels.Problem(w.kind, w.d, w.box_s, w.box_t, w.box_theta, w.n_spatial, w.n_param)
    out = odriver.offline(P, X, Y, w.tol, seed=0)
    kern = pkg.TTKernel.build_offline(torch.tensor(X), torch.tensor(Y), kind=w.kind, d=w.d, box_s=w.box_s,
                                      box_t=w.box_t, box_theta=w.box_theta, n_spatial=w.n_spatial,
                                      n_param=w.n_param, tol=w.tol, dtype=torch.float64, seed=0)
    inf = kern.info()
    assert inf["ranks"] == out["ranks"]
    U, V = kern.factors()
    M = kern.online_core(torch.tensor(th, device="cuda"))
    d = w.d
    worst_o = worst_g = 0.0
    for b in range(th.shape[0]):
        H = opttk.online_H(out["param"], th[b], P.box_theta, w.n_param)
        Ko = out["S"] @ H @ out["T"].T
        Kg = (U @ M[b] @ V.t()).cpu().numpy()
        e = rel(Kg, Ko)
        assert e <= 1e-10, (b, e)
        K = odense.dense_K(w.kind, X, Y, th[b])
        worst_o = max(worst_o, rel(Ko, K))
        worst_g = max(worst_g, rel(Kg, K))
    say(f"  |U M V^T - K| / |K| (2000 x 2000, worst theta): gpu {worst_g:.3e} oracle {worst_o:.3e}")
    assert abs(worst_g - worst_o) <= 1e-9


def test_global_workload_full_size_properties():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    w = synth.WORKLOADS["matern_global"]
    say(f"[full] {w.name}: Global-1 on {w.n_src} points")
    X, _ = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)[:4]
    kern = pkg.TTKernel.build_offline(torch.tensor(X, dtype=torch.float32), None, kind=w.kind, d=w.d,
                                      box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta, n_spatial=w.n_spatial,
                                      n_param=w.n_param, tol=w.tol, dtype=torch.float32, seed=0,
                                      symmetric_psd=True)
    Q, R = kern.global_factors()
    k = Q.shape[1]
    Qd = Q.double()
    orth = (Qd.t() @ Qd - torch.eye(k, dtype=torch.float64, device="cuda")).abs().max().item()
    U, V = kern.factors()
    A = torch.cat([U, V], dim=1).double()
    resid = (torch.linalg.norm(Qd @ torch.tensor(R, device="cuda") - A) / torch.linalg.norm(A)).item()
    say(f"  k = {k}, |Q^T Q - I| = {orth:.2e}, |QR - [U V]| / |[U V]| = {resid:.2e}")
    assert orth <= 1e-5 and resid <= 1e-6
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    W = kern.global_online(thd).double()
    for b in range(W.shape[0]):
        lam = torch.linalg.eigvalsh(0.5 * (W[b] + W[b].t()))
        assert lam.min().item() >= -1e-6 * lam.abs().max().item()
    x = torch.randn((4, w.n_src), device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    y = kern.global_apply(x, W=kern.global_online(thd)).double()
    for b in range(4):
        yb = Qd @ (W[b] @ (Qd.t() @ x[b].double()))
        assert (torch.linalg.norm(y[b] - yb) / torch.linalg.norm(yb)).item() <= 1e-5
        # x^T (Q W Q^T) x >= 0
        assert (x[b].double() @ y[b]).item() >= -1e-6 * torch.linalg.norm(x[b].double()).item() ** 2 * \
            torch.linalg.eigvalsh(W[b]).abs().max().item()


def test_batched_workload_full_size_matches_oracle():
    """The 1M + 1M point, 4096-theta workload (Matern in (l, nu)) in bench.py's
    launch configuration, against the free-running oracle's offline stage
    stored in tests/golden (written by make_oracle_offline.py from oracle/
    alone; the oracle's cross for it takes about 25 minutes of CPU):
    identical decisions up to the first one that is a tie within rounding
    (R6), then both TTs agree at sampled grid entries to the approximation
    level, and U M V^T, y, dX and dtheta agree with the oracle's S H T^T at
    sampled rows.  Also: converged build, the error against dense K (64
    thetas, 4000 x 4000 subsample) <= 1e-5, the adjoint identity and batched
    = plain apply."""
    torch = _torch()
    import paper_2406_06344_amd as pkg
    w = synth.WORKLOADS["matern_batched"]
    say(f"[full] {w.name}: {w.n_src} + {w.n_tgt} points, {w.n_theta} thetas")
    g = np.load(os.path.join(GOLDEN, "matern_batched_oracle.npz"))
    X, Y = synth.points(w, seed=0)
    th = synth.thetas(w, seed=1)
    B = th.shape[0]
    d, dt = w.d, w.d_theta
    kern = pkg.TTKernel.build_offline(torch.tensor(X, dtype=torch.float32), torch.tensor(Y, dtype=torch.float32),
                                      kind=w.kind, d=w.d, box_s=w.box_s, box_t=w.box_t, box_theta=w.box_theta,
                                      n_spatial=w.n_spatial, n_param=w.n_param, tol=w.tol, dtype=torch.float32,
                                      seed=0, max_sweeps=w.extra["max_sweeps"])
    inf = kern.info()
    say(f"  status {kern.status} ranks {inf['ranks']} cross {inf['cross_ranks']} sweeps {inf['sweeps']} "
        f"error {inf['sampled_error']:.3e}; oracle: ranks {list(g['ranks'])} cross {list(g['cross_ranks'])} "
        f"sweeps {int(g['sweeps'])} error {float(g['error']):.3e}")
    assert kern.status == 0 and bool(g["converged"])
    # 1. decisions against the free-running oracle
    L, R, log = kern.cross_record()
    lp, lm = g["log_pivot"], g["log_margin"]
    n_same = 0
    for a, r in zip(lp, log):
        if (int(a[0]), int(a[1]), int(a[2])) != (r["pivot_row"], r["pivot_col"], int(r["added"])):
            say(f"  first differing decision {n_same} (sweep {r['sweep']}, k {r['k']}): oracle margin "
                f"{lm[n_same]:.2e}, gpu margins {r['sample_margin']:.2e} / {r['search_margin']:.2e}")
            assert min(lm[n_same], r["sample_margin"], r["search_margin"]) < 1e-9, n_same
            break
        n_same += 1
    say(f"  decisions identical to the free-running oracle: {n_same} of {len(log)} (oracle {len(lp)})")
    if n_same == len(lp) == len(log):
        assert inf["cross_ranks"] == list(g["cross_ranks"]) and inf["ranks"] == list(g["ranks"])
    # 2. the two rounded TTs approximate the same grid tensor: sampled entries
    P = okernels.Problem(w.kind, w.d, w.box_s, w.box_t, w.box_theta, w.n_spatial, w.n_param)
    Go = [g[f"core{k}"] for k in range(P.D)]
    Gg = kern.cores()
    rng = np.random.default_rng(21)
    idx = np.stack([rng.integers(0, nj, 4000) for nj in P.n], axis=1)
    exact = P.entries(idx)
    vo, vg = ott.evaluate(Go, idx), ott.evaluate(Gg, idx)
    eo = np.abs(vo - exact).max() / np.abs(exact).max()
    eg = np.abs(vg - exact).max() / np.abs(exact).max()
    say(f"  sampled grid entries, max error / max entry: gpu {eg:.2e} oracle {eo:.2e} (tol {w.tol:g})")
    assert eg <= 10 * w.tol and eo <= 10 * w.tol
    # 3. U M V^T against the oracle's S H T^T at sampled rows, for a few thetas
    si = np.sort(rng.choice(w.n_src, 1500, replace=False))
    ti = np.sort(rng.choice(w.n_tgt, 1500, replace=False))
    S = opttk.phase3_source(opttk.factor_values(X[si], P.box_s, w.n_spatial), Go[:d])
    T = opttk.phase3_target(opttk.factor_values(Y[ti], P.box_t, w.n_spatial), Go[d + dt:])
    U, V = kern.factors()
    sel = [0, 1, 17, 1234, 4095, int(np.argmin(th[:, 0]))]
    M = kern.online_core(torch.tensor(th[sel], dtype=torch.float32, device="cuda"))
    worst = 0.0
    for j, b in enumerate(sel):
        Ko = S @ opttk.online_H(Go[d:d + dt], th[b], P.box_theta, w.n_param) @ T.T
        Kg = U[si].double().cpu().numpy() @ M[j].double().cpu().numpy() @ V[ti].double().cpu().numpy().T
        worst = max(worst, rel(Kg, Ko))
    say(f"  |U M V^T - S H T^T| / |S H T^T| on 1500 x 1500 sampled rows, worst of {len(sel)} thetas: {worst:.2e}")
    assert worst <= 1e-5
    # 4. error against dense K (the accuracy bar of the workload)
    si2 = np.sort(np.random.default_rng(11).choice(w.n_src, 4000, replace=False))
    ti2 = np.sort(np.random.default_rng(12).choice(w.n_tgt, 4000, replace=False))
    cols = np.linspace(0, B - 1, 64).astype(int)
    M64 = kern.online_core(torch.tensor(th[cols], dtype=torch.float32, device="cuda"))
    Us, Vs = U[si2].double(), V[ti2].double()
    errs = []
    for j, b in enumerate(cols):
        K = pkg.eval_dense(torch.tensor(X[si2]), torch.tensor(Y[ti2]), th[b], w.kind, w.d, dtype=torch.float64)
        errs.append((torch.linalg.norm(K - Us @ M64[j].double() @ Vs.t()) / torch.linalg.norm(K)).item())
    say(f"  error against dense K (64 thetas, 4000 x 4000): max {max(errs):.2e}, median {np.median(errs):.2e}")
    assert max(errs) <= 1e-5
    # 5. apply and backward at full size: adjoint identity, batched = plain, and
    #    the oracle's y, dX, dtheta for inputs supported on the sampled rows
    gen = torch.Generator(device="cuda").manual_seed(2)
    xb = torch.randn((B, w.n_tgt), generator=gen, device="cuda")
    gb = torch.randn((B, w.n_src), generator=gen, device="cuda")
    thd = torch.tensor(th, dtype=torch.float32, device="cuda")
    Yo, Wv = kern.apply(thd, xb, save_w=True)
    dX, dth = kern.apply_backward(thd, gb, W=Wv)
    adj = adjoint_gap(dX, xb, gb, Yo)
    say(f"  adjoint identity: max |<dX,x> - <g,y>| / (|g||y|) = {adj:.2e}")
    assert adj <= 1e-5
    Yp = kern.apply_plain(thd[[0, 1, 2047, 4095]], xb[[0, 1, 2047, 4095]])
    e = (torch.linalg.norm(Yp.double() - Yo[[0, 1, 2047, 4095]].double()) /
         torch.linalg.norm(Yo[[0, 1, 2047, 4095]].double())).item()
    say(f"  batched vs plain apply: {e:.2e}")
    assert e <= 1e-5 and torch.isfinite(dth).all()
    nb = 8
    xs = synth.rhs(1500, nb, seed=2)
    gs = synth.rhs(1500, nb, seed=3)
    xr = torch.zeros((nb, w.n_tgt), device="cuda")
    gr = torch.zeros((nb, w.n_src), device="cuda")
    xr[:, torch.tensor(ti)] = torch.tensor(xs.T, dtype=torch.float32, device="cuda")
    gr[:, torch.tensor(si)] = torch.tensor(gs.T, dtype=torch.float32, device="cuda")
    thb = thd[torch.tensor(sel[:nb] + [3, 5], device="cuda")][:nb]
    tho = thb.double().cpu().numpy()
    Yr, Wr = kern.apply(thb, xr, save_w=True)
    dXr, dthr = kern.apply_backward(thb, gr, W=Wr)
    Hs = [opttk.online_H(Go[d:d + dt], t, P.box_theta, w.n_param) for t in tho]
    dHs = [opttk.online_dH(Go[d:d + dt], t, P.box_theta, w.n_param) for t in tho]
    y_o = np.stack([S @ (Hs[b] @ (T.T @ xs[:, b])) for b in range(nb)])
    dx_o = np.stack([T @ (Hs[b].T @ (S.T @ gs[:, b])) for b in range(nb)])
    dth_o = np.array([[(S.T @ gs[:, b]) @ dHs[b][j] @ (T.T @ xs[:, b]) for j in range(dt)] for b in range(nb)])
    ey = rel(Yr[:, torch.tensor(si)].double().cpu().numpy(), y_o)
    ex = rel(dXr[:, torch.tensor(ti)].double().cpu().numpy(), dx_o)
    et = rel(dthr.double().cpu().numpy(), dth_o)
    say(f"  apply {ey:.2e} dX {ex:.2e} dtheta {et:.2e} (against the oracle's cores on the sampled rows)")
    assert ey <= 1e-5 and ex <= 1e-5 and et <= 1e-5


def test_uneven_pairs_full_size_properties():
    torch = _torch()
    import paper_2406_06344_amd as pkg
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
    say(f"[full] uneven pairs: {len(pairs)} pairs, {so} + {to} points")
    bt = pkg.TTBatch.build(pairs, torch.tensor(np.vstack(xs)), torch.tensor(np.vstack(ys)), "matern", 3,
                           base.box_theta, n_spatial=14, n_param=14, tol=1e-6, dtype=torch.float32, seed=0)
    inf = bt.info()
    say(f"  {inf['num_classes']} classes, factor grid {inf['factor_grid']}")
    B = 256
    th = torch.tensor(synth.thetas(base, count=B, seed=1), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(2)
    xb = torch.randn((B, to), generator=gen, device="cuda")
    gb = torch.randn((B, so), generator=gen, device="cuda")
    out = (torch.empty((B, so), device="cuda"), torch.empty((B, to), device="cuda"), torch.empty((B, 2), device="cuda"))
    Yo, dX, dth = bt.apply(th, xb, G=gb, out=out)
    adj = adjoint_gap(dX, xb, gb, Yo)
    say(f"  adjoint identity {adj:.2e}")
    assert adj <= 1e-5
    # replays of the captured graph reproduce the first call
    ref = [t.clone() for t in out]
    for _ in range(2):
        bt.apply(th, xb, G=gb, out=out)
        for a, b in zip(out, ref):
            assert (torch.linalg.norm(a.double() - b.double()) / torch.linalg.norm(b.double())).item() <= 1e-6
    # one pair against its own class kernel applied to its rows
    p0 = 7
    c = inf["class_of_pair"][p0]
    U, V = bt.factors(p0)
    ck = bt.class_kernel(c)
    M = ck.online_core(th[:3])
    q = pairs[p0]
    xr = torch.zeros((3, to), device="cuda")
    xr[:, q["tgt_off"]:q["tgt_off"] + q["n_tgt"]] = xb[:3, q["tgt_off"]:q["tgt_off"] + q["n_tgt"]]
    Yr = bt.apply(th[:3], xr)
    for b in range(3):
        yb = U.double() @ (M[b].double() @ (V.double().t() @ xr[b, q["tgt_off"]:q["tgt_off"] + q["n_tgt"]].double()))
        got = Yr[b, q["src_off"]:q["src_off"] + q["n_src"]].double()
        assert (torch.linalg.norm(got - yb) / torch.linalg.norm(yb)).item() <= 1e-5
