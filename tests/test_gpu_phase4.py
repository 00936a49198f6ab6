"""GPU parity of Phase 4 of Algorithm 2 (TT-Round of [S, G_{d+1}, ...,
G_{d+d_theta}, T^T], tt_kernel_phase4_round) against the oracle's
pttk.phase4_paper, which rounds that TT with its N-row outer cores directly.

The GPU takes S = Q_S R_S and T = Q_T R_T by a tall-skinny QR (blocks of 512
rows, batched Householder, levels of stacked R factors) and rounds the small
TT [R_S, G..., R_T^T]; the two are the same rounding in exact arithmetic.
Both sides start from the oracle's rounded cores on the same float32-rounded
points; 20000 sources and 9000 targets give three and two QR levels, with
ragged last blocks.  Checked: the ranks after rounding, the approximation
U' M'(theta) V'^T against S' H'(theta) T'^T (a gauge-free product), the
orthonormal columns of U' (Q_S times an orthonormal core; V' when there are
no parameter cores), and the batched apply on the compressed handle."""
import functools
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import dense as odense
from oracle import driver as odriver
from oracle import kernels as okernels
from oracle import pttk as opttk

CASES = {
    # kind, d, box_s, box_t, box_theta, n, tol
    "matern32_d2": ("matern32", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], 8, 1e-7),
    "matern_d1": ("matern", 1, [[0, 1]], [[2, 3]], [[0.5, 2.0], [0.5, 2.5]], 8, 1e-6),
    "exp_ttk": ("exp", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [], 8, 1e-8),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    return odense.rel_fro(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


@functools.lru_cache(maxsize=None)
def oracle_case(name, n_src=20000, n_tgt=9000):
    kind, d, bs, bt, bth, n, tol = CASES[name]
    fixed = [1.0] if not bth else None
    P = okernels.Problem(kind, d, bs, bt, bth, n, theta_fixed=fixed)
    rng = np.random.default_rng(3)
    X = rng.uniform(np.array(bs)[:, 0], np.array(bs)[:, 1], (n_src, d)).astype(np.float32).astype(np.float64)
    Y = rng.uniform(np.array(bt)[:, 0], np.array(bt)[:, 1], (n_tgt, d)).astype(np.float32).astype(np.float64)
    out = odriver.offline(P, X, Y, tol, seed=0)
    S2, G2, T2 = opttk.phase4_paper(out["S"], out["param"], out["T"], tol)
    return P, X, Y, out, (S2, G2, T2)


@pytest.mark.parametrize("name,dtype", [("matern32_d2", "f64"), ("matern_d1", "f64"), ("exp_ttk", "f64"),
                                        ("matern32_d2", "f32"), ("matern_d1", "f32")])
def test_phase4_matches_oracle(name, dtype):
    torch = _torch()
    import paper_2406_06344_amd as pkg
    kind, d, bs, bt, bth, n, tol = CASES[name]
    P, X, Y, out, (S2, G2, T2) = oracle_case(name)
    f64 = dtype == "f64"
    tdt = torch.float64 if f64 else torch.float32
    kw = {"theta_fixed": [1.0]} if not bth else {}
    kern = pkg.TTKernel.from_cores(out["cores"], torch.tensor(X), torch.tensor(Y), kind, d, bs, bt, bth,
                                   n_spatial=n, n_param=n, dtype=tdt, **kw)
    say(f"[phase4] {name} {dtype}: ranks before {kern.info()['ranks']}, r_s {kern.r_s} r_t {kern.r_t}")
    kern.phase4_round(tol)
    inf = kern.info()
    r_o = [S2.shape[1]] + [g.shape[2] for g in G2]
    r_g = inf["ranks"][d:d + P.dt + 1]
    say(f"  ranks after: gpu {r_g} oracle {r_o}")
    assert r_g == r_o and kern.r_s == S2.shape[1] and kern.r_t == T2.shape[1]
    U, V = kern.factors()
    U, V = U.double().cpu().numpy(), V.double().cpu().numpy()
    # the gauge leaves the first core left-orthonormal when a parameter core
    # carries the norm; with no parameter cores the last core is the
    # right-orthonormal one, so V' has orthonormal columns instead
    F = U if P.dt > 0 else V
    orth = np.abs(F.T @ F - np.eye(F.shape[1])).max()
    say(f"  |F^T F - I| for the orthonormal factor = {orth:.2e}")
    assert orth <= (1e-12 if f64 else 1e-5)
    bth_a = np.asarray(bth, float) if bth else np.zeros((0, 2))
    ths = [bth_a[:, 0], bth_a.mean(axis=1), bth_a[:, 1]] if bth else [np.zeros(0)]
    rng = np.random.default_rng(4)
    for th in ths:
        H = opttk.online_H(G2, th, bth_a, n) if bth else np.eye(S2.shape[1])
        ref = S2 @ H @ T2.T
        if bth:
            M = kern.online_core(torch.tensor(th[None, :], dtype=tdt)).double().cpu().numpy()[0]
        else:
            M = np.eye(kern.r_s)
        e = rel(U @ M @ V.T, ref)
        say(f"  theta {th}: |U'M'V'^T - S'H'T'^T|/|.| = {e:.2e}")
        assert e <= (1e-10 if f64 else 1e-5)
        if bth:   # the batched apply on the compressed handle
            xs = rng.standard_normal((2, Y.shape[0]))
            thb = torch.tensor(np.repeat(th[None, :], 2, axis=0), dtype=tdt)
            y = kern.apply(thb, torch.tensor(xs, dtype=tdt)).double().cpu().numpy()
            assert rel(y, xs @ ref.T) <= (1e-10 if f64 else 1e-5)
    # the spatial cores no longer describe U' and V'
    from paper_2406_06344_amd._lib import TTKError
    with pytest.raises(TTKError, match="UNSUPPORTED"):
        kern.cores()
