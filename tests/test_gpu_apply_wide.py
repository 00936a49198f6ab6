"""GPU parity of the batched apply and backward beyond the small ranks of
the main parity test (B > 16: the float32 matrix-core kernels for ranks up
to 128, the register-tiled kernels above; 2 <= B <= 16: the skinny
matrix-core kernels)
against the FP64 oracle on the same cores and float32-rounded inputs.

Cores are random TT cores with the ranks under test (d = 2, one parameter):
the apply, its backward pass and the online core depend on the cores only
through S, T and H(theta), which the oracle forms from the same cores
(Phase 3 of Algorithm 2, Algorithm 3).  Bars: relative Frobenius <= 1e-5 and
largest entry error <= 1e-5 of the largest entry, per output."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import dense as odense
from oracle import pttk as opttk

BOX_S = [[0.0, 1.0], [0.0, 1.0]]
BOX_T = [[2.0, 3.0], [0.0, 1.0]]
BOX_TH = [[0.5, 2.0]]
N_SP, N_PA = 16, 12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def random_cores(rs, rt, seed):
    """Nodal cores G_1..G_5 with ranks (1, 16, rs, rt, 16, 1), entries scaled
    so every chain product stays of order one."""
    rng = np.random.default_rng(seed)
    r = [1, N_SP, rs, rt, N_SP, 1]
    n = [N_SP, N_SP, N_PA, N_SP, N_SP]
    return [rng.standard_normal((r[k], n[k], r[k + 1])) / np.sqrt(r[k] * n[k]) for k in range(5)]


def errs(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return odense.rel_fro(got, ref), float(np.abs(got - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("rs,rt,ns,nt,B", [
    (100, 90, 3001, 2999, 200),     # MFMA path, ragged N (unaligned columns), ragged theta tiles
    (72, 75, 4096, 2048, 64),       # MFMA path, aligned columns (16-byte stores and loads)
    (128, 17, 1500, 2100, 513),     # the widest MFMA rank and a narrow one, 5 theta blocks + 1
    (130, 70, 1200, 1000, 80),      # rank above 128: the register-tiled float32 kernels
])
def test_wide_apply_and_backward_match_oracle(rs, rt, ns, nt, B):
    _check_apply_and_backward(rs, rt, ns, nt, B)


@pytest.mark.parametrize("rs,rt,ns,nt,B", [
    (100, 90, 3001, 2999, 16),      # 64-column group + 3 / 2 tail tiles, unaligned X and Y columns
    (72, 75, 4096, 2048, 16),       # group + 1 tail tile, aligned columns (16-byte X loads, Y stores)
    (128, 17, 1500, 2100, 5),       # two 64-column groups; two tail tiles only
    (40, 60, 999, 1001, 2),         # three tail tiles; a part-filled 64-column group
])
def test_skinny_apply_and_backward_match_oracle(rs, rt, ns, nt, B):
    """2 <= B <= 16: the float32 skinny matrix-core reduce and expand (every
    rank-dependent shape of their column split), same bars."""
    _check_apply_and_backward(rs, rt, ns, nt, B)


def _check_apply_and_backward(rs, rt, ns, nt, B):
    torch = _torch()
    import paper_2406_06344_amd as pkg
    say(f"[wide] r_s {rs} r_t {rt} N {ns} x {nt} B {B}")
    cores = random_cores(rs, rt, seed=rs + rt)
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, (ns, 2)).astype(np.float32).astype(np.float64)
    Y = rng.uniform([2, 0], [3, 1], (nt, 2)).astype(np.float32).astype(np.float64)
    th = rng.uniform(0.5, 2.0, (B, 1)).astype(np.float32).astype(np.float64)
    xb = rng.standard_normal((nt, B)).astype(np.float32).astype(np.float64)
    gb = rng.standard_normal((ns, B)).astype(np.float32).astype(np.float64)
    kern = pkg.TTKernel.from_cores(cores, torch.tensor(X), torch.tensor(Y), "matern32", 2, BOX_S, BOX_T, BOX_TH,
                                   n_spatial=N_SP, n_param=N_PA, dtype=torch.float32)
    assert (kern.r_s, kern.r_t) == (rs, rt)
    bs, bt, bth = np.array(BOX_S), np.array(BOX_T), np.array(BOX_TH)
    S = opttk.phase3_source(opttk.factor_values(X, bs, N_SP), cores[:2])
    T = opttk.phase3_target(opttk.factor_values(Y, bt, N_SP), cores[3:])
    Hs = [opttk.online_H(cores[2:3], t, bth, N_PA) for t in th]
    dHs = [opttk.online_dH(cores[2:3], t, bth, N_PA) for t in th]
    y_o, W_o = opttk.apply_batched(S, Hs, T, xb)
    dX_o, dth_o = opttk.backward_batched(S, Hs, dHs, T, xb, gb)
    tht = torch.tensor(th, dtype=torch.float32)
    Yg, Wg = kern.apply(tht, torch.tensor(xb.T.copy(), dtype=torch.float32), save_w=True)
    dXg, dthg = kern.apply_backward(tht, torch.tensor(gb.T.copy(), dtype=torch.float32), W=Wg)
    res = {"W": errs(Wg.cpu().numpy().T, W_o), "y": errs(Yg.cpu().numpy().T, y_o),
           "dX": errs(dXg.cpu().numpy().T, dX_o), "dtheta": errs(dthg.cpu().numpy(), dth_o)}
    say("  (rel Frobenius, max entry):", {k: (f"{a:.2e}", f"{b:.2e}") for k, (a, b) in res.items()})
    for k, (fro, mx) in res.items():
        assert fro <= 1e-5 and mx <= 1e-5, (k, fro, mx)
    # the backward without the saved W (W formed from X) and without dX
    gt = torch.tensor(gb.T.copy(), dtype=torch.float32)
    dX2, dth2 = kern.apply_backward(tht, gt, X=torch.tensor(xb.T.copy(), dtype=torch.float32))
    _, dth3 = kern.apply_backward(tht, gt, W=Wg, want_dx=False)
    assert errs(dX2.cpu().numpy().T, dX_o)[0] <= 1e-5
    for d in (dth2, dth3):
        fro, mx = errs(d.cpu().numpy(), dth_o)
        assert fro <= 1e-5 and mx <= 1e-5, (fro, mx)
    # the plain per-theta apply (other kernels) agrees with the batched one
    Yp = kern.apply_plain(tht[:5], torch.tensor(xb[:, :5].T.copy(), dtype=torch.float32))
    assert errs(Yp.cpu().numpy(), Yg[:5].cpu().numpy())[0] <= 1e-5


@pytest.mark.parametrize("B,npar", [(300, 16), (40, 12), (1000, 8)])
def test_online_core_two_parameters_matches_oracle(B, npar):
    """M(theta) and dM/dtheta for d_theta = 2 in float32 with B >= 32 (the
    matrix-core form: M = sum_{k1,k2} T_k1 T_k2 C_{k1 k2} with C the products of
    the parameter cores, in passes of 128 rows when n1 n2 > 128) against the
    oracle's Algorithm 3 on the same cores."""
    torch = _torch()
    import paper_2406_06344_amd as pkg
    rng = np.random.default_rng(B)
    r = [1, N_SP, 80, 150, 70, N_SP, 1]
    n = [N_SP, N_SP, npar, npar, N_SP, N_SP]
    cores = [rng.standard_normal((r[k], n[k], r[k + 1])) / np.sqrt(r[k] * n[k]) for k in range(6)]
    bth = np.array([[0.5, 2.0], [0.5, 2.5]])
    X = rng.uniform(0, 1, (50, 2))
    Y = rng.uniform([2, 0], [3, 1], (40, 2))
    kern = pkg.TTKernel.from_cores(cores, torch.tensor(X), torch.tensor(Y), "matern", 2, BOX_S, BOX_T, bth,
                                   n_spatial=N_SP, n_param=npar, dtype=torch.float32)
    th = rng.uniform(bth[:, 0], bth[:, 1], (B, 2)).astype(np.float32).astype(np.float64)
    M, dM = kern.online_core(torch.tensor(th, dtype=torch.float32), deriv=True)
    M, dM = M.double().cpu().numpy(), dM.double().cpu().numpy()
    Mo = np.stack([opttk.online_H(cores[2:4], t, bth, npar) for t in th])
    dMo = np.stack([np.stack(opttk.online_dH(cores[2:4], t, bth, npar)) for t in th])
    em, edm = errs(M, Mo), errs(dM, dMo)
    say(f"[online] B {B} n_param {npar}: M {em}, dM {edm}")
    assert em[0] <= 1e-6 and em[1] <= 2e-6 and edm[0] <= 1e-5 and edm[1] <= 1e-5
