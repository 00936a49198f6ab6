"""Uneven batches of source/target box pairs (an interaction list, as in the
FMM / H-matrix use of Section 1): one parametric TT per class of pairs with
the same relative geometry, Phase 3 for each pair's points, and the batched
apply and backward summed over the list.  Test infrastructure only: plain
FP64, one pair at a time.

Reading.  Every kernel here except the two test kernels depends on x and y
only through r = ||x - y||_2, so the grid tensor of a pair is unchanged by a
common translation, reflection of an axis, or permutation of the axes of
both boxes.  A pair is mapped to a canonical frame: for axis i let hs_i, ht_i
be the box sides and delta_i the offset of the target centre from the source
centre; the canonical axes are the pair's axes sorted by (hs, ht, |delta|),
reflected so every offset is >= 0, with the source box at [0, hs].  Pairs
with equal canonical boxes share one TT.  For the test kernels every pair is
its own class, in its own frame."""
import numpy as np

from . import driver, kernels, pttk

ISOTROPIC = {"se", "exp", "matern32", "matern52", "matern_nu", "matern", "mq", "tps",
             "laplace3d", "laplace2d", "biharmonic", "thinplate"}


def frame(box_s, box_t, isotropic=True):
    """Canonical frame of a pair: permutation perm (canonical axis j is pair
    axis perm[j]), signs, and the canonical source and target boxes."""
    bs = np.asarray(box_s, float)
    bt = np.asarray(box_t, float)
    d = bs.shape[0]
    if not isotropic:
        return {"perm": list(range(d)), "sign": [1.0] * d, "box_s": bs.tolist(), "box_t": bt.tolist(),
                "key": ("pair", tuple(bs.ravel()), tuple(bt.ravel())), "shift": [0.0] * d, "identity": True}
    hs = bs[:, 1] - bs[:, 0]
    ht = bt[:, 1] - bt[:, 0]
    cs = 0.5 * (bs[:, 0] + bs[:, 1])
    ct = 0.5 * (bt[:, 0] + bt[:, 1])
    delta = ct - cs
    rnd = lambda v: float(f"{v:.12e}")
    tup = [(rnd(hs[i]), rnd(ht[i]), rnd(abs(delta[i]))) for i in range(d)]
    perm = sorted(range(d), key=lambda i: (tup[i], i))
    sign = [1.0 if delta[i] >= 0 else -1.0 for i in perm]
    cbs, cbt = [], []
    for j, i in enumerate(perm):
        cbs.append([0.0, hs[i]])
        m = 0.5 * hs[i] + abs(delta[i])
        cbt.append([m - 0.5 * ht[i], m + 0.5 * ht[i]])
    return {"perm": perm, "sign": sign, "box_s": cbs, "box_t": cbt, "centre_s": cs.tolist(),
            "key": tuple(tup[i] for i in perm), "identity": False}


def to_canonical(P, fr):
    """Points of the pair (N, d) in the canonical frame."""
    P = np.asarray(P, float)
    if fr["identity"]:
        return P.copy()
    out = np.empty_like(P)
    for j, i in enumerate(fr["perm"]):
        h = fr["box_s"][j][1]
        out[:, j] = 0.5 * h + fr["sign"][j] * (P[:, i] - fr["centre_s"][i])
    return out


def classes(pairs, kind):
    """Class index of every pair and one canonical frame per class."""
    iso = kind in ISOTROPIC
    keys, cls, frames = {}, [], []
    for p in pairs:
        fr = frame(p["box_s"], p["box_t"], iso)
        if fr["key"] not in keys:
            keys[fr["key"]] = len(frames)
            frames.append(fr)
        cls.append(keys[fr["key"]])
    return cls, frames


def offline(kind, d, box_theta, n_spatial, n_param, pairs, X, Y, eps, seed=0, const=None):
    """One TT per class (cross, rounding, gauge), then Phase 3 per pair.
    pairs[i] has box_s, box_t, src_off, n_src, tgt_off, n_tgt; X, Y hold all
    source / target points (rows)."""
    cls, frames = classes(pairs, kind)
    builds = []
    for fr in frames:
        P = kernels.Problem(kind, d, fr["box_s"], fr["box_t"], box_theta, n_spatial, n_param, const)
        # the class build does not depend on points; one point per box keeps Phase 3 defined
        x0 = P.box_s[:, :1].T
        y0 = P.box_t[:, :1].T
        builds.append((P, driver.offline(P, x0, y0, eps, seed=seed)))
    S, T = [], []
    iso = kind in ISOTROPIC
    for p, c in zip(pairs, cls):
        fr = frame(p["box_s"], p["box_t"], iso)      # the pair's own map to the class frame
        P, out = builds[c]
        Xp = to_canonical(X[p["src_off"]:p["src_off"] + p["n_src"]], fr)
        Yp = to_canonical(Y[p["tgt_off"]:p["tgt_off"] + p["n_tgt"]], fr)
        rs, rt = out["ranks"][d], out["ranks"][d + P.dt]
        S.append(pttk.phase3_source(pttk.factor_values(Xp, P.box_s, n_spatial), out["cores"][:d])
                 if len(Xp) else np.zeros((0, rs)))
        T.append(pttk.phase3_target(pttk.factor_values(Yp, P.box_t, n_spatial), out["cores"][d + P.dt:])
                 if len(Yp) else np.zeros((0, rt)))
    return {"class": cls, "frames": frames, "builds": builds, "S": S, "T": T}


def online(ob, thetas):
    """H_c(theta_b) and dH_c/dtheta_j(theta_b) for every class."""
    Hs, dHs = [], []
    for P, out in ob["builds"]:
        Hs.append([pttk.online_H(out["param"], th, P.box_theta, P.n[P.d]) for th in thetas])
        dHs.append([pttk.online_dH(out["param"], th, P.box_theta, P.n[P.d]) for th in thetas])
    return Hs, dHs


def apply(ob, pairs, Hs, Xv, n_src_total):
    """Y[:, b] = sum over pairs of the pair's block S_p H_c(theta_b) T_p^T applied
    to the pair's rows of X[:, b], scattered to its source rows."""
    B = Xv.shape[1]
    Yv = np.zeros((n_src_total, B))
    for i, p in enumerate(pairs):
        c = ob["class"][i]
        xs = Xv[p["tgt_off"]:p["tgt_off"] + p["n_tgt"]]
        for b in range(B):
            Yv[p["src_off"]:p["src_off"] + p["n_src"], b] += ob["S"][i] @ (Hs[c][b] @ (ob["T"][i].T @ xs[:, b]))
    return Yv


def backward(ob, pairs, Hs, dHs, Xv, Gv, n_tgt_total):
    """Gradients of L = sum_b <g_b, y_b>: dX (targets x B) and dtheta (B x dt)."""
    B = Xv.shape[1]
    dX = np.zeros((n_tgt_total, B))
    dt = len(dHs[0][0]) if dHs and dHs[0] else 0
    dth = np.zeros((B, dt))
    for i, p in enumerate(pairs):
        c = ob["class"][i]
        S, T = ob["S"][i], ob["T"][i]
        xs = Xv[p["tgt_off"]:p["tgt_off"] + p["n_tgt"]]
        gs = Gv[p["src_off"]:p["src_off"] + p["n_src"]]
        for b in range(B):
            a = S.T @ gs[:, b]
            w = T.T @ xs[:, b]
            dX[p["tgt_off"]:p["tgt_off"] + p["n_tgt"], b] += T @ (Hs[c][b].T @ a)
            for j in range(dt):
                dth[b, j] += a @ dHs[c][b][j] @ w
    return dX, dth


def assemble(ob, pairs, H_per_class, n_src_total, n_tgt_total):
    """The block-sparse matrix sum_p E_s,p S_p H_c T_p^T E_t,p^T, written out
    densely (tiny cases only)."""
    K = np.zeros((n_src_total, n_tgt_total))
    for i, p in enumerate(pairs):
        c = ob["class"][i]
        K[p["src_off"]:p["src_off"] + p["n_src"], p["tgt_off"]:p["tgt_off"] + p["n_tgt"]] += \
            ob["S"][i] @ H_per_class[c] @ ob["T"][i].T
    return K
