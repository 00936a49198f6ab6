"""The library's working memory is pooled: a released buffer is handed out
again to a later allocation on the same thread, after one device
synchronisation.  A build whose buffers all come back from the pool (right
after a different build released them, and on another stream) must give the
same factors as the first build of the same problem, and a handle destroyed
while its stream still has work queued must not disturb a build that follows
at once on another stream."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PROBLEM = ("se", 2, [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], 1e-8)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _points(n_src, n_tgt, seed):
    kind, d, bs, bt, bth, tol = PROBLEM
    rng = np.random.default_rng(seed)
    X = rng.uniform(np.array(bs)[:, 0], np.array(bs)[:, 1], (n_src, d))
    Y = rng.uniform(np.array(bt)[:, 0], np.array(bt)[:, 1], (n_tgt, d))
    return X, Y


def _build(torch, pkg, stream, X, Y, n):
    kind, d, bs, bt, bth, tol = PROBLEM
    with torch.cuda.stream(stream):
        k = pkg.TTKernel.build_offline(torch.tensor(X), torch.tensor(Y), kind, d, bs, bt, bth, n_spatial=n,
                                       n_param=n, tol=tol, dtype=torch.float64, seed=0, stream=stream)
        U, V = k.factors(stream=stream)
    stream.synchronize()
    return k, U.cpu().numpy(), V.cpu().numpy()


def test_builds_from_pooled_memory_match_across_streams():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()   # default priority
    X, Y = _points(700, 500, seed=3)
    say("pool: first build on stream 1")
    k1, U1, V1 = _build(torch, pkg, s1, X, Y, 12)
    r1 = k1.info()["ranks"]
    del k1
    # another problem in between (other sizes), on the other stream
    X2, Y2 = _points(1300, 900, seed=4)
    say("pool: a different build on stream 2")
    k2, _, _ = _build(torch, pkg, s2, X2, Y2, 16)
    del k2
    say("pool: the first problem again on stream 2")
    k3, U3, V3 = _build(torch, pkg, s2, X, Y, 12)
    assert k3.info()["ranks"] == r1
    assert U3.shape == U1.shape and V3.shape == V1.shape
    scale = max(np.abs(U1).max(), np.abs(V1).max())
    assert np.abs(U3 - U1).max() <= 1e-13 * scale
    assert np.abs(V3 - V1).max() <= 1e-13 * scale


def test_handle_released_with_queued_work_then_build_on_other_stream():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    X, Y = _points(600, 400, seed=5)
    _, Uref, Vref = _build(torch, pkg, s1, X, Y, 12)
    kind, d, bs, bt, bth, tol = PROBLEM
    with torch.cuda.stream(s1):
        k = pkg.TTKernel.build_offline(torch.tensor(X), torch.tensor(Y), kind, d, bs, bt, bth, n_spatial=12,
                                       n_param=12, tol=tol, dtype=torch.float64, seed=0, stream=s1)
        th = torch.tensor([[1.0]], dtype=torch.float64, device="cuda")
        xb = torch.ones((1, Y.shape[0]), dtype=torch.float64, device="cuda")
        for _ in range(8):   # work left queued on stream 1 when the handle goes
            k.apply(th, xb, stream=s1)
    del k
    say("pool: build on stream 2 while stream 1 may still run")
    k2, U2, V2 = _build(torch, pkg, s2, X, Y, 12)
    s1.synchronize()
    scale = max(np.abs(Uref).max(), np.abs(Vref).max())
    assert np.abs(U2 - Uref).max() <= 1e-13 * scale
    assert np.abs(V2 - Vref).max() <= 1e-13 * scale
