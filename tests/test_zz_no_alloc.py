"""tt_kernel_apply_noalloc (the batched apply with a fixed per-device scratch
instead of allocations) against tt_kernel_apply, through the C ABI: two calls
in a row, the second with a smaller input, in float32 (matrix-core and
skinny paths) and float64; plus the size limit."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cores(rs, rt, seed):
    rng = np.random.default_rng(seed)
    r = [1, 16, rs, rt, 16, 1]
    n = [16, 16, 12, 16, 16]
    return [rng.standard_normal((r[k], n[k], r[k + 1])) / np.sqrt(r[k] * n[k]) for k in range(5)]


def _rel(a, b):
    a, b = a.double(), b.double()
    return ((a - b).norm() / b.norm()).item(), ((a - b).abs().max() / b.abs().max()).item()


@pytest.mark.parametrize("dtype_name,rs,rt,calls", [
    ("f32", 72, 75, [(300, 3001, 2999), (37, 3001, 2999)]),      # matrix-core path, then a smaller batch
    ("f32", 40, 33, [(16, 5000, 4000), (3, 5000, 4000)]),        # skinny path, then B = 3
    ("f64", 30, 28, [(70, 1500, 1300), (1, 1500, 1300)]),         # float64 tiled path, then the plain one
])
def test_noalloc_apply_matches_apply(dtype_name, rs, rt, calls):
    torch = _torch()
    import paper_2406_06344_amd as pkg
    from paper_2406_06344_amd import _lib
    lib = _lib.load()
    dt = torch.float32 if dtype_name == "f32" else torch.float64
    tol = 1e-5 if dtype_name == "f32" else 1e-12
    rng = np.random.default_rng(3)
    ns, nt = calls[0][1], calls[0][2]
    X = rng.uniform(0, 1, (ns, 2))
    Y = rng.uniform([2, 0], [3, 1], (nt, 2))
    kern = pkg.TTKernel.from_cores(_cores(rs, rt, rs), torch.tensor(X), torch.tensor(Y), "matern32", 2,
                                   [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], n_spatial=16, n_param=12,
                                   dtype=dt)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for i, (B, _, _) in enumerate(calls):
        say(f"[noalloc] {dtype_name} r {rs}/{rt} call {i}: B = {B}")
        th = torch.tensor(rng.uniform(0.5, 2.0, (B, 1)), dtype=dt, device="cuda")
        xb = torch.tensor(rng.standard_normal((B, nt)), dtype=dt, device="cuda")
        y_ref = torch.empty((B, ns), dtype=dt, device="cuda")
        w_ref = torch.empty((B, rt), dtype=dt, device="cuda")
        assert lib.tt_kernel_apply(kern._h, ctypes.c_void_p(th.data_ptr()), B, ctypes.c_void_p(xb.data_ptr()), nt,
                                   ctypes.c_void_p(y_ref.data_ptr()), ns, ctypes.c_void_p(w_ref.data_ptr()), st) == 0
        y = torch.full((B, ns), float("nan"), dtype=dt, device="cuda")
        w = torch.full((B, rt), float("nan"), dtype=dt, device="cuda")
        y2 = torch.full((B, ns), float("nan"), dtype=dt, device="cuda")
        torch.cuda.synchronize()
        # with the caller keeping W, then without
        assert lib.tt_kernel_apply_noalloc(kern._h, ctypes.c_void_p(th.data_ptr()), B, ctypes.c_void_p(xb.data_ptr()),
                                           nt, ctypes.c_void_p(y.data_ptr()), ns, ctypes.c_void_p(w.data_ptr()),
                                           st) == 0
        assert lib.tt_kernel_apply_noalloc(kern._h, ctypes.c_void_p(th.data_ptr()), B, ctypes.c_void_p(xb.data_ptr()),
                                           nt, ctypes.c_void_p(y2.data_ptr()), ns, None, st) == 0
        torch.cuda.synchronize()
        ey, ew, ey2 = _rel(y, y_ref), _rel(w, w_ref), _rel(y2, y_ref)
        say(f"  y {ey}, W {ew}, y without W {ey2}")
        for e in (ey, ew, ey2):
            assert e[0] <= tol and e[1] <= tol


def test_noalloc_rejects_oversize_batch_without_touching_outputs():
    torch = _torch()
    import paper_2406_06344_amd as pkg
    from paper_2406_06344_amd import _lib
    lib = _lib.load()
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (100, 2))
    Y = rng.uniform([2, 0], [3, 1], (90, 2))
    kern = pkg.TTKernel.from_cores(_cores(100, 110, 1), torch.tensor(X), torch.tensor(Y), "matern32", 2,
                                   [[0, 1], [0, 1]], [[2, 3], [0, 1]], [[0.5, 2.0]], n_spatial=16, n_param=12,
                                   dtype=torch.float32)
    B = 4096                                   # M(theta) alone is 4096 * 100 * 110 * 4 bytes > 64 MiB
    th = torch.ones((B, 1), device="cuda")
    xb = torch.ones((B, 90), device="cuda")
    y = torch.full((B, 100), 7.0, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = lib.tt_kernel_apply_noalloc(kern._h, ctypes.c_void_p(th.data_ptr()), B, ctypes.c_void_p(xb.data_ptr()), 90,
                                    ctypes.c_void_p(y.data_ptr()), 100, None, st)
    assert s == -1 and b"scratch" in lib.tt_kernel_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
