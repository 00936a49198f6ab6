"""The Python binding rejects mismatched shapes before any library call (the
C ABI receives only sizes and pointers and trusts them).  CPU only: every
case raises ValueError before a device tensor is made."""
import pytest
import torch

import paper_2406_06344_amd as pkg
from paper_2406_06344_amd import api


def _fake_kernel(d=3, d_theta=2, n_src=100, n_tgt=80, r_s=7, r_t=9):
    k = api.TTKernel.__new__(api.TTKernel)
    k._h = None
    k._borrowed = True
    k.params = api.make_params("matern" if d_theta == 2 else "matern32", d, [[0, 1]] * d, [[2, 3]] * d,
                               [[0.5, 2.0]] * d_theta)
    k.dtype = torch.float32
    k.n_src, k.n_tgt, k.r_s, k.r_t, k.d_theta, k.D = n_src, n_tgt, r_s, r_t, d_theta, 2 * d + d_theta
    return k


def test_apply_rejects_wrong_widths():
    k = _fake_kernel()
    th = torch.zeros((4, 2))
    with pytest.raises(ValueError, match="X"):
        k.apply(th, torch.zeros((4, 79)))                    # narrow X
    with pytest.raises(ValueError, match="theta"):
        k.apply(torch.zeros((3, 2)), torch.zeros((4, 80)))   # short theta
    with pytest.raises(ValueError, match="theta"):
        k.apply(torch.zeros((4, 1)), torch.zeros((4, 80)))   # theta width != d_theta
    with pytest.raises(ValueError, match="X"):
        k.apply_plain(th, torch.zeros((4, 81)))
    with pytest.raises(ValueError, match="theta"):
        k.online_core(torch.zeros((4, 3)))


def test_backward_rejects_wrong_shapes():
    k = _fake_kernel()
    th = torch.zeros((4, 2))
    with pytest.raises(ValueError, match="G"):
        k.apply_backward(th, torch.zeros((4, 99)), X=torch.zeros((4, 80)))
    with pytest.raises(ValueError, match="X"):
        k.apply_backward(th, torch.zeros((4, 100)), X=torch.zeros((5, 80)))
    with pytest.raises(ValueError, match="W"):
        k.apply_backward(th, torch.zeros((4, 100)), W=torch.zeros((4, 8)))
    with pytest.raises(ValueError, match="dtheta needs X"):
        k.apply_backward(th, torch.zeros((4, 100)))


def test_factor_rows_and_points_checks():
    k = _fake_kernel()
    with pytest.raises(ValueError, match="P"):
        k.factor_rows(torch.zeros((10, 2)))                  # d = 3 points expected
    with pytest.raises(ValueError, match="side"):
        k.factor_rows(torch.zeros((10, 3)), side=2)
    with pytest.raises(ValueError, match="X"):
        pkg.TTKernel.build_offline(torch.zeros((10, 2)), torch.zeros((10, 3)), "matern32", 3, [[0, 1]] * 3,
                                   [[2, 3]] * 3, [[0.5, 2.0]])


def test_entry_and_dense_checks():
    with pytest.raises(ValueError, match="idx"):
        pkg.eval_entries(torch.zeros((5, 6), dtype=torch.int32), "matern32", 3, [[0, 1]] * 3, [[2, 3]] * 3,
                         [[0.5, 2.0]], n_spatial=8)           # D = 7 columns expected
    with pytest.raises(ValueError, match="out of range"):
        pkg.eval_entries(torch.full((5, 7), 8, dtype=torch.int32), "matern32", 3, [[0, 1]] * 3, [[2, 3]] * 3,
                         [[0.5, 2.0]], n_spatial=8)
    with pytest.raises(ValueError, match="theta"):
        pkg.eval_dense(torch.zeros((4, 3)), torch.zeros((5, 3)), [1.0], "matern", 3)


def test_ttk_allows_no_theta():
    assert api._theta(None, 0, torch.float32) is None
    with pytest.raises(ValueError):
        api._theta(None, 1, torch.float32)
