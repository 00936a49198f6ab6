"""Python binding of the PTTK C ABI: argument marshalling only.

Every step runs in libttk.so; torch supplies device memory and the stream.
Shapes follow torch's row-major convention:
  points X, Y           (N, d)   -> passed structure-of-arrays (d, N)
  theta                 (B, d_theta)
  right-hand sides X    (B, N_t)  (row b = x_b; a column-major N_t x B matrix)
  outputs Y             (B, N_s)
  U, V                  (N_s, r_s), (N_t, r_t)
  M(theta)              (B, r_s, r_t)
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import KINDS, KIND_DTHETA, TTK_FP32, TTK_FP64, BatchInfo, Decision, Info, Pair, Params, check


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype_code(dtype):
    if dtype == torch.float32:
        return TTK_FP32
    if dtype == torch.float64:
        return TTK_FP64
    raise ValueError(f"unsupported dtype {dtype}")


def make_params(kind, d, box_s, box_t, box_theta=(), n_spatial=16, n_param=None, tol=1e-6,
                dtype=torch.float32, seed=0, max_rank=256, max_sweeps=200, init_card=2,
                init_max_it=10, n_test=0, kernel_const=0.0, symmetric_psd=False, theta_fixed=None):
    """theta_fixed: the kind's parameters held fixed (non-parametric TTK, d_theta = 0)."""
    p = Params()
    p.d = int(d)
    p.d_theta = KIND_DTHETA[kind]
    if theta_fixed is not None:
        tf = [float(v) for v in np.ravel(theta_fixed)]
        if len(tf) != KIND_DTHETA[kind]:
            raise ValueError(f"theta_fixed: {kind} has {KIND_DTHETA[kind]} parameters, got {len(tf)}")
        p.d_theta = 0
        for i, v in enumerate(tf):
            p.theta_fixed[i] = v
    p.n_spatial = int(n_spatial)
    p.n_param = int(n_spatial if n_param is None else n_param)
    p.kind = KINDS[kind]
    p.kernel_const = float(kernel_const)
    bs = np.asarray(box_s, float).reshape(-1)
    bt = np.asarray(box_t, float).reshape(-1)
    bp = np.asarray(box_theta, float).reshape(-1)
    for i, v in enumerate(bs):
        p.box_s[i] = v
    for i, v in enumerate(bt):
        p.box_t[i] = v
    for i, v in enumerate(bp):
        p.box_theta[i] = v
    p.tol = float(tol)
    p.max_rank = int(max_rank)
    p.max_sweeps = int(max_sweeps)
    p.init_card = int(init_card)
    p.init_max_it = int(init_max_it)
    p.n_test = int(n_test)
    p.seed = int(seed)
    p.dtype = _dtype_code(dtype)
    p.symmetric_psd = 1 if symmetric_psd else 0
    return p


def _soa(P, dtype, d=None, name="points"):
    """(N, d) points -> contiguous (d, N) on the current device."""
    if P.dim() != 2 or (d is not None and P.shape[1] != d):
        raise ValueError(f"{name}: expected shape (N, {d}), got {tuple(P.shape)}")
    return P.to(device="cuda", dtype=dtype).t().contiguous()


def _chk(t, name, rows, cols):
    """ValueError unless t is a (rows, cols) matrix (rows None: any); checked
    before anything reaches the device, since the library trusts sizes."""
    if t is None:
        raise ValueError(f"{name} is required")
    if t.dim() != 2 or (rows is not None and t.shape[0] != rows) or t.shape[1] != cols:
        raise ValueError(f"{name}: expected shape ({'B' if rows is None else rows}, {cols}), got {tuple(t.shape)}")
    return t


def _dev(t, dtype):
    return None if t is None else t.to(device="cuda", dtype=dtype).contiguous()


def _out(t, name, shape, dtype):
    """A caller-supplied output: exactly this shape and dtype, contiguous, on the GPU."""
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous cuda {dtype} tensor of shape {tuple(shape)}, got "
                         f"{tuple(t.shape)} {t.dtype} on {t.device} (contiguous={t.is_contiguous()})")
    return t


def _theta(theta, d_theta, dtype, B=None, convert=True):
    """theta as a contiguous (B, max(d_theta, 1)) device tensor.  Accepts
    (B, d_theta), or (B,) when d_theta <= 1; B must match when given.
    convert=False: validate and reshape only."""
    w = max(d_theta, 1)
    if theta is None:
        if d_theta == 0:
            return None            # no parameters: M = I
        raise ValueError("theta is required")
    if theta.dim() == 1 and w == 1:
        theta = theta.reshape(-1, 1)
    if theta.dim() != 2 or theta.shape[1] != w or (B is not None and theta.shape[0] != B):
        raise ValueError(f"theta: expected shape ({'B' if B is None else B}, {w}), got {tuple(theta.shape)}")
    return theta.to(device="cuda", dtype=dtype).contiguous() if convert else theta


class TTKernel:
    """Offline stage (U, V, parameter cores) held by the C library."""

    def __init__(self, handle, params, dtype, n_src, n_tgt, status=0):
        self._h = handle
        self.params = params
        self.dtype = dtype
        self.n_src = n_src
        self.n_tgt = n_tgt
        self.status = status
        inf = self.info()
        self.r_s, self.r_t, self.D = inf["r_s"], inf["r_t"], inf["D"]
        self.d_theta = params.d_theta

    # ----------------------------------------------------------- builds
    @classmethod
    def build_offline(cls, X, Y, kind, d, box_s, box_t, box_theta=(), n_spatial=16, n_param=None,
                      tol=1e-6, dtype=torch.float32, stream=None, **kw):
        """Y = None (or Y is X) with symmetric_psd=True builds PTTK-Global-1."""
        lib = _lib.load()
        p = make_params(kind, d, box_s, box_t, box_theta, n_spatial, n_param, tol, dtype, **kw)
        Xs = _soa(X, dtype, d, "X")
        Ys = Xs if (Y is None or Y is X) else _soa(Y, dtype, d, "Y")
        h = ctypes.c_void_p()
        st = check(lib.tt_kernel_build_offline(ctypes.byref(p), _ptr(Xs), Xs.shape[1], _ptr(Ys), Ys.shape[1],
                                               _stream_ptr(stream), ctypes.byref(h)))
        return cls(h, p, dtype, Xs.shape[1], Ys.shape[1], st)

    @classmethod
    def from_cores(cls, cores, X, Y, kind, d, box_s, box_t, box_theta=(), n_spatial=16, n_param=None,
                   dtype=torch.float32, stream=None, **kw):
        """cores: list of float64 arrays (r0, n, r1) (nodal basis, gauge as given)."""
        lib = _lib.load()
        p = make_params(kind, d, box_s, box_t, box_theta, n_spatial, n_param, 1e-6, dtype, **kw)
        ranks = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
        flat = np.concatenate([np.asarray(c, np.float64).reshape(-1, order="F") for c in cores])
        r_arr = (ctypes.c_int * len(ranks))(*ranks)
        c_arr = flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if len(cores) != 2 * int(d) + p.d_theta:
            raise ValueError(f"cores: expected {2 * int(d) + p.d_theta} cores, got {len(cores)}")
        Xs = _soa(X, dtype, d, "X")
        Ys = Xs if (Y is None or Y is X) else _soa(Y, dtype, d, "Y")
        h = ctypes.c_void_p()
        check(lib.tt_kernel_build_from_cores(ctypes.byref(p), r_arr, c_arr, _ptr(Xs), Xs.shape[1], _ptr(Ys),
                                             Ys.shape[1], _stream_ptr(stream), ctypes.byref(h)))
        return cls(h, p, dtype, Xs.shape[1], Ys.shape[1])

    def __del__(self):
        h = getattr(self, "_h", None)
        if getattr(self, "_borrowed", False):
            return
        if h is not None and h.value:
            try:
                _lib.load().tt_kernel_destroy(h)
            except Exception:
                pass
            self._h = None

    # ----------------------------------------------------------- queries
    def info(self):
        inf = Info()
        check(_lib.load().tt_kernel_get_info(self._h, ctypes.byref(inf)))
        D = inf.D
        return {"D": D, "r_s": inf.r_s, "r_t": inf.r_t, "ranks": list(inf.ranks)[:D + 1],
                "cross_ranks": list(inf.cross_ranks)[:D + 1], "kernel_evals": inf.kernel_evals,
                "sweeps": inf.sweeps, "n_decisions": inf.n_decisions, "sampled_error": inf.sampled_error,
                "init_max_cond": inf.init_max_cond, "min_margin": inf.min_margin,
                "t_cross_ms": inf.t_cross_ms, "t_round_ms": inf.t_round_ms, "t_factor_ms": inf.t_factor_ms,
                "n_src": inf.n_src, "n_tgt": inf.n_tgt}

    def factors(self, stream=None):
        U = torch.empty((self.n_src, self.r_s), dtype=self.dtype, device="cuda")
        V = torch.empty((self.n_tgt, self.r_t), dtype=self.dtype, device="cuda")
        check(_lib.load().tt_kernel_get_factors(self._h, _ptr(U), _ptr(V), _stream_ptr(stream)))
        return U, V

    def cores(self):
        inf = self.info()
        r = inf["ranks"]
        n = [self.params.n_spatial] * self.params.d + [self.params.n_param] * self.params.d_theta + \
            [self.params.n_spatial] * self.params.d
        sizes = [r[k] * n[k] * r[k + 1] for k in range(inf["D"])]
        buf = np.zeros(sum(sizes))
        check(_lib.load().tt_kernel_get_cores(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              buf.size))
        out, off = [], 0
        for k, s in enumerate(sizes):
            out.append(buf[off:off + s].reshape((r[k], n[k], r[k + 1]), order="F"))
            off += s
        return out

    def coeff_cores(self):
        """Coefficient-basis cores (Chebyshev basis along mode 2), float64."""
        inf = self.info()
        r = inf["ranks"]
        n = [self.params.n_spatial] * self.params.d + [self.params.n_param] * self.params.d_theta + \
            [self.params.n_spatial] * self.params.d
        sizes = [r[k] * n[k] * r[k + 1] for k in range(inf["D"])]
        buf = np.zeros(sum(sizes))
        check(_lib.load().tt_kernel_get_coeff_cores(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                    buf.size))
        out, off = [], 0
        for k, s in enumerate(sizes):
            out.append(buf[off:off + s].reshape((r[k], n[k], r[k + 1]), order="F"))
            off += s
        return out

    def cross_record(self):
        inf = self.info()
        D = inf["D"]
        r = inf["cross_ranks"]
        nl = sum(r[k] * k for k in range(1, D))
        nr = sum(r[k] * (D - k) for k in range(1, D))
        left = (ctypes.c_int32 * max(nl, 1))()
        right = (ctypes.c_int32 * max(nr, 1))()
        nd = inf["n_decisions"]
        dec = (Decision * max(nd, 1))()
        check(_lib.load().tt_kernel_get_cross(self._h, left, right, dec, nd))
        L, R = [None] * (D + 1), [None] * (D + 1)
        lo = ro = 0
        for k in range(1, D):
            L[k] = np.array(left[lo:lo + r[k] * k], dtype=np.int64).reshape(r[k], k)
            lo += r[k] * k
            R[k] = np.array(right[ro:ro + r[k] * (D - k)], dtype=np.int64).reshape(r[k], D - k)
            ro += r[k] * (D - k)
        names = [f[0] for f in Decision._fields_]
        decisions = [{n: getattr(dec[i], n) for n in names} for i in range(nd)]
        for rec in decisions:
            rec["added"] = bool(rec["added"])
        return L, R, decisions

    def factor_rows(self, P, side=0, out=None, stream=None):
        """Rows of U (side 0) or V (side 1) for points P (n, d) of the same box."""
        if side not in (0, 1):
            raise ValueError("side must be 0 (sources) or 1 (targets)")
        Ps = _soa(P, self.dtype, self.params.d, "P")
        n = Ps.shape[1]
        r = self.r_s if side == 0 else self.r_t
        if out is None:
            out = torch.empty((n, r), dtype=self.dtype, device="cuda")
        _out(out, "out", (n, r), self.dtype)
        check(_lib.load().tt_kernel_factor_rows(self._h, side, _ptr(Ps), n, _ptr(out), _stream_ptr(stream)))
        return out

    def factor_rows_soa(self, Ps, side, out, stream=None):
        """As factor_rows for points already in (d, n) device layout; no allocation."""
        if side not in (0, 1):
            raise ValueError("side must be 0 (sources) or 1 (targets)")
        _out(Ps, "Ps", (self.params.d, Ps.shape[1] if Ps.dim() == 2 else -1), self.dtype)
        _out(out, "out", (Ps.shape[1], self.r_s if side == 0 else self.r_t), self.dtype)
        check(_lib.load().tt_kernel_factor_rows(self._h, side, _ptr(Ps), Ps.shape[1], _ptr(out),
                                                _stream_ptr(stream)))
        return out

    # ------------------------------------------------------------ online
    def online_core(self, theta, deriv=False, stream=None):
        theta = _theta(theta, self.d_theta, self.dtype)
        B = theta.shape[0]
        M = torch.empty((B, self.r_t, self.r_s), dtype=self.dtype, device="cuda")
        dM = torch.empty((B, max(self.d_theta, 1), self.r_t, self.r_s), dtype=self.dtype,
                         device="cuda") if deriv else None
        check(_lib.load().tt_kernel_online_core(self._h, _ptr(theta), B, _ptr(M), _ptr(dM), _stream_ptr(stream)))
        Mt = M.transpose(1, 2)
        return (Mt, dM.transpose(2, 3)) if deriv else Mt

    def apply(self, theta, X, save_w=False, stream=None):
        """y_b = U M(theta_b) V^T x_b for every row x_b of X (B, N_t)."""
        B = _chk(X, "X", None, self.n_tgt).shape[0]
        theta = _dev(_theta(theta, self.d_theta, self.dtype, B, convert=False), self.dtype)
        X = _dev(X, self.dtype)
        Y = torch.empty((B, self.n_src), dtype=self.dtype, device="cuda")
        W = torch.empty((B, self.r_t), dtype=self.dtype, device="cuda") if save_w else None
        check(_lib.load().tt_kernel_apply(self._h, _ptr(theta), B, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
                                          _ptr(W), _stream_ptr(stream)))
        return (Y, W) if save_w else Y

    def apply_noalloc(self, theta, X, out, W=None, stream=None):
        """apply() through tt_kernel_apply_noalloc: the library allocates
        nothing (its working memory is a fixed per-device scratch).  out
        (B, N_s) and W (B, r_t, optional) are caller-owned device tensors."""
        B = _chk(X, "X", None, self.n_tgt).shape[0]
        theta = _theta(theta, self.d_theta, self.dtype, B, convert=False)
        _out(out, "out", (B, self.n_src), self.dtype)
        if W is not None:
            _out(W, "W", (B, self.r_t), self.dtype)
        theta, X = _dev(theta, self.dtype), _dev(X, self.dtype)
        check(_lib.load().tt_kernel_apply_noalloc(self._h, _ptr(theta), B, _ptr(X), X.stride(0), _ptr(out),
                                                  out.stride(0), _ptr(W), _stream_ptr(stream)))
        return out

    def project(self, X, side=1, out=None, stream=None):
        """W (B, r) with row b = F^T x_b: F = V for side 1 (X (B, N_t)), U for side 0 (X (B, N_s))."""
        if side not in (0, 1):
            raise ValueError("side must be 0 (U) or 1 (V)")
        n, r = (self.n_src, self.r_s) if side == 0 else (self.n_tgt, self.r_t)
        B = _chk(X, "X", None, n).shape[0]
        if out is None:
            out = torch.empty((B, r), dtype=self.dtype, device="cuda")
        _out(out, "out", (B, r), self.dtype)
        X = _dev(X, self.dtype)
        check(_lib.load().tt_kernel_project(self._h, side, _ptr(X), X.stride(0), B, _ptr(out), _stream_ptr(stream)))
        return out

    def apply_plain(self, theta, X, stream=None):
        B = _chk(X, "X", None, self.n_tgt).shape[0]
        theta = _dev(_theta(theta, self.d_theta, self.dtype, B, convert=False), self.dtype)
        X = _dev(X, self.dtype)
        Y = torch.empty((B, self.n_src), dtype=self.dtype, device="cuda")
        check(_lib.load().tt_kernel_apply_plain(self._h, _ptr(theta), B, _ptr(X), X.stride(0), _ptr(Y),
                                                Y.stride(0), _stream_ptr(stream)))
        return Y

    def apply_backward(self, theta, G, X=None, W=None, want_dx=True, want_dtheta=True, stream=None):
        B = _chk(G, "G", None, self.n_src).shape[0]
        theta = _theta(theta, self.d_theta, self.dtype, B, convert=False)
        if X is not None:
            _chk(X, "X", B, self.n_tgt)
        want_dth = want_dtheta and self.d_theta > 0
        if W is not None:
            _out(W, "W", (B, self.r_t), self.dtype)
        elif want_dth and X is None:
            raise ValueError("dtheta needs X or the W saved by apply(save_w=True)")
        theta, G, Xc = _dev(theta, self.dtype), _dev(G, self.dtype), _dev(X, self.dtype)
        dX = torch.empty((B, self.n_tgt), dtype=self.dtype, device="cuda") if want_dx else None
        dth = torch.empty((B, max(self.d_theta, 1)), dtype=self.dtype, device="cuda") if want_dth else None
        check(_lib.load().tt_kernel_apply_backward(self._h, _ptr(theta), B, _ptr(Xc), self.n_tgt, _ptr(W),
                                                   _ptr(G), G.stride(0), _ptr(dX), self.n_tgt, _ptr(dth),
                                                   _stream_ptr(stream)))
        return dX, dth

    # ------------------------------------------------ Global-1 (Algorithm 4)
    def global_factors(self, stream=None):
        """(Q (N, k), R (k, k) float64 numpy) of the thin QR [U V] = Q R."""
        lib = _lib.load()
        k = ctypes.c_int()
        check(lib.tt_kernel_global_factors(self._h, ctypes.byref(k), None, None, _stream_ptr(stream)))
        k = k.value
        Q = torch.empty((self.n_src, k), dtype=self.dtype, device="cuda")
        R = np.zeros((k, k), order="F")
        check(lib.tt_kernel_global_factors(self._h, None, _ptr(Q), R.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           _stream_ptr(stream)))
        return Q, R

    def global_online(self, theta, stream=None):
        """W(theta_b) (B, k, k): PSD part of R Hhat R^T."""
        lib = _lib.load()
        k = ctypes.c_int()
        check(lib.tt_kernel_global_factors(self._h, ctypes.byref(k), None, None, _stream_ptr(stream)))
        k = k.value
        theta = _theta(theta, self.d_theta, self.dtype)
        B = theta.shape[0]
        W = torch.empty((B, k, k), dtype=self.dtype, device="cuda")
        check(lib.tt_kernel_global_online(self._h, _ptr(theta), B, _ptr(W), _stream_ptr(stream)))
        return W.transpose(1, 2)   # stored column-major

    def phase4_round(self, eps, stream=None):
        """Phase 4 of Algorithm 2 in place: TT-Round of [S, parameter cores, T^T]
        with tolerance eps; U, V and the parameter cores become the rounded ones."""
        if not eps > 0:
            raise ValueError("eps must be positive")
        check(_lib.load().tt_kernel_phase4_round(self._h, float(eps), _stream_ptr(stream)))
        inf = self.info()
        self.r_s, self.r_t = inf["r_s"], inf["r_t"]
        return self

    def global2_online(self, theta, eps, stream=None):
        """PTTK-Global-2 for one theta (d_theta values): (Z (N, r_c), lam (r_c,))
        with K(X, X; theta) ~ Z diag(lam) Z^T, Z = Q Uhat."""
        lib = _lib.load()
        if not eps > 0:
            raise ValueError("eps must be positive")
        k = ctypes.c_int()
        check(lib.tt_kernel_global_factors(self._h, ctypes.byref(k), None, None, _stream_ptr(stream)))
        k = k.value
        th = None
        if self.d_theta:
            th = _theta(torch.as_tensor(theta, dtype=torch.float64).reshape(1, -1), self.d_theta, self.dtype, 1)
        Z = torch.empty((self.n_src, k), dtype=self.dtype, device="cuda")
        lam = torch.empty((k,), dtype=self.dtype, device="cuda")
        rc = ctypes.c_int()
        check(lib.tt_kernel_global2_online(self._h, _ptr(th), float(eps), _ptr(Z), k, _ptr(lam), ctypes.byref(rc),
                                           _stream_ptr(stream)))
        r = rc.value
        return Z[:, :r], lam[:r]

    def global2_apply(self, Z, lam, X, stream=None):
        """y_b = Z diag(lam) Z^T x_b for rows x_b of X (B, N), (Z, lam) from global2_online."""
        lib = _lib.load()
        rc = int(lam.shape[0])
        if Z.dim() != 2 or tuple(Z.shape) != (self.n_src, rc):
            raise ValueError(f"Z: expected shape ({self.n_src}, {rc}), got {tuple(Z.shape)}")
        B = _chk(X, "X", None, self.n_src).shape[0]
        X = _dev(X, self.dtype)
        Zc = Z.to(device="cuda", dtype=self.dtype).contiguous()
        lc = lam.to(device="cuda", dtype=self.dtype).contiguous()
        Y = torch.empty((B, self.n_src), dtype=self.dtype, device="cuda")
        check(lib.tt_kernel_global2_apply(self._h, _ptr(Zc), max(rc, 1), _ptr(lc), rc, B, _ptr(X), self.n_src,
                                          _ptr(Y), self.n_src, _stream_ptr(stream)))
        return Y

    def global_apply(self, X, theta=None, W=None, stream=None):
        """y_b = Q W_b Q^T x_b for rows x_b of X (B, N); theta (B, d_theta) or W (B, k, k)."""
        if (theta is None) == (W is None):
            raise ValueError("give exactly one of theta and W")
        B = _chk(X, "X", None, self.n_src).shape[0]
        if theta is not None:
            _theta(theta, self.d_theta, self.dtype, B, convert=False)
        X = _dev(X, self.dtype)
        Y = torch.empty((B, self.n_src), dtype=self.dtype, device="cuda")
        th = None
        Wc = None
        if theta is not None:
            th = _theta(theta, self.d_theta, self.dtype, B)
        else:
            k = ctypes.c_int()
            check(_lib.load().tt_kernel_global_factors(self._h, ctypes.byref(k), None, None, _stream_ptr(stream)))
            if W.dim() != 3 or tuple(W.shape) != (B, k.value, k.value):
                raise ValueError(f"W: expected shape ({B}, {k.value}, {k.value}), got {tuple(W.shape)}")
            Wc = W.to(device="cuda", dtype=self.dtype).transpose(1, 2).contiguous()   # column-major per matrix
        check(_lib.load().tt_kernel_global_apply(self._h, _ptr(th), _ptr(Wc), B, _ptr(X), self.n_src, _ptr(Y),
                                                 self.n_src, _stream_ptr(stream)))
        return Y


class _ApplyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, X, kern):
        Y, W = kern.apply(theta, X, save_w=True)
        ctx.kern = kern
        ctx.save_for_backward(theta, W)
        return Y

    @staticmethod
    def backward(ctx, gY):
        theta, W = ctx.saved_tensors
        kern = ctx.kern
        dX, dth = kern.apply_backward(theta, gY, W=W, want_dx=ctx.needs_input_grad[1],
                                      want_dtheta=ctx.needs_input_grad[0])
        if dth is not None:
            dth = dth.reshape(theta.shape)
        return dth, dX, None


def kernel_apply(kern: TTKernel, theta, X):
    """Differentiable y_b = U M(theta_b) V^T x_b (gradients in theta and X)."""
    return _ApplyFn.apply(theta, X, kern)


def eval_entries(idx, kind, d, box_s, box_t, box_theta=(), n_spatial=16, n_param=None, kernel_const=0.0,
                 theta_fixed=None, stream=None):
    """f_kappa at grid multi-indices idx (P, D) int32, on the device, float64."""
    lib = _lib.load()
    p = make_params(kind, d, box_s, box_t, box_theta, n_spatial, n_param, kernel_const=kernel_const,
                    theta_fixed=theta_fixed)
    D = 2 * int(d) + p.d_theta
    if idx.dim() != 2 or idx.shape[1] != D:
        raise ValueError(f"idx: expected shape (P, {D}), got {tuple(idx.shape)}")
    n = [p.n_spatial] * int(d) + [p.n_param] * p.d_theta + [p.n_spatial] * int(d)
    if idx.numel() and (int(idx.min()) < 0 or any(int(idx[:, j].max()) >= n[j] for j in range(D))):
        raise ValueError("idx: node index out of range")
    idx = idx.to(device="cuda", dtype=torch.int32).contiguous()
    out = torch.empty(idx.shape[0], dtype=torch.float64, device="cuda")
    check(lib.tt_kernel_eval_entries(ctypes.byref(p), _ptr(idx), idx.shape[0], _ptr(out), _stream_ptr(stream)))
    return out


def eval_dense(X, Y, theta, kind, d, dtype=torch.float64, kernel_const=0.0, stream=None):
    """Dense K(X, Y; theta) block on the device, rows = sources."""
    lib = _lib.load()
    p = make_params(kind, d, [[0, 1]] * d, [[0, 1]] * d, [[0, 1]] * KIND_DTHETA[kind], dtype=dtype,
                    kernel_const=kernel_const)
    if np.size(theta) != KIND_DTHETA[kind]:
        raise ValueError(f"theta: expected {KIND_DTHETA[kind]} values, got {np.size(theta)}")
    Xs, Ys = _soa(X, dtype, d, "X"), _soa(Y, dtype, d, "Y")
    nx, ny = Xs.shape[1], Ys.shape[1]
    K = torch.empty((ny, nx), dtype=dtype, device="cuda")       # column-major nx x ny
    th = (ctypes.c_double * 2)(*([float(v) for v in np.ravel(theta)] + [0.0, 0.0])[:2])
    check(lib.tt_kernel_eval_dense(ctypes.byref(p), _ptr(Xs), nx, _ptr(Ys), ny, th, _ptr(K), nx,
                                   _stream_ptr(stream)))
    return K.t()


class TTBatch:
    """An interaction list of source/target box pairs (one TT per geometry
    class, Phase 3 for every pair in one persistent launch, batched apply and
    backward as one captured graph).  pairs: list of dicts with box_s, box_t
    ((d, 2) boxes), src_off, n_src, tgt_off, n_tgt (rows of X / Y)."""

    def __init__(self, handle, params, dtype, pairs, n_x, n_y, status):
        self._h = handle
        self.params = params
        self.dtype = dtype
        self.pairs = pairs
        self.n_x, self.n_y = n_x, n_y
        self.status = status
        self.d_theta = params.d_theta

    @classmethod
    def build(cls, pairs, X, Y, kind, d, box_theta=(), n_spatial=16, n_param=None, tol=1e-6,
              dtype=torch.float32, stream=None, **kw):
        lib = _lib.load()
        p = make_params(kind, d, [[0, 1]] * d, [[2, 3]] * d, box_theta, n_spatial, n_param, tol, dtype, **kw)
        arr = (Pair * len(pairs))()
        for i, q in enumerate(pairs):
            bs = np.asarray(q["box_s"], float).reshape(-1)
            bt = np.asarray(q["box_t"], float).reshape(-1)
            for j in range(bs.size):
                arr[i].box_s[j] = bs[j]
                arr[i].box_t[j] = bt[j]
            arr[i].src_off, arr[i].n_src = int(q["src_off"]), int(q["n_src"])
            arr[i].tgt_off, arr[i].n_tgt = int(q["tgt_off"]), int(q["n_tgt"])
            if arr[i].src_off < 0 or arr[i].n_src < 0 or arr[i].src_off + arr[i].n_src > X.shape[0] or \
                    arr[i].tgt_off < 0 or arr[i].n_tgt < 0 or arr[i].tgt_off + arr[i].n_tgt > Y.shape[0]:
                raise ValueError(f"pair {i}: point range outside X ({X.shape[0]}) or Y ({Y.shape[0]})")
        Xs, Ys = _soa(X, dtype, d, "X"), _soa(Y, dtype, d, "Y")
        h = ctypes.c_void_p()
        st = check(lib.tt_kernel_batch_build(ctypes.byref(p), arr, len(pairs), _ptr(Xs), Xs.shape[1], _ptr(Ys),
                                             Ys.shape[1], _stream_ptr(stream), ctypes.byref(h)))
        return cls(h, p, dtype, pairs, Xs.shape[1], Ys.shape[1], st)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().tt_kernel_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def configure(self, use_graph=True, factor_grid=0, reduce_rows=0):
        check(_lib.load().tt_kernel_batch_configure(self._h, int(bool(use_graph)), int(factor_grid),
                                                    int(reduce_rows)))

    def refactor(self, X, Y, stream=None):
        """Phase 3 again for points (same layout); returns the SoA copies used."""
        if X.shape[0] != self.n_x or Y.shape[0] != self.n_y:
            raise ValueError(f"X, Y: expected {self.n_x} and {self.n_y} points")
        Xs, Ys = _soa(X, self.dtype, self.params.d, "X"), _soa(Y, self.dtype, self.params.d, "Y")
        check(_lib.load().tt_kernel_batch_factor(self._h, _ptr(Xs), _ptr(Ys), _stream_ptr(stream)))
        return Xs, Ys

    def refactor_soa(self, Xs, Ys, stream=None):
        _out(Xs, "Xs", (self.params.d, self.n_x), self.dtype)
        _out(Ys, "Ys", (self.params.d, self.n_y), self.dtype)
        check(_lib.load().tt_kernel_batch_factor(self._h, _ptr(Xs), _ptr(Ys), _stream_ptr(stream)))

    def info(self):
        lib = _lib.load()
        inf = BatchInfo()
        check(lib.tt_kernel_batch_get_info(self._h, ctypes.byref(inf), None, None))
        cop = (ctypes.c_int * max(inf.num_pairs, 1))()
        cr = (ctypes.c_int * (9 * max(inf.num_classes, 1)))()
        check(lib.tt_kernel_batch_get_info(self._h, None, cop, cr))
        D = 2 * self.params.d + self.params.d_theta
        return {"num_pairs": inf.num_pairs, "num_classes": inf.num_classes, "kernel_evals": inf.kernel_evals,
                "factor_rows": inf.factor_rows, "t_cross_ms": inf.t_cross_ms, "t_round_ms": inf.t_round_ms,
                "t_factor_ms": inf.t_factor_ms, "factor_grid": inf.factor_grid, "reduce_rows": inf.reduce_rows,
                "graph": bool(inf.graph), "class_of_pair": list(cop)[:inf.num_pairs],
                "class_ranks": [list(cr[9 * c:9 * c + D + 1]) for c in range(inf.num_classes)]}

    def class_kernel(self, c):
        """The TTKernel of class c (borrowed from the batch, canonical frame, no points)."""
        h = ctypes.c_void_p()
        check(_lib.load().tt_kernel_batch_get_class(self._h, int(c), ctypes.byref(h)))
        k = TTKernel.__new__(TTKernel)
        k._borrowed = True
        k._owner = self
        TTKernel.__init__(k, h, self.params, self.dtype, 0, 0)
        return k

    def factors(self, pair, stream=None):
        inf = self.info()
        c = inf["class_of_pair"][pair]
        r = inf["class_ranks"][c]
        d = self.params.d
        rs, rt = r[d], r[d + self.d_theta]
        q = self.pairs[pair]
        U = torch.empty((int(q["n_src"]), rs), dtype=self.dtype, device="cuda")
        V = torch.empty((int(q["n_tgt"]), rt), dtype=self.dtype, device="cuda")
        check(_lib.load().tt_kernel_batch_get_factors(self._h, int(pair), _ptr(U), _ptr(V), _stream_ptr(stream)))
        return U, V

    def apply(self, theta, X, G=None, want_dx=True, want_dtheta=True, out=None, stream=None):
        """Y (B, n_x) = sum over pairs; with G (B, n_x) also dX (B, n_y) and dtheta (B, d_theta).
        out: optional (Y, dX, dtheta) tensors to write into (keeps the captured graph valid)."""
        B = _chk(X, "X", None, self.n_y).shape[0]
        theta = _theta(theta, self.d_theta, self.dtype, B, convert=False)
        if G is not None:
            _chk(G, "G", B, self.n_x)
        theta, X = _dev(theta, self.dtype), _dev(X, self.dtype)
        if out is not None:
            Y, dX, dth = out
            _out(Y, "out[0] (Y)", (B, self.n_x), self.dtype)
            if G is not None and dX is not None:
                _out(dX, "out[1] (dX)", (B, self.n_y), self.dtype)
            if G is not None and dth is not None and self.d_theta > 0:
                _out(dth, "out[2] (dtheta)", (B, self.d_theta), self.dtype)
        else:
            Y = torch.empty((B, self.n_x), dtype=self.dtype, device="cuda")
            dX = torch.empty((B, self.n_y), dtype=self.dtype, device="cuda") if (G is not None and want_dx) \
                else None
            dth = torch.empty((B, max(self.d_theta, 1)), dtype=self.dtype, device="cuda") \
                if (G is not None and want_dtheta and self.d_theta > 0) else None
        Gc = _dev(G, self.dtype)
        check(_lib.load().tt_kernel_batch_apply(self._h, _ptr(theta), B, _ptr(X), self.n_y, _ptr(Y), self.n_x,
                                                _ptr(Gc), self.n_x, _ptr(dX), self.n_y, _ptr(dth),
                                                _stream_ptr(stream)))
        return (Y, dX, dth) if G is not None else Y


class HMatrix:
    """A parametric hierarchical matrix for K(X, X; theta): far blocks (the
    interaction lists of a uniform tree over the root box, every level >= 2)
    in the PTTK low-rank form through a pair batch, near blocks (neighbouring
    leaves) summed directly.  X: (N, d) points in the root box."""

    def __init__(self, handle, params, dtype, n):
        self._h = handle
        self.params = params
        self.dtype = dtype
        self.n = n
        self.d_theta = params.d_theta
        self.status = 0

    @classmethod
    def build(cls, X, kind, d, box, box_theta=(), leaf_points=64, n_spatial=16, n_param=None, tol=1e-6,
              dtype=torch.float32, stream=None, **kw):
        lib = _lib.load()
        if int(leaf_points) < 1:
            raise ValueError("leaf_points must be positive")
        p = make_params(kind, d, box, box, box_theta, n_spatial, n_param, tol, dtype, **kw)
        Xs = _soa(X, dtype, d, "X")
        h = ctypes.c_void_p()
        st = check(lib.tt_kernel_hmat_build(ctypes.byref(p), _ptr(Xs), Xs.shape[1], int(leaf_points),
                                            _stream_ptr(stream), ctypes.byref(h)))
        H = cls(h, p, dtype, Xs.shape[1])
        H.status = st   # 0, or TTK_WARN_NOT_CONVERGED (1): a class's cross stopped above tol
        return H

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().tt_kernel_hmat_destroy(h)
            except Exception:
                pass

    def info(self):
        inf = _lib.HmatInfo()
        check(_lib.load().tt_kernel_hmat_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _lib.HmatInfo._fields_}

    def lists(self):
        """(far (F, 7): level, source cell, target cell; near (M, 6); perm (N,))
        as numpy int32 arrays."""
        inf = self.info()
        far = np.zeros((max(inf["far_pairs"], 1), 7), dtype=np.int32)
        near = np.zeros((max(inf["near_pairs"], 1), 6), dtype=np.int32)
        perm = np.zeros(self.n, dtype=np.int32)
        P32 = ctypes.POINTER(ctypes.c_int32)
        check(_lib.load().tt_kernel_hmat_get_lists(self._h, far.ctypes.data_as(P32), near.ctypes.data_as(P32),
                                                   perm.ctypes.data_as(P32)))
        return far[:inf["far_pairs"]], near[:inf["near_pairs"]], perm

    def apply(self, theta, X, stream=None):
        """Y[b] = H(theta_b) X[b] for rows of X (B, N) and theta (B, d_theta)."""
        B = _chk(X, "X", None, self.n).shape[0]
        th = _theta(theta, self.d_theta, self.dtype, B) if self.d_theta else None
        X = _dev(X, self.dtype)
        Y = torch.empty((B, self.n), dtype=self.dtype, device="cuda")
        check(_lib.load().tt_kernel_hmat_apply(self._h, _ptr(th), B, _ptr(X), self.n, _ptr(Y), self.n,
                                               _stream_ptr(stream)))
        return Y
