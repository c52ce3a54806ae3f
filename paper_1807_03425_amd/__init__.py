"""Python binding of libsap.so, the gfx950 Secant-Avoidance Projection library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  If the library
has not been built, every entry point raises immediately; there is no
fallback of any kind.

    ctx = SapContext(X, P0, form="fused")       # X: N x n cuda tensor, P0: n x k float64
    res = ctx.min_secant()                       # dict: min_norm, i, j, certified, ...
    tr  = ctx.run(200)                           # per-iteration min / (i, j) / certified
    L   = SoftMinSecant.apply(P32, ctx, 0.01)    # differentiable soft-min (fused form)
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path
from typing import Optional

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libsap.so"

SAP_OK = 0
STATUS = {0: "SAP_OK", 1: "SAP_ERR_INVALID_ARG", 2: "SAP_ERR_NONFINITE",
          3: "SAP_ERR_NO_PAIRS", 4: "SAP_ERR_OUT_OF_MEMORY", 5: "SAP_ERR_DEVICE",
          6: "SAP_ERR_NOT_ORTHONORMAL", 7: "SAP_ERR_POISONED", 8: "SAP_ERR_UNSUPPORTED",
          9: "SAP_ERR_CAPACITY"}
SAP_F64, SAP_F32 = 0, 1
SAP_PLAIN, SAP_FUSED = 0, 1
SAP_STEP_LITERAL, SAP_STEP_NORMALIZED = 0, 1
SAP_GEMM_F64, SAP_GEMM_F32, SAP_GEMM_BF16 = 0, 1, 2
GEMMS = {"f64": SAP_GEMM_F64, "f32": SAP_GEMM_F32, "bf16": SAP_GEMM_BF16}


class SapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sap_config(C.Structure):
    _fields_ = [("N", C.c_int64), ("n", C.c_int32), ("k", C.c_int32),
                ("dtype", C.c_int32), ("form", C.c_int32), ("rule", C.c_int32),
                ("close_cap", C.c_int32), ("cand_cap", C.c_int32), ("gemm", C.c_int32),
                ("alpha", C.c_double),
                ("min_len", C.c_double), ("close_d", C.c_double)]


class sap_min_result(C.Structure):
    _fields_ = [("min_norm", C.c_double), ("runner_up", C.c_double), ("i", C.c_int64),
                ("j", C.c_int64), ("pair_index", C.c_int64), ("coarse_min", C.c_double),
                ("window", C.c_double), ("certified", C.c_int32), ("runner_up_exact", C.c_int32),
                ("n_rescored", C.c_int32), ("t", C.c_int32), ("n_units", C.c_int32),
                ("reserved", C.c_int32)]


class sap_info_t(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_dropped", C.c_int64), ("n_close", C.c_int64),
                ("close_d", C.c_double), ("e_abs", C.c_double), ("e_rel", C.c_double),
                ("radius", C.c_double), ("bytes_per_iter", C.c_int64),
                ("device_bytes", C.c_int64), ("n_tiles", C.c_int64)]


class sap_profile_t(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8)]


class sap_pca_info(C.Structure):
    _fields_ = [("sigma", C.c_double * 16), ("residual", C.c_double), ("ms", C.c_double),
                ("iters", C.c_int32), ("converged", C.c_int32)]


class sap_batch_problem(C.Structure):
    _fields_ = [("set", C.c_int32), ("k", C.c_int32), ("rule", C.c_int32),
                ("reserved", C.c_int32), ("alpha", C.c_double)]


class sap_batch_stats(C.Structure):
    _fields_ = [("init_ms", C.c_double), ("run_ms", C.c_double), ("n_pairs", C.c_int64),
                ("scratch_bytes", C.c_int64)]


PROFILE_SLOTS = ("gemm", "pass", "select", "sm_fwd", "sm_bwd", "sm_other", "select_gemm")

_lib: Optional[C.CDLL] = None

# name -> (restype, argtypes)
_SIGS = {
    "sap_init": (C.c_int, [C.POINTER(sap_config), C.c_void_p, C.c_int64, C.c_void_p,
                           C.c_void_p, C.POINTER(C.c_void_p)]),
    "sap_min_secant": (C.c_int, [C.c_void_p, C.POINTER(sap_min_result)]),
    "sap_step": (C.c_int, [C.c_void_p, C.POINTER(sap_min_result)]),
    "sap_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sap_get_P": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sap_set_P": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sap_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sap_pca_init": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(sap_pca_info), C.c_int32]),
    "sap_info": (C.c_int, [C.c_void_p, C.POINTER(sap_info_t)]),
    "sap_softmin_fwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "sap_softmin_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "sap_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "sap_profile_read": (C.c_int, [C.c_void_p, C.POINTER(sap_profile_t)]),
    "sap_batch_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_int32,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.POINTER(sap_batch_stats)]),
    "sap_batch_run_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(sap_batch_stats)]),
    "sap_destroy": (C.c_int, [C.c_void_p]),
    "sap_last_error": (C.c_char_p, [C.c_void_p]),
}


def lib() -> C.CDLL:
    """The loaded libsap.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, handle=None):
    if st != SAP_OK:
        msg = lib().sap_last_error(handle)
        raise SapError(st, msg.decode() if msg else "")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class SapContext:
    """One SAP problem on one GPU: borrowed X (N x n, cuda, float32/float64,
    unit stride along n) and the library-owned state derived from it."""

    def __init__(self, X, P0, form: str = "fused", alpha: float = 0.01,
                 min_len: float = 0.0, rule: str = "literal", close_d: float = -1.0,
                 close_cap: int = 0, cand_cap: int = 0, gemm: str = "f64", stream=None):
        import torch
        if X.dim() != 2 or X.device.type != "cuda" or X.stride(1) != 1:
            raise ValueError("X must be a 2-D cuda tensor with unit stride along n")
        if X.dtype not in (torch.float32, torch.float64):
            raise ValueError("X must be float32 or float64")
        P0 = P0.to(device=X.device, dtype=torch.float64).contiguous()
        N, n = X.shape
        if P0.dim() != 2 or P0.shape[0] != n:
            raise ValueError("P0 must be n x k")
        k = P0.shape[1]
        cfg = sap_config(N=N, n=n, k=k,
                         dtype=SAP_F64 if X.dtype == torch.float64 else SAP_F32,
                         form={"plain": SAP_PLAIN, "fused": SAP_FUSED}[form],
                         rule={"literal": SAP_STEP_LITERAL, "normalized": SAP_STEP_NORMALIZED}[rule],
                         close_cap=int(close_cap), cand_cap=int(cand_cap), gemm=GEMMS[gemm],
                         alpha=float(alpha), min_len=float(min_len),
                         close_d=float(close_d))
        self._X = X                      # keep the borrowed buffer alive
        self._stream = stream
        self.N, self.n, self.k, self.form = int(N), int(n), int(k), form
        self.dtype = X.dtype
        h = C.c_void_p()
        st = lib().sap_init(C.byref(cfg), _dptr(X), X.stride(0), _dptr(P0),
                            _stream_ptr(stream), C.byref(h))
        _check(st, None)
        self._h = h

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().sap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("SapContext is closed")
        return self._h

    # -- evaluation / iteration
    @staticmethod
    def _res(r: sap_min_result) -> dict:
        return dict(min_norm=r.min_norm, runner_up=r.runner_up, runner_up_exact=r.runner_up_exact,
                    i=r.i, j=r.j, pair_index=r.pair_index, coarse_min=r.coarse_min,
                    window=r.window, certified=r.certified, n_rescored=r.n_rescored, t=r.t,
                    n_window_tiles=r.n_units)

    def min_secant(self) -> dict:
        r = sap_min_result()
        _check(lib().sap_min_secant(self.handle, C.byref(r)), self.handle)
        return self._res(r)

    def step(self, sync: bool = True) -> Optional[dict]:
        if not sync:
            _check(lib().sap_step(self.handle, None), self.handle)
            return None
        r = sap_min_result()
        _check(lib().sap_step(self.handle, C.byref(r)), self.handle)
        return self._res(r)

    def run(self, iters: int, out: Optional[dict] = None) -> dict:
        import torch
        m = iters + 1
        dev = self._X.device
        if out is None:
            out = dict(min=torch.empty(m, dtype=torch.float64, device=dev),
                       ij=torch.empty((m, 2), dtype=torch.int64, device=dev),
                       certified=torch.empty(m, dtype=torch.int32, device=dev))
        _check(lib().sap_run(self.handle, int(iters), _dptr(out["min"]),
                             _dptr(out["ij"]) if out.get("ij") is not None else None,
                             _dptr(out["certified"]) if out.get("certified") is not None else None),
               self.handle)
        return out

    # -- state
    def get_P(self):
        import torch
        P = torch.empty((self.n, self.k), dtype=torch.float64, device=self._X.device)
        _check(lib().sap_get_P(self.handle, _dptr(P)), self.handle)
        return P

    def set_P(self, P):
        import torch
        P = P.to(device=self._X.device, dtype=torch.float64).contiguous()
        _check(lib().sap_set_P(self.handle, _dptr(P)), self.handle)

    def pca_init(self, set_P: bool = False):
        """Algorithm 1's initial projection: the top-k left singular vectors
        of the secant matrix (sap_pca_init).  Returns (P n x k float64 cuda
        tensor, info dict); with set_P it also becomes the current P."""
        import torch
        P = torch.empty((self.n, self.k), dtype=torch.float64, device=self._X.device)
        info = sap_pca_info()
        _check(lib().sap_pca_init(self.handle, _dptr(P), C.byref(info), 1 if set_P else 0), self.handle)
        return P, dict(sigma=list(info.sigma)[:self.k], residual=info.residual, ms=info.ms,
                       iters=info.iters, converged=info.converged)

    def set_stream(self, stream):
        self._stream = stream
        _check(lib().sap_set_stream(self.handle, _stream_ptr(stream)), self.handle)

    def info(self) -> dict:
        r = sap_info_t()
        _check(lib().sap_info(self.handle, C.byref(r)), self.handle)
        return {f: getattr(r, f) for f, _ in sap_info_t._fields_}

    # -- per-kernel timing
    def profile(self, on: bool = True):
        _check(lib().sap_profile_enable(self.handle, 1 if on else 0), self.handle)

    def profile_read(self) -> dict:
        r = sap_profile_t()
        _check(lib().sap_profile_read(self.handle, C.byref(r)), self.handle)
        return {name: dict(ms=r.ms[i], launches=r.launches[i])
                for i, name in enumerate(PROFILE_SLOTS)}

    # -- soft-min
    def softmin_fwd(self, P, tau: float):
        """Soft-min loss at P (1-element float32 tensor).  The handle keeps
        this forward's P, Y and L for the next softmin_bwd."""
        import torch
        P = P.to(device=self._X.device, dtype=torch.float32).contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=self._X.device)
        _check(lib().sap_softmin_fwd(self.handle, _dptr(P), float(tau), _dptr(loss)), self.handle)
        self._sm_token = getattr(self, "_sm_token", 0) + 1
        return loss

    def softmin_bwd(self, P, tau: float, grad_loss):
        """grad_loss * dL/dP at the P of the last softmin_fwd (same P, bit for
        bit, and the same tau; otherwise SapError INVALID_ARG)."""
        import torch
        P = P.to(device=self._X.device, dtype=torch.float32).contiguous()
        g = grad_loss.to(device=self._X.device, dtype=torch.float32).reshape(1).contiguous()
        dP = torch.empty_like(P)
        _check(lib().sap_softmin_bwd(self.handle, _dptr(P), float(tau), _dptr(g), _dptr(dP)),
               self.handle)
        return dP


def batch_run(X, sets, problems, P0s, iters: int, set_min_len=None, cand_cap: int = 0,
              stream=None, noalloc: bool = False) -> dict:
    """Run independent SAP problems on point subsets of X in one launch
    (sap_batch_run).

    X: N x n cuda tensor (float32/float64, unit stride along n).
    sets: list of 1-D integer index arrays (rows of X; the order defines the
        local indices of each set's pairs).
    problems: list of dicts with keys set, k, and optionally alpha (0.01),
        rule ("literal" | "normalized").
    P0s: list of n x k_b starting projections (one per problem).
    Returns dict(min=(B, iters+1) float64, ij=(B, iters+1, 2) int64,
    certified=(B, iters+1) int32 device tensors, P=[n x k_b float64 device
    tensors], stats=dict)."""
    import numpy as np
    import torch
    if X.dim() != 2 or X.device.type != "cuda" or X.stride(1) != 1:
        raise ValueError("X must be a 2-D cuda tensor with unit stride along n")
    if X.dtype not in (torch.float32, torch.float64):
        raise ValueError("X must be float32 or float64")
    dev = X.device
    N, n = X.shape
    offs = np.zeros(len(sets) + 1, dtype=np.int64)
    for s_i, ix in enumerate(sets):
        offs[s_i + 1] = offs[s_i] + len(ix)
    pts = np.ascontiguousarray(np.concatenate([np.asarray(ix, dtype=np.int32) for ix in sets]))
    ml = None if set_min_len is None else np.ascontiguousarray(set_min_len, dtype=np.float64)
    B = len(problems)
    probs = (sap_batch_problem * B)()
    ks = []
    for b, q in enumerate(problems):
        rule = {"literal": SAP_STEP_LITERAL, "normalized": SAP_STEP_NORMALIZED}[q.get("rule", "literal")]
        probs[b] = sap_batch_problem(int(q["set"]), int(q["k"]), rule, 0, float(q.get("alpha", 0.01)))
        ks.append(int(q["k"]))
    P0 = torch.cat([torch.as_tensor(P).to(device=dev, dtype=torch.float64).reshape(-1) for P in P0s]).contiguous()
    P_out = torch.empty_like(P0)
    m = iters + 1
    tmin = torch.empty((B, m), dtype=torch.float64, device=dev)
    tij = torch.empty((B, m, 2), dtype=torch.int64, device=dev)
    tcert = torch.empty((B, m), dtype=torch.int32, device=dev)
    st = sap_batch_stats()
    fn = lib().sap_batch_run_noalloc if noalloc else lib().sap_batch_run
    rc = fn(_dptr(X), SAP_F64 if X.dtype == torch.float64 else SAP_F32, N, n, X.stride(0),
            len(sets), offs.ctypes.data_as(C.c_void_p), pts.ctypes.data_as(C.c_void_p),
            ml.ctypes.data_as(C.c_void_p) if ml is not None else None, B, probs, _dptr(P0),
            int(iters), int(cand_cap), _dptr(P_out), _dptr(tmin), _dptr(tij), _dptr(tcert),
            _stream_ptr(stream), C.byref(st))
    _check(rc, None)
    Ps, off = [], 0
    for k in ks:
        Ps.append(P_out[off:off + n * k].reshape(n, k))
        off += n * k
    return dict(min=tmin, ij=tij, certified=tcert, P=Ps,
                stats=dict(init_ms=st.init_ms, run_ms=st.run_ms, n_pairs=st.n_pairs,
                           scratch_bytes=st.scratch_bytes))


def _make_softmin_function():
    import torch

    class SoftMinSecant(torch.autograd.Function):
        """L(P) = -tau log sum_{i<j} exp(-||P^T s_ij|| / tau) with the library's
        hand-written backward.  Gradients flow to P only."""

        @staticmethod
        def forward(fctx, P, sap_ctx: SapContext, tau: float):
            loss = sap_ctx.softmin_fwd(P.detach(), tau)
            fctx.sap_ctx, fctx.tau = sap_ctx, tau
            fctx.token = sap_ctx._sm_token
            fctx.save_for_backward(P.detach())
            return loss.reshape(())

        @staticmethod
        def backward(fctx, g):
            (P,) = fctx.saved_tensors
            c = fctx.sap_ctx
            if c._sm_token != fctx.token:
                # another forward ran since this one: recompute its state
                c.softmin_fwd(P, fctx.tau)
                fctx.token = c._sm_token
            dP = c.softmin_bwd(P, fctx.tau, g)
            return dP.to(P.dtype), None, None

    return SoftMinSecant


class _LazySoftMin:
    _fn = None

    def apply(self, *args):
        if _LazySoftMin._fn is None:
            _LazySoftMin._fn = _make_softmin_function()
        return _LazySoftMin._fn.apply(*args)


SoftMinSecant = _LazySoftMin()

__all__ = ["SapContext", "SoftMinSecant", "SapError", "lib", "LIB_PATH", "sap_config",
           "sap_min_result", "sap_info_t", "sap_profile_t", "sap_batch_problem", "sap_batch_stats",
           "sap_pca_info",
           "batch_run"]
