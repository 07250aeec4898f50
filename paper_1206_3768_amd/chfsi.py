"""Thin ctypes binding of libchfsi.so (include/chfsi.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; this module converts torch device
tensors to pointers and back.  It raises if the library is missing -- there is no CPU fallback.

Layout convention: the library is column-major.  A column-major ``rows x cols`` matrix lives in a
contiguous torch tensor of shape ``(cols, rows)`` (each row of the tensor is one column of the
matrix); :func:`to_device` and :func:`to_numpy` convert from and to numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfsi.so")
_lib = None

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}
DEG_FIXED, DEG_ANALYTIC, DEG_LEARNED, DEG_RANDOM = 0, 1, 2, 3
TRACE_COLS = 10
MLP_NPARAM = 8769
SUCCESS, ERR_ARG, ERR_NOT_HPD, ERR_NO_CONVERGENCE, ERR_NUMERIC, ERR_DEVICE, ERR_ALLOC, ERR_TOO_LARGE = range(8)
STATUS_NAMES = {0: "success", 1: "invalid argument", 2: "not HPD", 3: "no convergence", 4: "numeric",
                5: "device", 6: "alloc", 7: "exceeds the fixed scratch"}
NOALLOC_SCRATCH_BYTES = 64 << 20


class ChfsiError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nev", C.c_int), ("nex", C.c_int), ("deg", C.c_int), ("tol", C.c_double),
                ("max_loops", C.c_int), ("lanczos_steps", C.c_int), ("filter_precision", C.c_int),
                ("degree_policy", C.c_int), ("deg_min", C.c_int), ("deg_max", C.c_int),
                ("seed", C.c_ulonglong), ("have_bounds", C.c_int), ("mu1", C.c_double), ("a", C.c_double),
                ("trace", C.c_int), ("switch_residual", C.c_double), ("deg_margin", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("loops", C.c_int), ("nlocked", C.c_int), ("filtered_vectors", C.c_longlong),
                ("matvecs", C.c_longlong), ("filter_flops", C.c_double),
                ("t_reduce", C.c_double), ("t_lanczos", C.c_double), ("t_filter", C.c_double),
                ("t_qr", C.c_double), ("t_rr", C.c_double), ("t_resid", C.c_double), ("t_lock", C.c_double),
                ("t_back", C.c_double), ("t_total", C.c_double), ("mu1", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("norm_a", C.c_double), ("lanczos_steps", C.c_int),
                ("precision_switches", C.c_int), ("filter_launches", C.c_int), ("t_filter_kernels", C.c_double),
                ("t_filter_steps", C.c_double), ("status", C.c_int), ("factor_reused", C.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class LobpcgParams(C.Structure):
    _fields_ = [("nev", C.c_int), ("bs", C.c_int), ("maxiter", C.c_int), ("tol", C.c_double), ("gen", C.c_int),
                ("seed", C.c_ulonglong)]


class LobpcgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("nconv", C.c_int), ("matvecs", C.c_longlong), ("bmatvecs", C.c_longlong),
                ("dropped", C.c_int), ("t_reduce", C.c_double), ("t_iterate", C.c_double), ("t_total", C.c_double),
                ("restarts", C.c_int)]


class TilePlan(C.Structure):
    _fields_ = [("bm", C.c_int), ("bn", C.c_int), ("ksplit", C.c_int), ("fused", C.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("nev", C.c_int), ("nex", C.c_int), ("A", C.c_void_p), ("lda", C.c_int),
                ("S", C.c_void_p), ("lds", C.c_int), ("X", C.c_void_p), ("ldx", C.c_int),
                ("x_is_guess", C.c_int), ("lambda_", C.c_void_p), ("resid", C.c_void_p)]


EXPORTED = ["chfsi_default_params", "chfsi_create", "chfsi_destroy", "chfsi_solve", "chfsi_solve_batched",
            "chfsi_filter", "chfsi_reduce", "chfsi_reduce_explicit", "chfsi_lanczos", "chfsi_orthonormalize", "chfsi_rayleigh_ritz",
            "chfsi_zgemm", "chfsi_random_block", "chfsi_set_degree_model", "chfsi_get_trace", "chfsi_mlp_forward",
            "chfsi_mlp_loss_grad", "chfsi_mlp_adam", "chfsi_mlp_train", "chfsi_status_string",
            "chfsi_filter_kernel_time", "chfsi_autotune_filter", "chfsi_set_filter_plan",
            "chfsi_filter_launch_log", "chfsi_set_batched_plan", "chfsi_autotune_batched",
            "chfsi_batched_info", "chfsi_filter_noalloc", "chfsi_correlation", "chfsi_lobpcg",
            "chfsi_lobpcg_default_params", "chfsi_autotune_batched_tiles", "chfsi_set_batched_tiles"]


def load():
    """Loads libchfsi.so and declares the C signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1206_3768_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, u = C.c_void_p, C.c_int, C.c_double, C.c_ulonglong
    lib.chfsi_default_params.argtypes = [C.POINTER(Params)]
    lib.chfsi_default_params.restype = None
    lib.chfsi_create.argtypes = [C.POINTER(vp), i, vp]
    lib.chfsi_destroy.argtypes = [vp]
    lib.chfsi_solve.argtypes = [vp, i, vp, i, vp, i, vp, i, i, vp, vp, C.POINTER(Params), C.POINTER(Stats)]
    lib.chfsi_solve_batched.argtypes = [vp, i, C.POINTER(Problem), C.POINTER(Params), C.POINTER(Stats)]
    lib.chfsi_filter.argtypes = [vp, i, vp, i, vp, i, i, vp, i, d, d, d, i]
    lib.chfsi_filter_noalloc.argtypes = [vp, i, vp, i, vp, i, i, i, d, d, d]
    lib.chfsi_correlation.argtypes = [vp, i, i, vp, i, vp, i, vp, i, vp, i, vp, vp]
    lib.chfsi_lobpcg_default_params.argtypes = [C.POINTER(LobpcgParams)]
    lib.chfsi_lobpcg_default_params.restype = None
    lib.chfsi_lobpcg.argtypes = [vp, i, vp, i, vp, i, vp, i, i, vp, vp, C.POINTER(LobpcgParams), C.POINTER(LobpcgStats)]
    lib.chfsi_reduce.argtypes = [vp, i, vp, i, vp, i, vp, vp]
    lib.chfsi_reduce_explicit.argtypes = [vp, i, vp, i, vp, i, vp, vp]
    lib.chfsi_lanczos.argtypes = [vp, i, vp, i, i, u, vp, vp, vp, vp]
    lib.chfsi_orthonormalize.argtypes = [vp, i, i, vp, i, i, vp, i]
    lib.chfsi_rayleigh_ritz.argtypes = [vp, i, vp, i, i, vp, i, vp, vp]
    lib.chfsi_random_block.argtypes = [vp, u, u, i, i, vp, i]
    lib.chfsi_zgemm.argtypes = [vp, C.c_char, C.c_char, i, i, i, d, vp, i, vp, i, d, vp, i]
    lib.chfsi_set_degree_model.argtypes = [vp, vp, C.c_size_t]
    lib.chfsi_get_trace.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    lib.chfsi_mlp_forward.argtypes = [vp, vp, i, vp, C.c_float, C.c_float, vp]
    lib.chfsi_mlp_loss_grad.argtypes = [vp, vp, i, vp, vp, C.c_float, C.c_float, vp, vp]
    lib.chfsi_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i, C.c_float, C.c_float, C.c_float, C.c_float]
    lib.chfsi_mlp_train.argtypes = [vp, vp, i, vp, vp, C.c_float, C.c_float, i, i, C.c_float, u, vp]
    lib.chfsi_filter_kernel_time.argtypes = [vp, vp, vp]
    lib.chfsi_filter_launch_log.argtypes = [vp, vp, i, vp]
    lib.chfsi_autotune_filter.argtypes = [vp, i, i, i, C.POINTER(TilePlan), vp]
    lib.chfsi_set_filter_plan.argtypes = [vp, i, i, i, C.POINTER(TilePlan)]
    lib.chfsi_set_batched_plan.argtypes = [vp, C.POINTER(TilePlan), i, i]
    lib.chfsi_autotune_batched.argtypes = [vp, i, C.POINTER(Problem), C.POINTER(TilePlan), vp]
    lib.chfsi_autotune_batched_tiles.argtypes = [vp, i, C.POINTER(Problem), C.POINTER(TilePlan), vp]
    lib.chfsi_set_batched_tiles.argtypes = [vp, i, C.POINTER(Problem), C.POINTER(TilePlan)]
    lib.chfsi_batched_info.argtypes = [vp, vp, vp, vp, vp]
    lib.chfsi_status_string.argtypes = [i]
    lib.chfsi_status_string.restype = C.c_char_p
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return STATUS_NAMES.get(int(st), f"status {int(st)}")


def default_params(**kw) -> Params:
    p = Params()
    load().chfsi_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "filter_precision" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(p, k, v)
    return p


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def to_device(a: np.ndarray, device="cuda", dtype=None):
    """numpy (rows x cols) -> contiguous torch tensor (cols, rows) holding the column-major matrix."""
    import torch
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[:, None]
    t = torch.from_numpy(np.ascontiguousarray(a.T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def to_numpy(t) -> np.ndarray:
    """torch tensor (cols, rows) holding a column-major matrix -> numpy (rows x cols), Fortran order."""
    return np.asfortranarray(t.detach().cpu().numpy().T)


def filter_noalloc(H, Y, a: float, b: float, mu1: float, deg: int = 10, stream=None, n: Optional[int] = None,
                   m: Optional[int] = None, sync: bool = True) -> None:
    """chfsi_filter_noalloc on torch device tensors: FP64 filter of Y in place, no allocation, no
    handle; enqueued on `stream` (a torch.cuda.Stream, default the current stream)."""
    import torch
    n = H.shape[-1] if n is None else n
    m = Y.shape[0] if m is None else m
    s = torch.cuda.current_stream() if stream is None else stream
    st = load().chfsi_filter_noalloc(C.c_void_p(s.cuda_stream), n, _ptr(H), H.shape[-1], _ptr(Y), Y.shape[-1],
                                     m, deg, a, b, mu1)
    if st != SUCCESS:
        raise ChfsiError(st, "chfsi_filter_noalloc")
    if sync:
        s.synchronize()


@dataclass
class SolveResult:
    status: int
    lam: np.ndarray
    resid: np.ndarray
    stats: dict = field(default_factory=dict)


class Handle:
    """One library handle (device, stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.chfsi_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != 0:
            raise ChfsiError(st, "chfsi_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.chfsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise ChfsiError(st, what)

    # ---- whole solver ------------------------------------------------------------------------
    def solve(self, A, S, X, x_is_guess: bool, params: Params, n: Optional[int] = None,
              raise_on_error: bool = True) -> SolveResult:
        """A, S (or None), X: complex128 device tensors (column-major via shape (cols, rows)).
        X is overwritten with the Ritz vectors."""
        n = n or A.shape[-1]
        m = params.nev + params.nex
        lam = np.zeros(m)
        res = np.zeros(m)
        st = Stats()
        status = self.lib.chfsi_solve(self.h, n, _ptr(A), A.shape[-1], _ptr(S), 0 if S is None else S.shape[-1],
                                      _ptr(X), X.shape[-1], 1 if x_is_guess else 0,
                                      lam.ctypes.data, res.ctypes.data, C.byref(params), C.byref(st))
        if raise_on_error and status not in (0,):
            raise ChfsiError(status, "chfsi_solve")
        return SolveResult(status=int(status), lam=lam, resid=res, stats=st.as_dict())

    @staticmethod
    def _problems(problems: Sequence[dict]):
        cnt = len(problems)
        arr = (Problem * cnt)()
        outs = []
        for k, pr in enumerate(problems):
            m = pr["nev"] + pr["nex"]
            lam = np.zeros(m)
            res = np.zeros(m)
            outs.append((lam, res))
            A, S, X = pr["A"], pr.get("S"), pr["X"]
            arr[k] = Problem(A.shape[-1], pr["nev"], pr["nex"], _ptr(A), A.shape[-1], _ptr(S),
                             0 if S is None else S.shape[-1], _ptr(X), X.shape[-1], 1 if pr.get("x_is_guess") else 0,
                             lam.ctypes.data, res.ctypes.data)
        return arr, outs

    def solve_batched(self, problems: Sequence[dict], params: Params):
        """problems: dicts with keys A, S (or None), X, nev, nex, x_is_guess (device tensors in the
        layout of to_device).  Returns (status, [SolveResult])."""
        cnt = len(problems)
        arr, outs = self._problems(problems)
        st = (Stats * cnt)()
        status = self.lib.chfsi_solve_batched(self.h, cnt, arr, C.byref(params), st)
        results = [SolveResult(status=int(st[k].status), lam=outs[k][0], resid=outs[k][1], stats=st[k].as_dict())
                   for k in range(cnt)]
        return int(status), results

    def set_batched_plan(self, bm: Optional[int] = None, bn: Optional[int] = None, use_graph: bool = True,
                         lanes: int = 0):
        plan = None if bm is None else C.byref(TilePlan(bm, bn, 1, 0))
        self._check(self.lib.chfsi_set_batched_plan(self.h, plan, 1 if use_graph else 0, lanes),
                    "chfsi_set_batched_plan")

    def autotune_batched(self, problems: Sequence[dict]):
        """Tunes the persistent multi-problem filter tile on these problems; returns ((bm, bn), ms)."""
        arr, _ = self._problems(problems)
        plan = TilePlan()
        ms = np.zeros(1)
        self._check(self.lib.chfsi_autotune_batched(self.h, len(problems), arr, C.byref(plan), ms.ctypes.data),
                    "chfsi_autotune_batched")
        return (plan.bm, plan.bn), float(ms[0])

    def autotune_batched_tiles(self, problems: Sequence[dict]):
        """Tunes a tile per problem (per order and block width) and selects the kernel with a tile
        per problem; returns ([(bm, bn)] per problem, ms of one filter step of the whole batch)."""
        arr, _ = self._problems(problems)
        tiles = (TilePlan * len(problems))()
        ms = np.zeros(1)
        self._check(self.lib.chfsi_autotune_batched_tiles(self.h, len(problems), arr, tiles, ms.ctypes.data),
                    "chfsi_autotune_batched_tiles")
        return [(t.bm, t.bn) for t in tiles], float(ms[0])

    def set_batched_tiles(self, problems: Optional[Sequence[dict]], tiles: Optional[Sequence[tuple]]):
        """Sets the tile (bm, bn) of each problem's order and width (tiles None: back to one tile)."""
        if tiles is None:
            self._check(self.lib.chfsi_set_batched_tiles(self.h, 0, None, None), "chfsi_set_batched_tiles")
            return
        arr, _ = self._problems(problems)
        tp = (TilePlan * len(tiles))(*[TilePlan(bm, bn, 1, 0) for bm, bn in tiles])
        self._check(self.lib.chfsi_set_batched_tiles(self.h, len(problems), arr, tp), "chfsi_set_batched_tiles")

    def batched_info(self) -> dict:
        """Filter ms, filter flops, graph replays and kernel launches of the last solve_batched."""
        t = np.zeros(2)
        c = np.zeros(2, dtype=np.int32)
        self._check(self.lib.chfsi_batched_info(self.h, t.ctypes.data, t[1:].ctypes.data, c.ctypes.data,
                                                c[1:].ctypes.data), "chfsi_batched_info")
        return {"filter_ms": float(t[0]), "filter_flops": float(t[1]), "graph_launches": int(c[0]),
                "kernel_launches": int(c[1])}

    # ---- steps -------------------------------------------------------------------------------
    def filter(self, H, Y, a: float, b: float, mu1: float, deg=10, prec: int = FP64, n: Optional[int] = None):
        n = n or H.shape[-1]
        m = Y.shape[0]
        if np.isscalar(deg):
            dp, du = None, int(deg)
        else:
            dv = np.ascontiguousarray(deg, dtype=np.int32)
            dp, du = dv.ctypes.data, 0
        self._check(self.lib.chfsi_filter(self.h, n, _ptr(H), H.shape[-1], _ptr(Y), Y.shape[-1], m, dp, du,
                                          a, b, mu1, prec), "chfsi_filter")

    def filter_kernel_time(self):
        """(total ms, launches) of the filter-step kernels of the last solve/filter call."""
        t = np.zeros(1); c = np.zeros(1, dtype=np.int32)
        self._check(self.lib.chfsi_filter_kernel_time(self.h, t.ctypes.data, c.ctypes.data), "chfsi_filter_kernel_time")
        return float(t[0]), int(c[0])

    def filter_launch_log(self) -> np.ndarray:
        """Rows (n, width, prec, bm, bn, ksplit, mode, main_ms, step_ms) of the last solve/filter."""
        cnt = np.zeros(1, dtype=np.int32)
        self._check(self.lib.chfsi_filter_launch_log(self.h, None, 0, cnt.ctypes.data), "chfsi_filter_launch_log")
        rows = np.zeros((int(cnt[0]), 9))
        if len(rows):
            self._check(self.lib.chfsi_filter_launch_log(self.h, rows.ctypes.data, len(rows), cnt.ctypes.data),
                        "chfsi_filter_launch_log")
        return rows

    def autotune_filter(self, n: int, m: int, prec: int = FP64):
        """Times every tile plan of the n x m filter step; returns (plan dict, ms per step)."""
        p = TilePlan()
        ms = np.zeros(1)
        self._check(self.lib.chfsi_autotune_filter(self.h, n, m, prec, C.byref(p), ms.ctypes.data),
                    "chfsi_autotune_filter")
        return p.as_dict(), float(ms[0])

    def set_filter_plan(self, n: int, m: int, prec: int, plan: Optional[dict]):
        if plan is None:
            self._check(self.lib.chfsi_set_filter_plan(self.h, n, m, prec, None), "chfsi_set_filter_plan")
            return
        p = TilePlan(plan["bm"], plan["bn"], plan["ksplit"], plan.get("fused", 0))
        self._check(self.lib.chfsi_set_filter_plan(self.h, n, m, prec, C.byref(p)), "chfsi_set_filter_plan")

    def reduce(self, A, S, H, L):
        self._check(self.lib.chfsi_reduce(self.h, A.shape[-1], _ptr(A), A.shape[-1], _ptr(S), S.shape[-1],
                                          _ptr(H), _ptr(L)), "chfsi_reduce")

    def reduce_explicit(self, A, S, H, L):
        self._check(self.lib.chfsi_reduce_explicit(self.h, A.shape[-1], _ptr(A), A.shape[-1], _ptr(S), S.shape[-1],
                                                   _ptr(H), _ptr(L)), "chfsi_reduce_explicit")

    def lanczos(self, H, k: int, seed: int):
        th = np.zeros(k); zw = np.zeros(k); bk = np.zeros(1); ku = np.zeros(1, dtype=np.int32)
        self._check(self.lib.chfsi_lanczos(self.h, H.shape[-1], _ptr(H), H.shape[-1], k, seed, th.ctypes.data,
                                           zw.ctypes.data, bk.ctypes.data, ku.ctypes.data), "chfsi_lanczos")
        kk = int(ku[0])
        return th[:kk], zw[:kk], float(bk[0])

    def orthonormalize(self, Y, YL=None):
        n = Y.shape[-1]
        nl = 0 if YL is None else YL.shape[0]
        self._check(self.lib.chfsi_orthonormalize(self.h, n, Y.shape[0], _ptr(Y), n, nl, _ptr(YL),
                                                  n if YL is not None else 0), "chfsi_orthonormalize")

    def rayleigh_ritz(self, H, Y):
        m = Y.shape[0]
        th = np.zeros(m); r = np.zeros(m)
        self._check(self.lib.chfsi_rayleigh_ritz(self.h, H.shape[-1], _ptr(H), H.shape[-1], m, _ptr(Y),
                                                 Y.shape[-1], th.ctypes.data, r.ctypes.data), "chfsi_rayleigh_ritz")
        return th, r

    def correlation(self, Xp, Xc, S=None, n: Optional[int] = None, m: Optional[int] = None):
        """chfsi_correlation: (O device tensor (m, m) column-major, sin_pair, sin_sub host arrays)."""
        import torch
        n = Xc.shape[-1] if n is None else n
        m = Xc.shape[0] if m is None else m
        O = torch.empty((m, m), dtype=torch.complex128, device=Xc.device)
        sp, ss = np.zeros(m), np.zeros(m)
        self._check(self.lib.chfsi_correlation(self.h, n, m, _ptr(S), 0 if S is None else S.shape[-1], _ptr(Xp),
                                               Xp.shape[-1], _ptr(Xc), Xc.shape[-1], _ptr(O), m, sp.ctypes.data,
                                               ss.ctypes.data), "chfsi_correlation")
        return O, sp, ss

    def lobpcg(self, A, S, X, x_is_guess: bool, nev: int, bs: int = 0, tol: float = 1e-10, maxiter: int = 1000,
               gen: bool = False, seed: int = 0, n: Optional[int] = None, raise_on_error: bool = True) -> "SolveResult":
        """chfsi_lobpcg: X (torch, bs columns) in/out; returns the Ritz values, residuals and stats."""
        n = A.shape[-1] if n is None else n
        p = LobpcgParams()
        self.lib.chfsi_lobpcg_default_params(C.byref(p))
        p.nev, p.bs, p.tol, p.maxiter, p.gen, p.seed = nev, bs, tol, maxiter, 1 if gen else 0, seed
        m = X.shape[0]
        lam, res = np.zeros(m), np.zeros(m)
        st = LobpcgStats()
        s = self.lib.chfsi_lobpcg(self.h, n, _ptr(A), A.shape[-1], _ptr(S), 0 if S is None else S.shape[-1], _ptr(X),
                                  X.shape[-1], 1 if x_is_guess else 0, lam.ctypes.data, res.ctypes.data, C.byref(p),
                                  C.byref(st))
        if raise_on_error and s not in (SUCCESS, ERR_NO_CONVERGENCE):
            raise ChfsiError(s, "chfsi_lobpcg")
        return SolveResult(int(s), lam, res, {f: getattr(st, f) for f, _ in LobpcgStats._fields_})

    def random_block(self, seed: int, stream: int, n: int, m: int):
        import torch
        Y = torch.empty((m, n), dtype=torch.complex128, device=f"cuda:{self.device}")
        self._check(self.lib.chfsi_random_block(self.h, seed, stream, n, m, _ptr(Y), n), "chfsi_random_block")
        return Y

    def zgemm(self, ta: str, tb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B, ldb: int,
              beta: float, Cm, ldc: int):
        self._check(self.lib.chfsi_zgemm(self.h, ta.encode(), tb.encode(), m, n, k, alpha, _ptr(A), lda, _ptr(B),
                                         ldb, beta, _ptr(Cm), ldc), "chfsi_zgemm")

    # ---- degree network ----------------------------------------------------------------------
    def set_degree_model(self, blob: Optional[np.ndarray]):
        if blob is None:
            self._check(self.lib.chfsi_set_degree_model(self.h, None, 0), "chfsi_set_degree_model")
            return
        b = np.ascontiguousarray(blob, dtype=np.float32)
        self._check(self.lib.chfsi_set_degree_model(self.h, b.ctypes.data, b.nbytes), "chfsi_set_degree_model")

    def get_trace(self) -> np.ndarray:
        nb = C.c_size_t(0)
        self._check(self.lib.chfsi_get_trace(self.h, None, C.byref(nb)), "chfsi_get_trace")
        buf = np.zeros(nb.value // 8)
        nb2 = C.c_size_t(nb.value)
        self._check(self.lib.chfsi_get_trace(self.h, buf.ctypes.data, C.byref(nb2)), "chfsi_get_trace")
        return buf.reshape(-1, TRACE_COLS)

    def mlp_forward(self, P, X, dmin=4.0, dmax=30.0):
        import torch
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self._check(self.lib.chfsi_mlp_forward(self.h, _ptr(P), X.shape[0], _ptr(X), dmin, dmax, _ptr(out)),
                    "chfsi_mlp_forward")
        return out

    def mlp_loss_grad(self, P, X, y, dmin=4.0, dmax=30.0):
        import torch
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
        loss = np.zeros(1, dtype=np.float32)
        self._check(self.lib.chfsi_mlp_loss_grad(self.h, _ptr(P), X.shape[0], _ptr(X), _ptr(y), dmin, dmax, _ptr(g),
                                                 loss.ctypes.data), "chfsi_mlp_loss_grad")
        return float(loss[0]), g

    def mlp_adam(self, P, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.chfsi_mlp_adam(self.h, _ptr(P), _ptr(g), _ptr(m), _ptr(v), t, lr, beta1, beta2, eps),
                    "chfsi_mlp_adam")

    def mlp_train(self, P, X, y, epochs=20, batch=256, lr=1e-3, seed=0, dmin=4.0, dmax=30.0):
        hist = np.zeros(max(epochs, 1), dtype=np.float32)
        self._check(self.lib.chfsi_mlp_train(self.h, _ptr(P), X.shape[0], _ptr(X), _ptr(y), dmin, dmax, epochs,
                                             batch, lr, seed, hist.ctypes.data), "chfsi_mlp_train")
        return hist[:epochs]
