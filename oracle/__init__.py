"""CPU FP64 reference ("oracle") for Chebyshev-filtered subspace iteration.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
benchmark's ``cpu_baseline`` leg.  The product package never imports it.

The C sources (``chfsi_oracle.c``, ``mlp_oracle.c``) are compiled with gcc into
``liboracle.so``; this module wraps them with ctypes over numpy arrays (complex128, Fortran
order).  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "chfsi_oracle.c"), os.path.join(_HERE, "mlp_oracle.c"),
         os.path.join(_HERE, "lobpcg_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP, FP64, no fast-math except C99 limited-range complex
    multiplication, which drops only the inf/nan recovery of __muldc3)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range",
               "-o", _LIB_PATH + ".tmp"] + _SRCS + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    dp, ip = C.c_void_p, C.c_int
    lib.orc_philox4x64.argtypes = [dp, dp, dp]
    lib.orc_random_block.argtypes = [C.c_uint64, C.c_uint64, ip, ip, dp, ip]
    lib.orc_zgemm.argtypes = [C.c_char, C.c_char, ip, ip, ip, _Z, dp, ip, dp, ip, _Z, dp, ip]
    lib.orc_cholesky.argtypes = [ip, dp, ip, dp, ip]
    lib.orc_cholesky.restype = ip
    lib.orc_trsm_lower.argtypes = [ip, ip, dp, ip, dp, ip]
    lib.orc_trsm_lower_h.argtypes = [ip, ip, dp, ip, dp, ip]
    lib.orc_reduce.argtypes = [ip, dp, ip, dp, ip, dp, ip]
    lib.orc_qr.argtypes = [ip, ip, dp, ip, dp, ip]
    lib.orc_qr.restype = ip
    lib.orc_jacobi.argtypes = [ip, dp, ip, dp, dp, ip]
    lib.orc_jacobi.restype = ip
    lib.orc_lanczos.argtypes = [ip, dp, ip, ip, C.c_uint64, dp, dp, dp]
    lib.orc_lanczos.restype = ip
    lib.orc_bounds.argtypes = [ip, dp, dp, C.c_double, ip, ip, dp, dp, dp]
    lib.orc_filter.argtypes = [ip, dp, ip, ip, dp, ip, dp, ip, C.c_double, C.c_double, C.c_double]
    lib.orc_residuals.argtypes = [ip, ip, dp, ip, dp, ip, dp, dp]
    lib.orc_analytic_degree.argtypes = [C.c_double] * 5 + [ip, ip]
    lib.orc_analytic_degree.restype = ip
    lib.orc_solve.argtypes = [ip, dp, ip, dp, ip, dp, ip, ip, dp, dp, dp, dp]
    lib.orc_solve.restype = ip
    lib.orc_num_threads.restype = ip
    lib.orc_mlp_nparams.restype = ip
    lib.orc_mlp_forward.argtypes = [dp, ip, dp, C.c_double, C.c_double, dp]
    lib.orc_mlp_loss_grad.argtypes = [dp, ip, dp, dp, C.c_double, C.c_double, dp]
    lib.orc_mlp_loss_grad.restype = C.c_double
    lib.orc_adam_step.argtypes = [ip, dp, dp, dp, dp, ip, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.orc_set_library_hooks.argtypes = [dp, dp, dp]
    lib.orc_correlation.argtypes = [ip, ip, dp, ip, dp, ip, dp, ip, dp, ip, dp, dp]
    _lib = lib
    return lib


# ---- optional library primitives ----------------------------------------------------------------
# The C reference writes its dense product, triangular solves and Cholesky factor as plain loops,
# which stream the whole matrix once per column: fine up to a few thousand, hours at order 8192.
# use_library_products(True) routes exactly those three primitives to numpy's matmul and LAPACK
# (scipy ztrsm / zpotrf) -- library routines with the same definitions -- while every step of the
# method above them stays the C code.

_GEMM_T = C.CFUNCTYPE(None, C.c_char, C.c_char, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p,
                      C.c_int, C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_int)
_TRSM_T = C.CFUNCTYPE(None, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int)
_CHOL_T = C.CFUNCTYPE(C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int)
_hooks = None


def _view(ptr: int, rows: int, cols: int, ld: int) -> np.ndarray:
    """Column-major rows x cols matrix with leading dimension ld at address ptr (no copy)."""
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols), dtype=np.complex128, order="F")
    buf = (C.c_double * (2 * (ld * (cols - 1) + rows))).from_address(ptr)
    return np.ndarray((rows, cols), dtype=np.complex128, buffer=buf, strides=(16, 16 * ld))


def _gemm_cb(ta, tb, m, n, k, ar, ai, A, lda, B, ldb, br, bi, Cp, ldc):
    ta, tb = ta.decode(), tb.decode()
    out = _view(Cp, m, n, ldc)
    if k == 0:
        prod = np.zeros((m, n), dtype=np.complex128)
    else:
        a = _view(A, m, k, lda) if ta == "N" else _view(A, k, m, lda).conj().T
        b = _view(B, k, n, ldb) if tb == "N" else _view(B, n, k, ldb).conj().T
        prod = a @ b
    res = complex(ar, ai) * prod
    if br != 0.0 or bi != 0.0:
        res += complex(br, bi) * out
    out[...] = res


def _trsm_cb(conj_trans, n, nrhs, L, ldl, B, ldb):
    import scipy.linalg as sla
    if n == 0 or nrhs == 0:
        return
    lo = _view(L, n, n, ldl)
    b = _view(B, n, nrhs, ldb)
    b[...] = sla.solve_triangular(lo, b, lower=True, trans="C" if conj_trans else "N", check_finite=False)


def _chol_cb(n, S, lds, L, ldl):
    import scipy.linalg as sla
    s = _view(S, n, n, lds)
    lo = _view(L, n, n, ldl)
    try:
        f = sla.cholesky(np.tril(s), lower=True, check_finite=False)
    except np.linalg.LinAlgError:
        return 1
    if not np.all(np.isfinite(f)):
        return 1
    lo[...] = np.tril(f)
    return 0


def use_library_products(on: bool = True) -> None:
    """Routes the reference's dense products, triangular solves and Cholesky factor to numpy /
    LAPACK (on) or back to its plain loops (off)."""
    global _hooks
    lib = _load()
    if on:
        _hooks = (_GEMM_T(_gemm_cb), _TRSM_T(_trsm_cb), _CHOL_T(_chol_cb))
        lib.orc_set_library_hooks(C.cast(_hooks[0], C.c_void_p), C.cast(_hooks[1], C.c_void_p),
                                  C.cast(_hooks[2], C.c_void_p))
    else:
        lib.orc_set_library_hooks(None, None, None)
        _hooks = None


def _p(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def _zmat(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.complex128))


class _Z(C.Structure):
    """complex double passed by value (two SSE-class doubles, as the x86-64 ABI passes _Complex)."""
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


def _cplx(z) -> _Z:
    z = complex(z)
    return _Z(z.real, z.imag)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ---- building blocks ---------------------------------------------------------------------------

def philox4x64(counter: Sequence[int], key: Sequence[int]) -> np.ndarray:
    ctr = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64(_p(ctr), _p(k), _p(out))
    return out


def random_block(seed: int, stream: int, n: int, m: int) -> np.ndarray:
    y = np.zeros((n, m), dtype=np.complex128, order="F")
    _load().orc_random_block(seed, stream, n, m, _p(y), n)
    return y


def zgemm(ta: str, tb: str, A, B, alpha=1.0, beta=0.0, Cm=None) -> np.ndarray:
    A = _zmat(A); B = _zmat(B)
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    out = np.zeros((m, n), dtype=np.complex128, order="F") if Cm is None else _zmat(Cm).copy(order="F")
    _load().orc_zgemm(ta.encode(), tb.encode(), m, n, k, _cplx(alpha), _p(A), A.shape[0], _p(B),
                      B.shape[0], _cplx(beta), _p(out), m)
    return out


def cholesky(S):
    S = _zmat(S)
    n = S.shape[0]
    L = np.zeros((n, n), dtype=np.complex128, order="F")
    st = _load().orc_cholesky(n, _p(S), n, _p(L), n)
    return L, int(st)


def trsm_lower(L, B, conj_trans: bool = False) -> np.ndarray:
    L = _zmat(L); X = _zmat(B).copy(order="F")
    n, nrhs = X.shape
    f = _load().orc_trsm_lower_h if conj_trans else _load().orc_trsm_lower
    f(n, nrhs, _p(L), n, _p(X), n)
    return X


def reduce(A, L) -> np.ndarray:
    A = _zmat(A); L = _zmat(L)
    n = A.shape[0]
    H = np.zeros((n, n), dtype=np.complex128, order="F")
    _load().orc_reduce(n, _p(A), n, _p(L), n, _p(H), n)
    return H


def qr(Y):
    Q = _zmat(Y).copy(order="F")
    n, m = Q.shape
    R = np.zeros((m, m), dtype=np.complex128, order="F")
    st = _load().orc_qr(n, m, _p(Q), n, _p(R), m)
    return Q, R, int(st)


def jacobi(G):
    G = _zmat(G)
    m = G.shape[0]
    w = np.zeros(m)
    V = np.zeros((m, m), dtype=np.complex128, order="F")
    sweeps = _load().orc_jacobi(m, _p(G), m, _p(w), _p(V), m)
    return w, V, int(sweeps)


def lanczos(H, k: int, seed: int):
    H = _zmat(H)
    n = H.shape[0]
    theta = np.zeros(k); zw = np.zeros(k); bk = np.zeros(1)
    kk = _load().orc_lanczos(n, _p(H), n, k, seed, _p(theta), _p(zw), _p(bk))
    return theta[:kk], zw[:kk], float(bk[0])


def bounds(theta, zw, beta_k: float, m: int, n: int):
    theta = np.ascontiguousarray(theta, dtype=np.float64); zw = np.ascontiguousarray(zw, dtype=np.float64)
    out = np.zeros(3)
    o = out.ctypes.data
    _load().orc_bounds(len(theta), _p(theta), _p(zw), beta_k, m, n, C.c_void_p(o), C.c_void_p(o + 8),
                       C.c_void_p(o + 16))
    return float(out[0]), float(out[1]), float(out[2])   # mu1, a, b


def cheb_filter(H, Y, a: float, b: float, mu1: float, deg=10) -> np.ndarray:
    H = _zmat(H); Yo = _zmat(Y).copy(order="F")
    n, m = Yo.shape
    if np.isscalar(deg):
        _load().orc_filter(n, _p(H), n, m, _p(Yo), n, None, int(deg), a, b, mu1)
    else:
        d = np.ascontiguousarray(deg, dtype=np.int32)
        _load().orc_filter(n, _p(H), n, m, _p(Yo), n, _p(d), 0, a, b, mu1)
    return Yo


def residuals(HY, Y, theta) -> np.ndarray:
    HY = _zmat(HY); Y = _zmat(Y); th = np.ascontiguousarray(theta, dtype=np.float64)
    n, m = Y.shape
    r = np.zeros(m)
    _load().orc_residuals(n, m, _p(HY), n, _p(Y), n, _p(th), _p(r))
    return r


def analytic_degree(theta, r, a, b, thr, dmin=4, dmax=30) -> int:
    return int(_load().orc_analytic_degree(theta, r, a, b, thr, dmin, dmax))


def correlation(Xp, Xc, S=None):
    """Scalar products O = Xp^H S Xc of successive eigenvector blocks, the sine of the angle of each
    pair (xp_i, xc_i) and the sines of the principal angles between the spans (ascending)."""
    Xp = _zmat(Xp); Xc = _zmat(Xc)
    n, m = Xc.shape
    Sm = None if S is None else _zmat(S)
    O = np.zeros((m, m), dtype=np.complex128, order="F")
    sp = np.zeros(m); ss = np.zeros(m)
    _load().orc_correlation(n, m, None if Sm is None else _p(Sm), n, _p(Xp), n, _p(Xc), n, _p(O), m, _p(sp), _p(ss))
    return O, sp, ss


# ---- the solver --------------------------------------------------------------------------------

class _Params(C.Structure):
    _fields_ = [("nev", C.c_int), ("nex", C.c_int), ("deg", C.c_int), ("tol", C.c_double),
                ("max_loops", C.c_int), ("lanczos_steps", C.c_int), ("degree_policy", C.c_int),
                ("deg_min", C.c_int), ("deg_max", C.c_int), ("seed", C.c_uint64),
                ("have_bounds", C.c_int), ("mu1", C.c_double), ("a", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("loops", C.c_int), ("nlocked", C.c_int), ("lanczos_steps", C.c_int),
                ("filtered_vectors", C.c_longlong), ("matvecs", C.c_longlong), ("mu1", C.c_double),
                ("a", C.c_double), ("b", C.c_double), ("norm_a", C.c_double), ("lock_threshold", C.c_double)]


STATUS = {0: "ok", 1: "bad argument", 2: "not HPD", 3: "no convergence", 4: "numeric"}


@dataclass
class SolveResult:
    status: int
    lam: np.ndarray
    resid: np.ndarray
    X: np.ndarray
    stats: dict = field(default_factory=dict)


def solve(A, S=None, nev=32, nex=16, deg=10, tol=1e-10, X0=None, max_loops=50, lanczos_steps=25,
          degree_policy=0, deg_min=4, deg_max=30, seed=0, bounds: Optional[tuple] = None) -> SolveResult:
    """Algorithm 1 with reduction and back-transform.  ``X0`` given = warm start (generalized
    coordinates); ``bounds`` = (mu1, a) from the previous problem of the sequence."""
    A = _zmat(A)
    n = A.shape[0]
    m = nev + nex
    Sm = None if S is None else _zmat(S)
    X = np.zeros((n, m), dtype=np.complex128, order="F") if X0 is None else _zmat(X0).copy(order="F")
    lam = np.zeros(m); res = np.zeros(m)
    p = _Params(nev, nex, deg, tol, max_loops, lanczos_steps, degree_policy, deg_min, deg_max, seed,
                1 if bounds is not None else 0, bounds[0] if bounds else 0.0, bounds[1] if bounds else 0.0)
    st = _Stats()
    status = _load().orc_solve(n, _p(A), n, None if Sm is None else _p(Sm), n, _p(X), n,
                               0 if X0 is None else 1, _p(lam), _p(res), C.byref(p), C.byref(st))
    stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
    return SolveResult(status=int(status), lam=lam, resid=res, X=X, stats=stats)


# ---- LOBPCG (the paper's second solver; GEN on the pencil, STD after the reduction) -------------

class _LobpcgParams(C.Structure):
    _fields_ = [("nev", C.c_int), ("bs", C.c_int), ("maxiter", C.c_int), ("gen", C.c_int), ("tol", C.c_double),
                ("seed", C.c_uint64)]


class _LobpcgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("nconv", C.c_int), ("matvecs", C.c_longlong), ("bmatvecs", C.c_longlong),
                ("dropped", C.c_int)]


def lobpcg_block_size(nev: int) -> int:
    """Table 3: the LOBPCG block is 1.05 nev."""
    return int(math.ceil(1.05 * nev))


def lobpcg(A, S=None, nev=16, bs=None, tol=1e-10, X0=None, maxiter=1000, gen=False, seed=0) -> SolveResult:
    """Block LOBPCG without preconditioner; ``gen`` iterates on the pencil (A, S) directly,
    otherwise on H = L^{-1} A L^{-H} (S given) and back-transforms."""
    A = _zmat(A)
    n = A.shape[0]
    bs = lobpcg_block_size(nev) if bs is None else bs
    Sm = None if S is None else _zmat(S)
    X = np.zeros((n, bs), dtype=np.complex128, order="F") if X0 is None else _zmat(X0).copy(order="F")
    lam = np.zeros(bs); res = np.zeros(bs)
    p = _LobpcgParams(nev, bs, maxiter, 1 if gen else 0, tol, seed)
    st = _LobpcgStats()
    status = _load().orc_lobpcg(n, _p(A), n, None if Sm is None else _p(Sm), n, _p(X), n, 0 if X0 is None else 1,
                                _p(lam), _p(res), C.byref(p), C.byref(st))
    stats = {f: getattr(st, f) for f, _ in _LobpcgStats._fields_}
    return SolveResult(status=int(status), lam=lam, resid=res, X=X, stats=stats)


# ---- the degree network ------------------------------------------------------------------------

def mlp_nparams() -> int:
    return int(_load().orc_mlp_nparams())


def mlp_forward(P, X, dmin=4.0, dmax=30.0) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.float64); X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros(X.shape[0])
    _load().orc_mlp_forward(_p(P), X.shape[0], _p(X), dmin, dmax, _p(out))
    return out


def mlp_loss_grad(P, X, y, dmin=4.0, dmax=30.0):
    P = np.ascontiguousarray(P, dtype=np.float64); X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(mlp_nparams())
    loss = _load().orc_mlp_loss_grad(_p(P), X.shape[0], _p(X), _p(y), dmin, dmax, _p(g))
    return float(loss), g


def adam_step(P, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place on P, m, v (float64 arrays)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().orc_adam_step(len(P), _p(P), _p(g), _p(m), _p(v), t, lr, beta1, beta2, eps)
