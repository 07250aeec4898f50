"""Seeded synthetic inputs: sequences of correlated dense Hermitian (generalized) eigenproblems.

This module is shared by the tests, the benchmark and the CPU reference; it contains none of the
eigensolver's arithmetic, only the construction of the pencils (A, S) and their known spectra.

The paper's workloads are FLAPW pencils (Section 2, Table 1): dense, complex Hermitian A, HPD
overlap B, n between 2,000 and 20,000, the wanted fraction of the spectrum at most 15-20 %, and
successive problems of a sequence strongly correlated (eigenvector deviation angles ~1e-4 after a
few cycles, Section 2.2).  Those matrices are not available, so these generators stand in for
them with the same shapes and structure:

* spectrum: a clustered low part of ``n_low`` values uniform in [-1, -0.5] and the rest uniform
  in [-0.4, 1];
* eigenvectors: a unitary Q = R2 R1 P B with B block diagonal of Haar-distributed 64 x 64 blocks
  (QR of a complex Gaussian, diagonal of R rotated to be real positive; Mezzadri 2007), P a
  random permutation and R1, R2 Householder reflections along complex Gaussian vectors.  Q is
  dense, and it costs O(n^2) to build and apply where a Haar matrix of order n costs O(n^3).  The
  perturbations below have a unitarily invariant law, so for a standard problem the statistics of
  a whole sequence do not depend on which eigenbasis Q is used;
* overlap (generalized problems): S = I + G G^H / n with G a complex Gaussian n x 64;
* "designed form": A0 = S^{1/2} Q diag(lam) Q^H S^{1/2}, so the pencil (A0, S) has exactly the
  spectrum ``lam`` and S-orthonormal eigenvectors X = S^{-1/2} Q.  S^{+-1/2} = I + G f(G^H G/n) G^H
  are rank-64 corrections of I (f from the 64 x 64 eigen-decomposition of G^H G / n), so A0 costs
  O(n^2) as well;
* sequence: A_{l+1} = A_l + eps_l (E_l + E_l^H) / 2 with E_l an i.i.d. complex Gaussian
  (real and imaginary parts N(0, 1/2)) drawn from its own stream, which makes successive
  problems correlated with a shrinking step, as in the self-consistent cycle of Section 2.1.

All arrays are complex128 in Fortran (column-major) order, the layout of the C-ABI library.
Every random draw comes from numpy's PCG64 with one ``SeedSequence`` child per purpose, so a
(seed, purpose) pair always yields the same numbers.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Iterator, List, Optional

import numpy as np

# stream indices of the SeedSequence children, one per purpose
_STREAM_LAM, _STREAM_Q, _STREAM_G, _STREAM_START = 0, 1, 2, 3
_STREAM_E0 = 16  # E_l uses child _STREAM_E0 + l


_PANEL = 256          # columns per independent draw panel of complex_gaussian
_TILE = 128           # tile edge of the Hermitian symmetrisation
_POOL = None


def _pool():
    global _POOL
    if _POOL is None:
        from concurrent.futures import ThreadPoolExecutor
        _POOL = ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))
    return _POOL


def _rng(seed: int, stream: int) -> np.random.Generator:
    ss = np.random.SeedSequence([int(seed), int(stream)])
    return np.random.Generator(np.random.PCG64(ss))


def complex_gaussian(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """i.i.d. complex normal entries, real and imaginary parts N(0, 1/2), Fortran order.

    Columns are drawn in panels of 256: panel p (columns 256 p ..) from child p of rng.spawn, column
    by column, real then imaginary part of each entry; the panels are filled in parallel."""
    buf = empty_f(2 * rows, cols, np.float64).T       # (cols, 2 rows), C order
    npan = max(1, (cols + _PANEL - 1) // _PANEL)
    kids = rng.spawn(npan)

    def fill(p):
        kids[p].standard_normal(out=buf[p * _PANEL:(p + 1) * _PANEL])
        buf[p * _PANEL:(p + 1) * _PANEL] *= math.sqrt(0.5)

    if npan == 1:
        fill(0)
    else:
        list(_pool().map(fill, range(npan)))
    return buf.view(np.complex128).T          # (rows, cols), Fortran-ordered view


def hermitian_part_(M: np.ndarray) -> np.ndarray:
    """M <- (M + M^H) / 2 in place, tile by tile; the result is exactly Hermitian."""
    n = M.shape[0]
    b = _TILE

    def row(i):
        blk = M[i:i + b, i:i + b]
        M[i:i + b, i:i + b] = 0.5 * (blk + blk.conj().T)
        for j in range(i + b, n, b):
            Z = 0.5 * (M[i:i + b, j:j + b] + M[j:j + b, i:i + b].conj().T)
            M[i:i + b, j:j + b] = Z
            M[j:j + b, i:i + b] = Z.conj().T

    list(_pool().map(row, range(0, n, b)))
    return M


def _gemm(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a @ b through torch (threaded BLAS) for Fortran or C ordered operands; Fortran-ordered result
    (computed as the C-ordered (b^T a^T))."""
    import torch
    return (torch.from_numpy(b).T @ torch.from_numpy(a).T).numpy().T


def empty_f(rows: int, cols: int, dtype=np.complex128, zero: bool = False) -> np.ndarray:
    """Fortran-ordered array whose memory comes from torch's allocator (large blocks get huge-page
    aligned memory, which is much cheaper to touch first than numpy's)."""
    import torch
    tdt = {np.complex128: torch.complex128, np.float64: torch.float64}[np.dtype(dtype).type]
    t = (torch.zeros if zero else torch.empty)((cols, rows), dtype=tdt)
    return t.numpy().T


def _tt(M: np.ndarray):
    """Fortran-ordered numpy matrix -> torch tensor of its transpose sharing the memory (torch
    runs the n^2 passes multithreaded)."""
    import torch
    return torch.from_numpy(M.T)


def add_(a: np.ndarray, b: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    """a += alpha b for Fortran-ordered matrices, in place."""
    _tt(a).add_(_tt(b), alpha=alpha)
    return a


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed n x n unitary: QR of a complex Gaussian with R's diagonal made real
    positive (Mezzadri 2007), Fortran order."""
    q, r = np.linalg.qr(complex_gaussian(rng, n, n))
    d = np.diag(r)
    return np.asfortranarray(q * (d / np.abs(d))[None, :])


def split_spectrum(rng: np.random.Generator, n: int, n_low: int) -> np.ndarray:
    """``n_low`` values uniform in [-1, -0.5] and ``n - n_low`` uniform in [-0.4, 1], sorted."""
    lo = rng.uniform(-1.0, -0.5, size=n_low)
    hi = rng.uniform(-0.4, 1.0, size=n - n_low)
    return np.sort(np.concatenate([lo, hi]))


class StructuredUnitary:
    """Q = R2 R1 P B (see the module docstring), applied without forming it."""

    def __init__(self, rng: np.random.Generator, n: int, block: int = 64):
        self.n = n
        sizes = [block] * (n // block) + ([n % block] if n % block else [])
        self.blocks = [haar_unitary(rng, sz) for sz in sizes]
        self.perm = rng.permutation(n)          # P e_i = e_{perm[i]}
        self.u = []
        for _ in range(2):
            v = complex_gaussian(rng, n, 1)[:, 0]
            self.u.append(np.ascontiguousarray(v / np.linalg.norm(v)))

    def apply(self, Y: np.ndarray) -> np.ndarray:
        """Q Y for Y (n x k); Fortran-ordered result."""
        Z = np.empty_like(Y)
        o = 0
        for b in self.blocks:
            Z[o:o + b.shape[0]] = b @ Y[o:o + b.shape[0]]
            o += b.shape[0]
        W = np.empty_like(Z)
        W[self.perm] = Z
        for u in self.u:                          # R = I - 2 u u^H
            W -= 2.0 * np.outer(u, u.conj() @ W)
        return np.asfortranarray(W)

    def sandwich(self, lam: np.ndarray) -> np.ndarray:
        """Q diag(lam) Q^H, exactly Hermitian, Fortran order."""
        import torch
        n = self.n
        M = empty_f(n, n, zero=True)
        o = 0
        for b in self.blocks:
            k = b.shape[0]
            idx = self.perm[o:o + k]
            M[np.ix_(idx, idx)] = (b * lam[o:o + k][None, :]) @ b.conj().T
            o += k
        Mt = _tt(M)                               # M^T
        for un in self.u:                         # R M R = M - 2 u w^H - 2 w u^H + 4 c u u^H, w = M u
            u = torch.from_numpy(un)
            w = torch.mv(Mt.T, u)
            c = float(torch.vdot(u, w).real)
            Mt.addr_(w.conj(), u, alpha=-2.0)     # (u w^H)^T = conj(w) u^T
            Mt.addr_(u.conj(), w, alpha=-2.0)
            Mt.addr_(u.conj(), u, alpha=4.0 * c)
        return hermitian_part_(M)


@dataclasses.dataclass
class Overlap:
    """S = I + G G^H / n and the rank-r factors of S^{+-1/2} = I + K diag(f / n) K^H, K = G U."""
    S: np.ndarray
    K: np.ndarray
    f_half: np.ndarray        # f(d) = (sqrt(1 + d) - 1) / d        -> S^{1/2}
    f_mhalf: np.ndarray       # f(d) = (1 / sqrt(1 + d) - 1) / d    -> S^{-1/2}

    def apply_mhalf(self, Y: np.ndarray) -> np.ndarray:
        n = self.S.shape[0]
        return np.asfortranarray(Y + self.K @ ((self.f_mhalf / n)[:, None] * (self.K.conj().T @ Y)))

    def sandwich_half(self, M: np.ndarray) -> np.ndarray:
        """S^{1/2} M S^{1/2} for Hermitian M (overwritten): M + [K T] [[F W F, F], [F, 0]] [K T]^H
        with T = M K, W = K^H T, F = diag(f / n); exactly Hermitian."""
        import torch
        K = self.K
        r = K.shape[1]
        T = _gemm(M, K)
        F = np.diag(self.f_half / M.shape[0]).astype(np.complex128)
        W = K.conj().T @ T
        core = np.zeros((2 * r, 2 * r), dtype=np.complex128)
        core[:r, :r] = F @ W @ F
        core[:r, r:] = F
        core[r:, :r] = F
        L = torch.from_numpy(np.ascontiguousarray(np.concatenate([K, T], axis=1)))
        # M^T += (L core L^H)^T = conj(L) core^T L^T
        _tt(M).addmm_(L.conj() @ torch.from_numpy(core.T.copy()), L.T)
        return hermitian_part_(M)


def overlap(rng: np.random.Generator, n: int, rank: int = 64, kappa: float = 0.0) -> Overlap:
    """HPD overlap with its square roots.  kappa = 0: S = I + G G^H / n with G an n x rank complex
    Gaussian (condition number about 2.4).  kappa > 1: S = I + Q diag(s - 1) Q^H with Q an n x rank
    orthonormal block (QR of a complex Gaussian) and s logarithmically spaced from 1/kappa to 1, so
    that S has the eigenvalue 1 (n - rank times) and s, and its condition number is exactly kappa:
    a nearly linearly dependent basis, as the ill-conditioned overlap of a FLAPW basis."""
    if kappa and kappa > 1.0:
        return _overlap_conditioned(rng, n, rank, kappa)
    import torch
    g = complex_gaussian(rng, n, rank)
    gt = torch.from_numpy(np.ascontiguousarray(g))
    S = empty_f(n, n)
    torch.mm(gt.conj(), gt.T, out=_tt(S))     # S^T = conj(G) G^T
    _tt(S).mul_(1.0 / n)
    hermitian_part_(S)
    S[np.diag_indices(n)] += 1.0
    gh = g.conj().T
    d, U = np.linalg.eigh(gh @ g / n)
    d = np.maximum(d, 0.0)
    safe = np.where(d > 1e-12, d, 1.0)
    sq = np.sqrt(1.0 + d)
    fh = np.where(d > 1e-12, (sq - 1.0) / safe, 0.5 - d / 8.0)
    fm = np.where(d > 1e-12, (1.0 / sq - 1.0) / safe, -0.5 + 3.0 * d / 8.0)
    return Overlap(S=S, K=np.asfortranarray(g @ U), f_half=fh, f_mhalf=fm)


def _overlap_conditioned(rng: np.random.Generator, n: int, rank: int, kappa: float) -> Overlap:
    import torch
    q, _ = np.linalg.qr(complex_gaussian(rng, n, rank))
    q = np.asfortranarray(q)
    s = np.logspace(-math.log10(kappa), 0.0, rank)
    d = s - 1.0                                   # S = I + Q diag(d) Q^H
    qt = torch.from_numpy(np.ascontiguousarray(q))
    S = empty_f(n, n)
    # S^T = conj(Q) diag(d) Q^T
    torch.mm(qt.conj() * torch.from_numpy(d)[None, :], qt.T, out=_tt(S))
    hermitian_part_(S)
    S[np.diag_indices(n)] += 1.0
    # the Overlap factors use K diag(f / n) K^H: K = sqrt(n) Q, f = sqrt(1 + d) - 1 (S^{1/2}) and
    # 1 / sqrt(1 + d) - 1 (S^{-1/2})
    return Overlap(S=S, K=np.asfortranarray(q * math.sqrt(n)), f_half=np.sqrt(s) - 1.0, f_mhalf=1.0 / np.sqrt(s) - 1.0)


def overlap_matrix(rng: np.random.Generator, n: int, rank: int = 64) -> np.ndarray:
    """HPD overlap S = I + G G^H / n with G an n x rank complex Gaussian."""
    return overlap(rng, n, rank).S


def hermitian_noise(rng: np.random.Generator, n: int) -> np.ndarray:
    """(E + E^H) / 2 with E an i.i.d. complex Gaussian (exactly Hermitian), Fortran order."""
    return hermitian_part_(complex_gaussian(rng, n, n))


@dataclasses.dataclass
class Pencil:
    """One problem of a sequence.  ``S`` is None for a standard problem."""
    A: np.ndarray
    S: Optional[np.ndarray]
    lam_exact: Optional[np.ndarray]   # exact spectrum when A is in designed form (cycle 0)
    X_exact: Optional[np.ndarray]     # exact S-orthonormal eigenvectors (designed form), n x n
    cycle: int = 0
    overlap: Optional["Overlap"] = None   # S with its square roots (generalized problems)


@dataclasses.dataclass
class SequenceSpec:
    """Recipe of a correlated sequence of (generalized) Hermitian eigenproblems."""
    n: int
    n_low: int
    generalized: bool
    cycles: int
    eps0: float
    eps_decay: float
    seed: int = 0
    nev: int = 32
    nex: int = 16
    deg: int = 10
    kappa: float = 0.0     # condition number of S (0: S = I + G G^H / n, about 2.4)

    def eps(self, cycle: int) -> float:
        return self.eps0 * self.eps_decay ** cycle


def designed_pencil(spec: SequenceSpec, keep_vectors: bool = True, vector_cols: Optional[int] = None) -> Pencil:
    """Cycle-0 pencil in designed form: exact spectrum and eigenvectors are known (the first
    ``vector_cols`` eigenvectors, all by default)."""
    n = spec.n
    lam = split_spectrum(_rng(spec.seed, _STREAM_LAM), n, spec.n_low)
    q = StructuredUnitary(_rng(spec.seed, _STREAM_Q), n)
    m = n if vector_cols is None else vector_cols
    qm = q.apply(np.eye(n, m, dtype=np.complex128)) if keep_vectors else None
    a = q.sandwich(lam)
    if spec.generalized:
        ov = overlap(_rng(spec.seed, _STREAM_G), n, kappa=spec.kappa)
        s = ov.S
        a = ov.sandwich_half(a)
        x = ov.apply_mhalf(qm) if keep_vectors else None
    else:
        ov = None
        s = None
        x = qm
    return Pencil(A=a, S=s, lam_exact=lam, X_exact=x, cycle=0, overlap=ov)


def sequence(spec: SequenceSpec, keep_vectors: bool = False) -> Iterator[Pencil]:
    """Yield the pencils of cycles 0 .. spec.cycles-1 (A_{l+1} = A_l + eps_l (E_l + E_l^H)/2).

    With an ill-conditioned overlap (spec.kappa > 1) the perturbation is S^{1/2} ((E_l + E_l^H)/2)
    S^{1/2}: A and S of a nearly dependent basis share its small directions, and a perturbation of
    the operator enters both through the basis (a plain E would put eigenvalues of order
    eps ||E|| kappa into the pencil).  Every term is exactly Hermitian, so every A_l is as well."""
    p = designed_pencil(spec, keep_vectors=keep_vectors)
    yield p
    a = p.A
    for ell in range(1, spec.cycles):
        e = hermitian_noise(_rng(spec.seed, _STREAM_E0 + ell - 1), spec.n)
        if spec.kappa and spec.kappa > 1.0:
            e = p.overlap.sandwich_half(e)
        a_next = empty_f(spec.n, spec.n)
        _tt(a_next).copy_(_tt(a))
        a = add_(a_next, e, spec.eps(ell - 1))
        yield Pencil(A=a, S=p.S, lam_exact=None, X_exact=None, cycle=ell)


def random_block(seed: int, n: int, m: int) -> np.ndarray:
    """A seeded complex Gaussian n x m block (caller-side random start)."""
    return complex_gaussian(_rng(seed, _STREAM_START), n, m)


# ---- the workloads -------------------------------------------------------------------------------

def config_single_standard(seed: int = 0) -> SequenceSpec:
    """Single standard problem, n=512: 64 clustered low values, nev 32, nex 16, degree 10."""
    return SequenceSpec(n=512, n_low=64, generalized=False, cycles=1, eps0=0.0, eps_decay=1.0,
                        seed=seed, nev=32, nex=16, deg=10)


def config_generalized_sequence(seed: int = 0, n: int = 2048, cycles: int = 10) -> SequenceSpec:
    """10-cycle generalized sequence, n=2048, lowest 5 % clustered, eps_l = 1e-2 * 0.5^l, nev 128, nex 64, deg 12."""
    return SequenceSpec(n=n, n_low=int(math.ceil(0.05 * n)), generalized=True, cycles=cycles,
                        eps0=1e-2, eps_decay=0.5, seed=seed, nev=128 * n // 2048, nex=64 * n // 2048, deg=12)


def config_mixed_precision(seed: int = 0, n: int = 8192, cycles: int = 5) -> SequenceSpec:
    """5-cycle generalized sequence, n=8192, 1/8 of the spectrum clustered, eps_l = 5e-3 * 0.6^l, nev 400, nex 80."""
    return SequenceSpec(n=n, n_low=n // 8, generalized=True, cycles=cycles, eps0=5e-3, eps_decay=0.6,
                        seed=seed, nev=400 * n // 8192, nex=80 * n // 8192, deg=12)


def config_ill_conditioned(seed: int = 0, n: int = 2048, cycles: int = 3, kappa: float = 1e6) -> SequenceSpec:
    """The n = 2048 generalized sequence with an overlap of condition number kappa (1e6): the
    ill-conditioned B of the paper's FLAPW problems (Section 2.1); nev 128, nex 64, degree 12."""
    spec = config_generalized_sequence(seed=seed, n=n, cycles=cycles)
    spec.kappa = kappa
    return spec


def config_learned_degree(seed: int = 0, n: int = 4096, cycles: int = 20) -> SequenceSpec:
    """20-cycle standard sequence, n=4096, 1/8 clustered, eps_l = 1e-2 * 0.5^l, nev 256, nex 64."""
    return SequenceSpec(n=n, n_low=n // 8, generalized=False, cycles=cycles, eps0=1e-2, eps_decay=0.5,
                        seed=seed, nev=256 * n // 4096, nex=64 * n // 4096, deg=12)


@dataclasses.dataclass
class KPointProblem:
    n: int
    nev: int
    nex: int
    A: np.ndarray
    S: np.ndarray
    X0: np.ndarray          # warm start: the exact eigenvectors of the unperturbed pencil, n x m
    lam_prev: np.ndarray    # the unperturbed spectrum (first m values)


def kpoint_sizes(count: int = 32, seed: int = 0, n_lo: int = 1500, n_hi: int = 6000) -> List[int]:
    rng = _rng(seed, 99)
    return [int(v) for v in rng.integers(n_lo, n_hi + 1, size=count)]


def kpoint_problem(k: int, n: int, seed: int = 0, eps: float = 1e-3, min_nex: int = 0) -> KPointProblem:
    """k-point problem k of one SCF cycle: a designed generalized pencil perturbed by eps, warm start
    from the unperturbed eigenvectors.  nev = ceil(0.06 n), nex = max(ceil(0.2 nev), min_nex)."""
    nev = int(math.ceil(0.06 * n))
    nex = max(int(math.ceil(0.2 * nev)), int(min_nex))
    spec = SequenceSpec(n=n, n_low=int(math.ceil(0.05 * n)), generalized=True, cycles=1, eps0=eps,
                        eps_decay=1.0, seed=1000 * (seed + 1) + k, nev=nev, nex=nex, deg=12)
    m = nev + nex
    p = designed_pencil(spec, keep_vectors=True, vector_cols=m)
    a = add_(p.A, hermitian_noise(_rng(spec.seed, _STREAM_E0), n), eps)
    return KPointProblem(n=n, nev=nev, nex=nex, A=a, S=p.S, X0=np.asfortranarray(p.X_exact[:, :m]),
                         lam_prev=p.lam_exact[:m].copy())
