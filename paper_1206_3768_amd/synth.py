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
* eigenvectors: a Haar-distributed unitary Q (QR of a complex Gaussian, diagonal of R rotated to
  be real positive; Mezzadri 2007);
* overlap (generalized problems): S = I + G G^H / n with G a complex Gaussian n x 64;
* "designed form": A0 = L Q diag(lam) Q^H L^H with S = L L^H, so the pencil (A0, S) has exactly the
  spectrum ``lam`` and S-orthonormal eigenvectors X = L^{-H} Q;
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
from typing import Iterator, List, Optional

import numpy as np
import scipy.linalg as sla

# stream indices of the SeedSequence children, one per purpose
_STREAM_LAM, _STREAM_Q, _STREAM_G, _STREAM_START = 0, 1, 2, 3
_STREAM_E0 = 16  # E_l uses child _STREAM_E0 + l


def _rng(seed: int, stream: int) -> np.random.Generator:
    ss = np.random.SeedSequence([int(seed), int(stream)])
    return np.random.Generator(np.random.PCG64(ss))


def complex_gaussian(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """i.i.d. complex normal entries, real and imaginary parts N(0, 1/2), Fortran order.

    The draws fill the matrix column by column, real then imaginary part of each entry."""
    buf = np.empty((cols, 2 * rows))
    rng.standard_normal(out=buf)
    buf *= math.sqrt(0.5)
    return buf.view(np.complex128).T          # (rows, cols), Fortran-ordered view


def _t(a: np.ndarray):
    """Fortran-ordered complex matrix -> torch tensor of its transpose (C-contiguous, no copy)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.T))


def _from_t(t) -> np.ndarray:
    """torch tensor holding a transpose -> Fortran-ordered numpy matrix (no copy)."""
    return t.numpy().T


def _to_fortran(t) -> np.ndarray:
    """torch matrix -> Fortran-ordered numpy array with the same entries (threaded transpose copy)."""
    return t.T.contiguous().numpy().T


def haar_unitary_t(rng: np.random.Generator, n: int):
    """Haar-distributed n x n unitary as a torch tensor: QR of a complex Gaussian (an i.i.d. matrix,
    taken in whichever memory order it was drawn) with R's diagonal made real positive."""
    import torch
    z = torch.from_numpy(complex_gaussian(rng, n, n).T)      # C-contiguous; still i.i.d. Gaussian
    q, r = torch.linalg.qr(z)
    d = torch.diagonal(r)
    return q * (d / d.abs())[None, :]


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed n x n unitary, Fortran order."""
    return _to_fortran(haar_unitary_t(rng, n))


def split_spectrum(rng: np.random.Generator, n: int, n_low: int) -> np.ndarray:
    """``n_low`` values uniform in [-1, -0.5] and ``n - n_low`` uniform in [-0.4, 1], sorted."""
    lo = rng.uniform(-1.0, -0.5, size=n_low)
    hi = rng.uniform(-0.4, 1.0, size=n - n_low)
    return np.sort(np.concatenate([lo, hi]))


def overlap_matrix(rng: np.random.Generator, n: int, rank: int = 64) -> np.ndarray:
    """HPD overlap S = I + G G^H / n with G an n x rank complex Gaussian."""
    import torch
    g = torch.from_numpy(complex_gaussian(rng, rank, n).T)   # n x rank, i.i.d.
    s = (g @ g.conj().T) / n
    s = 0.5 * (s + s.conj().T)
    s.diagonal().add_(1.0)
    return _to_fortran(s)


def hermitian_noise(rng: np.random.Generator, n: int) -> np.ndarray:
    """(E + E^H) / 2 with E an i.i.d. complex Gaussian (exactly Hermitian in floating point)."""
    et = _t(complex_gaussian(rng, n, n))      # E^T
    return _from_t(0.5 * (et + et.conj().T))   # (E^T + conj(E))/2 = ((E + E^H)/2)^T


@dataclasses.dataclass
class Pencil:
    """One problem of a sequence.  ``S`` is None for a standard problem."""
    A: np.ndarray
    S: Optional[np.ndarray]
    lam_exact: Optional[np.ndarray]   # exact spectrum when A is in designed form (cycle 0)
    X_exact: Optional[np.ndarray]     # exact S-orthonormal eigenvectors (designed form), n x n
    cycle: int = 0


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

    def eps(self, cycle: int) -> float:
        return self.eps0 * self.eps_decay ** cycle


def designed_pencil(spec: SequenceSpec, keep_vectors: bool = True) -> Pencil:
    """Cycle-0 pencil in designed form: exact spectrum and eigenvectors are known."""
    import torch
    n = spec.n
    lam = split_spectrum(_rng(spec.seed, _STREAM_LAM), n, spec.n_low)
    q = haar_unitary_t(_rng(spec.seed, _STREAM_Q), n)
    lt = torch.from_numpy(lam)
    if spec.generalized:
        s = overlap_matrix(_rng(spec.seed, _STREAM_G), n)
        lchol = torch.linalg.cholesky(torch.from_numpy(s))
        lq = lchol @ q
        a = (lq * lt[None, :]) @ lq.conj().T
        x = torch.linalg.solve_triangular(lchol.conj().T, q, upper=True) if keep_vectors else None
    else:
        s = None
        a = (q * lt[None, :]) @ q.conj().T
        x = q if keep_vectors else None
    a = 0.5 * (a + a.conj().T)
    return Pencil(A=_to_fortran(a), S=s, lam_exact=lam, X_exact=None if x is None else _to_fortran(x), cycle=0)


def sequence(spec: SequenceSpec, keep_vectors: bool = False) -> Iterator[Pencil]:
    """Yield the pencils of cycles 0 .. spec.cycles-1 (A_{l+1} = A_l + eps_l (E_l + E_l^H)/2).

    Every term is exactly Hermitian, so every A_l is exactly Hermitian as well."""
    p = designed_pencil(spec, keep_vectors=keep_vectors)
    yield p
    a = p.A
    for ell in range(1, spec.cycles):
        e = hermitian_noise(_rng(spec.seed, _STREAM_E0 + ell - 1), spec.n)
        e *= spec.eps(ell - 1)
        a = a + e
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


def kpoint_problem(k: int, n: int, seed: int = 0, eps: float = 1e-3) -> KPointProblem:
    """k-point problem k of one SCF cycle: a designed generalized pencil perturbed by eps, warm start
    from the unperturbed eigenvectors.  nev = ceil(0.06 n), nex = ceil(0.2 nev)."""
    nev = int(math.ceil(0.06 * n))
    nex = int(math.ceil(0.2 * nev))
    spec = SequenceSpec(n=n, n_low=int(math.ceil(0.05 * n)), generalized=True, cycles=1, eps0=eps,
                        eps_decay=1.0, seed=1000 * (seed + 1) + k, nev=nev, nex=nex, deg=12)
    p = designed_pencil(spec, keep_vectors=True)
    e = hermitian_noise(_rng(spec.seed, _STREAM_E0), n)
    e *= eps
    a = p.A + e
    m = nev + nex
    return KPointProblem(n=n, nev=nev, nex=nex, A=a, S=p.S, X0=np.asfortranarray(p.X_exact[:, :m]),
                         lam_prev=p.lam_exact[:m].copy())
