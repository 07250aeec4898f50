"""Pins of the oracle's block LOBPCG (the paper's second solver, Section 3.1; the GEN vs STD
comparison of Table 2) against what the mathematics fixes, independently of its own code:

  - the nev smallest eigenpairs of a Hermitian matrix / pencil (LAPACK's eigvalsh / eigh, the plain
    definition) to the solver's accuracy: |lambda - lambda_ref| <= 1e-10 max(|lambda_ref|, 1e-3),
    residuals <= 1e-10, S-orthonormal vectors to 1e-12;
  - a designed pencil with an ill-conditioned overlap (kappa(S) = 1e3), iterated directly (GEN) and
    after the reduction (STD), against its exact spectrum;
  - a block as large as the space: one Rayleigh-Ritz step on the whole space is exact;
  - the convergence rate of the three-term (conjugate-direction) recurrence: on a spectrum with
    relative gap g, one vector needs about sqrt(1/g) ln(2/tol) / 2 iterations (the rate of
    conjugate gradients / Chebyshev acceleration), while steepest descent (the recurrence without
    its third block) needs about ln(2/tol) / (2 g); the test bounds the count by twice the former,
    far below the latter;
  - a warm start from the exact eigenvectors converges without iterating.
"""
import math

import numpy as np
import pytest

from paper_1206_3768_amd import synth


def cg(n, m, rng):
    return (rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))) / math.sqrt(2)


def herm(n, rng):
    g = cg(n, n, rng)
    return np.asfortranarray(0.5 * (g + g.conj().T))


def _check_pairs(r, ref, nev, X, S=None):
    lam = r.lam[:nev]
    assert np.all(np.abs(lam - ref[:nev]) <= 1e-10 * np.maximum(np.abs(ref[:nev]), 1e-3)), np.abs(lam - ref[:nev]).max()
    assert r.resid[:nev].max() <= 1e-10
    Sm = np.eye(X.shape[0]) if S is None else S
    G = X.conj().T @ Sm @ X
    assert np.abs(G - np.eye(G.shape[0])).max() <= 1e-12


def test_lobpcg_standard_matches_eigvalsh(orc):
    rng = np.random.default_rng(1)
    A = herm(120, rng)
    r = orc.lobpcg(A, None, nev=10, tol=1e-10, seed=3)
    assert r.status == 0
    assert r.X.shape[1] == orc.lobpcg_block_size(10) == 11
    _check_pairs(r, np.linalg.eigvalsh(A), 10, r.X)


@pytest.mark.parametrize("gen", [False, True])
def test_lobpcg_ill_conditioned_pencil_gen_and_std(orc, gen):
    spec = synth.SequenceSpec(n=150, n_low=10, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=3, kappa=1e3)
    p = synth.designed_pencil(spec)
    r = orc.lobpcg(p.A, p.S, nev=12, tol=1e-10, gen=gen, seed=3)
    assert r.status == 0
    _check_pairs(r, p.lam_exact, 12, r.X, p.S)


def test_lobpcg_gen_needs_more_iterations_than_std_on_ill_conditioned_overlap(orc):
    """Table 2's finding on a synthetic pencil: with an ill-conditioned S the iteration on the
    pencil is much slower than on the reduced problem."""
    spec = synth.SequenceSpec(n=150, n_low=10, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=3, kappa=1e3)
    p = synth.designed_pencil(spec)
    std = orc.lobpcg(p.A, p.S, nev=12, tol=1e-10, gen=False, seed=3)
    gen = orc.lobpcg(p.A, p.S, nev=12, tol=1e-10, gen=True, seed=3)
    assert std.status == 0 and gen.status == 0
    assert gen.stats["iters"] > 3 * std.stats["iters"]
    assert gen.stats["bmatvecs"] > 0 and std.stats["bmatvecs"] == 0


def test_lobpcg_block_of_the_whole_space_is_exact(orc):
    rng = np.random.default_rng(2)
    A = herm(12, rng)
    r = orc.lobpcg(A, None, nev=12, bs=12, tol=1e-10, seed=1)
    assert r.status == 0 and r.stats["iters"] <= 1
    assert np.allclose(r.lam, np.linalg.eigvalsh(A), rtol=0, atol=1e-13)


def test_lobpcg_convergence_rate_of_the_three_term_recurrence(orc):
    """One vector on a diagonal spectrum: lambda_1 = 0, lambda_2 = g, the rest in [0.5, 1]."""
    n, g, tol = 400, 1e-3, 1e-10
    rng = np.random.default_rng(4)
    d = np.concatenate([[0.0, g], np.sort(rng.uniform(0.5, 1.0, n - 2))])
    A = np.asfortranarray(np.diag(d).astype(complex))
    r = orc.lobpcg(A, None, nev=1, bs=1, tol=tol, seed=5, maxiter=5000)
    assert r.status == 0
    assert abs(r.lam[0]) <= 1e-10
    cg_rate = 0.5 * math.sqrt(1.0 / g) * math.log(2.0 / tol)    # about 380
    sd_rate = 0.5 / g * math.log(2.0 / tol)                     # about 12000
    assert r.stats["iters"] <= 2 * cg_rate < sd_rate / 10
    # the eigenvector is the first unit vector up to a phase
    assert abs(abs(r.X[0, 0]) - 1.0) <= 1e-9


def test_lobpcg_warm_start_from_eigenvectors(orc):
    rng = np.random.default_rng(6)
    A = herm(80, rng)
    w, V = np.linalg.eigh(A)
    X0 = np.asfortranarray(V[:, :9])
    r = orc.lobpcg(A, None, nev=8, bs=9, tol=1e-10, X0=X0, seed=1)
    assert r.status == 0 and r.stats["iters"] == 1
    assert np.allclose(r.lam, w[:9], rtol=0, atol=1e-13)
