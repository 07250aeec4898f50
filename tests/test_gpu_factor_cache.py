"""The handle's cached Cholesky factor of the overlap: a solve whose S equals (bit for bit) the last
factored overlap reuses the factor, and its results are bit-identical to those of a fresh handle
(the factor is the same deterministic computation); a changed S is factored again."""
import numpy as np
import pytest

from paper_1206_3768_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return torch


def _solve(h, pen, spec, X=None):
    from paper_1206_3768_amd import chfsi
    m = spec.nev + spec.nex
    dX = chfsi.to_device(np.zeros((spec.n, m), dtype=complex) if X is None else X)
    r = h.solve(chfsi.to_device(pen.A), chfsi.to_device(pen.S), dX, X is not None,
                chfsi.default_params(nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1))
    return r, chfsi.to_numpy(dX)


def test_factor_reused_for_an_equal_overlap_and_refactored_for_a_changed_one(torch_dev, orc):
    from paper_1206_3768_amd import chfsi
    spec = synth.SequenceSpec(n=300, n_low=16, generalized=True, cycles=2, eps0=1e-2, eps_decay=0.5, seed=21,
                              nev=16, nex=8, deg=10)
    pens = list(synth.sequence(spec))
    h = chfsi.Handle(0)
    r0, X0 = _solve(h, pens[0], spec)
    assert r0.status == 0 and r0.stats["factor_reused"] == 0
    r1, X1 = _solve(h, pens[1], spec, X0)             # same S (a new device copy of it)
    assert r1.status == 0 and r1.stats["factor_reused"] == 1
    fresh = chfsi.Handle(0)
    f1, Y1 = _solve(fresh, pens[1], spec, X0)
    assert f1.stats["factor_reused"] == 0
    assert np.array_equal(r1.lam, f1.lam) and np.array_equal(X1, Y1)
    ref = orc.solve(pens[1].A, pens[1].S, nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1)
    assert np.all(np.abs(r1.lam[:spec.nev] - ref.lam[:spec.nev]) <= 1e-10 * np.maximum(np.abs(ref.lam[:spec.nev]), 1e-3))
    # one entry of S changed (still Hermitian positive definite): factored again
    S2 = pens[1].S.copy()
    S2[7, 7] += 1e-3
    pen2 = synth.Pencil(A=pens[1].A, S=S2, lam_exact=None, X_exact=None, cycle=1)
    r2, _ = _solve(h, pen2, spec, X0)
    f2, _ = _solve(fresh, pen2, spec, X0)
    assert r2.status == 0 and r2.stats["factor_reused"] == 0
    assert np.array_equal(r2.lam, f2.lam)
    ev = __import__("scipy.linalg", fromlist=["eigh"]).eigh(pens[1].A, S2, eigvals_only=True,
                                                          subset_by_index=[0, spec.nev - 1])
    assert np.all(np.abs(r2.lam[:spec.nev] - ev) <= 1e-10 * np.maximum(np.abs(ev), 1e-3))
    # a different order is factored afresh as well
    spec3 = synth.SequenceSpec(n=200, n_low=12, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=22,
                               nev=12, nex=6, deg=10)
    p3 = synth.designed_pencil(spec3, keep_vectors=False)
    r3, _ = _solve(h, p3, spec3)
    assert r3.status == 0 and r3.stats["factor_reused"] == 0
    assert np.all(np.abs(r3.lam[:12] - p3.lam_exact[:12]) <= 1e-10)
    h.close()
    fresh.close()
