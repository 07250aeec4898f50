"""Parity at the benchmark's full sizes, in the configuration bench.py times, checked by properties
that hold at any size (the oracle is too slow here): the pencils of cycle 0 are in designed form,
so their exact spectrum is known, and residuals are recomputed on the host for sampled columns,
independently of the library.

  c2: n = 2048 generalized, nev 128, nex 64, degree 12, FP64;
  c3: n = 8192 generalized, nev 400, nex 80, degree 12 (the bench's headline workload), with the
      FP64, FP32, BF16x3 and BF16x6 filters; cycle 0 against its designed spectrum, and the whole
      5-cycle warm-started sequence against the eigenvalues the CPU oracle computed for it
      (tests/golden/c3_oracle_eigenvalues.json, written by tests/golden/make_c3_golden.py).
"""
import json
import os

import numpy as np
import pytest

from paper_1206_3768_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_3768_amd import autotune, chfsi
    h = chfsi.Handle(0)
    autotune.load(h)   # the committed MI355X plan table, as bench.py uses it
    return h


def _check(res, p, nev, X, cols):
    lam = res.lam[:nev]
    ref = p.lam_exact[:nev]
    normA = np.abs(p.A).sum(axis=0).max()   # ||A||_1 >= ||A||_2 (Hermitian)
    assert np.all(np.abs(lam - ref) <= 1e-10 * np.maximum(np.abs(ref), 1e-3 * normA)), np.max(np.abs(lam - ref))
    assert res.resid[:nev].max() <= 1e-10
    # host residuals ||A x - lam S x|| / ||A||_lo (||A||_lo = largest column norm) on sampled columns
    lo = np.sqrt((np.abs(p.A) ** 2).sum(axis=0).max())
    for j in cols:
        r = p.A @ X[:, j] - lam[j] * (p.S @ X[:, j])
        assert np.linalg.norm(r) / lo <= 2e-10, (j, np.linalg.norm(r) / lo)
    # S-orthonormality of the sampled columns
    Xs = X[:, cols]
    G = Xs.conj().T @ (p.S @ Xs)
    assert np.abs(G - np.eye(len(cols))).max() <= 1e-12


def test_c2_full_size_fp64_matches_designed_spectrum(hd):
    from paper_1206_3768_amd import chfsi
    spec = synth.config_generalized_sequence()
    p = synth.designed_pencil(spec, keep_vectors=False)
    m = spec.nev + spec.nex
    dX = chfsi.to_device(np.zeros((spec.n, m), dtype=complex))
    res = hd.solve(chfsi.to_device(p.A), chfsi.to_device(p.S), dX, False,
                   chfsi.default_params(nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1))
    assert res.status == 0
    _check(res, p, spec.nev, chfsi.to_numpy(dX), [0, 1, 63, 64, 102, 103, 127])


@pytest.fixture(scope="module")
def c3_cycle0():
    spec = synth.config_mixed_precision()
    return spec, synth.designed_pencil(spec, keep_vectors=False)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_c3_full_size_low_precision_filter_matches_designed_spectrum(hd, c3_cycle0, prec):
    from paper_1206_3768_amd import chfsi
    spec, p = c3_cycle0
    m = spec.nev + spec.nex
    print(f"c3 cycle 0, {prec} filter", flush=True)
    dX = chfsi.to_device(np.zeros((spec.n, m), dtype=complex))
    res = hd.solve(chfsi.to_device(p.A), chfsi.to_device(p.S), dX, False,
                   chfsi.default_params(nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1,
                                        filter_precision=chfsi.PRECISIONS[prec]))
    assert res.status == 0
    assert res.stats["precision_switches"] > 0
    _check(res, p, spec.nev, chfsi.to_numpy(dX), [0, 1, 199, 200, 398, 399])


GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle_eigenvalues.json")


@pytest.fixture(scope="module")
def c3_sequence(hd):
    from paper_1206_3768_amd import sequence
    if not os.path.exists(GOLDEN_C3):
        pytest.skip("reference eigenvalues of the n = 8192 sequence not generated")
    with open(GOLDEN_C3) as fh:
        gold = {c["cycle"]: np.array([float(v) for v in c["lam"]]) for c in json.load(fh)["cycles"]}
    seq = sequence.Sequence(synth.config_mixed_precision(), handle=hd)
    yield seq, gold
    seq.A.clear()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_c3_sequence_every_eigenpair_against_oracle(c3_sequence, prec):
    """The bench's headline workload: cycle 0 from a random block, each later cycle warm-started
    from the previous solution; every one of the 400 converged eigenvalues of every cycle against
    the CPU oracle's, and the residuals, with the FP64 filter and each low-precision filter."""
    seq, gold = c3_sequence
    spec = seq.spec
    for c in range(spec.cycles):
        print(f"c3 cycle {c}, {prec} filter", flush=True)
        r = seq.solve(c, warm=c > 0, store=True, filter_precision=prec)
        assert r.status == 0, (c, r.status)
        assert r.resid[:spec.nev].max() <= 1e-10
        if c not in gold:
            continue
        ref = gold[c]
        err = np.abs(r.lam[:spec.nev] - ref)
        assert np.all(err <= 1e-10 * np.maximum(np.abs(ref), 1e-3)), (c, float(err.max()))


def test_c4_full_size_batch_matches_single_solves(hd):
    """Three k-point problems at the sizes of the batched workload (n in [1500, 6000]): one batch
    against single solves of the same problems, and host residuals of sampled columns."""
    from paper_1206_3768_amd import chfsi
    kps = [synth.kpoint_problem(k, n) for k, n in enumerate((1601, 3203, 5870))]
    probs = [dict(A=chfsi.to_device(kp.A), S=chfsi.to_device(kp.S), X=chfsi.to_device(kp.X0), nev=kp.nev,
                  nex=kp.nex, x_is_guess=1) for kp in kps]
    single = []
    for kp, pr in zip(kps, probs):
        X = chfsi.to_device(kp.X0)
        r = hd.solve(pr["A"], pr["S"], X, True, chfsi.default_params(nev=kp.nev, nex=kp.nex, deg=12, tol=1e-10))
        assert r.status == 0
        single.append(r.lam[:kp.nev].copy())
    st, res = hd.solve_batched(probs, chfsi.default_params(nev=1, nex=0, deg=12, tol=1e-10))
    assert st == 0
    for kp, pr, r, lam1 in zip(kps, probs, res, single):
        lam = r.lam[:kp.nev]
        assert np.all(np.abs(lam - lam1) <= 1e-12 * np.maximum(np.abs(lam1), 1e-3))
        X = chfsi.to_numpy(pr["X"])
        lo = np.sqrt((np.abs(kp.A) ** 2).sum(axis=0).max())
        for j in (0, kp.nev // 2, kp.nev - 1):
            rr = kp.A @ X[:, j] - lam[j] * (kp.S @ X[:, j])
            assert np.linalg.norm(rr) / lo <= 2e-10


def test_ill_conditioned_n2048_sequence_against_oracle(hd, orc):
    """The n = 2048 sequence with an overlap of condition number 1e6 (config_ill_conditioned), three
    warm-started cycles through the Hermitian two-sided reduction: every converged eigenvalue
    against the oracle's (its products, solves and Cholesky factor in LAPACK at this size), and
    LAPACK's generalized solver; residuals <= 1e-10, loops within one of the oracle's."""
    import scipy.linalg as sla
    from paper_1206_3768_amd import chfsi
    spec = synth.config_ill_conditioned()
    m = spec.nev + spec.nex
    X = Xo = bnd = bnd_o = None
    orc.use_library_products(True)
    try:
        for pen in synth.sequence(spec):
            print(f"ill-conditioned n=2048 cycle {pen.cycle}", flush=True)
            ref = orc.solve(pen.A, pen.S, nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1, X0=Xo,
                            bounds=bnd_o)
            assert ref.status == 0
            dX = chfsi.to_device(np.zeros((spec.n, m), dtype=complex) if X is None else X)
            prm = chfsi.default_params(nev=spec.nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=1)
            if bnd is not None:
                prm.have_bounds, prm.mu1, prm.a = 1, bnd[0], bnd[1]
            r = hd.solve(chfsi.to_device(pen.A), chfsi.to_device(pen.S), dX, X is not None, prm)
            assert r.status == 0
            ev = sla.eigh(pen.A, pen.S, eigvals_only=True, subset_by_index=[0, spec.nev - 1])
            for lam_ref in (ref.lam[:spec.nev], ev):
                assert np.all(np.abs(r.lam[:spec.nev] - lam_ref) <= 1e-10 * np.maximum(np.abs(lam_ref), 1e-3))
            assert r.resid[:spec.nev].max() <= 1e-10
            assert abs(r.stats["loops"] - ref.stats["loops"]) <= 1
            X = chfsi.to_numpy(dX)
            Xo, bnd, bnd_o = ref.X, (float(r.lam[0]), float(r.lam[m - 1])), (float(ref.lam[0]), float(ref.lam[m - 1]))
    finally:
        orc.use_library_products(False)
