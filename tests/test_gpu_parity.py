"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on identical seeded inputs.

Tolerances (each a rounding-error estimate of the operation with a safety margin):
  FP64 products / filter  : max-abs error <= 1e-12 * max|reference|
  FP32 filter             : <= 2e-4 * max|reference|      (u32 = 6e-8, n up to 512, degree 10)
  BF16x6 filter           : <= 2e-4 * max|reference|      (dropped split terms ~ 2^-24)
  BF16x3 filter           : <= 4e-3 * max|reference|      (dropped split terms ~ 2^-16)
  eigenvalues             : |lam_gpu - lam_ref| <= 1e-10 max(|lam_ref|, 1e-3 ||A||)
  residuals               : ||A x - lam S x|| / ||A||_lo <= 1e-10
  orthonormality          : ||X^H S X - I||_max <= 1e-12
  invariant subspaces     : every principal angle <= 1e-8
  loop count              : within +-1 of the oracle
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1206_3768_amd import synth

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(77)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return torch


@pytest.fixture(scope="module")
def hd(torch_dev):
    from paper_1206_3768_amd import chfsi
    h = chfsi.Handle(0)
    yield h
    h.close()


def dev(a):
    from paper_1206_3768_amd import chfsi
    return chfsi.to_device(np.asarray(a, dtype=np.complex128))


def host(t):
    from paper_1206_3768_amd import chfsi
    return chfsi.to_numpy(t)


def cgauss(n, m, rng=RNG):
    return np.asfortranarray((rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))) / math.sqrt(2))


def herm(n, rng=RNG):
    g = cgauss(n, n, rng)
    return np.asfortranarray(0.5 * (g + g.conj().T))


def relerr(x, ref):
    return np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300)


# ---- random numbers: bit-exact ------------------------------------------------------------------

def test_random_block_bit_exact(hd, orc):
    for (seed, stream, n, m) in [(0, 1, 300, 7), (123456789, 2, 97, 1), (5, 1, 1, 1)]:
        got = host(hd.random_block(seed, stream, n, m))
        ref = orc.random_block(seed, stream, n, m)
        assert np.array_equal(np.ascontiguousarray(got).view(np.uint64),
                              np.ascontiguousarray(ref).view(np.uint64)), (seed, stream, n, m)


# ---- dense product (MFMA kernel) ----------------------------------------------------------------

@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("mnk", [(1, 1, 1), (37, 11, 300), (130, 70, 33), (64, 64, 64), (200, 5, 1500)])
def test_zgemm_parity(hd, orc, ta, tb, mnk):
    import torch
    m, n, k = mnk
    A = cgauss(m, k) if ta == "N" else cgauss(k, m)
    B = cgauss(k, n) if tb == "N" else cgauss(n, k)
    Cm = cgauss(m, n)
    ref = orc.zgemm(ta, tb, A, B, alpha=0.75, beta=-0.5, Cm=Cm)
    dA, dB, dC = dev(A), dev(B), dev(Cm)
    hd.zgemm(ta, tb, m, n, k, 0.75, dA, A.shape[0], dB, B.shape[0], -0.5, dC, m)
    assert relerr(host(dC), ref) <= 1e-13 * max(1.0, math.sqrt(k))


def test_zgemm_empty_k_scales_c(hd, orc):
    Cm = cgauss(20, 3)
    dC = dev(Cm)
    dA = dev(np.zeros((20, 1)))
    hd.zgemm("N", "N", 20, 3, 0, 1.0, dA, 20, dA, 1, 2.0, dC, 20)
    assert np.allclose(host(dC), 2.0 * Cm, rtol=0, atol=0)


# ---- Chebyshev filter --------------------------------------------------------------------------

def _filter_case(n, m, seed=3):
    rng = np.random.default_rng(seed)
    spec = synth.SequenceSpec(n=n, n_low=max(1, n // 8), generalized=False, cycles=1, eps0=0, eps_decay=1, seed=seed)
    p = synth.designed_pencil(spec, keep_vectors=False)
    Y0 = cgauss(n, m, rng)
    return p.A, Y0, -0.45, 1.05, -1.0


@pytest.mark.parametrize("n,m,deg", [(300, 37, 10), (64, 64, 1), (129, 3, 7), (512, 48, 12)])
def test_filter_fp64_parity(hd, orc, n, m, deg):
    H, Y0, a, b, mu1 = _filter_case(n, m)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=deg)
    dH, dY = dev(H), dev(Y0)
    hd.filter(dH, dY, a, b, mu1, deg=deg, prec=0)
    assert relerr(host(dY), ref) <= 1e-12


def test_filter_fp64_degree_zero_is_identity(hd, orc):
    H, Y0, a, b, mu1 = _filter_case(100, 5)
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=0, prec=0)
    assert np.array_equal(host(dY), Y0)


def test_filter_per_column_degrees_parity(hd, orc):
    H, Y0, a, b, mu1 = _filter_case(300, 9)
    degs = [3, 0, 12, 7, 7, 1, 12, 2, 5]
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=degs)
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=degs, prec=0)
    assert relerr(host(dY), ref) <= 1e-12


@pytest.mark.parametrize("prec,tol", [(1, 2e-4), (3, 2e-4), (2, 4e-3)])
def test_filter_low_precision_against_fp64_oracle(hd, orc, prec, tol):
    H, Y0, a, b, mu1 = _filter_case(512, 48)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=10)
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=10, prec=prec)
    err = relerr(host(dY), ref)
    assert err <= tol, err


@pytest.mark.parametrize("n,m", [(4096, 768), (8192, 480)])
def test_filter_bf16x3_wide_tiles_against_fp64_filter(hd, torch_dev, n, m):
    """The BF16x3 filter on 128 x 128 tiles (taken when they still give a workgroup per CU: with a
    K split at n = 4096, w = 768, without one at the n = 8192 block of the sequence) against the FP64
    filter of the same library (itself checked against the oracle above), the two-term split's
    tolerance 4e-3 of the largest entry."""
    from paper_1206_3768_amd import chfsi
    g = torch_dev.Generator(device="cuda").manual_seed(5)
    A = torch_dev.randn((n, n), dtype=torch_dev.complex128, device="cuda", generator=g) * (1.0 / math.sqrt(2 * n))
    A = (0.5 * (A + A.conj().T)).contiguous()
    Y0 = torch_dev.randn((m, n), dtype=torch_dev.complex128, device="cuda", generator=g)
    Y1, Y2 = Y0.clone(), Y0.clone()
    hd.filter(A, Y1, -0.3, 1.2, -1.0, deg=3, prec=chfsi.FP64)
    hd.filter(A, Y2, -0.3, 1.2, -1.0, deg=3, prec=chfsi.BF16X3)
    log = hd.filter_launch_log()
    assert np.all(log[:, 3] == 128)   # the wide-tile kernel ran every step
    ref = host(Y1)
    assert relerr(host(Y2), ref) <= 4e-3


def test_filter_closed_form_diagonal(hd, orc):
    # diagonal H: (Y_d)_j = T_d((h_j - c)/e) / T_d((mu1 - c)/e) (Y_0)_j
    n, d = 200, 9
    h = np.sort(RNG.uniform(-1, 1, n))
    H = np.diag(h).astype(complex)
    Y0 = cgauss(n, 4)
    a, b, mu1 = -0.5, 1.2, -1.0
    c, e = (a + b) / 2, (b - a) / 2

    def T(t):
        t = np.asarray(t, dtype=float)
        return np.where(np.abs(t) <= 1, np.cos(d * np.arccos(np.clip(t, -1, 1))),
                        np.sign(t) ** d * np.cosh(d * np.arccosh(np.maximum(np.abs(t), 1))))
    ref = (T((h - c) / e) / T((mu1 - c) / e))[:, None] * Y0
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=d, prec=0)
    assert relerr(host(dY), ref) <= 1e-12


# ---- reduction, Lanczos, QR, Rayleigh-Ritz ------------------------------------------------------

@pytest.mark.parametrize("entry", ["reduce", "reduce_explicit"])
@pytest.mark.parametrize("n,kappa", [(40, 0.0), (64, 0.0), (257, 0.0), (1100, 0.0), (300, 1e6), (700, 1e6)])
def test_reduce_parity(hd, orc, torch_dev, n, kappa, entry):
    """The Hermitian two-sided reduction against the oracle's two triangular solves, in both of the
    library's forms: 64-column panels with lower-triangle rank-2k updates and one solve with a
    block-lower right-hand side (reduce), and two products with the explicit inverse L^{-1} that
    end each tile's inner dimension at the diagonal (reduce_explicit).  One panel or tile row (40,
    64), several with a ragged last one (257), the recursive splits (1100), and overlaps of
    condition number 1e6.  H's rounding grows with kappa(L) = sqrt(kappa)."""
    spec = synth.SequenceSpec(n=n, n_low=max(4, n // 20), generalized=True, cycles=1, eps0=0, eps_decay=1, seed=8,
                              kappa=kappa)
    p = synth.designed_pencil(spec, keep_vectors=False)
    Lr, st = orc.cholesky(p.S)
    Hr = orc.reduce(p.A, Lr)
    n = spec.n
    dH = torch_dev.empty((n, n), dtype=torch_dev.complex128, device="cuda")
    dL = torch_dev.empty((n, n), dtype=torch_dev.complex128, device="cuda")
    getattr(hd, entry)(dev(p.A), dev(p.S), dH, dL)
    H = host(dH)
    assert np.array_equal(H, H.conj().T)
    # both factors carry rounding amplified by the conditioning of the factorisation, which grows
    # like sqrt(kappa(S)) (first-order perturbation of the Cholesky factor)
    assert relerr(host(dL), Lr) <= 1e-13 * max(1.0, math.sqrt(kappa) / 10.0)
    assert relerr(H, Hr) <= 1e-12 * max(1.0, math.sqrt(kappa) / 10.0)
    # the designed spectrum survives the reduction
    assert np.max(np.abs(np.linalg.eigvalsh(H) - p.lam_exact)) <= 1e-12 * max(1.0, math.sqrt(kappa) / 10.0)


def test_reduce_above_4096_by_sampled_identities(hd, torch_dev):
    """n = 4160 (65 panels, several levels of the block-lower solve).  Checked without the oracle
    (too slow at this size) on sampled entries: (L L^H)_ij = S_ij and (L H L^H)_ij = A_ij, H exactly
    Hermitian, L lower."""
    spec = synth.SequenceSpec(n=4160, n_low=200, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=5)
    p = synth.designed_pencil(spec, keep_vectors=False)
    n = spec.n
    dH = torch_dev.empty((n, n), dtype=torch_dev.complex128, device="cuda")
    dL = torch_dev.empty((n, n), dtype=torch_dev.complex128, device="cuda")
    hd.reduce(dev(p.A), dev(p.S), dH, dL)
    H, L = host(dH), host(dL)
    assert np.array_equal(H, H.conj().T)
    assert np.all(np.triu(L, 1) == 0)
    rng = np.random.default_rng(3)
    idx = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(24, 2))] + [(0, 0), (n - 1, n - 1), (n - 1, 0), (4096, 63)]
    scale_a = np.abs(p.A).max()
    for i, j in idx:
        assert abs(L[i] @ L[j].conj() - p.S[i, j]) <= 1e-12 * np.abs(p.S).max()
        assert abs(L[i] @ H @ L[j].conj() - p.A[i, j]) <= 1e-11 * scale_a


@pytest.mark.parametrize("entry", ["reduce", "reduce_explicit"])
@pytest.mark.parametrize("n,bad", [(40, 5), (1100, 1050)])
def test_reduce_rejects_non_hpd(hd, torch_dev, n, bad, entry):
    from paper_1206_3768_amd import chfsi
    S = np.eye(n, dtype=complex)
    S[bad, bad] = -1
    dH = torch_dev.empty((n, n), dtype=torch_dev.complex128, device="cuda")
    with pytest.raises(chfsi.ChfsiError) as ei:
        getattr(hd, entry)(dev(herm(n)), dev(S), dH, dH.clone())
    assert ei.value.status == 2


def test_lanczos_parity(hd, orc):
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec, keep_vectors=False)
    for k in (10, 25, 60):
        th_r, zw_r, bk_r = orc.lanczos(p.A, k, seed=11)
        th, zw, bk = hd.lanczos(dev(p.A), k, 11)
        assert np.max(np.abs(th - th_r)) <= 1e-12
        assert np.max(np.abs(zw - zw_r)) <= 1e-10
        assert abs(bk - bk_r) <= 1e-10 * max(1.0, bk_r)


def test_lanczos_parity_eight_loads_in_flight(hd, orc):
    # above n = 3072 the matrix-vector product keeps eight loads in flight per lane
    n = 4096
    H = herm(n, np.random.default_rng(41)) / math.sqrt(n)
    th_r, zw_r, bk_r = orc.lanczos(H, 25, seed=7)
    th, zw, bk = hd.lanczos(dev(H), 25, 7)
    assert np.max(np.abs(th - th_r)) <= 1e-12 * np.abs(th_r).max()
    assert np.max(np.abs(zw - zw_r)) <= 1e-10
    assert abs(bk - bk_r) <= 1e-10 * max(1.0, bk_r)


def test_orthonormalize_parity(hd, orc):
    n, m, nl = 400, 30, 12
    YL, _, _ = orc.qr(cgauss(n, nl))
    Y = cgauss(n, m)
    # reference: CGS twice against YL, then QR with a positive real diagonal
    Yr = Y.copy()
    for _ in range(2):
        Yr = Yr - YL @ (YL.conj().T @ Yr)
    Qr, _, _ = orc.qr(Yr)
    dY = dev(Y)
    hd.orthonormalize(dY, dev(YL))
    Q = host(dY)
    assert relerr(Q, Qr) <= 1e-11
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-13
    assert np.abs(YL.conj().T @ Q).max() <= 1e-13


def test_orthonormalize_ill_conditioned_block(hd, orc):
    # nearly collinear columns (condition ~1e12): the shifted first pass keeps the result orthonormal
    n, m = 300, 10
    base = cgauss(n, 1)
    Y = base + 1e-12 * cgauss(n, m) + np.linspace(0, 1e-6, m)[None, :] * cgauss(n, m)
    dY = dev(Y)
    hd.orthonormalize(dY)
    Q = host(dY)
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-12
    # span check: the first column is the normalised first input column
    assert abs(abs(np.vdot(Q[:, 0], Y[:, 0])) / np.linalg.norm(Y[:, 0]) - 1) <= 1e-12


def test_rayleigh_ritz_parity(hd, orc):
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec, keep_vectors=False)
    Y, _, _ = orc.qr(cgauss(512, 24))
    G = Y.conj().T @ p.A @ Y
    w, W, _ = orc.jacobi(G)
    Yr = Y @ W
    rr = orc.residuals(p.A @ Yr, Yr, w)
    dY = dev(Y)
    th, r = hd.rayleigh_ritz(dev(p.A), dY)
    assert np.max(np.abs(th - w)) <= 1e-13
    gaps = np.minimum(np.diff(np.r_[-np.inf, w]), np.diff(np.r_[w, np.inf]))
    # eigenvector columns are unique (phase normalised) for simple eigenvalues
    col_err = np.max(np.abs(host(dY) - Yr), axis=0)
    assert np.all(col_err <= 1e-13 / np.minimum(gaps, 1.0) + 1e-12)
    assert np.allclose(r, rr, rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("n,m", [(1024, 192), (1024, 480)])
def test_rayleigh_ritz_parity_many_jacobi_blocks(hd, orc, n, m):
    """Rayleigh quotients of the solver's real block widths: the block-Jacobi eigensolver meets its
    16-index blocks in round-robin order (12 blocks and 11 rounds per sweep at m = 192, 30 blocks
    and 29 rounds at m = 480).  Eigenvalues element by element against the oracle's cyclic Jacobi of
    the same Rayleigh quotient, within the rounding of forming it in another order (2 (n + m) u ||G||),
    eigenvector columns of simple eigenvalues within that over the gap."""
    rng = np.random.default_rng(m)
    H = herm(n, rng) / math.sqrt(n)
    Y, _, _ = orc.qr(cgauss(n, m, rng))
    G = orc.zgemm("C", "N", Y, orc.zgemm("N", "N", H, Y))
    w, W, _ = orc.jacobi(G)
    Yr = Y @ W
    normG = np.abs(w).max()
    tol = 2.0 * (n + m) * 1.1e-16 * normG
    dY = dev(Y)
    th, r = hd.rayleigh_ritz(dev(H), dY)
    assert np.max(np.abs(th - w)) <= tol, np.max(np.abs(th - w)) / normG
    gaps = np.minimum(np.diff(np.r_[-np.inf, w]), np.diff(np.r_[w, np.inf]))
    simple = gaps > 1e-6 * normG
    col_err = np.max(np.abs(host(dY) - Yr), axis=0)
    assert np.all(col_err[simple] <= 10.0 * tol / gaps[simple] + 1e-12), np.max(col_err[simple] * gaps[simple])
    rr = orc.residuals(H @ Yr, Yr, w)
    assert np.allclose(r, rr, rtol=1e-6, atol=10.0 * tol)


def test_rayleigh_ritz_with_converged_columns(hd, orc):
    """Columns that are exact eigenvectors give rows of Y^H H Y without off-diagonal coupling; the
    eigensolver deflates them and must still return every pair, in ascending order."""
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec)
    rng = np.random.default_rng(12)
    exact = [3, 10, 11, 40, 200, 500]                      # eigenvector indices taken exactly
    R = cgauss(512, 18, rng)
    E = p.X_exact[:, exact]
    R -= E @ (E.conj().T @ R)
    R, _, _ = orc.qr(R)
    Y = np.concatenate([R, E], axis=1)
    Y = np.asfortranarray(Y[:, rng.permutation(Y.shape[1])])   # interleave exact and random columns
    G = Y.conj().T @ p.A @ Y
    w, W, _ = orc.jacobi(G)
    Yr = Y @ W
    rr = orc.residuals(p.A @ Yr, Yr, w)
    dY = dev(Y)
    th, r = hd.rayleigh_ritz(dev(p.A), dY)
    assert np.max(np.abs(th - w)) <= 1e-13
    assert all(np.min(np.abs(th - p.lam_exact[e])) <= 1e-13 for e in exact)
    Yg = host(dY)
    assert np.abs(Yg.conj().T @ Yg - np.eye(Y.shape[1])).max() <= 1e-13
    assert np.allclose(r, rr, rtol=1e-6, atol=1e-13)


# ---- the whole solver --------------------------------------------------------------------------

def _angles(X, Y, S=None):
    if S is not None:
        L = np.linalg.cholesky(S)
        X = L.conj().T @ X
        Y = L.conj().T @ Y
    return sla.subspace_angles(X, Y)


def _check_solution(res, ref_lam, nev, normA, X, S, tol=1e-10):
    lam = res.lam[:nev]
    assert np.all(np.abs(lam - ref_lam[:nev]) <= 1e-10 * np.maximum(np.abs(ref_lam[:nev]), 1e-3 * normA)), \
        np.max(np.abs(lam - ref_lam[:nev]))
    assert res.resid[:nev].max() <= tol
    m = X.shape[1]
    G = X.conj().T @ (X if S is None else S @ X)
    assert np.abs(G - np.eye(m)).max() <= 1e-12


def test_solve_config1_matches_oracle(hd, orc):
    from paper_1206_3768_amd import chfsi
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec)
    ref = orc.solve(p.A, None, nev=32, nex=16, deg=10, tol=1e-10, seed=1)
    dX = dev(np.zeros((512, 48), dtype=complex))
    prm = chfsi.default_params(nev=32, nex=16, deg=10, tol=1e-10, seed=1)
    res = hd.solve(dev(p.A), None, dX, False, prm)
    X = host(dX)
    normA = np.linalg.norm(p.A, 2)
    _check_solution(res, p.lam_exact, 32, normA, X, None)
    assert np.all(np.abs(res.lam[:32] - ref.lam[:32]) <= 1e-10 * np.maximum(np.abs(ref.lam[:32]), 1e-3))
    assert _angles(X[:, :32], ref.X[:, :32]).max() <= 1e-8
    assert _angles(X[:, :32], p.X_exact[:, :32]).max() <= 1e-8
    assert abs(res.stats["loops"] - ref.stats["loops"]) <= 1


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_solve_mixed_precision_recovers_fp64_accuracy(hd, orc, prec):
    from paper_1206_3768_amd import chfsi
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec)
    dX = dev(np.zeros((512, 48), dtype=complex))
    prm = chfsi.default_params(nev=32, nex=16, deg=10, tol=1e-10, seed=1, filter_precision=prec)
    res = hd.solve(dev(p.A), None, dX, False, prm)
    X = host(dX)
    _check_solution(res, p.lam_exact, 32, np.linalg.norm(p.A, 2), X, None)
    assert _angles(X[:, :32], p.X_exact[:, :32]).max() <= 1e-8


def test_solve_generalized_sequence_matches_oracle(hd, orc):
    from paper_1206_3768_amd import chfsi
    spec = synth.config_generalized_sequence(n=384, cycles=3)
    X_ref = None
    b_ref = None
    X_gpu = None
    b_gpu = None
    for pen in synth.sequence(spec):
        ref = orc.solve(pen.A, pen.S, nev=spec.nev, nex=spec.nex, deg=12, tol=1e-10, X0=X_ref, bounds=b_ref, seed=3)
        assert ref.status == 0
        dX = dev(X_gpu if X_gpu is not None else np.zeros((spec.n, spec.nev + spec.nex), dtype=complex))
        kw = dict(nev=spec.nev, nex=spec.nex, deg=12, tol=1e-10, seed=3)
        if b_gpu is not None:
            kw.update(have_bounds=1, mu1=b_gpu[0], a=b_gpu[1])
        res = hd.solve(dev(pen.A), dev(pen.S), dX, X_gpu is not None, chfsi.default_params(**kw))
        X = host(dX)
        ev, evec = sla.eigh(pen.A, pen.S)
        _check_solution(res, ev, spec.nev, np.linalg.norm(pen.A, 2), X, pen.S)
        assert np.all(np.abs(res.lam[:spec.nev] - ref.lam[:spec.nev]) <=
                      1e-10 * np.maximum(np.abs(ref.lam[:spec.nev]), 1e-3))
        assert _angles(X[:, :spec.nev], ref.X[:, :spec.nev], pen.S).max() <= 1e-8
        assert abs(res.stats["loops"] - ref.stats["loops"]) <= 1
        X_ref, b_ref = ref.X, (ref.lam[0], ref.lam[-1])
        X_gpu, b_gpu = X, (res.lam[0], res.lam[-1])


def test_solve_generalized_above_recursion_size_matches_designed_spectrum(hd):
    """n = 1100: the Cholesky factorisation and the triangular solves of the reduction and of the
    back-transform take their recursive branch; the pencil's spectrum is known exactly."""
    from paper_1206_3768_amd import chfsi
    spec = synth.SequenceSpec(n=1100, n_low=55, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=4)
    p = synth.designed_pencil(spec)
    nev, nex = 40, 16
    dX = dev(np.zeros((spec.n, nev + nex), dtype=complex))
    res = hd.solve(dev(p.A), dev(p.S), dX, False, chfsi.default_params(nev=nev, nex=nex, deg=12, tol=1e-10, seed=2))
    _check_solution(res, p.lam_exact, nev, np.linalg.norm(p.A, 2), host(dX), p.S)


def test_solve_ill_conditioned_sequence_matches_oracle(hd, orc):
    """Overlap of condition number 1e6 (the ill-conditioned B of FLAPW pencils), two warm-started
    cycles: eigenvalues against the oracle's and LAPACK's, residuals <= 1e-10, loops within one of
    the oracle's; S-orthonormality carries the rounding of L^{-H} (kappa(L) = 1e3): 1e-11."""
    from paper_1206_3768_amd import chfsi
    spec = synth.SequenceSpec(n=320, n_low=16, generalized=True, cycles=2, eps0=1e-2, eps_decay=0.5, seed=8,
                              nev=16, nex=8, deg=12, kappa=1e6)
    X = Xo = bnd = None
    for pen in synth.sequence(spec):
        m = spec.nev + spec.nex
        ref = orc.solve(pen.A, pen.S, nev=spec.nev, nex=spec.nex, deg=12, tol=1e-10, seed=2, X0=Xo, bounds=bnd)
        assert ref.status == 0
        dX = dev(np.zeros((spec.n, m), dtype=complex) if X is None else X)
        prm = chfsi.default_params(nev=spec.nev, nex=spec.nex, deg=12, tol=1e-10, seed=2)
        if bnd is not None:
            prm.have_bounds, prm.mu1, prm.a = 1, bnd[0], bnd[1]
        r = hd.solve(dev(pen.A), dev(pen.S), dX, X is not None, prm)
        assert r.status == 0
        ev = sla.eigh(pen.A, pen.S, eigvals_only=True)[:spec.nev]
        for lam_ref in (ref.lam[:spec.nev], ev):
            assert np.all(np.abs(r.lam[:spec.nev] - lam_ref) <= 1e-10 * np.maximum(np.abs(lam_ref), 1e-3))
        assert r.resid[:spec.nev].max() <= 1e-10
        Xg = host(dX)
        assert np.abs(Xg.conj().T @ pen.S @ Xg - np.eye(m)).max() <= 1e-11
        assert abs(r.stats["loops"] - ref.stats["loops"]) <= 1
        X, Xo, bnd = Xg, ref.X, (float(r.lam[0]), float(r.lam[m - 1]))


def test_solve_analytic_degree_policy(hd):
    from paper_1206_3768_amd import chfsi
    spec = synth.config_single_standard()
    p = synth.designed_pencil(spec)
    dX = dev(np.zeros((512, 48), dtype=complex))
    prm = chfsi.default_params(nev=32, nex=16, deg=10, tol=1e-10, seed=1, degree_policy=1)
    res = hd.solve(dev(p.A), None, dX, False, prm)
    _check_solution(res, p.lam_exact, 32, np.linalg.norm(p.A, 2), host(dX), None)


def test_solve_error_paths(hd):
    from paper_1206_3768_amd import chfsi
    spec = synth.SequenceSpec(n=96, n_low=8, generalized=True, cycles=1, eps0=0, eps_decay=1, seed=2)
    p = synth.designed_pencil(spec, keep_vectors=False)
    S = p.S.copy()
    S[4, 4] = -3.0
    dX = dev(np.zeros((96, 12), dtype=complex))
    prm = chfsi.default_params(nev=8, nex=4, deg=8)
    assert hd.solve(dev(p.A), dev(S), dX, False, prm, raise_on_error=False).status == 2
    A = p.A.copy()
    A[3, 7] = np.nan
    assert hd.solve(dev(A), dev(p.S), dX, False, prm, raise_on_error=False).status == 4
    prm2 = chfsi.default_params(nev=8, nex=4, deg=2, max_loops=1, tol=1e-14)
    r = hd.solve(dev(p.A), dev(p.S), dX, False, prm2, raise_on_error=False)
    assert r.status == 3 and r.stats["loops"] == 1
    prm3 = chfsi.default_params(nev=90, nex=20)
    assert hd.solve(dev(p.A), dev(p.S), dX, False, prm3, raise_on_error=False).status == 1


# ---- degree network ----------------------------------------------------------------------------

def test_mlp_forward_and_gradient_parity(hd, orc, torch_dev):
    rng = np.random.default_rng(4)
    P = (rng.standard_normal(8769) * 0.2).astype(np.float32)
    X = rng.standard_normal((300, 5)).astype(np.float32)
    y = rng.uniform(4, 30, 300).astype(np.float32)
    dP = torch_dev.from_numpy(P).cuda()
    dXf = torch_dev.from_numpy(X).cuda()
    dy = torch_dev.from_numpy(y).cuda()
    out = hd.mlp_forward(dP, dXf).cpu().numpy()
    ref = orc.mlp_forward(P.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(out - ref) / np.abs(ref)) <= 1e-5
    loss, g = hd.mlp_loss_grad(dP, dXf, dy)
    loss_r, g_r = orc.mlp_loss_grad(P.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    assert abs(loss - loss_r) <= 1e-4 * loss_r
    g = g.cpu().numpy()
    assert np.max(np.abs(g - g_r)) <= 1e-4 * np.max(np.abs(g_r))


def test_adam_step_parity(hd, orc, torch_dev):
    rng = np.random.default_rng(5)
    P = rng.standard_normal(8769).astype(np.float32)
    g = rng.standard_normal(8769).astype(np.float32)
    m = (rng.standard_normal(8769) * 0.1).astype(np.float32)
    v = np.abs(rng.standard_normal(8769) * 0.1).astype(np.float32)
    dP, dg, dm, dv = [torch_dev.from_numpy(x.copy()).cuda() for x in (P, g, m, v)]
    hd.mlp_adam(dP, dg, dm, dv, 3, lr=1e-2)
    P64, m64, v64 = P.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    orc.adam_step(P64, g.astype(np.float64), m64, v64, 3, lr=1e-2)
    assert np.max(np.abs(dP.cpu().numpy() - P64)) <= 1e-5
    assert np.max(np.abs(dm.cpu().numpy() - m64)) <= 1e-6


# ---- every tile plan of the filter kernel --------------------------------------------------------

@pytest.mark.parametrize("plan", [dict(bm=64, bn=64, ksplit=1, fused=0), dict(bm=64, bn=64, ksplit=4, fused=0),
                                  dict(bm=64, bn=64, ksplit=4, fused=1), dict(bm=32, bn=64, ksplit=2, fused=0),
                                  dict(bm=64, bn=32, ksplit=8, fused=1), dict(bm=32, bn=32, ksplit=1, fused=0),
                                  dict(bm=32, bn=32, ksplit=16, fused=0), dict(bm=32, bn=32, ksplit=3, fused=1)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-4)])
def test_filter_every_tile_plan(hd, orc, plan, prec, tol):
    n, m = 520, 70                      # ragged in both tile sizes
    H, Y0, a, b, mu1 = _filter_case(n, m)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=6)
    hd.set_filter_plan(n, m, prec, plan)
    try:
        dY = dev(Y0)
        hd.filter(dev(H), dY, a, b, mu1, deg=6, prec=prec)
    finally:
        hd.set_filter_plan(n, m, prec, None)
    assert relerr(host(dY), ref) <= tol


@pytest.mark.parametrize("plan", [dict(bm=64, bn=64, ksplit=1, fused=0), dict(bm=64, bn=64, ksplit=4, fused=1),
                                  dict(bm=128, bn=128, ksplit=1, fused=0), dict(bm=128, bn=128, ksplit=2, fused=1),
                                  dict(bm=128, bn=128, ksplit=8, fused=1)])
@pytest.mark.parametrize("prec,tol", [(2, 4e-3), (3, 2e-4)])
def test_filter_every_bf16_plan(hd, orc, plan, prec, tol):
    """The BF16-split kernels under every plan the tuner may pick (64 x 64 tiles, the pipelined
    128 x 128 kernel for the two-term split, K split in the kernel) against the FP64 oracle filter;
    128 x 128 tiles are refused for the three-term split, whose planes do not fit the LDS."""
    from paper_1206_3768_amd import chfsi
    n, m = 520, 70
    if prec == 3 and plan["bm"] == 128:
        with pytest.raises(chfsi.ChfsiError):
            hd.set_filter_plan(n, m, prec, plan)
        return
    H, Y0, a, b, mu1 = _filter_case(n, m)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=6)
    hd.set_filter_plan(n, m, prec, plan)
    try:
        dY = dev(Y0)
        hd.filter(dev(H), dY, a, b, mu1, deg=6, prec=prec)
        used = hd.filter_launch_log()[-1]
    finally:
        hd.set_filter_plan(n, m, prec, None)
    assert relerr(host(dY), ref) <= tol
    # the tile as asked; the K split as asked up to the rounding of its slices to 32 rows of K
    assert used[3] == plan["bm"] and (used[5] > 1) == (plan["ksplit"] > 1) and used[5] <= plan["ksplit"]


@pytest.mark.parametrize("prec", [2, 3])
def test_autotune_filter_bf16_returns_a_valid_plan(hd, orc, prec):
    plan, ms = hd.autotune_filter(320, 48, prec)
    assert plan["bm"] == plan["bn"] and plan["bm"] in ((64, 128) if prec == 2 else (64,)) and ms > 0
    H, Y0, a, b, mu1 = _filter_case(320, 48)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=5)
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=5, prec=prec)
    hd.set_filter_plan(320, 48, prec, None)
    assert relerr(host(dY), ref) <= (4e-3 if prec == 2 else 2e-4)


def test_autotune_filter_returns_a_valid_plan(hd, orc):
    plan, ms = hd.autotune_filter(256, 40, 0)
    assert plan["bm"] in (32, 64) and plan["bn"] in (32, 64) and plan["ksplit"] >= 1 and ms > 0
    H, Y0, a, b, mu1 = _filter_case(256, 40)
    ref = orc.cheb_filter(H, Y0, a, b, mu1, deg=5)
    dY = dev(Y0)
    hd.filter(dev(H), dY, a, b, mu1, deg=5, prec=0)
    hd.set_filter_plan(256, 40, 0, None)
    assert relerr(host(dY), ref) <= 1e-12
