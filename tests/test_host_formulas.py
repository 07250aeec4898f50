"""CPU checks of closed-form shortcuts the GPU path takes (no GPU, no oracle): each is checked
against its exact counterpart from LAPACK (numpy / scipy)."""

import numpy as np
import scipy.linalg as sla


def _orthonormal(n, m, rng):
    g = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    q, _ = np.linalg.qr(g)
    return q


def test_first_order_cholesky_qr_pass_is_second_order_accurate():
    """Last Cholesky-QR pass in first-order form: for Q with Q^H Q = I + E (E small), R = I + F with
    F = strict upper triangle of E plus half its diagonal matches the exact Cholesky factor of
    Q^H Q to O(|E|^2), and Q (I - F) is orthonormal to O(|E|^2)."""
    rng = np.random.default_rng(7)
    n, m = 300, 40
    q0 = _orthonormal(n, m, rng)
    for delta in (1e-5, 1e-7, 1e-9):
        k = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        q = q0 @ (np.eye(m) + delta * k)
        g = q.conj().T @ q
        e = g - np.eye(m)
        ne = np.abs(e).sum(axis=1).max()
        f = np.triu(e, 1) + np.diag(0.5 * np.real(np.diag(e)))
        r_exact = sla.cholesky(g, lower=False)          # G = R^H R, R upper, real positive diagonal
        assert np.abs(r_exact - (np.eye(m) + f)).max() <= 4 * ne ** 2 + 1e-15
        q1 = q @ (np.eye(m) - f)
        orth = np.abs(q1.conj().T @ q1 - np.eye(m)).max()
        assert orth <= 8 * ne ** 2 + 1e-14, (delta, ne, orth)
    # at the size where the GPU takes the shortcut (max row sum of |E| <= 1e-9) the error is at the
    # level of rounding
    assert 8 * (1e-9) ** 2 < 1e-16


def test_first_order_factor_is_wrong_without_the_half_diagonal():
    """Guard against a plausible slip: taking the full diagonal of E in F doubles the first-order
    error on the diagonal, and the result is no longer orthonormal to second order."""
    rng = np.random.default_rng(8)
    n, m = 200, 20
    q = _orthonormal(n, m, rng) @ (np.eye(m) + 1e-6 * rng.standard_normal((m, m)))
    g = q.conj().T @ q
    e = g - np.eye(m)
    f_wrong = np.triu(e)
    q1 = q @ (np.eye(m) - f_wrong)
    assert np.abs(q1.conj().T @ q1 - np.eye(m)).max() > 1e-8
