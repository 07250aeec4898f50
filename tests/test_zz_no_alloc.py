"""The allocation-free filter (chfsi_filter_noalloc) against chfsi_filter, the entry point it is a
variant of, and the CPU oracle: FP64, one degree for every column, through the C ABI.

Two calls in a row share the library's fixed scratch; the second one is smaller, so a result that
depended on what the first call left there would show.  Tolerance: the FP64 filter's
1e-12 * max|reference| (rounding of degree-d products of norm-1 operators, plus a margin for the
split-K plans, which may differ between the two entry points)."""
import ctypes as C
import math

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


@pytest.fixture(scope="module")
def hd(torch_dev):
    from paper_1206_3768_amd import chfsi
    h = chfsi.Handle(0)
    yield h
    h.close()


def _case(n, m, seed):
    rng = np.random.default_rng(seed)
    spec = synth.SequenceSpec(n=n, n_low=max(1, n // 8), generalized=False, cycles=1, eps0=0, eps_decay=1, seed=seed)
    p = synth.designed_pencil(spec, keep_vectors=False)
    Y0 = np.asfortranarray((rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))) / math.sqrt(2))
    return p.A, Y0


def _relerr(x, ref):
    return np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300)


def test_noalloc_filter_matches_filter_and_oracle_on_two_calls(hd, orc):
    from paper_1206_3768_amd import chfsi
    a, b, mu1 = -0.45, 1.05, -1.0
    # (n, m, degree): a split-K plan with several tiles and an odd degree (final copy from the
    # second block), then a smaller ragged case with an even degree
    for n, m, d, seed in [(1100, 150, 11, 5), (300, 37, 10, 6)]:
        print(f"noalloc filter n={n} m={m} degree {d}", flush=True)
        A, Y0 = _case(n, m, seed)
        dA = chfsi.to_device(A)
        Y1 = chfsi.to_device(Y0)
        Y2 = chfsi.to_device(Y0)
        chfsi.filter_noalloc(dA, Y1, a, b, mu1, deg=d)
        hd.filter(dA, Y2, a, b, mu1, deg=d, prec=chfsi.FP64)
        got, base = chfsi.to_numpy(Y1), chfsi.to_numpy(Y2)
        assert _relerr(got, base) <= 1e-12
        ref = orc.cheb_filter(A, Y0, a, b, mu1, deg=d)
        assert _relerr(got, ref) <= 1e-12


def test_noalloc_filter_full_size_n2048(hd):
    """The n = 2048 sequence's block (m = 192, degree 12): same result as chfsi_filter."""
    from paper_1206_3768_amd import chfsi
    A, Y0 = _case(2048, 192, 9)
    dA = chfsi.to_device(A)
    Y1, Y2 = chfsi.to_device(Y0), chfsi.to_device(Y0)
    chfsi.filter_noalloc(dA, Y1, -0.45, 1.05, -1.0, deg=12)
    hd.filter(dA, Y2, -0.45, 1.05, -1.0, deg=12, prec=chfsi.FP64)
    assert _relerr(chfsi.to_numpy(Y1), chfsi.to_numpy(Y2)) <= 1e-12


def test_noalloc_filter_rejects_what_does_not_fit(torch_dev):
    """Sizes beyond the fixed scratch and invalid arguments are refused on the host before anything
    is enqueued (the small tensors are never touched)."""
    from paper_1206_3768_amd import chfsi
    lib = chfsi.load()
    H = torch_dev.zeros((4, 4), dtype=torch_dev.complex128, device="cuda")
    Y = torch_dev.zeros((4, 4), dtype=torch_dev.complex128, device="cuda")
    s = C.c_void_p(torch_dev.cuda.current_stream().cuda_stream)
    n, m = 8192, chfsi.NOALLOC_SCRATCH_BYTES // (16 * 8192) + 1
    assert lib.chfsi_filter_noalloc(s, n, H.data_ptr(), n, Y.data_ptr(), n, m, 4, -0.5, 1.0, -1.0) == chfsi.ERR_TOO_LARGE
    assert lib.chfsi_filter_noalloc(s, 4, H.data_ptr(), 4, Y.data_ptr(), 4, 4, 4, 0.5, 0.2, -1.0) == chfsi.ERR_ARG
    assert lib.chfsi_filter_noalloc(s, 4, H.data_ptr(), 3, Y.data_ptr(), 4, 4, 4, -0.5, 1.0, -1.0) == chfsi.ERR_ARG
    assert lib.chfsi_filter_noalloc(s, 4, H.data_ptr(), 4, Y.data_ptr(), 4, 0, 4, -0.5, 1.0, -1.0) == chfsi.SUCCESS
    assert lib.chfsi_status_string(chfsi.ERR_TOO_LARGE).startswith(b"input exceeds")
