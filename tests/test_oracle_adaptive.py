"""CPU pins of the oracle's Lanczos bounds and adaptive Chebyshev order
(arXiv:1203.6208, section "Decomposition of the diffusion tensor": the
interval must contain the spectrum of D; N_Ch from eq. nint, then increased
until E_f < tol)."""
import math

import numpy as np
import pytest

from paper_1203_6208_amd import inputs


@pytest.fixture(scope="module")
def d100(orc):
    w = inputs.workload("n100")
    pos = w.positions()
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    return w, D, np.linalg.eigvalsh(D)


def test_lanczos_reproduces_a_diagonal_spectrum(orc):
    """Krylov space of a diagonal matrix with distinct entries from a start
    vector with every component nonzero: after dim steps the Ritz values are
    the entries (a dropped or misplaced term of the recurrence breaks it)."""
    d = np.array([0.3, 1.7, 2.2, 0.05, 4.0, 3.1, 0.9, 2.9, 1.1, 0.6])
    a, b = orc.lanczos(np.diag(d), np.ones(len(d)) + 0.1 * np.arange(len(d)), len(d))
    _, _, th = orc.lanczos_bounds(a, b, 0.0)
    assert np.allclose(np.sort(th), np.sort(d), rtol=0, atol=1e-12)
    assert abs(b[-1]) < 1e-10   # the Krylov space is exhausted


def test_lanczos_bounds_bracket_the_spectrum(orc, d100):
    w, D, lam = d100
    st = np.random.default_rng(3).standard_normal(D.shape[0])
    for k in (20, 40):
        a, b = orc.lanczos(D, st, k)
        lo, hi, th = orc.lanczos_bounds(a, b, 0.0)
        assert lo <= lam[0] and hi >= lam[-1]
        assert lam[0] - 1e-12 <= th[0] and th[-1] <= lam[-1] + 1e-12   # Ritz values interlace
    assert abs(th[-1] - lam[-1]) < 1e-10 * lam[-1]                  # lambda_max converged at k = 40


def test_adaptive_order_is_minimal(orc, d100):
    w, D, lam = d100
    lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
    dw = w.noise(m=2).reshape(2, -1)
    tol = 1e-4
    n, ds = orc.cheb_adaptive(D, dw, lo, hi, tol, 200)
    start = math.floor(math.sqrt(hi / lo) + 0.5) + 1
    assert n > start
    ef = [orc.sqrt_error(D, dw[j], ds[j]) for j in range(2)]
    assert max(ef) < tol
    prev = orc.cheb_sqrt(D, dw, n - 1, lo, hi)
    assert max(orc.sqrt_error(D, dw[j], prev[j]) for j in range(2)) >= tol
    assert np.allclose(ds, orc.cheb_sqrt(D, dw, n, lo, hi), rtol=0, atol=0)


def test_adaptive_order_starts_at_the_nint_rule(orc, d100):
    """With a tolerance every order meets, N_Ch = nint(sqrt(dmax/dmin)) + 1,
    nint rounding half away from zero (eq. nint)."""
    w, D, lam = d100
    dw = w.noise(m=1).reshape(1, -1)
    for lo, hi in ((0.05, 6.0), (0.07, 5.5), (0.25, 6.25)):
        n, _ = orc.cheb_adaptive(D, dw, lo, hi, 10.0, 500)
        assert n == math.floor(math.sqrt(hi / lo) + 0.5) + 1
    # exact half-way case: hi/lo = 42.25, sqrt = 6.5 -> nint 7 -> N_Ch 8
    n, _ = orc.cheb_adaptive(D, dw, 0.25, 10.5625, 10.0, 500)
    assert n == 8
