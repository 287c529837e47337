"""Pins of the oracle's reverse mode of u = D(R) F + p(D(R)) dW (the
differentiation form; pair-term derivatives of eq. M1, b1/b2, cor5 and the
cosine of eq. M2, adjoint of the recurrence eq. cheb1-cheb3 on a fixed
interval).  The analytic gradient is checked against central finite
differences of the oracle's own forward u (no shared formula), on every
coordinate of a small box that has overlapping pairs, self-images and
images beyond the first shell, and along random directions at N = 100."""
import numpy as np
import pytest

from paper_1203_6208_amd import inputs


def _setup(w, seed, close_pair=None):
    rng = np.random.default_rng(seed)
    pos = w.positions()
    if close_pair is not None:
        i, j, dist = close_pair
        u = rng.standard_normal(3)
        pos[j] = pos[i] + dist * u / np.linalg.norm(u)
    n = w.n
    F = rng.standard_normal((n, 3))
    dw = rng.standard_normal((n, 3)) * 0.03
    g = rng.standard_normal((n, 3))
    return pos, F, dw, g


def _interval(orc, w, pos):
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    lam = np.linalg.eigvalsh(D)
    return D, 0.9 * lam[0], 1.1 * lam[-1]


def _L(orc, w, pos, F, dw, g, nch, lo, hi):
    u = orc.u_forward(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, nch, lo, hi)
    return float(np.sum(g * u))


def test_gradient_matches_central_differences_every_coordinate(orc):
    """N = 20 (2 chains x 10 beads): beads 3 and 14 at 0.4 a (overlap form,
    series region), beads 5 and 6 at 1.2 a; 12 Chebyshev terms.  Central
    differences with h = 1e-6 on all 60 coordinates agree to 1e-7 of the
    largest gradient component."""
    w = inputs.Workload("g20", 2, 10, 1.0, nch=12, seed=inputs.POSITION_SEED_BASE + 301)
    pos, F, dw, g = _setup(w, 1, close_pair=(3, 14, 0.2))
    pos[6] = pos[5] + np.array([0.6, 0.0, 0.0])
    _, lo, hi = _interval(orc, w, pos)
    gpos, gF = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, 12, lo, hi)
    h = 1e-6
    fd = np.zeros_like(pos)
    for b in range(w.n):
        for i in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[b, i] += h
            p2[b, i] -= h
            fd[b, i] = (_L(orc, w, p1, F, dw, g, 12, lo, hi)
                        - _L(orc, w, p2, F, dw, g, 12, lo, hi)) / (2 * h)
    scale = np.max(np.abs(gpos))
    assert scale > 0
    assert np.max(np.abs(gpos - fd)) < 1e-7 * scale


def test_gradient_wrt_forces_is_D_g(orc):
    w = inputs.Workload("g20", 2, 10, 1.0, nch=8, seed=inputs.POSITION_SEED_BASE + 302)
    pos, F, dw, g = _setup(w, 2)
    D, lo, hi = _interval(orc, w, pos)
    _, gF = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, 8, lo, hi, rows=[0])
    assert np.max(np.abs(gF.reshape(-1) - D @ g.reshape(-1))) < 1e-13 * np.max(np.abs(gF))
    # u is linear in F: the directional derivative along F is exact
    e = np.random.default_rng(3).standard_normal(F.shape)
    l0 = _L(orc, w, pos, F, dw, g, 8, lo, hi)
    l1 = _L(orc, w, pos, F + e, dw, g, 8, lo, hi)
    assert abs((l1 - l0) - np.sum(gF * e)) < 1e-11 * abs(l1 - l0)


def test_gradient_is_translation_invariant(orc):
    """L(R + t) = L(R): the bead gradients sum to zero, and a rigid
    translation by a box vector leaves them unchanged."""
    w = inputs.Workload("g20", 2, 10, 1.0, nch=10, seed=inputs.POSITION_SEED_BASE + 303)
    pos, F, dw, g = _setup(w, 4, close_pair=(1, 12, 0.5))
    _, lo, hi = _interval(orc, w, pos)
    g1, _ = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, 10, lo, hi)
    assert np.max(np.abs(g1.sum(axis=0))) < 1e-11 * np.max(np.abs(g1))
    g2, _ = orc.u_vjp(pos + np.array([w.L, -2 * w.L, 0.0]), w.L, w.a, w.alpha, w.rc, w.n2max,
                      F, dw, g, 10, lo, hi)
    assert np.max(np.abs(g1 - g2)) < 1e-10 * np.max(np.abs(g1))


def test_gradient_directional_n100(orc):
    """N = 100 workload, 20 Chebyshev terms: five random directions, central
    differences (h = 1e-6) against the gradient to 1e-7; the rows variant
    equals the full gradient on a subset of beads."""
    w = inputs.workload("n100")
    pos, F, dw, g = _setup(w, 5)
    _, lo, hi = _interval(orc, w, pos)
    gpos, _ = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, 20, lo, hi)
    rng = np.random.default_rng(6)
    h = 1e-6
    for _ in range(5):
        e = rng.standard_normal(pos.shape)
        fd = (_L(orc, w, pos + h * e, F, dw, g, 20, lo, hi)
              - _L(orc, w, pos - h * e, F, dw, g, 20, lo, hi)) / (2 * h)
        an = float(np.sum(gpos * e))
        assert abs(fd - an) < 1e-7 * np.sum(np.abs(gpos * e))
    rows = [0, 17, 55, 99]
    gr, _ = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, 20, lo, hi, rows=rows)
    assert np.max(np.abs(gr - gpos[rows])) == 0.0
