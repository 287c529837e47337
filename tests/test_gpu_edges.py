"""Degenerate and limiting sizes of the single-box path through the C ABI,
against the oracle (arXiv:1203.6208, eq. DFmodified, cheb1-cheb3, sde):

  * one bead (its periodic images only: the self term, no real-space image
    within r_c = 0.58 L, and the reciprocal sum), a chain of one bead (no
    spring): D.v, one Euler step;
  * one bead tile exactly (N = 64) and one bead past it (N = 65: a second
    bead tile holding a single bead), D.v for 1..4 vectors on the vector
    units and 16 vectors on the matrix cores, and a step;
  * the smallest and the largest Chebyshev order (N_Ch = 2 and 512).

FP64 throughout, to rel 1e-12 (N_Ch = 512: 1e-11, 511 products of
rounding-level differences through a stable recurrence).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1203_6208_amd import inputs  # noqa: E402
from paper_1203_6208_amd import rpy  # noqa: E402

TOL = 1e-12
BASE = inputs.POSITION_SEED_BASE + 4400


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _single_bead():
    """One chain of one bead; the box of a two-bead chain at c/c* = 0.01
    (L = 6.5, so that 4a < L)."""
    w = inputs.Workload("one", 1, 2, 0.01, nch=20, seed=BASE)
    w.nchains, w.bpc, w.n = 1, 1, 1
    return w


def _workload(n):
    if n == 1:
        return _single_bead()
    nc, bpc = {64: (4, 16), 65: (5, 13)}[n]
    return inputs.Workload(f"edge{n}", nc, bpc, 1.0, nch=20, seed=BASE + n)


@pytest.mark.parametrize("n", [1, 64, 65])
def test_apply_and_step_at_edge_sizes(orc, n):
    _say(f"edge size N={n}")
    w = _workload(n)
    pos = w.positions()
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    lam = np.linalg.eigvalsh(D)
    lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
    ctx = rpy.context_for(w, max_rhs=16)
    ctx.build(_cuda(pos))
    for m in (1, 2, 3, 4, 16):
        v = np.random.default_rng(n + m).standard_normal((m, w.n, 3))
        out = ctx.apply(_cuda(v)).cpu().numpy().reshape(m, -1)
        assert _rel(out, orc.matvec(D, v.reshape(m, -1))) < TOL, m
    dw = w.noise(seed=BASE + 50 + n)[0]
    bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, d_min=lo, d_max=hi)
    tpos = _cuda(pos)
    drift, noise, ef = ctx.step(tpos, bp, dw=_cuda(dw), want=True)
    ref = orc.bd_step(pos, nchains=w.nchains, bpc=w.bpc, L=w.L, a=w.a, alpha=w.alpha, rc=w.rc,
                      n2max=w.n2max, dt=w.dt, nch=w.nch, dmin=lo, dmax=hi, dw=dw)
    if n == 1:   # no spring: the drift is zero
        assert float(drift.abs().max()) == 0.0
    else:
        assert _rel(drift.cpu().numpy(), ref["drift"]) < TOL
    assert _rel(noise.cpu().numpy(), ref["ds"]) < TOL
    assert _rel(tpos.cpu().numpy(), ref["pos"]) < TOL
    assert abs(float(ef.item()) ** 2 - ref["ef"] ** 2) < 1e-12
    assert ctx.status() == 0


@pytest.mark.parametrize("nch,tol", [(2, TOL), (512, 1e-11)])
def test_extreme_chebyshev_orders(orc, nch, tol):
    """N_Ch = 2 (one product: dS = c_0/2 dW + c_1 V_1) and N_Ch = 512 (the
    largest order the library accepts) at N = 65, three vectors."""
    _say(f"chebyshev order {nch}")
    w = _workload(65)
    pos = w.positions()
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    lam = np.linalg.eigvalsh(D)
    lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
    ctx = rpy.context_for(w, max_rhs=3)
    ctx.build(_cuda(pos))
    dw = w.noise(m=3, seed=BASE + 99)
    ds = ctx.sqrt_apply(_cuda(dw), nch, lo, hi).cpu().numpy().reshape(3, -1)
    ref = orc.cheb_sqrt(D, dw.reshape(3, -1), nch, lo, hi)
    assert _rel(ds, ref) < tol
    if nch == 512:   # converged: the dense square root itself
        lam_, Q = np.linalg.eigh(D)
        exact = (Q * np.sqrt(lam_)) @ Q.T @ dw.reshape(3, -1).T
        assert _rel(ds, exact.T) < 1e-10
