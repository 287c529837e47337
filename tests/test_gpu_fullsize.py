"""GPU parity at the full sizes of the benchmark and of the N = 1000
trajectory workload, against the dense CPU oracle (arXiv:1203.6208).

N = 4000 (80 chains x 50 beads, c/c* = 2, narrow-Gaussian excluded volume):
the dense oracle D (real-space images by brute force, the full +-k set with
direct cosines) is formed once per module.  Every launch configuration the
benchmark times is compared with it:
  * one whole FP64 bd_step -- springs + excluded volume, the folded product
    of [F, U+, dW] (the three-vector tile product with non-temporal loads),
    the paper's bound rule, N_Ch = 30 (28 one-vector products, non-temporal
    loads), E_f and the Euler update -- to rel 1e-12;
  * rpy_apply with 2, 3 and 4 vectors (the non-temporal tile products);
  * bd_step with the Chebyshev products in FP32 and in BF16, within the
    bound propagated from the rounding of the stored real-space part.
N = 1000 (40 chains x 25 beads, c/c* = 1, M = 4.6): five FP64 steps with
host noise, per-chain R_e^2 and R_g^2 (section "Testing and verification",
eq. Re2, Rg2) against the oracle trajectory, and alpha-independence of D at
these cutoffs.

Mixed-precision bound (the derivation of tests/test_gpu_block.py): only the
stored real-space part Drs is rounded, |E_ij| <= eps |Drs_ij| with eps =
2^-24 (FP32) or 2^-8 (BF16), the vector-unit product accumulates in FP64, so
||E||_2 <= eta = eps max_i sum_j |Drs_ij| (E is symmetric) and, with the
spectrum of D inside [d_min, d_max],
    ||d dS||_2 <= sum_p |c_p| 2 p (p + 1) eta ||dW||_2 / (d_max - d_min).
"""
import math
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
BOUNDS_C = 60.0   # the benchmark's constant of the paper's rule at N = 4000
EPS = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def n4000(orc):
    w = inputs.workload("n4000")
    pos = w.positions()
    _say("n4000: dense oracle D (about 20 s on 16 host threads)")
    Drs = orc.real_space_matrix(pos, w.L, w.a, w.alpha, w.rc)
    D = orc.recip_space_matrix(pos, w.L, w.a, w.alpha, w.n2max)
    D += Drs
    F = orc.spring_forces(pos, w.nchains, w.bpc) + orc.ev_forces(
        pos, w.L, w.ev["zstar"], w.ev["dstar"], w.ev["rcut"])
    return w, pos, D, Drs, F


def _oracle_step(orc, w, pos, D, F, dw, nch, dmin, dmax):
    """The oracle's Euler step on a given dense D (the order of oracle.bd_step,
    which would rebuild D)."""
    n = w.n
    ud = orc.matvec(D, F.reshape(1, -1)).reshape(n, 3)
    ds = orc.cheb_sqrt(D, dw.reshape(1, -1), nch, dmin, dmax).reshape(n, 3)
    ef = orc.sqrt_error(D, dw, ds)
    return ud, ds, ef, orc.euler(pos, w.dt, ud, ds)


def test_bd_step_n4000_f64_end_to_end(n4000, orc):
    """One whole FP64 step of the benchmark workload against the oracle."""
    _say("bd_step n4000 f64")
    w, pos, D, _, F = n4000
    dw = w.noise()[0]
    ctx = rpy.context_for(w)
    tpos = _cuda(pos)
    bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, bounds_rule=rpy.BOUNDS_PAPER,
                            bounds_C=BOUNDS_C, ev=w.ev)
    drift, noise, ef = ctx.step(tpos, bp, dw=_cuda(dw), want=True)
    lo, hi = orc.bounds_rule(D, w.n, BOUNDS_C)
    ud, ds, ef_ref, new = _oracle_step(orc, w, pos, D, F, dw, w.nch, lo, hi)
    assert _rel(drift.cpu().numpy(), ud) < TOL
    assert _rel(noise.cpu().numpy(), ds) < TOL
    assert _rel(tpos.cpu().numpy() - pos, new - pos) < TOL
    assert _rel(tpos.cpu().numpy(), new) < TOL
    assert abs(ef.item() ** 2 - ef_ref ** 2) < 1e-12
    assert ctx.status() == 0
    _say(f"  E_f {ef.item():.4f} on [{lo:.4f}, {hi:.2f}]")


@pytest.mark.parametrize("m", [2, 3, 4])
def test_apply_n4000_multi_vector(n4000, orc, m):
    """Products of 2-4 vectors stream the 384 MB of tiles with non-temporal
    loads in stored order: every output element against the dense oracle."""
    _say(f"apply n4000 m={m}")
    w, pos, D, _, _ = n4000
    ctx = rpy.context_for(w, max_rhs=4)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(40 + m).standard_normal((m, w.n, 3))
    out = ctx.apply(_cuda(v)).cpu().numpy().reshape(m, -1)
    ref = orc.matvec(D, v.reshape(m, -1))
    assert _rel(out, ref) < TOL


def test_apply_n4000_block_f64(n4000, orc):
    """Sixteen vectors at once on the FP64 matrix cores (the packed planes as
    16x16x4 FP64 operands, FP64 partials per tile column): every output
    element against the dense oracle."""
    _say("apply n4000 block f64 m=16")
    w, pos, D, _, _ = n4000
    ctx = rpy.context_for(w, max_rhs=16)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(4016).standard_normal((16, w.n, 3))
    out = ctx.apply(_cuda(v)).cpu().numpy().reshape(16, -1)
    ref = orc.matvec(D, v.reshape(16, -1))
    assert _rel(out, ref) < TOL


def _prop_bound(orc, Drs, eps, nch, lo, hi, dw):
    c = orc.cheb_coeffs(nch, lo, hi)
    eta = eps * np.max(np.abs(Drs).sum(axis=1))
    amp = sum(abs(c[p]) * 2 * p * (p + 1) for p in range(1, nch)) / (hi - lo)
    return amp * eta * np.linalg.norm(dw)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_bd_step_n4000_low_precision(n4000, orc, prec):
    """bd_step with FP32 or BF16 Chebyshev products (FP64 drift, bounds,
    reciprocal sums and recurrence) against the oracle's FP64 step: the drift
    to 1e-12, dS and the displacement within the propagated bound.  The
    interval of the paper's rule at C = 60 contains the spectrum of this D
    (lambda in [0.0298, 47.3] against [0.0275, 239]), which the bound needs."""
    _say(f"bd_step n4000 {prec}")
    w, pos, D, Drs, F = n4000
    dw = w.noise()[0]
    ctx = rpy.context_for(w, lowp=prec)
    tpos = _cuda(pos)
    bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, bounds_rule=rpy.BOUNDS_PAPER,
                            bounds_C=BOUNDS_C, prec=prec, ev=w.ev)
    drift, noise, _ = ctx.step(tpos, bp, dw=_cuda(dw), want=True)
    lo, hi = orc.bounds_rule(D, w.n, BOUNDS_C)
    ud, ds, _, new = _oracle_step(orc, w, pos, D, F, dw, w.nch, lo, hi)
    assert _rel(drift.cpu().numpy(), ud) < TOL
    bound = _prop_bound(orc, Drs, EPS[prec], w.nch, lo, hi, dw)
    err = float(np.linalg.norm(noise.cpu().numpy() - ds))
    _say(f"  ||d dS|| {err:.3e} (bound {bound:.3e}), rel {err / np.linalg.norm(ds):.3e}")
    assert err <= bound
    disp_err = float(np.linalg.norm(tpos.cpu().numpy() - new))
    assert disp_err <= bound / math.sqrt(2) + 1e-12 * np.linalg.norm(new)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_bd_step_n100_low_precision(orc, prec):
    """The same comparison at N = 100 (two bead tiles, a ragged tail) on an
    interval around the exact spectrum, three steps with host noise."""
    _say(f"bd_step n100 {prec}")
    w = inputs.workload("n100")
    ctx = rpy.context_for(w, lowp=prec)
    tpos = _cuda(w.positions())
    for step in range(3):
        # each step is compared on its own: the oracle steps from the GPU's
        # positions
        gpos0 = tpos.cpu().numpy()
        D = orc.diffusion_matrix(gpos0, w.L, w.a, w.alpha, w.rc, w.n2max)
        Drs = orc.real_space_matrix(gpos0, w.L, w.a, w.alpha, w.rc)
        lam = np.linalg.eigvalsh(D)
        lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
        bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, d_min=lo, d_max=hi, prec=prec)
        dw = w.noise(seed=7000 + step)[0]
        drift, noise, _ = ctx.step(tpos, bp, dw=_cuda(dw), want=True)
        F = orc.spring_forces(gpos0, w.nchains, w.bpc)
        ud, ds, _, new = _oracle_step(orc, w, gpos0, D, F, dw, w.nch, lo, hi)
        assert _rel(drift.cpu().numpy(), ud) < TOL
        bound = _prop_bound(orc, Drs, EPS[prec], w.nch, lo, hi, dw)
        err = float(np.linalg.norm(noise.cpu().numpy() - ds))
        assert err <= bound, (step, err, bound)
        assert float(np.linalg.norm(tpos.cpu().numpy() - new)) <= bound / math.sqrt(2) + 1e-12


def test_trajectory_n1000_observables(orc):
    """N = 1000 workload: five FP64 steps (paper's rule, C = 40, which
    brackets this D's spectrum [0.037, 20.3]; N_Ch = 30; host noise).  After
    every step the per-chain R_e^2 and R_g^2 of the GPU trajectory, its
    positions, drift and dS equal the oracle trajectory's to rel 1e-12."""
    w = inputs.workload("n1000")
    pos = w.positions()
    ctx = rpy.context_for(w)
    tpos = _cuda(pos)
    bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, bounds_rule=rpy.BOUNDS_PAPER, bounds_C=40.0)
    okw = dict(nchains=w.nchains, bpc=w.bpc, L=w.L, a=w.a, alpha=w.alpha, rc=w.rc,
               n2max=w.n2max, dt=w.dt, nch=w.nch, bounds_C=40.0)
    for step in range(5):
        _say(f"trajectory n1000 step {step}")
        dw = w.noise(seed=9000 + step)[0]
        drift, noise, _ = ctx.step(tpos, bp, dw=_cuda(dw), want=True)
        ref = orc.bd_step(pos, dw=dw, **okw)
        assert _rel(drift.cpu().numpy(), ref["drift"]) < TOL
        assert _rel(noise.cpu().numpy(), ref["ds"]) < TOL
        assert _rel(tpos.cpu().numpy(), ref["pos"]) < TOL
        pos = ref["pos"]
        re2, rg2 = ctx.observables(tpos)
        o_re2, o_rg2 = orc.chain_observables(pos, w.nchains, w.bpc)
        assert _rel(re2.cpu().numpy(), o_re2) < TOL
        assert _rel(rg2.cpu().numpy(), o_rg2) < TOL
    assert ctx.status() == 0


def test_alpha_independence_n1000():
    """At M = alpha r_c = 4.6 both Ewald truncations are below 1e-6 (the factor
    of eq. M2 at k = K is 5.9e-7, erfc(M) 8e-11), so D.v does not depend on
    how the sum is split: alpha L = 6 (the workload) against alpha L = 7.5 at
    the same M."""
    w = inputs.workload("n1000")
    w2 = inputs.Workload("n1000_aL7.5", w.nchains, w.bpc, w.c_over_cstar, alphaL=7.5, M=w.M,
                         nch=w.nch, seed=w.seed)
    pos = _cuda(w.positions())
    v = _cuda(np.random.default_rng(12).standard_normal((1, w.n, 3)))
    ys = []
    for wl in (w, w2):
        ctx = rpy.context_for(wl)
        ctx.build(pos)
        ys.append(ctx.apply(v).cpu().numpy())
    d = _rel(ys[1], ys[0])
    _say(f"alpha-independence at M = {w.M}: {d:.2e}")
    assert d < 1e-6
