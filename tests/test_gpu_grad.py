"""GPU parity of the differentiation form: the reverse mode of
u = D(R) F + p(D(R)) dW (rpy_u_vjp) and of the forces (rpy_forces_vjp)
through the C ABI, against the oracle's reverse mode (itself pinned by
central differences), against central differences of the GPU forward, and
through torch.autograd over checkpointed trajectories.

Tolerances: u to 1e-12 (as every FP64 product).  The gradient is a sum over
pairs, images and wave vectors of terms of both signs, each carrying a
relative rounding error near 1e-15 of its own size; it is compared norm-wise
to 1e-10 of its largest component.  Central differences with h = 1e-6 carry
a rounding error near 1e-10 relative to the sum of the directional
derivative's terms (measured: 3e-11 to 1e-10 at N = 2000); they are compared
to 1e-8 for the u term and to 1e-6 for the forces and for trajectories.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1203_6208_amd import diff, inputs  # noqa: E402
from paper_1203_6208_amd import rpy  # noqa: E402

GTOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _case(orc, w, seed, nch, close=None):
    rng = np.random.default_rng(seed)
    pos = w.positions()
    if close is not None:
        i, j, dist = close
        u = rng.standard_normal(3)
        pos[j] = pos[i] + dist * u / np.linalg.norm(u)
    F = rng.standard_normal((w.n, 3))
    dw = rng.standard_normal((w.n, 3)) * 0.03
    g = rng.standard_normal((w.n, 3))
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    lam = np.linalg.eigvalsh(D)
    return pos, F, dw, g, 0.9 * lam[0], 1.1 * lam[-1]


@pytest.mark.parametrize("name,close", [("n100", None), ("g150", (7, 120, 0.15))])
def test_u_and_vjp_match_oracle(orc, name, close):
    """u and (dL/dR, dL/dF) for L = g.u: N = 100 (two tiles) and N = 150
    (three tiles, ragged tail, a pair at 0.3 a: overlap form in its series
    region), 20 Chebyshev terms, V_p kept by the forward or recomputed."""
    _say(f"grad {name}")
    w = inputs.workload("n100") if name == "n100" else \
        inputs.Workload("g150", 10, 15, 1.5, nch=20, seed=inputs.POSITION_SEED_BASE + 311)
    nch = 20
    pos, F, dw, g, lo, hi = _case(orc, w, 7, nch, close)
    rc = rpy.context_for(w, max_rhs=16, cheb_keep=nch, grad=1)
    u = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    vh = torch.empty((nch, w.n, 3), dtype=torch.float64, device="cuda")
    tp, tF, tdw, tg = _cuda(pos), _cuda(F), _cuda(dw), _cuda(g)
    rpy.rpy_u_forward(rc.handle, tp, tF, tdw, nch, lo, hi, u, vh)
    want_u = orc.u_forward(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, nch, lo, hi)
    assert _rel(u.cpu().numpy(), want_u) < 1e-12
    gp_o, gF_o = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, nch, lo, hi)
    for keep in (vh, None):
        gp = torch.empty_like(tp)
        gF = torch.empty_like(tp)
        rpy.rpy_u_vjp(rc.handle, tp, tF, tdw, tg, nch, lo, hi, gp, gF, keep)
        e_p = _rel(gp.cpu().numpy(), gp_o)
        e_F = _rel(gF.cpu().numpy(), gF_o)
        _say(f"  keep={keep is not None} rel err dL/dR {e_p:.2e} dL/dF {e_F:.2e}")
        assert e_F < 1e-12
        assert e_p < GTOL
    rc.close()


def _crosses_cutoff(pos, e, h, moved, L, rc):
    """Whether some periodic image of a pair with a moved bead crosses
    |r| = r_c between pos - h e and pos + h e (the truncated real-space sum
    jumps there by the size of M1(r_c), about 1e-5, which would enter a
    difference quotient as 1e-5 / (2 h))."""
    n = np.arange(-1, 2)
    img = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3) * L
    d0 = pos[moved][:, None, :] - pos[None, :, :]           # [moved, N, 3]
    shift = L * np.round(d0 / L)     # nearest image at pos, kept for both signs
    inside = []
    for sgn in (1.0, -1.0):
        p = pos + sgn * h * e
        d = p[moved][:, None, :] - p[None, :, :] - shift     # |d_i| <= L/2 + O(h)
        r2 = np.zeros(d.shape[:2] + (len(img),))
        for c in range(3):
            r2 += (d[:, :, None, c] + img[None, None, :, c]) ** 2
        inside.append(r2 <= rc * rc)
    return bool(np.any(inside[0] != inside[1]))


def test_vjp_central_differences_n2000(orc):
    """The differentiation workload (N = 2000, 40 chains x 50 beads), N_Ch =
    30: 20 random directions, each moving 100 random beads, central
    differences of the GPU forward with h = 1e-6 against the adjoint's
    directional derivative; directions along which an image crosses the
    real-space cutoff are redrawn (the truncated sum is discontinuous there;
    a direction moving all 2000 beads crosses about 1.5 images per
    difference).  Then the adjoint against the oracle's reverse mode on 6
    sampled beads (the oracle builds the dense 6000 x 6000 D)."""
    _say("grad n2000")
    w = inputs.workload("n2000")
    nch = 30
    rng = np.random.default_rng(21)
    pos = w.positions()
    F = rng.standard_normal((w.n, 3))
    dw = rng.standard_normal((w.n, 3)) * np.sqrt(w.dt)
    g = rng.standard_normal((w.n, 3))
    rc = rpy.context_for(w, max_rhs=16, cheb_keep=nch, grad=1)
    rc.build(_cuda(pos))
    lo, hi, _, _ = rc.lanczos_bounds(60, seed=1, margin=0.05)
    tp, tF, tdw, tg = _cuda(pos), _cuda(F), _cuda(dw), _cuda(g)
    gp = torch.empty_like(tp)
    rpy.rpy_u_vjp(rc.handle, tp, tF, tdw, tg, nch, lo, hi, gp, None, None)
    gpn = gp.cpu().numpy()
    u = torch.empty_like(tp)
    h = 1e-6
    errs = []
    redrawn = 0
    while len(errs) < 20:
        moved = np.sort(rng.choice(w.n, size=100, replace=False))
        e = np.zeros(pos.shape)
        e[moved] = rng.standard_normal((100, 3))
        if _crosses_cutoff(pos, e, h, moved, w.L, w.rc):
            redrawn += 1
            assert redrawn < 20
            continue
        rpy.rpy_u_forward(rc.handle, _cuda(pos + h * e), tF, tdw, nch, lo, hi, u)
        lp = float(torch.sum(tg * u))
        rpy.rpy_u_forward(rc.handle, _cuda(pos - h * e), tF, tdw, nch, lo, hi, u)
        lm = float(torch.sum(tg * u))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(gpn * e))
        errs.append(abs(fd - an) / np.sum(np.abs(gpn * e)))
    _say(f"  max FD rel err {max(errs):.2e} ({redrawn} directions redrawn)")
    assert max(errs) < 1e-8
    rows = [0, 1, 777, 1024, 1500, 1999]
    gr, _ = orc.u_vjp(pos, w.L, w.a, w.alpha, w.rc, w.n2max, F, dw, g, nch, lo, hi, rows=rows)
    e_o = float(np.max(np.abs(gpn[rows] - gr)) / np.max(np.abs(gpn)))
    _say(f"  sampled oracle rel err {e_o:.2e}")
    assert e_o < GTOL
    rc.close()


@pytest.mark.parametrize("name", ["n100", "n2000"])
def test_forces_vjp_central_differences(orc, name):
    """(dF/dR)^T gF for springs + narrow-Gaussian excluded volume (N = 100:
    all-pairs kernel; N = 2000: cell list) against central differences of the
    oracle's forces along 5 random directions."""
    _say(f"forces vjp {name}")
    w = inputs.workload(name)
    ev = dict(inputs.NG_EV)
    if name == "n100":
        ev["rcut"] = 3.5   # below L/2 = 3.86: minimum image holds
    rng = np.random.default_rng(31)
    pos = w.positions()
    gF = rng.standard_normal((w.n, 3))
    rc = rpy.context_for(w)
    out = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    rpy.rpy_forces_vjp(rc.handle, _cuda(pos), ev["zstar"], ev["dstar"], ev["rcut"], _cuda(gF), out)
    gp = out.cpu().numpy()

    def Ftot(p):
        return orc.spring_forces(p, w.nchains, w.bpc) + orc.ev_forces(
            p, w.L, ev["zstar"], ev["dstar"], ev["rcut"])

    h = 1e-6
    for _ in range(5):
        e = rng.standard_normal(pos.shape)
        fd = float(np.sum(gF * (Ftot(pos + h * e) - Ftot(pos - h * e)))) / (2 * h)
        an = float(np.sum(gp * e))
        assert abs(fd - an) < 1e-6 * np.sum(np.abs(gp * e))
    rc.close()


def test_trajectory_gradient_checkpointed():
    """MSD after 6 steps of the N = 100 workload with excluded volume: the
    gradient with respect to the initial positions and to a spring-stiffness
    factor is the same with checkpoints every 2 steps and without
    checkpointing (bit for bit), and matches central differences of the
    trajectory (GPU forward) along 3 directions and in the stiffness."""
    _say("trajectory")
    w = inputs.workload("n100")
    ev = dict(inputs.NG_EV)
    ev["rcut"] = 3.5
    nch = 20
    rc = rpy.context_for(w, max_rhs=16, cheb_keep=nch, grad=1)
    pos0 = _cuda(w.positions())
    rc.build(pos0)
    lo, hi, _, _ = rc.lanczos_bounds(40, seed=2, margin=0.1)
    dt = 1e-3

    def run(p0, k, every):
        return diff.trajectory(p0, rc, 6, dt, nch, lo, hi, seed=5, ev=ev, spring=k, every=every)

    grads = []
    for every in (2, 0):
        p0 = pos0.clone().requires_grad_(True)
        k = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        m = diff.msd(run(p0, k, every), p0)
        m.backward()
        grads.append((p0.grad.clone(), k.grad.clone(), float(m)))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    gp, gk, _ = grads[0]
    rng = np.random.default_rng(41)
    h = 1e-6
    with torch.no_grad():
        one = torch.tensor(1.0, dtype=torch.float64, device="cuda")
        for _ in range(3):
            e = _cuda(rng.standard_normal((w.n, 3)))
            fp = float(diff.msd(run(pos0 + h * e, one, 0), pos0 + h * e))
            fm = float(diff.msd(run(pos0 - h * e, one, 0), pos0 - h * e))
            fd = (fp - fm) / (2 * h)
            an = float(torch.sum(gp * e))
            assert abs(fd - an) < 1e-6 * float(torch.sum(torch.abs(gp * e))), (fd, an)
        fp = float(diff.msd(run(pos0, one + h, 0), pos0))
        fm = float(diff.msd(run(pos0, one - h, 0), pos0))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - float(gk)) < 1e-6 * max(abs(fd), 1e-12), (fd, float(gk))
    rc.close()


def test_vjp_needs_grad_context():
    w = inputs.workload("n100")
    rc = rpy.context_for(w, cheb_keep=20)
    t = _cuda(w.positions())
    with pytest.raises(rpy.RpyError):
        rpy.rpy_u_vjp(rc.handle, t, t, t, t, 20, 0.1, 2.0, torch.empty_like(t))
    rc.close()


def test_u_entry_points_reject_invalid():
    """Interval, order and n_cheb > cheb_keep are refused before any launch."""
    w = inputs.workload("n100")
    rc = rpy.context_for(w, max_rhs=16, cheb_keep=10, grad=1)
    t = _cuda(w.positions())
    u = torch.empty_like(t)
    for nch, lo, hi in ((1, 0.1, 2.0), (10, 0.0, 2.0), (10, 2.0, 1.0), (10, 0.1, float("inf"))):
        with pytest.raises(rpy.RpyError):
            rpy.rpy_u_forward(rc.handle, t, t, t, nch, lo, hi, u)
    with pytest.raises(rpy.RpyError):   # more terms than kept vectors
        rpy.rpy_u_vjp(rc.handle, t, t, t, t, 11, 0.1, 2.0, torch.empty_like(t))
    with pytest.raises(rpy.RpyError):   # excluded volume with rcut >= L/2
        rpy.rpy_forces_vjp(rc.handle, t, 1.0, 0.5, 0.6 * w.L, t, torch.empty_like(t))
    rc.close()
