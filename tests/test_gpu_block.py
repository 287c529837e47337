"""GPU parity of the matrix-core block product (5..16 vectors at once on the
packed planes of the stored real-space tiles: FP64 tiles with FP64
accumulation, FP32 or BF16 tiles with FP32 accumulation inside a tile)
through the C ABI against the CPU oracle (arXiv:1203.6208, eq. DFmodified;
the product is the one every Chebyshev term of eq. cheb1-cheb3 takes).

Bounds are elementwise and worst-case, from the rounding of what is stored:
only the real-space part (self term, M1 images, M*) is held in low precision,
so with Drs that part and v the vectors,

    |y_i - (D v)_i| <= eps * sum_j |Drs_ij| |v_j|

  FP32: eps = 2^-24 (tile entry) + 2^-24 (vector entry) + 400 * 2^-24 (FP32
        accumulation over the 192 products of a tile row, with margin);
  BF16: eps = 2^-8 (tile entry: 8-bit significand, round to nearest)
        + 2^-15 (the vector enters as a hi + lo BF16 pair, error <= 2^-16 |v|,
        plus the FP32 conversion) + 800 * 2^-24 (FP32 accumulation over the
        384 hi and lo products).
The reciprocal sum and the sum over tiles are FP64 and add nothing at this
scale.  The same kernel is also compared with the vector-unit path of the
same precision (1..4 vectors): both read the same stored tiles, so they
differ only by the vector rounding and the FP32 summation order.
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

U24 = 2.0 ** -24
EPS = {"f32": 2 * U24 + 400 * U24, "bf16": 2.0 ** -8 + 2.0 ** -15 + 800 * U24}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _check_bound(got, ref, Drs, v, eps):
    """|got - ref| <= eps sum_j |Drs_ij| |v_j| for every row and vector."""
    got = np.asarray(got).reshape(v.shape[0], -1)
    ref = np.asarray(ref).reshape(v.shape[0], -1)
    scale = np.abs(v.reshape(v.shape[0], -1)) @ np.abs(Drs).T
    err = np.abs(got - ref)
    worst = float(np.max(err / np.maximum(eps * scale, 1e-300)))
    assert worst <= 1.0, f"error reaches {worst:.3g} of the bound"
    return worst


@pytest.fixture(scope="module")
def n100(orc):
    w = inputs.workload("n100")
    pos = w.positions()
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    Drs = orc.real_space_matrix(pos, w.L, w.a, w.alpha, w.rc)
    return w, pos, D, Drs


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("m", [5, 16])
def test_block_apply_n100(n100, orc, prec, m):
    """N = 100: two bead tiles (three stored tiles, one off the diagonal, a
    ragged last tile and a partly idle workgroup); m = 5 leaves 11 of the 16
    block columns empty."""
    _say(f"block apply n100 {prec} m={m}")
    w, pos, D, Drs = n100
    ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(100 + m).standard_normal((m, w.n, 3))
    out = ctx.apply(_cuda(v), prec=prec).cpu().numpy().reshape(m, -1)
    ref = orc.matvec(D, v.reshape(m, -1))
    _check_bound(out, ref, Drs, v, EPS[prec])
    # the vector-unit path on the same stored tiles, 4 + 1 vectors at a time
    valu = np.concatenate([ctx.apply(_cuda(v[j:j + 4]), prec=prec).cpu().numpy()
                           for j in range(0, m, 4)]).reshape(m, -1)
    tol = 2 * EPS["f32"] if prec == "f32" else 2 * (2.0 ** -15 + 800 * U24)
    _check_bound(out, valu, Drs, v, tol)


@pytest.mark.parametrize("m", [5, 16])
def test_block_apply_f64_n100(n100, orc, m):
    """FP64 tiles on the FP64 matrix cores (16x16x4, FP64 accumulation): to
    rel 1e-12 against the oracle, and against the vector-unit FP64 product
    of the same vectors four at a time."""
    _say(f"block apply n100 f64 m={m}")
    w, pos, D, _ = n100
    ctx = rpy.context_for(w, max_rhs=16)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(200 + m).standard_normal((m, w.n, 3))
    out = ctx.apply(_cuda(v)).cpu().numpy().reshape(m, -1)
    ref = orc.matvec(D, v.reshape(m, -1))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    valu = np.concatenate([ctx.apply(_cuda(v[j:j + 4])).cpu().numpy()
                           for j in range(0, m, 4)]).reshape(m, -1)
    assert np.max(np.abs(out - valu)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_block_apply_n1000(orc, prec):
    """N = 1000: 16 bead tiles per side, 136 stored tiles (120 off the
    diagonal), 16 vectors."""
    _say(f"block apply n1000 {prec}")
    w = inputs.workload("n1000")
    pos = w.positions()
    D = orc.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    Drs = orc.real_space_matrix(pos, w.L, w.a, w.alpha, w.rc)
    ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(1000).standard_normal((16, w.n, 3))
    out = ctx.apply(_cuda(v), prec=prec).cpu().numpy().reshape(16, -1)
    ref = orc.matvec(D, v.reshape(16, -1))
    if prec == "f64":
        assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        _check_bound(out, ref, Drs, v, EPS[prec])


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_block_apply_n4000_sampled_rows(orc, prec):
    """The precision-form workload (N = 4000, 2016 stored tiles, 16 vectors)
    in the launch the benchmark times: sampled block rows against oracle
    rows, covering the first and last bead tile and a tile boundary."""
    _say(f"block apply n4000 {prec}")
    w = inputs.workload("n4000")
    pos = w.positions()
    rows = [0, 1, 63, 64, 2047, 3968, 3999]
    R = orc.diffusion_rows(pos, rows, w.L, w.a, w.alpha, w.rc, w.n2max)
    Rrs = orc.real_space_rows(pos, rows, w.L, w.a, w.alpha, w.rc)
    ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
    ctx.build(_cuda(pos))
    v = np.random.default_rng(4000).standard_normal((16, w.n, 3))
    out = ctx.apply(_cuda(v), prec=prec).cpu().numpy().reshape(16, w.n, 3)
    got = out[:, rows, :].reshape(16, -1)
    ref = (R @ v.reshape(16, -1).T).T
    _check_bound(got, ref, Rrs, v, EPS[prec])


def test_block_chebyshev_f64_n100(n100, orc):
    """16 simultaneous dW through the Chebyshev recurrence (N_Ch = 20) on the
    FP64 block product (FP64 tiles and accumulation on the matrix cores; each
    product after the first reads the operands its predecessor's epilogue
    packed), against the oracle's FP64 recurrence (eq. cheb1-cheb3) to the
    FP64 parity tolerance."""
    _say("block chebyshev n100 f64")
    w, pos, D, Drs = n100
    ctx = rpy.context_for(w, max_rhs=16)
    ctx.build(_cuda(pos))
    lam = np.linalg.eigvalsh(D)
    lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
    nch = 20
    dw = w.noise(m=16)
    ds = ctx.sqrt_apply(_cuda(dw), nch, lo, hi).cpu().numpy().reshape(16, -1)
    ref = orc.cheb_sqrt(D, dw.reshape(16, -1), nch, lo, hi)
    rel = float(np.max(np.abs(ds - ref)) / np.max(np.abs(ref)))
    assert rel < 1e-12, rel


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_block_chebyshev_n100(n100, orc, prec):
    """16 simultaneous dW through the Chebyshev recurrence (N_Ch = 20) on the
    block product, against the oracle's FP64 recurrence (eq. cheb1-cheb3).

    Worst-case propagation: each product D V is replaced by D V + E V with
    ||E||_2 <= ||E||_inf <= eta = eps max_i sum_j |Drs_ij|.  With
    Y = (2 D - (d_max + d_min)) / (d_max - d_min) the error of V_p obeys
    dV_p = 2 Y dV_{p-1} - dV_{p-2} + f_p, ||f_p|| <= 4 eta ||dW|| / (d_max - d_min)
    (||V_q|| <= ||dW|| since |T_q| <= 1 on the spectrum), so
    dV_p = sum_q U_{p-q}(Y) f_q with ||U_n(Y)|| <= n + 1, and
    ||d dS||_2 <= sum_p |c_p| 2 p (p + 1) eta ||dW||_2 / (d_max - d_min)."""
    _say(f"block chebyshev n100 {prec}")
    w, pos, D, Drs = n100
    ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
    ctx.build(_cuda(pos))
    lam = np.linalg.eigvalsh(D)
    lo, hi = 0.9 * lam[0], 1.1 * lam[-1]
    nch = 20
    dw = w.noise(m=16)
    ds = ctx.sqrt_apply(_cuda(dw), nch, lo, hi, prec=prec).cpu().numpy().reshape(16, -1)
    ref = orc.cheb_sqrt(D, dw.reshape(16, -1), nch, lo, hi)
    c = orc.cheb_coeffs(nch, lo, hi)
    eta = EPS[prec] * np.max(np.abs(Drs).sum(1))
    amp = sum(abs(c[p]) * 2 * p * (p + 1) for p in range(1, nch)) / (hi - lo)
    for j in range(16):
        bound = amp * eta * np.linalg.norm(dw[j])
        err = float(np.linalg.norm(ds[j] - ref[j]))
        assert err <= bound, (j, err, bound)
    _say(f"  rel err {np.max(np.abs(ds - ref)) / np.max(np.abs(ref)):.3g}")
