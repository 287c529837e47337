"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rpy.h, rejects invalid parameters with the documented
codes, and its real-space pair code (the same source the build kernel runs,
compiled for the host) matches the oracle."""
import ctypes
import math
import os
import re
import zlib

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpy.h")
LIB = os.path.join(ROOT, "paper_1203_6208_amd", "librpy.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="librpy.so not built")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert "rpy_ewald_build" in names and "bd_step" in names and "chebyshev_sqrt_apply" in names
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n


@pytest.fixture(scope="module")
def rpy():
    from paper_1203_6208_amd import rpy as m
    return m


def _params(rpy, **over):
    from paper_1203_6208_amd import inputs
    w = inputs.workload("n100")
    kw = dict(n_beads=w.n, n_chains=w.nchains, beads_per_chain=w.bpc, box_l=w.L, a=w.a,
              alpha=w.alpha, r_c=w.rc, k_c=w.kc, lowp="f64", max_rhs=1)
    kw.update(over)
    return rpy.make_params(**kw)


@pytest.mark.parametrize("over,code", [
    (dict(n_beads=0, n_chains=0), -1),
    (dict(box_l=-1.0), -1),
    (dict(a=0.0), -1),
    (dict(alpha=float("nan")), -1),
    (dict(r_c=0.0), -1),
    (dict(k_c=0.0), -1),
    (dict(n_chains=9), -1),
    (dict(max_rhs=17), -1),
    (dict(a=2.0), -2),
])
def test_create_rejects_invalid(rpy, over, code):
    """Parameter validation happens before any device call (error path)."""
    p = _params(rpy, **over)
    h = ctypes.c_void_p()
    rc = rpy._lib.rpy_create(ctypes.byref(h), ctypes.byref(p))
    assert rc == code
    assert not h.value
    assert rpy.rpy_strerror(rc)


def test_strerror_codes(rpy):
    for c in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(rpy.rpy_strerror(c), str)


def _oracle_block(orc, p, rt0, rt1):
    pos = np.array([rt0, rt1])
    D = orc.real_space_matrix(pos, p.box_l, p.a, p.alpha, p.r_c)
    return D[0:3, 3:6], D[0:3, 0:3]


@pytest.mark.parametrize("case", ["random", "overlap", "tiny", "zero", "contact", "near_half"])
@pytest.mark.parametrize("wl", ["n100", "n1000"])
def test_host_pair_block_matches_oracle(rpy, orc, case, wl):
    """The pair kernel (M1, the overlap term Omega_B - S with the small-r
    series, M* beyond r_c, all images) equals the oracle's brute-force
    block, including coincident beads and r just below 2a."""
    from paper_1203_6208_amd import inputs
    w = inputs.workload(wl)
    p = _params(rpy, n_beads=w.n, n_chains=w.nchains, beads_per_chain=w.bpc, box_l=w.L,
                alpha=w.alpha, r_c=w.rc, k_c=w.kc)
    # a fixed seed per case (str hashes are salted per process)
    rng = np.random.default_rng(zlib.crc32(f"{case}/{wl}".encode()))
    for _ in range(5):
        x0 = rng.uniform(0, w.L, 3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        r = {"random": rng.uniform(2 * w.a, w.L), "overlap": rng.uniform(0.05, 1.98) * w.a,
             "tiny": 10 ** rng.uniform(-6, -2) * w.a, "zero": 0.0,
             "contact": 2 * w.a * (1 - 1e-7), "near_half": 0.5 * w.L * 0.999}[case]
        x1 = x0 + r * u
        rt = orc.wrap(np.array([x0, x1]), w.L)
        off, diag = _oracle_block(orc, p, rt[0], rt[1])
        got = np.array(rpy.rpy_host_pair_block(p, rt[0] - rt[1], False)).reshape(3, 3)
        assert np.max(np.abs(got - off)) < 1e-13, (case, r)
        gd = np.array(rpy.rpy_host_pair_block(p, [0.0, 0.0, 0.0], True)).reshape(3, 3)
        assert np.max(np.abs(gd - diag)) < 1e-13


def _batch_create(rpy, ps, lowp=0, tb=64):
    arr = (rpy.RpyParams * max(len(ps), 1))(*ps)
    h = ctypes.c_void_p()
    rc = rpy._lib.rpy_batch_create(ctypes.byref(h), arr, len(ps), lowp, tb)
    return rc, h


@pytest.mark.parametrize("case", ["empty", "tile48", "bf16", "kset", "badbox", "geom"])
def test_batch_create_rejects_invalid(rpy, case):
    """Batch parameter validation happens before any device call: every box
    is checked as rpy_create checks it, all boxes must share one integer
    wave-vector set, tiles are 32 or 64 beads, FP64 or FP32 tiles only."""
    ok = [_params(rpy), _params(rpy, box_l=_params(rpy).box_l * 1.3,
                                alpha=_params(rpy).alpha / 1.3, r_c=_params(rpy).r_c * 1.3,
                                k_c=_params(rpy).k_c / 1.3)]
    ps, lowp, tb, code = ok, 0, 64, -1
    if case == "empty":
        ps = []
    elif case == "tile48":
        tb = 48
    elif case == "bf16":
        lowp = 2
    elif case == "kset":
        ps = ok + [_params(rpy, k_c=_params(rpy).k_c * 1.5)]
    elif case == "badbox":
        ps = ok + [_params(rpy, n_chains=7)]
    elif case == "geom":
        ps = ok + [_params(rpy, a=2.0)]
        code = -2
    rc, h = _batch_create(rpy, ps, lowp, tb)
    assert rc == code
    assert not h.value
    assert rpy.rpy_strerror(rc)


@pytest.mark.parametrize("over", [dict(lma=2), dict(lma=1, grad=1, cheb_keep=4),
                                  dict(lma=1)])
def test_create_rejects_invalid_lma(rpy, over):
    """The low-memory form needs max(r_c, 2a) <= L/3 (the n100 workload has
    r_c = 0.58 L) and excludes the reverse-mode buffers."""
    p = _params(rpy, **over)
    h = ctypes.c_void_p()
    rc = rpy._lib.rpy_create(ctypes.byref(h), ctypes.byref(p))
    assert rc == -1
    assert not h.value
    assert rpy.rpy_strerror(rc)
