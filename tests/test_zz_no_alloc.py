"""The allocation-free forces entry point (rpy_forces_noalloc) through the C
ABI against rpy_forces on a context: two calls in a row on one stream, the
second with fewer beads (the static scratch keeps the first call's contents),
and the refusal of a size beyond its scratch.  The forces are the Hookean
springs (section "Governing equation") plus the narrow-Gaussian excluded
volume; both entry points run the same kernels, so they agree bit for bit.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1203_6208_amd import inputs  # noqa: E402
from paper_1203_6208_amd import rpy  # noqa: E402


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _noalloc(w, pos, ev, out):
    """The entry point called through ctypes directly, on torch's stream."""
    code = rpy._lib.rpy_forces_noalloc(w.n, w.nchains, w.bpc, ctypes.c_double(w.L),
                                       ctypes.c_void_p(pos.data_ptr()),
                                       ctypes.c_double(ev["zstar"]), ctypes.c_double(ev["dstar"]),
                                       ctypes.c_double(ev["rcut"]),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code


def test_forces_noalloc_matches_context_forces(orc):
    ws = [inputs.workload("n4000"), inputs.workload("n1000")]
    ev = dict(inputs.NG_EV)
    pos = [_cuda(w.positions()) for w in ws]
    outs = [torch.full((w.n, 3), np.nan, dtype=torch.float64, device="cuda") for w in ws]
    # two calls in a row, the second smaller (6 and 4 cells per side)
    for w, p, o in zip(ws, pos, outs):
        print(f"rpy_forces_noalloc N={w.n}", flush=True)
        assert _noalloc(w, p, ev, o) == rpy.RPY_OK
    torch.cuda.synchronize()
    for w, p, o in zip(ws, pos, outs):
        ctx = rpy.context_for(w)
        ref = torch.empty_like(o)
        rpy.rpy_forces(ctx.handle, p, ev["zstar"], ev["dstar"], ev["rcut"], ref)
        torch.cuda.synchronize()
        got, want = o.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
        assert np.array_equal(got, want)
        pw = w.positions()
        orc_f = orc.spring_forces(pw, w.nchains, w.bpc) + orc.ev_forces(
            pw, w.L, ev["zstar"], ev["dstar"], ev["rcut"])
        assert np.max(np.abs(got - orc_f)) <= 1e-12 * np.max(np.abs(orc_f))
        del ctx
    sys.stdout.flush()


def test_forces_noalloc_refuses_beyond_its_scratch():
    w = inputs.Workload("big", 1, 65537, 1.0)
    pos = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    assert _noalloc(w, pos, dict(inputs.NG_EV), out) == rpy.RPY_EINVAL
    assert "65536" in rpy.rpy_strerror(rpy.RPY_EINVAL)
