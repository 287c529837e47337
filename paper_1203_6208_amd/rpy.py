"""Thin ctypes binding of ``librpy.so`` (declared in ``include/rpy.h``).

Argument marshalling only: every entry point forwards torch tensors' device
pointers and the current HIP stream to the C ABI of the same name.  All
computation happens in the HIP kernels of the library.  Importing this module
raises if the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpy.so")

RPY_OK, RPY_EINVAL, RPY_EGEOM, RPY_ENONFINITE, RPY_ETOL, RPY_ENOMEM, RPY_EHIP = 0, -1, -2, -3, -4, -5, -6
PREC = {"f64": 0, "f32": 1, "bf16": 2}
BOUNDS_EXPLICIT, BOUNDS_PAPER, BOUNDS_DILUTE = 0, 1, 2


class RpyError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with {code}: {rpy_strerror(code)}")
        self.code = code


class RpyParams(ctypes.Structure):
    _fields_ = [("n_beads", ctypes.c_int32), ("n_chains", ctypes.c_int32),
                ("beads_per_chain", ctypes.c_int32), ("lowp", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("cheb_keep", ctypes.c_int32),
                ("grad", ctypes.c_int32), ("lma", ctypes.c_int32),
                ("box_l", ctypes.c_double), ("a", ctypes.c_double),
                ("alpha", ctypes.c_double), ("r_c", ctypes.c_double),
                ("k_c", ctypes.c_double)]


class BdParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("ev_zstar", ctypes.c_double),
                ("ev_dstar", ctypes.c_double), ("ev_rcut", ctypes.c_double),
                ("bounds_C", ctypes.c_double), ("d_min", ctypes.c_double),
                ("d_max", ctypes.c_double), ("tol", ctypes.c_double),
                ("n_cheb", ctypes.c_int32), ("bounds_rule", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("n_max", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)
_v = ctypes.c_void_p
_d = ctypes.c_double
_i = ctypes.c_int
_P = ctypes.POINTER
_SIG = {
    "rpy_create": (_i, [_P(_v), _P(RpyParams)]),
    "rpy_destroy": (None, [_v]),
    "rpy_ewald_build": (_i, [_v, _v, _v]),
    "rpy_apply": (_i, [_v, _v, _v, _i, _i, _v]),
    "rpy_bounds": (_i, [_v, _i, _d, _P(_d), _P(_d), _v]),
    "chebyshev_sqrt_apply": (_i, [_v, _v, _v, _i, _i, _d, _d, _d, _i, _P(_i), _v, _v]),
    "rpy_order_stats": (_i, [_v, _P(ctypes.c_int64), _P(_d), _P(_i), _P(ctypes.c_int64), _v]),
    "bd_step": (_i, [_v, _v, _P(BdParams), _v, ctypes.c_uint64, ctypes.c_uint64, _v, _v, _v, _v]),
    "rpy_status": (_i, [_v, _v]),
    "rpy_real_space_dense": (_i, [_v, _v, _v]),
    "rpy_observables": (_i, [_v, _v, _v, _v, _v]),
    "rpy_forces": (_i, [_v, _v, _d, _d, _d, _v, _v]),
    "rpy_gaussian_noise": (_i, [_v, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, _d, _v]),
    "rpy_philox4x32_10": (_i, [_v, _v, ctypes.c_int64, _v]),
    "rpy_host_pair_block": (_i, [_P(RpyParams), _P(_d), _i, _P(_d)]),
    "rpy_num_kvectors": (_i, [_v]),
    "rpy_profile_enable": (_i, [_v, _i]),
    "rpy_profile_read": (_i, [_v, _i, _P(ctypes.c_int64), _P(_d)]),
    "rpy_strerror": (ctypes.c_char_p, [_i]),
    "rpy_lanczos_bounds": (_i, [_v, _i, ctypes.c_uint64, _v, _d, _P(_d), _P(_d), _P(_d), _P(_d), _v]),
    "chebyshev_sqrt_adaptive": (_i, [_v, _v, _v, _i, _i, _i, _d, _d, _d, _i, _P(_i), _v, _v]),
    "rpy_u_forward": (_i, [_v, _v, _v, _v, _i, _d, _d, _v, _v, _v]),
    "rpy_u_vjp": (_i, [_v, _v, _v, _v, _v, _v, _i, _d, _d, _v, _v, _v]),
    "rpy_forces_vjp": (_i, [_v, _v, _d, _d, _d, _v, _v, _v]),
    "rpy_forces_noalloc": (_i, [_i, _i, _i, _d, _v, _d, _d, _d, _v, _v]),
    "rpy_batch_create": (_i, [_P(_v), _P(RpyParams), _i, _i, _i]),
    "rpy_batch_destroy": (None, [_v]),
    "rpy_batch_padded_beads": (ctypes.c_int64, [_v]),
    "rpy_batch_offsets": (_i, [_v, _P(ctypes.c_int64)]),
    "rpy_batch_build": (_i, [_v, _v, _v]),
    "rpy_batch_apply": (_i, [_v, _v, _v, _i, _i, _v]),
    "rpy_batch_chebyshev": (_i, [_v, _v, _v, _i, _i, _d, _d, _d, _i, _v, _v, _v]),
    "rpy_batch_step": (_i, [_v, _v, _P(BdParams), ctypes.c_uint64, ctypes.c_uint64, _v, _v, _v,
                            _v]),
    "rpy_batch_run": (_i, [_v, _v, _P(BdParams), ctypes.c_uint64, ctypes.c_uint64, _i, _v]),
    "rpy_batch_observables": (_i, [_v, _v, _v, _v, _v]),
    "rpy_batch_status": (_i, [_v, _v]),
    "rpy_batch_set_variant": (_i, [_v, _i, _i]),
    "rpy_batch_graph_nodes": (ctypes.c_int64, [_v]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name}: need a contiguous {dtype} tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _check(code: int, what: str):
    if code != RPY_OK:
        raise RpyError(code, what)


def rpy_strerror(code: int) -> str:
    return _lib.rpy_strerror(int(code)).decode()


def make_params(*, n_beads, n_chains, beads_per_chain, box_l, a, alpha, r_c, k_c,
                lowp="f64", max_rhs=1, cheb_keep=0, grad=0, lma=0) -> RpyParams:
    return RpyParams(int(n_beads), int(n_chains), int(beads_per_chain), PREC[lowp],
                     int(max_rhs), int(cheb_keep), int(grad), int(lma), float(box_l), float(a),
                     float(alpha), float(r_c), float(k_c))


def rpy_create(params: RpyParams) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.rpy_create(ctypes.byref(h), ctypes.byref(params)), "rpy_create")
    return h


def rpy_destroy(ctx) -> None:
    _lib.rpy_destroy(ctx)


def rpy_ewald_build(ctx, pos: torch.Tensor, stream=None) -> None:
    _check(_lib.rpy_ewald_build(ctx, _dev(pos, "pos"), _stream(stream)), "rpy_ewald_build")


def rpy_apply(ctx, v: torch.Tensor, out: torch.Tensor, m: int, prec="f64", stream=None):
    _check(_lib.rpy_apply(ctx, _dev(v, "v"), _dev(out, "out"), int(m), PREC[prec],
                          _stream(stream)), "rpy_apply")
    return out


def rpy_bounds(ctx, C: float, rule=BOUNDS_PAPER, stream=None):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(_lib.rpy_bounds(ctx, int(rule), float(C), ctypes.byref(lo), ctypes.byref(hi),
                           _stream(stream)), "rpy_bounds")
    return lo.value, hi.value


def chebyshev_sqrt_apply(ctx, dw: torch.Tensor, out: torch.Tensor, m: int, n_cheb: int,
                         d_min: float, d_max: float, prec="f64", e_f: torch.Tensor = None,
                         tol: float = 0.0, want_n: bool = False, stream=None,
                         allow_etol=False):
    """Fixed order (tol <= 0) or adaptive order up to n_cheb (tol > 0).
    Returns the order used when want_n (that synchronises), else None.
    RPY_ETOL raises unless allow_etol."""
    n = ctypes.c_int()
    code = _lib.chebyshev_sqrt_apply(ctx, _dev(dw, "dw"), _dev(out, "out"), int(m), int(n_cheb),
                                     float(d_min), float(d_max), float(tol), PREC[prec],
                                     ctypes.byref(n) if want_n else None, _dev(e_f, "e_f"),
                                     _stream(stream))
    if not (code == RPY_OK or (allow_etol and code == RPY_ETOL)):
        _check(code, "chebyshev_sqrt_apply")
    return n.value if want_n else None


def rpy_order_stats(ctx, stream=None):
    """(calls, mean N_Ch, max N_Ch, calls that missed the tolerance) of the
    adaptive calls since the last read; resets them."""
    calls, mx, missed = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64()
    mean = ctypes.c_double()
    _check(_lib.rpy_order_stats(ctx, ctypes.byref(calls), ctypes.byref(mean), ctypes.byref(mx),
                                ctypes.byref(missed), _stream(stream)), "rpy_order_stats")
    return calls.value, mean.value, mx.value, missed.value


def rpy_lanczos_bounds(ctx, n_iter: int, seed: int = 0, start: torch.Tensor = None,
                       margin: float = 0.05, stream=None):
    """(d_min, d_max, alpha[n_iter], beta[n_iter]) from the FP64 Lanczos
    recurrence on D of the last build."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    a = (ctypes.c_double * int(n_iter))()
    b = (ctypes.c_double * int(n_iter))()
    _check(_lib.rpy_lanczos_bounds(ctx, int(n_iter), int(seed), _dev(start, "start"), float(margin),
                                   ctypes.byref(lo), ctypes.byref(hi), a, b, _stream(stream)),
           "rpy_lanczos_bounds")
    return lo.value, hi.value, list(a), list(b)


def chebyshev_sqrt_adaptive(ctx, dw: torch.Tensor, out: torch.Tensor, m: int, n_start: int,
                            n_max: int, d_min: float, d_max: float, tol: float, prec="f64",
                            e_f: torch.Tensor = None, stream=None, allow_etol=False):
    """Adaptive-order square root; returns the order used.  RPY_ETOL raises
    unless allow_etol (then the order n_max is returned)."""
    n = ctypes.c_int()
    code = _lib.chebyshev_sqrt_adaptive(ctx, _dev(dw, "dw"), _dev(out, "out"), int(m),
                                        int(n_start), int(n_max), float(d_min), float(d_max),
                                        float(tol), PREC[prec], ctypes.byref(n), _dev(e_f, "e_f"),
                                        _stream(stream))
    if not (code == RPY_OK or (allow_etol and code == RPY_ETOL)):
        _check(code, "chebyshev_sqrt_adaptive")
    return n.value


def make_bd_params(*, dt, n_cheb, bounds_rule=BOUNDS_EXPLICIT, d_min=0.0, d_max=0.0,
                   bounds_C=8.0, prec="f64", ev=None, tol=0.0, n_max=0) -> BdParams:
    ev = ev or {}
    return BdParams(float(dt), float(ev.get("zstar", 0.0)), float(ev.get("dstar", 0.0)),
                    float(ev.get("rcut", 0.0)), float(bounds_C), float(d_min), float(d_max),
                    float(tol), int(n_cheb), int(bounds_rule), PREC[prec], int(n_max))


def bd_step(ctx, pos: torch.Tensor, bp: BdParams, dw: torch.Tensor = None, seed: int = 0,
            step: int = 0, drift: torch.Tensor = None, noise: torch.Tensor = None,
            e_f: torch.Tensor = None, stream=None) -> None:
    _check(_lib.bd_step(ctx, _dev(pos, "pos"), ctypes.byref(bp), _dev(dw, "dw"),
                        ctypes.c_uint64(seed), ctypes.c_uint64(step), _dev(drift, "drift"),
                        _dev(noise, "noise"), _dev(e_f, "e_f"), _stream(stream)), "bd_step")


def rpy_status(ctx, stream=None) -> int:
    return _lib.rpy_status(ctx, _stream(stream))


def rpy_real_space_dense(ctx, out: torch.Tensor, stream=None):
    _check(_lib.rpy_real_space_dense(ctx, _dev(out, "out"), _stream(stream)),
           "rpy_real_space_dense")
    return out


def rpy_observables(ctx, pos, re2, rg2, stream=None):
    _check(_lib.rpy_observables(ctx, _dev(pos, "pos"), _dev(re2, "re2"), _dev(rg2, "rg2"),
                                _stream(stream)), "rpy_observables")


def rpy_forces(ctx, pos, zstar, dstar, rcut, out, stream=None):
    _check(_lib.rpy_forces(ctx, _dev(pos, "pos"), float(zstar), float(dstar), float(rcut),
                           _dev(out, "out"), _stream(stream)), "rpy_forces")
    return out


def rpy_forces_noalloc(n_beads, n_chains, beads_per_chain, box_l, pos, zstar, dstar, rcut, out,
                       stream=None):
    _check(_lib.rpy_forces_noalloc(int(n_beads), int(n_chains), int(beads_per_chain),
                                   float(box_l), _dev(pos, "pos"), float(zstar), float(dstar),
                                   float(rcut), _dev(out, "out"), _stream(stream)),
           "rpy_forces_noalloc")
    return out


def rpy_gaussian_noise(out: torch.Tensor, seed: int, step: int, dt: float, stream=None):
    _check(_lib.rpy_gaussian_noise(_dev(out, "out"), out.numel(), ctypes.c_uint64(seed),
                                   ctypes.c_uint64(step), float(dt), _stream(stream)),
           "rpy_gaussian_noise")
    return out


def rpy_philox4x32_10(ctr_key: torch.Tensor, out: torch.Tensor, stream=None):
    n = ctr_key.numel() // 6
    _check(_lib.rpy_philox4x32_10(_dev(ctr_key, "ctr_key", torch.int32), _dev(out, "out", torch.int32),
                                  n, _stream(stream)), "rpy_philox4x32_10")
    return out


def rpy_host_pair_block(params: RpyParams, d, self_pair: bool):
    dd = (ctypes.c_double * 3)(*[float(x) for x in d])
    out = (ctypes.c_double * 9)()
    _check(_lib.rpy_host_pair_block(ctypes.byref(params), dd, int(bool(self_pair)), out),
           "rpy_host_pair_block")
    return [out[i] for i in range(9)]


def rpy_u_forward(ctx, pos, F, dw, n_cheb, d_min, d_max, u, vh=None, stream=None):
    """u = D(pos) F + p(D(pos)) dW on the fixed interval; vh [n_cheb, N, 3]
    receives the V_p when given."""
    _check(_lib.rpy_u_forward(ctx, _dev(pos, "pos"), _dev(F, "F"), _dev(dw, "dw"), int(n_cheb),
                              float(d_min), float(d_max), _dev(u, "u"), _dev(vh, "vh"),
                              _stream(stream)), "rpy_u_forward")
    return u


def rpy_u_vjp(ctx, pos, F, dw, g, n_cheb, d_min, d_max, g_pos, g_F=None, vh=None, stream=None):
    _check(_lib.rpy_u_vjp(ctx, _dev(pos, "pos"), _dev(F, "F"), _dev(dw, "dw"), _dev(vh, "vh"),
                          _dev(g, "g"), int(n_cheb), float(d_min), float(d_max),
                          _dev(g_pos, "g_pos"), _dev(g_F, "g_F"), _stream(stream)), "rpy_u_vjp")
    return g_pos, g_F


def rpy_forces_vjp(ctx, pos, zstar, dstar, rcut, gF, g_pos, stream=None):
    _check(_lib.rpy_forces_vjp(ctx, _dev(pos, "pos"), float(zstar), float(dstar), float(rcut),
                               _dev(gF, "gF"), _dev(g_pos, "g_pos"), _stream(stream)),
           "rpy_forces_vjp")
    return g_pos


PROF_SYMV, PROF_BUILD, PROF_KSPACE, PROF_EPI, PROF_OTHER, PROF_SYMV_MULTI = range(6)


def rpy_profile_enable(ctx, cap: int) -> None:
    _check(_lib.rpy_profile_enable(ctx, int(cap)), "rpy_profile_enable")


def rpy_profile_read(ctx, kind: int):
    n, t = ctypes.c_int64(), ctypes.c_double()
    _check(_lib.rpy_profile_read(ctx, int(kind), ctypes.byref(n), ctypes.byref(t)),
           "rpy_profile_read")
    return n.value, t.value


def rpy_num_kvectors(ctx) -> int:
    return _lib.rpy_num_kvectors(ctx)


class Context:
    """Owns one rpy_ctx; methods forward to the entry points above."""

    def __init__(self, **kw):
        self.params = make_params(**kw)
        self.n = self.params.n_beads
        self.handle = rpy_create(self.params)

    def close(self):
        if self.handle is not None and self.handle.value:
            rpy_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, pos, stream=None):
        rpy_ewald_build(self.handle, pos, stream)

    def apply(self, v, prec="f64", stream=None):
        v = v.reshape(-1, self.n, 3).contiguous()
        out = torch.empty_like(v)
        rpy_apply(self.handle, v, out, v.shape[0], prec, stream)
        return out

    def sqrt_apply(self, dw, n_cheb, d_min, d_max, prec="f64", want_ef=False, tol=0.0,
                   want_n=False, stream=None, allow_etol=False):
        """dS (and E_f when want_ef, the order used when want_n)."""
        dw = dw.reshape(-1, self.n, 3).contiguous()
        out = torch.empty_like(dw)
        ef = torch.empty(dw.shape[0], dtype=torch.float64, device=dw.device) if want_ef else None
        n = chebyshev_sqrt_apply(self.handle, dw, out, dw.shape[0], n_cheb, d_min, d_max, prec,
                                 ef, tol, want_n, stream, allow_etol)
        res = (out,) + ((ef,) if want_ef else ()) + ((n,) if want_n else ())
        return res if len(res) > 1 else out

    def bounds(self, C, rule=BOUNDS_PAPER, stream=None):
        return rpy_bounds(self.handle, C, rule, stream)

    def order_stats(self, stream=None):
        return rpy_order_stats(self.handle, stream)

    def lanczos_bounds(self, n_iter, seed=0, start=None, margin=0.05, stream=None):
        if start is not None:
            start = start.reshape(self.n, 3).contiguous()
        return rpy_lanczos_bounds(self.handle, n_iter, seed, start, margin, stream)

    def sqrt_adaptive(self, dw, d_min, d_max, tol, n_max, n_start=0, prec="f64", stream=None,
                      allow_etol=False):
        """(dS, E_f, N_Ch used)."""
        dw = dw.reshape(-1, self.n, 3).contiguous()
        out = torch.empty_like(dw)
        ef = torch.empty(dw.shape[0], dtype=torch.float64, device=dw.device)
        n = chebyshev_sqrt_adaptive(self.handle, dw, out, dw.shape[0], n_start, n_max, d_min,
                                    d_max, tol, prec, ef, stream, allow_etol)
        return out, ef, n

    def real_space_dense(self, stream=None):
        out = torch.empty((3 * self.n, 3 * self.n), dtype=torch.float64, device="cuda")
        return rpy_real_space_dense(self.handle, out, stream)

    def step(self, pos, bp, dw=None, seed=0, step=0, want=False, e_f=None, stream=None):
        drift = noise = None
        ef = e_f
        if want:
            drift = torch.empty_like(pos)
            noise = torch.empty_like(pos)
            if ef is None:
                ef = torch.empty(1, dtype=torch.float64, device=pos.device)
        bd_step(self.handle, pos, bp, dw, seed, step, drift, noise, ef, stream)
        return (drift, noise, ef) if want else None

    def observables(self, pos, re2=None, rg2=None, stream=None):
        """Per-chain R_e^2, R_g^2 (device [n_chains] each)."""
        nc = self.params.n_chains
        if re2 is None:
            re2 = torch.empty(nc, dtype=torch.float64, device=pos.device)
        if rg2 is None:
            rg2 = torch.empty(nc, dtype=torch.float64, device=pos.device)
        rpy_observables(self.handle, pos, re2, rg2, stream)
        return re2, rg2

    def status(self, stream=None):
        return rpy_status(self.handle, stream)

    def num_kvectors(self):
        return rpy_num_kvectors(self.handle)


def context_for(workload, lowp="f64", max_rhs=1, cheb_keep=0, grad=0, lma=0) -> Context:
    """Context for an ``inputs.Workload``."""
    return Context(n_beads=workload.n, n_chains=workload.nchains,
                   beads_per_chain=workload.bpc, box_l=workload.L, a=workload.a,
                   alpha=workload.alpha, r_c=workload.rc, k_c=workload.kc, lowp=lowp,
                   max_rhs=max_rhs, cheb_keep=cheb_keep, grad=grad, lma=lma)


# ------------------------------------------------------------------ batches
def rpy_batch_create(params, lowp="f64", tile_beads=64) -> ctypes.c_void_p:
    arr = (RpyParams * len(params))(*params)
    h = ctypes.c_void_p()
    _check(_lib.rpy_batch_create(ctypes.byref(h), arr, len(params), PREC[lowp], int(tile_beads)),
           "rpy_batch_create")
    return h


def rpy_batch_destroy(b) -> None:
    _lib.rpy_batch_destroy(b)


def rpy_batch_padded_beads(b) -> int:
    return int(_lib.rpy_batch_padded_beads(b))


def rpy_batch_offsets(b, nbox: int):
    out = (ctypes.c_int64 * (nbox + 1))()
    _check(_lib.rpy_batch_offsets(b, out), "rpy_batch_offsets")
    return [int(x) for x in out]


def rpy_batch_build(b, pos, stream=None):
    _check(_lib.rpy_batch_build(b, _dev(pos, "pos"), _stream(stream)), "rpy_batch_build")


def rpy_batch_apply(b, v, out, m, prec="f64", stream=None):
    _check(_lib.rpy_batch_apply(b, _dev(v, "v"), _dev(out, "out"), int(m), PREC[prec],
                                _stream(stream)), "rpy_batch_apply")
    return out


def rpy_batch_chebyshev(b, dw, out, n_cheb, bounds_rule=BOUNDS_PAPER, C=8.0, d_min=0.0,
                        d_max=0.0, prec="f64", e_f=None, bounds=None, stream=None):
    _check(_lib.rpy_batch_chebyshev(b, _dev(dw, "dw"), _dev(out, "out"), int(n_cheb),
                                    int(bounds_rule), float(C), float(d_min), float(d_max),
                                    PREC[prec], _dev(e_f, "e_f"), _dev(bounds, "bounds"),
                                    _stream(stream)), "rpy_batch_chebyshev")
    return out


def rpy_batch_step(b, pos, bp: BdParams, seed=0, step=0, drift=None, noise=None, e_f=None,
                   stream=None):
    _check(_lib.rpy_batch_step(b, _dev(pos, "pos"), ctypes.byref(bp), ctypes.c_uint64(seed),
                               ctypes.c_uint64(step), _dev(drift, "drift"), _dev(noise, "noise"),
                               _dev(e_f, "e_f"), _stream(stream)), "rpy_batch_step")


def rpy_batch_run(b, pos, bp: BdParams, seed=0, step0=0, n_steps=1, stream=None):
    _check(_lib.rpy_batch_run(b, _dev(pos, "pos"), ctypes.byref(bp), ctypes.c_uint64(seed),
                              ctypes.c_uint64(step0), int(n_steps), _stream(stream)),
           "rpy_batch_run")


def rpy_batch_observables(b, pos, re2, rg2, stream=None):
    _check(_lib.rpy_batch_observables(b, _dev(pos, "pos"), _dev(re2, "re2"), _dev(rg2, "rg2"),
                                      _stream(stream)), "rpy_batch_observables")


def rpy_batch_status(b, stream=None) -> int:
    return _lib.rpy_batch_status(b, _stream(stream))


SF_SPREAD, SF_FRONT = 0, 1
LOADS_STREAM, LOADS_CACHED = 0, 1


def rpy_batch_set_variant(b, sf_place=SF_SPREAD, tile_loads=LOADS_STREAM):
    _check(_lib.rpy_batch_set_variant(b, int(sf_place), int(tile_loads)),
           "rpy_batch_set_variant")


def rpy_batch_graph_nodes(b) -> int:
    return int(_lib.rpy_batch_graph_nodes(b))


class Batch:
    """Owns one rpy_batch over ``inputs.Workload`` boxes; converts between the
    per-box ``[N_b, 3]`` arrays and the padded global layout."""

    def __init__(self, workloads, lowp="f64", tile_beads=64):
        self.workloads = list(workloads)
        ps = [make_params(n_beads=w.n, n_chains=w.nchains, beads_per_chain=w.bpc, box_l=w.L,
                          a=w.a, alpha=w.alpha, r_c=w.rc, k_c=w.kc) for w in self.workloads]
        self.tile_beads = int(tile_beads)
        self.handle = rpy_batch_create(ps, lowp, tile_beads)
        self.nbox = len(ps)
        self.G = rpy_batch_padded_beads(self.handle)
        self.bead0 = rpy_batch_offsets(self.handle, self.nbox)
        self.nchain = sum(w.nchains for w in self.workloads)

    def close(self):
        if self.handle is not None and self.handle.value:
            rpy_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, per_box, m=None, device="cuda"):
        """Per-box arrays [N_b, 3] (or [m, N_b, 3]) -> padded [G, 3] ([m, G, 3])."""
        lead = () if m is None else (m,)
        out = torch.zeros(lead + (self.G, 3), dtype=torch.float64)
        for b, x in enumerate(per_box):
            t = torch.as_tensor(x, dtype=torch.float64)
            out[..., self.bead0[b]:self.bead0[b] + self.workloads[b].n, :] = t
        return out.to(device).contiguous()

    def unpack(self, x):
        """Padded [..., G, 3] -> list of per-box [..., N_b, 3] (same device)."""
        return [x[..., self.bead0[b]:self.bead0[b] + w.n, :] for b, w in enumerate(self.workloads)]

    def build(self, pos, stream=None):
        rpy_batch_build(self.handle, pos, stream)

    def set_variant(self, sf_place=SF_SPREAD, tile_loads=LOADS_STREAM):
        rpy_batch_set_variant(self.handle, sf_place, tile_loads)

    def graph_nodes(self):
        return rpy_batch_graph_nodes(self.handle)

    def apply(self, v, prec="f64", stream=None):
        v = v.reshape(-1, self.G, 3).contiguous()
        out = torch.empty_like(v)
        rpy_batch_apply(self.handle, v, out, v.shape[0], prec, stream)
        return out

    def chebyshev(self, dw, n_cheb, bounds_rule=BOUNDS_PAPER, C=8.0, d_min=0.0, d_max=0.0,
                  prec="f64", stream=None):
        """(dS [G, 3], E_f [nbox], bounds [nbox, 2])."""
        dw = dw.reshape(self.G, 3).contiguous()
        out = torch.empty_like(dw)
        ef = torch.empty(self.nbox, dtype=torch.float64, device=dw.device)
        bnd = torch.empty((self.nbox, 2), dtype=torch.float64, device=dw.device)
        rpy_batch_chebyshev(self.handle, dw, out, n_cheb, bounds_rule, C, d_min, d_max, prec, ef,
                            bnd, stream)
        return out, ef, bnd

    def step(self, pos, bp, seed=0, step=0, want=False, stream=None):
        drift = noise = ef = None
        if want:
            drift = torch.empty_like(pos)
            noise = torch.empty_like(pos)
            ef = torch.empty(self.nbox, dtype=torch.float64, device=pos.device)
        rpy_batch_step(self.handle, pos, bp, seed, step, drift, noise, ef, stream)
        return (drift, noise, ef) if want else None

    def run(self, pos, bp, seed=0, step0=0, n_steps=1, stream=None):
        rpy_batch_run(self.handle, pos, bp, seed, step0, n_steps, stream)

    def observables(self, pos, stream=None):
        re2 = torch.empty(self.nchain, dtype=torch.float64, device=pos.device)
        rg2 = torch.empty(self.nchain, dtype=torch.float64, device=pos.device)
        rpy_batch_observables(self.handle, pos, re2, rg2, stream)
        return re2, rg2

    def status(self, stream=None):
        return rpy_batch_status(self.handle, stream)
