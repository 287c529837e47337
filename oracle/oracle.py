"""ctypes wrapper around ``liboracle.so`` (plain C, FP64, libquadmath).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here.
The HIP product path never falls back to it.

Every function takes and returns numpy float64 arrays in the layouts the paper
fixes (arXiv:1203.6208, section "Governing equation"): positions ``[N, 3]``,
vectors ``[m, N, 3]``, the dense diffusion matrix ``[3N, 3N]`` with row
``3*nu + i``.  Each wrapper cites the passage the C routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpy_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math), OpenMP over rows."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", _SRC,
               "-lquadmath", "-lm", "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i, p = ctypes.c_double, ctypes.c_int, _dp
        sig = {
            "orc_rpy_branch_a": (None, [d, d, p, p]),
            "orc_rpy_branch_b": (None, [d, d, p, p]),
            "orc_m1_coeffs": (None, [d, d, d, p, p]),
            "orc_mstar_coeffs": (None, [d, p, p]),
            "orc_self_coeff": (d, [d, d]),
            "orc_m2_scalar": (d, [d, d, d, d]),
            "orc_wrap": (None, [i, p, d, p]),
            "orc_real_space": (None, [i, p, d, d, d, d, p]),
            "orc_real_space_rows": (None, [i, p, d, d, d, d, i, _ip, p]),
            "orc_recip_space_rows": (None, [i, p, d, d, d, i, i, _ip, p]),
            "orc_u_vjp_rows": (None, [i, p, d, d, d, d, i, p, p, p, i, d, d, i, _ip, p, p]),
            "orc_self_term_rows": (None, [i, d, d, i, _ip, p]),
            "orc_self_term": (None, [i, d, d, p]),
            "orc_recip_space": (None, [i, p, d, d, d, i, p]),
            "orc_count_kvectors": (i, [i]),
            "orc_matvec": (None, [i, p, i, p, p]),
            "orc_rows_matvec": (None, [i, i, p, p, p]),
            "orc_set_threads": (None, [i]),
            "orc_max_threads": (i, []),
            "orc_cheb_coeffs": (None, [i, d, d, p]),
            "orc_cheb_sqrt": (None, [i, p, i, p, i, d, d, p]),
            "orc_sqrt_error": (d, [i, p, p, p]),
            "orc_bounds_rule": (None, [i, p, d, p, p]),
            "orc_bounds_dilute": (None, [i, p, p, p]),
            "orc_cheb_adaptive": (i, [i, p, i, p, i, i, d, d, d, p]),
            "orc_lanczos": (None, [i, p, p, i, p, p]),
            "orc_spring_forces": (None, [i, i, p, p]),
            "orc_ev_forces": (None, [i, p, d, d, d, d, p]),
            "orc_euler": (None, [i, p, d, p, p, p]),
            "orc_chain_observables": (None, [i, i, p, p, p]),
            "orc_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "orc_gaussian_noise": (None, [ctypes.c_long, ctypes.c_uint64,
                                          ctypes.c_uint64, d, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def set_threads(n: int) -> None:
    """Set the OpenMP thread count the oracle uses (environment-level)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))


def use_threads(n: int) -> None:
    """Set the OpenMP team size of the oracle's later parallel loops (takes
    effect in a process whose OpenMP runtime has already started)."""
    _L().orc_set_threads(int(n))


def max_threads() -> int:
    """The team size the oracle's parallel loops use now."""
    return int(_L().orc_max_threads())


# ---------------------------------------------------------------- pair terms
def rpy_branch_a(r: float, a: float):
    """RPY branch A, r >= 2a (eq. b1): returns (Omega1, Omega2)."""
    o1, o2 = ctypes.c_double(), ctypes.c_double()
    _L().orc_rpy_branch_a(r, a, ctypes.byref(o1), ctypes.byref(o2))
    return o1.value, o2.value


def rpy_branch_b(r: float, a: float):
    """RPY branch B, 0 < r <= 2a (eq. b2): returns (Omega1, Omega2)."""
    o1, o2 = ctypes.c_double(), ctypes.c_double()
    _L().orc_rpy_branch_b(r, a, ctypes.byref(o1), ctypes.byref(o2))
    return o1.value, o2.value


def m1_coeffs(r: float, a: float, alpha: float):
    """Real-space Ewald kernel M1(r) (eq. M1): (coef of I, coef of rhat rhat)."""
    c1, c2 = ctypes.c_double(), ctypes.c_double()
    _L().orc_m1_coeffs(r, a, alpha, ctypes.byref(c1), ctypes.byref(c2))
    return c1.value, c2.value


def mstar_coeffs(x: float):
    """Overlap correction M*(x), x = r/a (eq. cor5, corrected rr term)."""
    c1, c2 = ctypes.c_double(), ctypes.c_double()
    _L().orc_mstar_coeffs(x, ctypes.byref(c1), ctypes.byref(c2))
    return c1.value, c2.value


def self_coeff(a: float, alpha: float) -> float:
    """Self term 1 - 6 a alpha/sqrt(pi) + 40 a^3 alpha^3/(3 sqrt(pi)) (eq. DF)."""
    return _L().orc_self_coeff(a, alpha)


def m2_scalar(k: float, a: float, alpha: float, vol: float) -> float:
    """m(k) with M2(k) = m(k)(I - khat khat) (eq. M2)."""
    return _L().orc_m2_scalar(k, a, alpha, vol)


def count_kvectors(n2max: int) -> int:
    """Size of the full wave-vector set {n != 0, |n|^2 <= n2max}."""
    return _L().orc_count_kvectors(int(n2max))


# ------------------------------------------------------------------- matrix
def wrap(pos, L: float) -> np.ndarray:
    """Wrapped positions L*(r/L - floor(r/L))."""
    pos = _f64(pos)
    out = np.empty_like(pos)
    _L().orc_wrap(pos.shape[0], _ptr(pos), L, _ptr(out))
    return out


def real_space_matrix(pos, L, a, alpha, rc) -> np.ndarray:
    """Self term plus the real-space lattice sum of M1 with the overlap
    correction M* (eq. DFmodified, first, second and last terms), dense."""
    pos = _f64(pos)
    n = pos.shape[0]
    rt = wrap(pos, L)
    D = np.zeros((3 * n, 3 * n))
    _L().orc_real_space(n, _ptr(rt), L, a, alpha, rc, _ptr(D))
    _L().orc_self_term(n, a, alpha, _ptr(D))
    return D


def recip_space_matrix(pos, L, a, alpha, n2max) -> np.ndarray:
    """Reciprocal-space sum over the full +-k set (eq. DFmodified, third term)."""
    pos = _f64(pos)
    n = pos.shape[0]
    rt = wrap(pos, L)
    D = np.zeros((3 * n, 3 * n))
    _L().orc_recip_space(n, _ptr(rt), L, a, alpha, int(n2max), _ptr(D))
    return D


def diffusion_matrix(pos, L, a, alpha, rc, n2max) -> np.ndarray:
    """Full periodic diffusion matrix D (eq. DFmodified read as a matrix)."""
    return real_space_matrix(pos, L, a, alpha, rc) + recip_space_matrix(
        pos, L, a, alpha, n2max)


def diffusion_rows(pos, rows, L, a, alpha, rc, n2max) -> np.ndarray:
    """Block rows of the full periodic D for the listed beads: [3*len(rows), 3N]
    (same sums as diffusion_matrix, restricted to those rows)."""
    pos = _f64(pos)
    n = pos.shape[0]
    rt = wrap(pos, L)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.intc))
    rp = r.ctypes.data_as(_ip)
    D = np.zeros((3 * len(r), 3 * n))
    _L().orc_real_space_rows(n, _ptr(rt), L, a, alpha, rc, len(r), rp, _ptr(D))
    _L().orc_self_term_rows(n, a, alpha, len(r), rp, _ptr(D))
    _L().orc_recip_space_rows(n, _ptr(rt), L, a, alpha, int(n2max), len(r), rp, _ptr(D))
    return D


def real_space_rows(pos, rows, L, a, alpha, rc) -> np.ndarray:
    """Block rows of the self term plus the real-space sum (eq. DFmodified,
    first, second and last terms) for the listed beads: [3*len(rows), 3N]."""
    pos = _f64(pos)
    n = pos.shape[0]
    rt = wrap(pos, L)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.intc))
    rp = r.ctypes.data_as(_ip)
    D = np.zeros((3 * len(r), 3 * n))
    _L().orc_real_space_rows(n, _ptr(rt), L, a, alpha, rc, len(r), rp, _ptr(D))
    _L().orc_self_term_rows(n, a, alpha, len(r), rp, _ptr(D))
    return D


def matvec(D, V) -> np.ndarray:
    """D . V for V of shape [m, 3N] (or [3N])."""
    D = _f64(D)
    V = _f64(V)
    shp = V.shape
    V2 = V.reshape(-1, D.shape[0])
    out = np.empty_like(V2)
    _L().orc_matvec(D.shape[0], _ptr(D), V2.shape[0], _ptr(V2), _ptr(out))
    return out.reshape(shp)


def rows_matvec(R, v) -> np.ndarray:
    """R . v for a block of rows R [r, c] and a vector v [c] (plain loop)."""
    R, v = _f64(R), _f64(v).ravel()
    out = np.empty(R.shape[0])
    _L().orc_rows_matvec(R.shape[0], R.shape[1], _ptr(R), _ptr(v), _ptr(out))
    return out


# ---------------------------------------------------------------- chebyshev
def cheb_coeffs(nch: int, dmin: float, dmax: float) -> np.ndarray:
    """Chebyshev coefficients c_p of sqrt on [dmin, dmax] (eq. cheb1)."""
    c = np.empty(nch)
    _L().orc_cheb_coeffs(int(nch), dmin, dmax, _ptr(c))
    return c


def cheb_sqrt(D, dw, nch: int, dmin: float, dmax: float) -> np.ndarray:
    """Fixman-Chebyshev dS ~ sqrt(D) dW (eq. cheb1-cheb3); dw is [m, 3N]."""
    D = _f64(D)
    dw = _f64(dw)
    shp = dw.shape
    W = dw.reshape(-1, D.shape[0])
    out = np.empty_like(W)
    _L().orc_cheb_sqrt(D.shape[0], _ptr(D), W.shape[0], _ptr(W), int(nch),
                       dmin, dmax, _ptr(out))
    return out.reshape(shp)


def cheb_adaptive(D, dw, dmin: float, dmax: float, tol: float, nmax: int, nch0: int = 0):
    """The paper's adaptive order (eq. nint, then N_Ch + 1 until every E_f <
    tol, at most nmax); returns (N_Ch, dS)."""
    D = _f64(D)
    dw = _f64(dw)
    shp = dw.shape
    W = dw.reshape(-1, D.shape[0])
    out = np.empty_like(W)
    n = _L().orc_cheb_adaptive(D.shape[0], _ptr(D), W.shape[0], _ptr(W), int(nch0), int(nmax),
                               dmin, dmax, tol, _ptr(out))
    return int(n), out.reshape(shp)


def lanczos(D, start, k: int):
    """alpha[k], beta[k] of the plain Lanczos recurrence from `start`."""
    D, start = _f64(D), _f64(start).ravel()
    a, b = np.empty(k), np.empty(k)
    _L().orc_lanczos(D.shape[0], _ptr(D), _ptr(start), int(k), _ptr(a), _ptr(b))
    return a, b


def lanczos_bounds(alpha, beta, margin: float):
    """Chebyshev interval from Lanczos coefficients: the extreme Ritz values
    theta of the tridiagonal T_k widened by their residual bounds
    beta_k |s_k| (s the unit eigenvector of T_k) and by the relative margin:
      d_min = (theta_min - r_min)(1 - margin), d_max = (theta_max + r_max)(1 + margin);
    if that d_min is not positive, d_min = theta_min / 2."""
    alpha, beta = np.asarray(alpha, float), np.asarray(beta, float)
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    th, S = np.linalg.eigh(T)
    r = abs(beta[k - 1]) * np.abs(S[k - 1, :])
    lo = (th[0] - r[0]) * (1.0 - margin)
    hi = (th[-1] + r[-1]) * (1.0 + margin)
    if not lo > 0:
        lo = th[0] / 2
    return float(lo), float(hi), th


def sqrt_error(D, dw, ds) -> float:
    """E_f of the square-root estimate (error estimate after eq. fmin)."""
    D, dw, ds = _f64(D), _f64(dw).ravel(), _f64(ds).ravel()
    return _L().orc_sqrt_error(D.shape[0], _ptr(D), _ptr(dw), _ptr(ds))


def bounds_rule(D, nbeads: int, C: float):
    """Paper's semidilute rule (eq. lmax-lmin-dilute, fmax, fmin): (dmin, dmax)."""
    D = _f64(D)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _L().orc_bounds_rule(int(nbeads), _ptr(D), C, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def bounds_dilute(D, nbeads: int):
    """Dilute rule (eq. lmax-lmin-dilute): d_max = 2 U+.D.U+/(3N),
    d_min = U-.D.U-/(2 3N); returns (dmin, dmax)."""
    D = _f64(D)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _L().orc_bounds_dilute(int(nbeads), _ptr(D), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


# ------------------------------------------------------------ forces/update
def spring_forces(pos, nchains: int, bpc: int) -> np.ndarray:
    """Hookean spring forces F_mu = Q_mu - Q_{mu-1} (section "Governing equation")."""
    pos = _f64(pos)
    F = np.empty_like(pos)
    _L().orc_spring_forces(int(nchains), int(bpc), _ptr(pos), _ptr(F))
    return F


def ev_forces(pos, L, zstar, dstar, rcut) -> np.ndarray:
    """Narrow-Gaussian excluded-volume forces over all images within rcut."""
    pos = _f64(pos)
    rt = wrap(pos, L)
    F = np.zeros_like(pos)
    _L().orc_ev_forces(pos.shape[0], _ptr(rt), L, zstar, dstar, rcut, _ptr(F))
    return F


def euler(pos, dt, ud, ds) -> np.ndarray:
    """r + (dt/4) D.F + dS/sqrt(2) (eq. sde, kappa = 0)."""
    pos, ud, ds = _f64(pos), _f64(ud), _f64(ds)
    out = np.empty_like(pos)
    _L().orc_euler(pos.size, _ptr(pos), dt, _ptr(ud), _ptr(ds), _ptr(out))
    return out


def chain_observables(pos, nchains: int, bpc: int):
    """Per-chain (R_e^2, R_g^2) (section "Testing and verification")."""
    pos = _f64(pos)
    re2, rg2 = np.empty(nchains), np.empty(nchains)
    _L().orc_chain_observables(int(nchains), int(bpc), _ptr(pos), _ptr(re2), _ptr(rg2))
    return re2, rg2


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block (Salmon et al., SC'11)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _L().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def gaussian_noise(count: int, seed: int, step: int, dt: float) -> np.ndarray:
    """dW ~ N(0, dt) from Philox4x32-10 + Box-Muller (mapping documented in C)."""
    out = np.empty(int(count))
    _L().orc_gaussian_noise(int(count), ctypes.c_uint64(seed), ctypes.c_uint64(step),
                            dt, _ptr(out))
    return out


# --------------------------------------------------------------- full step
def bd_step(pos, *, nchains, bpc, L, a, alpha, rc, n2max, dt, nch, dmin=None,
            dmax=None, bounds_C=None, dw=None, seed=0, step=0, ev=None):
    """One Euler step (eq. sde) with Fixman-Chebyshev noise: forces, D,
    drift D.F, bounds (explicit or the paper's rule), dS, update.

    Returns dict with new positions, drift, dS, dW, dmin, dmax, E_f."""
    pos = _f64(pos)
    n = pos.shape[0]
    D = diffusion_matrix(pos, L, a, alpha, rc, n2max)
    F = spring_forces(pos, nchains, bpc)
    if ev is not None:
        F = F + ev_forces(pos, L, ev["zstar"], ev["dstar"], ev["rcut"])
    ud = matvec(D, F.reshape(1, -1)).reshape(n, 3)
    if dmin is None or dmax is None:
        dmin, dmax = bounds_rule(D, n, bounds_C)
    if dw is None:
        dw = gaussian_noise(3 * n, seed, step, dt)
    dw = _f64(dw).reshape(n, 3)
    ds = cheb_sqrt(D, dw.reshape(1, -1), nch, dmin, dmax).reshape(n, 3)
    ef = sqrt_error(D, dw, ds)
    new = euler(pos, dt, ud, ds)
    return {"pos": new, "drift": ud, "ds": ds, "dw": dw, "dmin": dmin,
            "dmax": dmax, "ef": ef, "F": F}


# ---------------------------------------------------------- differentiation
def u_forward(pos, L, a, alpha, rc, n2max, F, dw, nch, dmin, dmax) -> np.ndarray:
    """u = D(R) F + p(D(R)) dW: the drift product plus the Chebyshev sum of
    eq. cheb1-cheb3 on a fixed interval (the quantity whose reverse mode
    u_vjp computes)."""
    D = diffusion_matrix(pos, L, a, alpha, rc, n2max)
    n3 = D.shape[0]
    return (matvec(D, _f64(F).reshape(1, n3)) +
            cheb_sqrt(D, _f64(dw).reshape(1, n3), nch, dmin, dmax)).reshape(-1, 3)


def u_vjp(pos, L, a, alpha, rc, n2max, F, dw, g, nch, dmin, dmax, rows=None):
    """Reverse mode of u_forward for L = g.u: (dL/dR for the listed beads
    [len(rows), 3] (all beads when rows is None), dL/dF = D g [N, 3]).
    Pair-term derivatives of eq. M1, b1/b2, cor5 and M2 written out in
    rpy_oracle.c; the interval is held fixed."""
    pos = _f64(pos)
    n = pos.shape[0]
    r = np.arange(n, dtype=np.intc) if rows is None else np.asarray(rows, dtype=np.intc)
    r = np.ascontiguousarray(r)
    gpos = np.zeros((len(r), 3))
    gF = np.zeros((n, 3))
    _L().orc_u_vjp_rows(n, _ptr(pos), L, a, alpha, rc, int(n2max), _ptr(_f64(F)),
                        _ptr(_f64(dw)), _ptr(_f64(g)), int(nch), dmin, dmax, len(r),
                        r.ctypes.data_as(_ip), _ptr(gpos), _ptr(gF))
    return gpos, gF

