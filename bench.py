"""Benchmark: Brownian-dynamics steps per second at N = 4000 beads.

One step = the whole hot path of the semidilute Ewald-RPY Brownian-dynamics
method (arXiv:1203.6208): wrap + cell list + spring and excluded-volume
forces, real-space tile build of D, the FP64 drift product D.F, the
Chebyshev interval, the Fixman-Chebyshev products for sqrt(D).dW (each the
stored real-space tiles plus the reciprocal sum), device noise and the Euler
update.  Inputs are resident in HBM before the timed region starts.

The headline `value` is the plain FP64 step at a stated accuracy of the
square root: N_Ch from eq. nint, raised one term at a time until E_f < 1e-2
(the paper's procedure, run on the device with no host synchronisation),
on the interval of an FP64 Lanczos estimate of the extreme eigenvalues
(5% margin) that is refreshed every 50 steps inside the timed region.  The
fixed-order steps (N_Ch = 30 on the paper's bound rule, the configuration
of the previous headline, and the paper's rule with the adaptive order) are
reported beside it with their E_f; the FP32 and BF16 product forms under
`forms`, with their errors against the FP64 oracle.  `roofline` is for the
dominant kernel (the one-vector packed tile product), timed live with HIP
events on the stream the library launches on.  `cpu_baseline` times the CPU
oracle on a bounded sample of the same step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Bytes moved by one tile-product launch at N = 4000, from two rocprofv3
# counter runs (FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000, scale factors
# calibrated on 1 GiB device copies in the same process).  FETCH_SIZE counts
# what the L2 fetches over the fabric, Infinity-Cache hits included.  Valid only for the
# kernel source they were measured on (sha256 of the kernel's source files);
# otherwise reported as null.
TRAFFIC = {"src_sha256": "9708caa00cf7f2dfb4401bcffc1e9d40314e85844f0a5881ae71da0b2507a829",
           "files": ("rpy_apply.hip", "rpy_sf.h", "rpy_internal.h"),
           "bytes_per_launch": 404568114}
# The matrix-core tile kernel (k_block_tiles) of a 16-vector product: tile and
# vector reads plus the per-tile FP64/FP32 partial sums it writes.
TRAFFIC_BLOCK = {"src_sha256": "a8c5b8b032e98909eaaa0615d5f4e928507f6de593cdc81e6e8dc0c21f087a7d",
                 "files": ("rpy_block.hip", "rpy_internal.h"),
                 "bytes_per_launch": {"f64": 420300874 + 97542144,
                                      "f32": 215952215 + 48771689,
                                      "bf16": 111220975 + 48771088}}
# The batched FP32 tile product over the 256-box ensemble (k_bsymv<64, float, 1>),
# same calibration (FETCH x 2.0, WRITE x 1.0).
TRAFFIC_BATCH = {"src_sha256": "3f4d6f7ef76d80f5d4d67d3389d5c42216a1e5d5650dc93e70b33bf6bf01bfda",
                 "files": ("rpy_batch.hip", "rpy_internal.h"),
                 "bytes_per_launch": 4845338478}
METRIC = "BD steps/s at N=4000 (Ewald-RPY D·F + Chebyshev √D·dW) vs plain FP64"
BOUNDS_C = 60.0   # C of the paper's bound rule; chosen so that d_min < lambda_min here
TOL_EF = 1e-2     # E_f tolerance of the headline's adaptive order
# E_f is measured against the FP64 quadratic form dW.D.dW; BF16 tiles leave a
# floor of about 0.02 at N = 4000, so the BF16 adaptive form asks for 3e-2.
TOL_BY_PREC = {"f64": TOL_EF, "f32": TOL_EF, "bf16": 3e-2}
N_MAX = 160       # N_Ch the context keeps (the adaptive order's largest possible)
SLACK = 12        # the adaptive search runs to eq. nint + SLACK at most (with
                  # eq. nint + 6 the paper-rule form missed E_f < 1e-2 in 12 of
                  # 250 steps: its order drifts up to nint + 6 over a refresh period)
LANCZOS_STEPS = 60
LANCZOS_MARGIN = 0.05
REFRESH = 250     # steps between Lanczos refreshes of the interval (0.25 time units at dt = 1e-3)
ORACLE_REF = os.path.join(ROOT, "tests", "golden", "n4000_oracle.npz")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=REFRESH,
                    help="timed steps (default: one Lanczos refresh period, the refresh included)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batching form (for profiling)")
    ap.add_argument("--diff-only", action="store_true",
                    help="run only the differentiation form (for profiling)")
    ap.add_argument("--lma-only", action="store_true",
                    help="run only the high/low-memory crossover study")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the eigenvalue, batching, differentiation and crossover studies")
    ap.add_argument("--oracle-table", action="store_true",
                    help="also time the CPU oracle at N = 100, 1000, 2000, 4000 on one thread "
                         "and on all threads (about a minute of host time)")
    ap.add_argument("--oracle-table-seconds", type=float, default=2.5,
                    help="host seconds per cell of the oracle table")
    ap.add_argument("--theta-steps", type=int, default=3000,
                    help="steps per state of the theta-statics grid")
    ap.add_argument("--studies-only", action="store_true",
                    help="run only the eigenvalue scaling and theta-statics studies")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a device copy of this size (HBM counter calibration)")
    return ap.parse_args()


class Stepper:
    """bd_step on one context in one of the step configurations:
      "adaptive"        Lanczos interval (refreshed every REFRESH steps, the
                        refresh counted in the step that does it) + adaptive
                        order to E_f < tol (the headline);
      "paper_fixed"     paper's rule at C = BOUNDS_C, N_Ch = w.nch;
      "paper_adaptive"  paper's rule at C = BOUNDS_C + adaptive order."""

    def __init__(self, w, prec, kind, torch, rpy, tol=TOL_EF):
        self.w, self.kind, self.rpy = w, kind, rpy
        adapt = kind != "paper_fixed"
        self.ctx = rpy.context_for(w, lowp=prec, cheb_keep=N_MAX if adapt else 0)
        self.tpos = torch.from_numpy(w.positions()).cuda()
        if kind == "paper_fixed":
            self.bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, bounds_rule=rpy.BOUNDS_PAPER,
                                         bounds_C=BOUNDS_C, prec=prec, ev=w.ev)
        elif kind == "paper_adaptive":
            # the rule fixes d_max / d_min = C N^0.6, hence eq. nint
            n0 = math.floor(math.sqrt(BOUNDS_C * w.n ** 0.6) + 0.5) + 1
            self.bp = rpy.make_bd_params(dt=w.dt, n_cheb=0, bounds_rule=rpy.BOUNDS_PAPER,
                                         bounds_C=BOUNDS_C, prec=prec, ev=w.ev, tol=tol,
                                         n_max=min(N_MAX, n0 + SLACK))
        else:
            self.bp = rpy.make_bd_params(dt=w.dt, n_cheb=0, bounds_rule=rpy.BOUNDS_EXPLICIT,
                                         prec=prec, ev=w.ev, tol=tol, n_max=N_MAX)
        self.i = 0

    def refresh(self):
        self.ctx.build(self.tpos)
        lo, hi, _, _ = self.ctx.lanczos_bounds(LANCZOS_STEPS, seed=1000 + self.i,
                                               margin=LANCZOS_MARGIN)
        self.bp.d_min, self.bp.d_max = lo, hi
        n0 = math.floor(math.sqrt(hi / lo) + 0.5) + 1   # eq. nint
        self.bp.n_max = min(N_MAX, n0 + SLACK)

    def step(self, seed, e_f=None):
        if self.kind == "adaptive" and self.i % REFRESH == 0:
            self.refresh()
        self.ctx.step(self.tpos, self.bp, seed=seed, step=self.i, e_f=e_f)
        self.i += 1


def time_form(w, prec, steps, warmup, torch, rpy, kind="adaptive"):
    """Steps/s of bd_step with Chebyshev products in `prec` in the step
    configuration `kind`; E_f of every timed step is kept on the device."""
    st = Stepper(w, prec, kind, torch, rpy, tol=TOL_BY_PREC[prec])
    for _ in range(warmup):
        st.step(seed=1)
    if kind != "paper_fixed":
        st.ctx.order_stats()   # forget the warm-up orders
    st.i = 0                    # the timed region starts with a refresh
    efs = torch.empty(steps, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        st.step(seed=2, e_f=efs[i:i + 1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = st.ctx.status()
    res = {"steps_per_s": steps / wall, "ms_per_step": 1e3 * wall / steps, "status": status,
           "E_f_max": float(efs.max()), "E_f_mean": float(efs.mean())}
    if kind == "paper_fixed":
        res["n_cheb"] = w.nch
    else:
        calls, mean_n, max_n, missed = st.ctx.order_stats()
        res.update({"n_cheb_mean": mean_n, "n_cheb_max": max_n, "tol": st.bp.tol,
                    "missed_tol": missed, "adaptive_calls": calls})
    if kind == "adaptive":
        res.update({"interval": [st.bp.d_min, st.bp.d_max], "lanczos_steps": LANCZOS_STEPS,
                    "refresh_every": REFRESH})
    return st, wall, res


def profile_pass(st, rpy, steps, torch):
    """The same steps with HIP event pairs around every launch, per kernel
    class (a Lanczos refresh falls outside: the pass starts mid-interval)."""
    ctx = st.ctx
    st.i = 1
    rpy.rpy_profile_enable(ctx.handle, (N_MAX + 8) * steps + 64)
    for i in range(steps):
        st.step(seed=3)
    torch.cuda.synchronize()
    out = {}
    names = {rpy.PROF_SYMV: "tile_product", rpy.PROF_SYMV_MULTI: "tile_product_2_to_4_vectors",
             rpy.PROF_BUILD: "tile_build", rpy.PROF_KSPACE: "sf_reduce",
             rpy.PROF_EPI: "kspace_epilogue", rpy.PROF_OTHER: "forces_noise_side_stream"}
    for k, nm in names.items():
        n, ms = rpy.rpy_profile_read(ctx.handle, k)
        out[nm] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / max(n, 1)}
    rpy.rpy_profile_enable(ctx.handle, 0)
    return out


def form_errors(w, torch, rpy):
    """Error of each product precision against the FP64 oracle, at the
    workload's initial state: D.F with the precision's stored tiles, and the
    N_Ch = 30 Chebyshev sum p(D) dW on the paper's interval (C = 60) for one
    dW and for the 16-vector block (the matrix-core block product in FP32 and
    BF16).  The oracle's values are read from tests/golden/n4000_oracle.npz,
    written by the oracle alone; they cover the block rows of every 8th bead,
    over which the norm-wise relative errors ||y - y_oracle|| / ||y_oracle||
    are taken.  (bd_step always takes its drift in FP64.)"""
    ref = np.load(ORACLE_REF)
    rows = torch.from_numpy(ref["rows"]).cuda()
    lo, hi, nch = float(ref["dmin"]), float(ref["dmax"]), int(ref["n_cheb"])
    pos = torch.from_numpy(w.positions()).cuda()
    dw1 = torch.from_numpy(w.noise()[0]).cuda()
    dw16 = torch.from_numpy(w.noise(m=16)).cuda()
    cuda = {k: torch.from_numpy(ref[k]).cuda() for k in ("drift", "ds1", "ds16")}

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    out = {"reference": "tests/golden/n4000_oracle.npz (CPU oracle, rows of every 8th bead)",
           "interval": [lo, hi], "n_cheb": nch, "E_f_oracle_m1": float(ref["ef1"])}
    for prec in ("f64", "f32", "bf16"):
        ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
        F = torch.empty_like(pos)
        rpy.rpy_forces(ctx.handle, pos, w.ev["zstar"], w.ev["dstar"], w.ev["rcut"], F)
        ctx.build(pos)
        y = ctx.apply(F, prec=prec).reshape(w.n, 3)
        ds1, ef1 = ctx.sqrt_apply(dw1, nch, lo, hi, prec=prec, want_ef=True)
        ds16 = ctx.sqrt_apply(dw16, nch, lo, hi, prec=prec)
        torch.cuda.synchronize()
        out[prec] = {"rel_err_DF": rel(y[rows], cuda["drift"]),
                     "rel_err_sqrtD_dW_m1": rel(ds1.reshape(w.n, 3)[rows], cuda["ds1"]),
                     "rel_err_sqrtD_dW_m16": rel(ds16.reshape(16, w.n, 3)[:, rows], cuda["ds16"]),
                     "E_f_m1": float(ef1[0])}
        del ctx
    return out


def time_block(w, prec, reps, torch, rpy):
    """sqrt(D) dW for a block of 16 dW vectors (N_Ch - 1 = 29 products of D
    with 16 vectors) on the step's D and bounds, each product one pass of the
    matrix-core block product over the packed tiles of the given precision
    (tile kernel with the vector packing, FP64 structure factors and their
    reduction, FP64 back-projection + epilogue).  Per-stage times come from
    HIP event pairs on the library's stream."""
    ctx = rpy.context_for(w, lowp=prec, max_rhs=16)
    pos = torch.from_numpy(w.positions()).cuda()
    dw16 = torch.from_numpy(w.noise(m=16)).cuda()
    ctx.build(pos)
    lo, hi = ctx.bounds(BOUNDS_C)
    for _ in range(2):
        ctx.sqrt_apply(dw16, w.nch, lo, hi, prec=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.sqrt_apply(dw16, w.nch, lo, hi, prec=prec)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    rpy.rpy_profile_enable(ctx.handle, 64 * w.nch)
    ctx.sqrt_apply(dw16, w.nch, lo, hi, prec=prec)
    torch.cuda.synchronize()
    nprod = w.nch - 1
    stage = {}
    for kinds, nm in (((rpy.PROF_SYMV, rpy.PROF_SYMV_MULTI), "tile_product"),
                      ((rpy.PROF_KSPACE,), "structure_factors"),
                      ((rpy.PROF_EPI,), "back_projection_epilogue")):
        ms = sum(rpy.rpy_profile_read(ctx.handle, k)[1] for k in kinds)
        stage[nm + "_us"] = 1e3 * ms / nprod
    rpy.rpy_profile_enable(ctx.handle, 0)
    gbs = tile_bytes(w.n, prec) / (stage["tile_product_us"] * 1e-6) / 1e9
    del ctx
    return {"ms_per_block": 1e3 * wall, "us_per_product": 1e6 * wall / nprod,
            **stage, "tile_product_GBs": gbs, "tile_product_hbm_frac": gbs / HBM_PEAK_GBS,
            "tile_product_traffic": measured_traffic(TRAFFIC_BLOCK, prec),
            "vector_products_per_s": 16 * nprod / wall}


def eigen_study(w, torch, rpy):
    """Chebyshev interval and order at the bench state (section
    "Decomposition of the diffusion tensor"): FP64 Lanczos bounds (60 steps)
    against the paper's rule at C = 8 and at the bench's C and against the
    oracle's exact extreme eigenvalues (tests/golden/n4000_oracle.npz), the
    order of eq. nint for each, and the order the adaptive procedure needs
    for E_f < 1e-2 and 1e-3 on one dW with the Lanczos interval."""
    ref = np.load(ORACLE_REF)
    ctx = rpy.context_for(w, max_rhs=1, cheb_keep=256)
    pos = torch.from_numpy(w.positions()).cuda()
    ctx.build(pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lo, hi, _, _ = ctx.lanczos_bounds(LANCZOS_STEPS, seed=1, margin=LANCZOS_MARGIN)
    t_lz = time.perf_counter() - t0
    out = {"exact_oracle": {"lambda_min": float(ref["lam_min"]), "lambda_max": float(ref["lam_max"]),
                            "n_cheb_rule": math.floor(math.sqrt(ref["lam_max"] / ref["lam_min"])
                                                      + 0.5) + 1},
           f"lanczos_{LANCZOS_STEPS}": {"d_min": lo, "d_max": hi, "seconds": t_lz,
                                        "margin": LANCZOS_MARGIN,
                                        "n_cheb_rule": math.floor(math.sqrt(hi / lo) + 0.5) + 1}}
    for C in (8.0, BOUNDS_C):
        a, b = ctx.bounds(C)
        out[f"paper_rule_C{C:g}"] = {"d_min": a, "d_max": b,
                                     "n_cheb_rule": math.floor(math.sqrt(b / a) + 0.5) + 1}
    a, b = ctx.bounds(0.0, rule=rpy.BOUNDS_DILUTE)
    out["dilute_rule"] = {"d_min": a, "d_max": b,
                          "n_cheb_rule": math.floor(math.sqrt(b / a) + 0.5) + 1}
    dw = torch.from_numpy(w.noise()[0]).cuda()
    for tol in (1e-2, 1e-3):
        _, ef, n = ctx.sqrt_apply(dw, 256, lo, hi, tol=tol, want_ef=True, want_n=True,
                                  allow_etol=True)
        out[f"adaptive_tol_{tol:g}"] = {"n_cheb": n, "E_f": float(ef[0])}
    del ctx
    return out


def trajectory_n1000(torch, rpy, inputs, steps=1000, refresh=100):
    """The N = 1000 workload (40 chains x 25 beads, c/c* = 1, alpha r_c =
    4.6): `steps` FP64 steps with D rebuilt every step, N_Ch = 30 on a
    Lanczos interval (60 steps, 5% margin) refreshed every `refresh` steps,
    device noise.  Steps/s, the E_f of every step, the status, and the chain
    averages of R_e^2 and R_g^2 (section "Testing and verification") at the
    start and at the end.  Its first five steps are compared with the oracle
    trajectory in tests/test_gpu_fullsize.py."""
    w = inputs.workload("n1000")
    ctx = rpy.context_for(w)
    tpos = torch.from_numpy(w.positions()).cuda()
    bp = rpy.make_bd_params(dt=w.dt, n_cheb=w.nch, bounds_rule=rpy.BOUNDS_EXPLICIT)
    re0, rg0 = ctx.observables(tpos)
    efs = torch.empty(steps, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i % refresh == 0:
            ctx.build(tpos)
            lo, hi, _, _ = ctx.lanczos_bounds(LANCZOS_STEPS, seed=2000 + i, margin=LANCZOS_MARGIN)
            bp.d_min, bp.d_max = lo, hi
        ctx.step(tpos, bp, seed=11, step=i, e_f=efs[i:i + 1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    re2, rg2 = ctx.observables(tpos)
    st = ctx.status()
    del ctx
    return {"workload": "n1000: 40 x 25 beads, c/c*=1, h*=0.28, theta (no EV), alpha L=6, "
                        "alpha r_c=4.6, N_Ch=30, dt=1e-3",
            "steps": steps, "seconds": wall, "steps_per_s": steps / wall, "status": st,
            "lanczos_refresh_every": refresh, "E_f_max": float(efs.max()),
            "E_f_mean": float(efs.mean()),
            "Re2_mean": [float(re0.mean()), float(re2.mean())],
            "Rg2_mean": [float(rg0.mean()), float(rg2.mean())],
            "Re2_theta": 3.0 * (w.bpc - 1), "Rg2_theta": inputs.theta_rg2(w.bpc)}


EIGEN_SIZES = (100, 200, 400, 1000, 2000, 4000)
EIGEN_REPLICAS = 3
EIGEN_LANCZOS = 1500
THETA_BPC = (20, 40)
THETA_CONC = (3e-4, 3e-3, 3e-2, 0.3, 1.0, 3.0)


def ritz_extremes(alpha, beta):
    """Extreme Ritz values of a k-step Lanczos run and their residual bounds
    |beta_k s_k| (s_k the last component of the unit Ritz vector): the
    tridiagonal has diagonal alpha[0..k-1] and off-diagonal beta[0..k-2];
    beta[k-1] is the norm of the last residual."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    k = len(a)
    T = np.diag(a) + np.diag(b[:k - 1], 1) + np.diag(b[:k - 1], -1)
    ev, vec = np.linalg.eigh(T)   # k <= 512: the dense solver is cheap and robust
    return (float(ev[0]), float(ev[-1]), abs(b[k - 1] * vec[-1, 0]),
            abs(b[k - 1] * vec[-1, -1]))


def power_fit(ns, ys):
    """Least-squares fit y = A N^p on log-log axes: (p, A)."""
    p, la = np.polyfit(np.log(np.asarray(ns, dtype=np.float64)),
                       np.log(np.asarray(ys, dtype=np.float64)), 1)
    return float(p), float(math.exp(la))


def eigen_scaling(torch, rpy, inputs, sizes=EIGEN_SIZES, replicas=EIGEN_REPLICAS,
                  n_iter=EIGEN_LANCZOS):
    """How the extreme eigenvalues of D grow with N at the state of the
    paper's eigenvalue study (section "Decomposition of the diffusion
    tensor": N_b = 10, c = 4.44 c*, a = 0.5): for each N and start
    conformation, lambda_max and lambda_min of D from an FP64 Lanczos run
    (min(`n_iter`, 2N) steps in the 3N-dimensional space, extreme Ritz values
    with their residual bounds), and
    Fixman's estimates lambda^F = U.D.U / 3N with U = U+ and U- (eq.
    lmax-lmin-dilute, from the dilute rule's interval: d_max = 2 lambda^F_max,
    d_min = lambda^F_min / 2).  Fits lambda_max / lambda^F_max = A N^p
    (eq. fmax: 0.35 N^0.6) and lambda_max / lambda_min = C N^q (eq. fmin:
    C = 8, q = 0.6), and the prefactors with the exponent held at 0.6."""
    states = []
    for n in sizes:
        for r in range(replicas):
            w = inputs.eigen_state(n, r)
            ctx = rpy.context_for(w, max_rhs=2)
            ctx.build(torch.from_numpy(w.positions()).cuda())
            a, b = ctx.bounds(0.0, rule=rpy.BOUNDS_DILUTE)
            _, _, al, be = ctx.lanczos_bounds(min(n_iter, 2 * n), seed=7 + r, margin=0.0)
            del ctx
            tmin, tmax, rmin, rmax = ritz_extremes(al, be)
            states.append({"N": n, "replica": r, "L": w.L, "lambda_min": tmin,
                           "lambda_max": tmax, "residual_min": rmin, "residual_max": rmax,
                           "lambda_max_fixman": 0.5 * b, "lambda_min_fixman": 2.0 * a,
                           "max_over_fixman": tmax / (0.5 * b), "max_over_min": tmax / tmin})
    ns = [s["N"] for s in states]
    p1, a1 = power_fit(ns, [s["max_over_fixman"] for s in states])
    p2, c2 = power_fit(ns, [s["max_over_min"] for s in states])
    pf, lf = power_fit(ns, [s["lambda_max_fixman"] for s in states])
    pm, lm = power_fit(ns, [s["lambda_min"] for s in states])
    at06 = lambda key: float(np.mean([s[key] / s["N"] ** 0.6 for s in states]))
    return {"state": "N_b=10, c=4.44 c*, a=0.5, theta conformations (random walks), "
                     "alpha L=6, alpha r_c=3.5",
            "lanczos_steps": n_iter, "replicas": replicas, "states": states,
            "fit": {"max_over_fixman": {"exponent": p1, "prefactor": a1,
                                        "prefactor_at_0.6": at06("max_over_fixman")},
                    "max_over_min": {"exponent": p2, "prefactor": c2,
                                     "prefactor_at_0.6": at06("max_over_min")},
                    "lambda_max_fixman": {"exponent": pf, "prefactor": lf},
                    "lambda_min": {"exponent": pm, "prefactor": lm}},
            "paper": {"max_over_fixman": "0.35 N^0.6 (eq. fmax)",
                      "max_over_min": "C N^0.6, C = 8 at this state (eq. fmin)"}}


def theta_statics(torch, rpy, inputs, steps=3000, replicas=2, every=10, refresh=250,
                  tol=TOL_EF, bpcs=THETA_BPC, concs=THETA_CONC):
    """Theta-solvent statics on the paper's grid (section "Testing and
    verification", theta solvents): N_c = 20 chains of N_b = 20 and 40
    beads, a = 0.5, dt = 0.01, c/c* from 3e-4 to 3 by the box length, FP64
    with hydrodynamic interaction, N_Ch by eq. nint raised until E_f < tol on
    a Lanczos interval (80 steps, margin 0.2) refreshed every `refresh`
    steps; `replicas` independent boxes per state.  The start is an
    equilibrium sample, so every window of the run samples equilibrium;
    <R_e^2> and <R_g^2> are averaged over time (every `every` steps) and
    chains, with the standard error from the spread of the per-chain
    averages over all replicas, against eq. Re2 and Rg2.  The runs are
    shorter than the longest relaxation time of a 40-bead chain, so the
    averages stay close to those of the start conformations (`*_start`,
    same chains at t = 0), which carry the sampling error of the start: the
    per-chain R_g^2 of a 40-bead random walk has a relative spread of about
    0.5 and a long upper tail, so a low sample mean comes with a small
    sample spread (for 20 start chains drawn from the generator, the mean
    lies more than 2 standard errors below the exact value in 6% of draws,
    where a normal sample would give 2.3%)."""
    out = []
    for bpc in bpcs:
        for cc in concs:
            series = {"Re2": [], "Rg2": []}
            start = {"Re2": [], "Rg2": []}
            res = {"N_b": bpc, "c_over_cstar": cc, "steps": steps, "replicas": replicas,
                   "seconds": 0.0, "n_cheb_mean": 0.0, "n_cheb_max": 0, "missed_tol": 0,
                   "E_f_max": 0.0, "status": []}
            for rep in range(replicas):
                w = inputs.theta_state(bpc, cc, replica=rep)
                res["N"], res["L"] = w.n, w.L
                ctx = rpy.context_for(w, cheb_keep=N_MAX)
                pos = torch.from_numpy(w.positions()).cuda()
                bp = rpy.make_bd_params(dt=w.dt, n_cheb=0, bounds_rule=rpy.BOUNDS_EXPLICIT,
                                        tol=tol, n_max=N_MAX)
                ns = steps // every
                re2 = torch.empty((ns, w.nchains), dtype=torch.float64, device="cuda")
                rg2 = torch.empty_like(re2)
                efs = torch.empty(steps, dtype=torch.float64, device="cuda")
                re0, rg0 = ctx.observables(pos)
                start["Re2"].append(re0.cpu().numpy())
                start["Rg2"].append(rg0.cpu().numpy())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i in range(steps):
                    if i % refresh == 0:
                        ctx.build(pos)
                        lo, hi, _, _ = ctx.lanczos_bounds(80, seed=300 + i, margin=0.2)
                        bp.d_min, bp.d_max = lo, hi
                        bp.n_max = min(N_MAX, math.floor(math.sqrt(hi / lo) + 0.5) + 1 + SLACK)
                    ctx.step(pos, bp, seed=17 + rep, step=i, e_f=efs[i:i + 1])
                    if (i + 1) % every == 0:
                        r = (i + 1) // every - 1
                        ctx.observables(pos, re2[r], rg2[r])
                torch.cuda.synchronize()
                res["seconds"] += time.perf_counter() - t0
                calls, mean_n, max_n, missed = ctx.order_stats()
                res["n_cheb_mean"] += mean_n / replicas
                res["n_cheb_max"] = max(res["n_cheb_max"], max_n)
                res["missed_tol"] += missed
                res["E_f_max"] = max(res["E_f_max"], float(efs.max()))
                res["status"].append(ctx.status())
                series["Re2"].append(re2.mean(dim=0).cpu().numpy())
                series["Rg2"].append(rg2.mean(dim=0).cpu().numpy())
                del ctx
            res["steps_per_s"] = steps * replicas / res["seconds"]
            for nm, exact in (("Re2", 3.0 * (bpc - 1)), ("Rg2", inputs.theta_rg2(bpc))):
                per_chain = np.concatenate(series[nm])
                mean = float(per_chain.mean())
                se = float(per_chain.std(ddof=1) / math.sqrt(len(per_chain)))
                res[nm] = mean
                res[nm + "_se"] = se
                res[nm + "_exact"] = exact
                res[nm + "_dev_in_se"] = (mean - exact) / se
                res[nm + "_start"] = float(np.concatenate(start[nm]).mean())
            out.append(res)
    return {"states": out, "tol": tol, "every": every, "lanczos_refresh_every": refresh}


def batch_study(torch, rpy, inputs, steps=5, per_box=True):
    """Batching form: the 256-box ragged ensemble (N 125..1989 in whole chains
    of 10..50 beads, c/c* 0.5..3, no excluded volume), FP64 core with FP32
    Chebyshev products (N_Ch = 30, paper rule), every step one HIP graph
    replay.  Tile size, structure-factor placement and tile-load policy from
    the autotuner (its whole table is reported), compared with both fixed
    tile sizes in the default variant;
    the same ensemble with FP64 products, and box by box through the
    single-box library (FP64, one bd_step per box) as the plain baseline.
    Throughput is aggregate box-steps/s (boxes x steps / s)."""
    from paper_1203_6208_amd import autotune
    ws = inputs.batch_boxes()
    nbox = len(ws)
    beads = sum(w.n for w in ws)
    bp32 = rpy.make_bd_params(dt=1e-3, n_cheb=30, bounds_rule=rpy.BOUNDS_PAPER,
                              bounds_C=BOUNDS_C, prec="f32")
    bp64 = rpy.make_bd_params(dt=1e-3, n_cheb=30, bounds_rule=rpy.BOUNDS_PAPER,
                              bounds_C=BOUNDS_C, prec="f64")
    pos_np = [w.positions() for w in ws]
    t0 = time.perf_counter()
    best, times = autotune.tune_batch(ws, bp32, lowp="f32", steps=3, positions=pos_np)
    t_tune = time.perf_counter() - t0
    table = [dict(c.as_dict(), ms_per_step=1e3 * t, box_steps_per_s=nbox / t)
             for c, t in sorted(times.items(), key=lambda kv: kv[1])]
    out = {"boxes": nbox, "beads": beads, "n_cheb": 30,
           "autotune": {"best": best.as_dict(), "seconds_tuning": t_tune,
                        "search_space": "tile_beads {32, 64} x sf_place {spread, front} x "
                                        "tile_loads {stream, cached}, 3 graph replays each",
                        "table": table}}

    def graph_rate(lowp, bp, config):
        B = autotune.make_batch(ws, config, lowp=lowp)
        pos = B.pack(pos_np)
        B.run(pos, bp, seed=1, step0=0, n_steps=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.run(pos, bp, seed=1, step0=1, n_steps=steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = B.status()
        return B, pos, wall / steps, st

    B, pos, sec, st = graph_rate("f32", bp32, best)
    out["f32_autotuned"] = {"box_steps_per_s": nbox / sec, "ensemble_steps_per_s": 1.0 / sec,
                            "ms_per_step": 1e3 * sec, "status": st, **best.as_dict(),
                            "graph_nodes_per_step": B.graph_nodes()}
    # one FP32 product (tile kernel + reduction + back-projection) timed with events
    v = B.pack([np.ones((w.n, 3)) for w in ws], m=1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    B.apply(v, prec="f32")
    e0.record()
    for _ in range(5):
        B.apply(v, prec="f32")
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / 5
    alg = sum(3 * w.n * (w.n + 1) for w in ws) * 4   # packed symmetric 3 x 3 blocks, FP32
    out["f32_product"] = {"us": us, "algorithmic_bytes": alg,
                          "GBs": alg / (us * 1e-6) / 1e9,
                          "hbm_frac": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                          "tile_kernel_traffic_bytes": (measured_traffic(TRAFFIC_BATCH)
                                                        if best == autotune.Config() else None)}
    # accuracy of the FP32 form on one step against FP64 products (same state)
    B64 = autotune.make_batch(ws, best, lowp="f64")
    p64 = B64.pack(pos_np)
    p32 = B.pack(pos_np)
    d64, n64, _ = B64.step(p64, bp64, seed=5, step=0, want=True)
    d32, n32, _ = B.step(p32, bp32, seed=5, step=0, want=True)
    torch.cuda.synchronize()
    e_n = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
              for a, b in zip(B.unpack(n32), B64.unpack(n64)))
    e_d = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
              for a, b in zip(B.unpack(d32), B64.unpack(d64)))
    out["f32_vs_f64_max_box_rel_err"] = {"dS": e_n, "drift": e_d}
    del B, B64, pos, p64, p32
    for tb in (32, 64):   # fixed tiles with the default variant
        fixed = autotune.Config(tile_beads=tb)
        if fixed == best:
            out[f"f32_fixed_tile{tb}"] = dict(out["f32_autotuned"])
            continue
        Bx, px, sx, stx = graph_rate("f32", bp32, fixed)
        out[f"f32_fixed_tile{tb}"] = {"box_steps_per_s": nbox / sx, "ms_per_step": 1e3 * sx}
        del Bx, px
    Bd, pd, sd, std = graph_rate("f64", bp64, best)
    out["f64_batched"] = {"box_steps_per_s": nbox / sd, "ms_per_step": 1e3 * sd, "status": std}
    del Bd, pd
    torch.cuda.empty_cache()
    if per_box:
        ctxs = [rpy.context_for(w) for w in ws]
        tp = [torch.from_numpy(p).cuda() for p in pos_np]
        bps = [rpy.make_bd_params(dt=1e-3, n_cheb=30, bounds_rule=rpy.BOUNDS_PAPER,
                                  bounds_C=BOUNDS_C, prec="f64") for _ in ws]
        for c, p, b in zip(ctxs, tp, bps):
            c.step(p, b, seed=1, step=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c, p, b in zip(ctxs, tp, bps):
            c.step(p, b, seed=1, step=1)
        torch.cuda.synchronize()
        sp = time.perf_counter() - t0
        out["f64_box_by_box"] = {"box_steps_per_s": nbox / sp, "ms_per_ensemble_step": 1e3 * sp}
        for c in ctxs:
            c.close()
        del ctxs, tp
    out["speedup_autotuned_f32_vs_box_by_box_f64"] = (
        out["f32_autotuned"]["box_steps_per_s"] / out["f64_box_by_box"]["box_steps_per_s"]
        if per_box else None)
    return out


def diff_study(torch, rpy, inputs, n_steps=100, every=10):
    """Differentiation form at N = 2000 (40 chains x 50 beads, c/c* = 1,
    narrow-Gaussian excluded volume): the mean-square displacement after a
    100-step trajectory and its gradient with respect to the initial
    positions and a spring-stiffness factor, through torch.autograd with a
    checkpoint every 10 steps.  The Chebyshev interval is fixed for the
    trajectory (60-step Lanczos bounds at the start, 5% margin).  Reports
    forward and backward wall times, their ratio, the plain library step
    (bd_step, FP64) for comparison, peak device memory, and the gradient's
    agreement with central differences of the GPU forward along 4 directions
    that move 100 beads each."""
    from paper_1203_6208_amd import diff
    w = inputs.workload("n2000")
    nch = w.nch
    rc = rpy.context_for(w, max_rhs=16, cheb_keep=nch, grad=1)
    pos0 = torch.from_numpy(w.positions()).cuda()
    rc.build(pos0)
    lo, hi, _, _ = rc.lanczos_bounds(60, seed=1, margin=0.05)
    ev = dict(w.ev)
    dt = w.dt

    def run(p0, k, every_):
        return diff.trajectory(p0, rc, n_steps, dt, nch, lo, hi, seed=9, ev=ev, spring=k,
                               every=every_)

    one = torch.tensor(1.0, dtype=torch.float64, device="cuda")
    with torch.no_grad():                       # warm-up and no-grad forward
        run(pos0, one, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(pos0, one, 0)
        torch.cuda.synchronize()
        t_nograd = time.perf_counter() - t0
    def grad_pass(every_):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        p0 = pos0.clone().requires_grad_(True)
        k = one.clone().requires_grad_(True)
        t0 = time.perf_counter()
        m = diff.msd(run(p0, k, every_), p0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return (float(m.detach()), float(k.grad), p0.grad.detach(), t1 - t0, t2 - t1,
                (torch.cuda.max_memory_allocated() - base) / 1e6)

    grad_pass(every)                            # warm-up (first-use costs)
    mval, kgrad, gp, t_fwd, t_bwd, peak = grad_pass(every)
    _, _, gp0, t_fwd0, t_bwd0, peak0 = grad_pass(0)
    same = bool(torch.equal(gp, gp0))
    # plain library step for comparison
    bp = rpy.make_bd_params(dt=dt, n_cheb=nch, bounds_rule=rpy.BOUNDS_EXPLICIT, d_min=lo,
                            d_max=hi, ev=ev)
    pp = pos0.clone()
    rc.step(pp, bp, seed=1, step=0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for i in range(n_steps):
        rc.step(pp, bp, seed=1, step=i)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t3
    # u-term gradient against central differences (sparse directions)
    rng = np.random.default_rng(3)
    pos = w.positions()
    F = torch.from_numpy(rng.standard_normal((w.n, 3))).cuda()
    dW = torch.from_numpy(rng.standard_normal((w.n, 3)) * math.sqrt(dt)).cuda()
    g = torch.from_numpy(rng.standard_normal((w.n, 3))).cuda()
    gpos = torch.empty_like(pos0)
    rpy.rpy_u_vjp(rc.handle, pos0, F, dW, g, nch, lo, hi, gpos, None, None)
    u = torch.empty_like(pos0)
    errs = []
    h = 1e-6
    for _ in range(4):
        moved = rng.choice(w.n, size=100, replace=False)
        e = np.zeros(pos.shape)
        e[moved] = rng.standard_normal((100, 3))
        te = torch.from_numpy(e).cuda()
        rpy.rpy_u_forward(rc.handle, pos0 + h * te, F, dW, nch, lo, hi, u)
        lp = float(torch.sum(g * u))
        rpy.rpy_u_forward(rc.handle, pos0 - h * te, F, dW, nch, lo, hi, u)
        lm = float(torch.sum(g * u))
        an = float(torch.sum(gpos * te))
        errs.append(abs((lp - lm) / (2 * h) - an) / float(torch.sum(torch.abs(gpos * te))))
    rc.close()
    return {"workload": "n2000: 40 x 50 beads, c/c*=1, EV z*=1 d*=0.5, N_Ch=30, dt=1e-3",
            "steps": n_steps, "checkpoint_every": every, "msd": mval,
            "d_msd_d_spring": kgrad, "grad_pos_norm": float(torch.linalg.norm(gp)),
            "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
            "peak_mem_MB": peak,
            "no_checkpoint": {"forward_s": t_fwd0, "backward_s": t_bwd0,
                              "backward_over_forward": t_bwd0 / t_fwd0, "peak_mem_MB": peak0,
                              "same_gradient_bits": same},
            "forward_nograd_s": t_nograd, "plain_bd_step_s": t_plain,
            "fd_check_u_term": {"directions": 4, "h": h, "max_rel_err": max(errs),
                                "note": "directions move 100 beads; see the differentiation "
                                        "tests for the cutoff-crossing rule"}}


def lma_study(torch, rpy, inputs, sizes=(2000, 8000, 16000, 32000)):
    """High-memory (stored real-space tiles, alpha L = 6) against low-memory
    (matrix-free cell-list recomputation, alpha L = 12 and 14) forms at
    c/c* = 1 with 50-bead chains: FP64 product (m = 1) and build times from
    HIP events on the library's stream, a full bd_step (N_Ch = 30, paper
    rule), the bytes the stored form keeps, and the relative difference of
    D.v between the two forms (both truncate the same Ewald sum at
    M = 3.5, so they agree to the truncation error, not to rounding)."""
    out = []
    for n in sizes:
        row = {"N": n}
        forms = {"hma": (6.0, 0), "lma_aL12": (12.0, 1), "lma_aL14": (14.0, 1)}
        ref = None
        for name, (aL, lma) in forms.items():
            w = inputs.Workload(f"x{n}", n // 50, 50, 1.0, alphaL=aL, nch=30,
                                seed=inputs.POSITION_SEED_BASE + 500 + n)
            ctx = rpy.context_for(w, lma=lma)
            pos = torch.from_numpy(w.positions()).cuda()
            v = torch.from_numpy(np.random.default_rng(1).standard_normal((1, w.n, 3))).cuda()
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            ctx.build(pos)
            y = ctx.apply(v)
            torch.cuda.synchronize()
            e0.record()
            ctx.build(pos)
            e1.record()
            for _ in range(5):
                y = ctx.apply(v)
            e2.record()
            torch.cuda.synchronize()
            bp = rpy.make_bd_params(dt=1e-3, n_cheb=30, bounds_rule=rpy.BOUNDS_PAPER,
                                    bounds_C=BOUNDS_C)
            p2 = pos.clone()
            ctx.step(p2, bp, seed=1, step=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(3):
                ctx.step(p2, bp, seed=1, step=i)
            torch.cuda.synchronize()
            st = (time.perf_counter() - t0) / 3
            rec = {"alphaL": aL, "n_k_half": ctx.num_kvectors(),
                   "build_ms": e0.elapsed_time(e1), "product_ms": e1.elapsed_time(e2) / 5,
                   "step_ms": 1e3 * st,
                   "stored_GB": 0.0 if lma else tile_bytes(n, "f64") / 1e9}
            if ref is None:
                ref = y
            else:
                rec["rel_diff_vs_hma"] = float(torch.max(torch.abs(y - ref)) /
                                               torch.max(torch.abs(ref)))
            row[name] = rec
            ctx.close()
            del ctx, y
            torch.cuda.empty_cache()
        out.append(row)
        print(f"# lma {row}", file=sys.stderr, flush=True)
    return out


def cpu_baseline(w, seconds):
    """Oracle on a bounded sample of one step: block rows of D (real space,
    self term, reciprocal sum over the full +-k set) for a subset of beads, and
    the 31 dense row-times-vector products of those rows; scaled to N beads."""
    import oracle
    oracle.build(force=False)
    pos = w.positions()
    rng = np.random.default_rng(0)
    v = rng.standard_normal(3 * w.n)

    def sample(nb):
        rows = np.linspace(0, w.n - 1, nb).astype(int)
        t0 = time.perf_counter()
        R = oracle.diffusion_rows(pos, rows, w.L, w.a, w.alpha, w.rc, w.n2max)
        t1 = time.perf_counter()
        for _ in range(2 + w.nch - 1):
            oracle.rows_matvec(R, v)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    # the oracle's loops are parallel over rows: probe with one row per thread
    threads = oracle.max_threads()
    p = min(w.n, max(4, threads))
    tb, tm = sample(p)
    per_bead = (tb + tm) / p
    nb = int(max(p, min(w.n, seconds / max(per_bead, 1e-9))))
    tb, tm = sample(nb)
    t_step = (tb + tm) * w.n / nb
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"D block rows of {nb} of {w.n} beads (real space + self + reciprocal "
                       f"over 1236 k, brute force) plus {2 + w.nch - 1} row-block products; "
                       f"{tb + tm:.1f} s measured, scaled by N/{nb}; forces and update omitted "
                       f"(O(N))")}


def host_description():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def oracle_table(seconds):
    """The oracle's cost on the host, on one thread and on all of its threads,
    for the workloads of N = 100, 1000, 2000 and 4000 beads: one build of D
    (real-space sum, self term and the reciprocal sum over the full +-k set),
    one product D.v, one sqrt(D).dW (N_Ch - 1 products) for 1 and 16 vectors,
    and one step (build + 2 + N_Ch - 1 products; forces and update are O(N)
    and left out).  Rows of D are sampled at evenly spaced beads (all rows
    where that fits the time per cell) and the times scaled by N / rows; the
    products are the oracle's plain row loops on the sampled rows, scaled the
    same way."""
    import oracle
    from paper_1203_6208_amd import inputs
    oracle.build(force=False)
    allth = oracle.max_threads()
    out = {"host": host_description(), "threads_all": allth,
           "seconds_per_cell": seconds, "rows": []}
    for name in ("n100", "n1000", "n2000", "n4000"):
        w = inputs.workload(name)
        pos = w.positions()
        v = np.random.default_rng(0).standard_normal(3 * w.n)

        def sample(nb):
            rows = np.linspace(0, w.n - 1, nb).round().astype(int)
            t0 = time.perf_counter()
            R = oracle.diffusion_rows(pos, rows, w.L, w.a, w.alpha, w.rc, w.n2max)
            t1 = time.perf_counter()
            reps, t2 = 0, t1
            while reps < 3 or (t2 - t1 < 0.2 and reps < 1000):
                oracle.rows_matvec(R, v)
                reps += 1
                t2 = time.perf_counter()
            return t1 - t0, (t2 - t1) / reps

        for th in sorted({1, allth}):
            oracle.use_threads(th)
            # the loops are parallel over rows: sample whole rounds of th rows
            p = min(w.n, max(2, th))
            tb, tm = sample(p)
            nb = int(seconds / max((tb + tm) / p, 1e-9))
            nb = min(w.n, max(p, nb // p * p))
            tb, tm = sample(nb)
            scale = w.n / nb
            build, prod = tb * scale, tm * scale
            row = {"workload": name, "n_beads": w.n, "n_cheb": w.nch, "threads": th,
                   "rows_sampled": nb, "build_s": build, "product_s": prod,
                   "sqrt_m1_s": (w.nch - 1) * prod, "sqrt_m16_s": 16 * (w.nch - 1) * prod,
                   "step_s": build + (2 + w.nch - 1) * prod}
            out["rows"].append(row)
            print(f"# oracle table {row}", file=sys.stderr, flush=True)
    oracle.use_threads(allth)
    return out


def tile_bytes(n, prec):
    """Algorithmic bytes one product streams, whatever the number of vectors:
    the packed tiles keep the 6 distinct entries of each symmetric 3 x 3
    bead-pair block for the N(N+1)/2 pairs i <= j."""
    esize = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    return 3 * n * (n + 1) * esize


def measured_traffic(t=TRAFFIC, key=None):
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_1203_6208_amd", "csrc", f), "rb").read()
                   for f in t["files"])
    if hashlib.sha256(src).hexdigest() != t["src_sha256"]:
        return None
    return t["bytes_per_launch"] if key is None else t["bytes_per_launch"][key]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library and this benchmark run on one GPU only (asked for --gpus "
              f"{args.gpus}); sharding across GPUs is designed, not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1203_6208_amd import inputs, rpy

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(nb, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# calibration copy: {nb * 8} bytes read and written per launch", file=sys.stderr)
        del a, b
    if args.lma_only:
        print(json.dumps({"lma": lma_study(torch, rpy, inputs)}))
        return
    if args.diff_only:
        print(json.dumps({"differentiation": diff_study(torch, rpy, inputs)}))
        return
    if args.studies_only:
        print(json.dumps({"eigen_scaling": eigen_scaling(torch, rpy, inputs),
                          "theta_statics": theta_statics(torch, rpy, inputs,
                                                         steps=args.theta_steps)}))
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_study(torch, rpy, inputs, steps=args.steps,
                                               per_box=False)}))
        return
    w = inputs.workload("n4000")
    print(f"# workload n4000 N={w.n} L={w.L:.4f} alpha={w.alpha:.5f} rc={w.rc:.4f} "
          f"n2max={w.n2max}", file=sys.stderr, flush=True)
    st, wall, head = time_form(w, "f64", args.steps, args.warmup, torch, rpy, kind="adaptive")
    ms_step = 1e3 * wall / args.steps
    value = args.steps / wall
    print(f"# f64 headline: {json.dumps(head)}", file=sys.stderr, flush=True)
    prof = profile_pass(st, rpy, min(args.steps, 20), torch)
    del st
    alg_bytes = tile_bytes(w.n, "f64")
    sym = prof["tile_product"]
    achieved = alg_bytes / (sym["avg_us"] * 1e-6) / 1e9
    print(f"# profile {json.dumps(prof)}", file=sys.stderr, flush=True)
    configs = {"adaptive_lanczos": head}
    forms = {}
    if not args.no_forms:
        for kind in ("paper_fixed", "paper_adaptive"):
            s2, _, r2 = time_form(w, "f64", args.steps, args.warmup, torch, rpy, kind=kind)
            del s2
            configs[kind] = r2
            print(f"# f64 {kind}: {json.dumps(r2)}", file=sys.stderr, flush=True)
        for prec in ("f32", "bf16"):
            forms[prec] = {}
            for kind in ("adaptive", "paper_fixed"):
                s2, _, r2 = time_form(w, prec, args.steps, args.warmup, torch, rpy, kind=kind)
                pr2 = profile_pass(s2, rpy, max(4, min(args.steps, 20) // 2), torch)
                del s2
                r2["speedup_vs_f64_same_configuration"] = (
                    r2["steps_per_s"] / configs["adaptive_lanczos" if kind == "adaptive"
                                                else kind]["steps_per_s"])
                r2["tile_product_avg_us"] = pr2["tile_product"]["avg_us"]
                r2["tile_product_GBs"] = (tile_bytes(w.n, prec)
                                          / (pr2["tile_product"]["avg_us"] * 1e-6) / 1e9)
                forms[prec][kind] = r2
                print(f"# {prec} {kind}: {json.dumps(r2)}", file=sys.stderr, flush=True)
        for prec in ("f64", "f32", "bf16"):
            forms.setdefault(prec, {})["block_m16"] = time_block(w, prec, 5, torch, rpy)
            print(f"# block m16 {prec}: {forms[prec]['block_m16']}", file=sys.stderr, flush=True)
        errs = form_errors(w, torch, rpy)
        print(f"# errors vs oracle {json.dumps(errs)}", file=sys.stderr, flush=True)
        forms["errors_vs_oracle"] = errs
    studies = not (args.no_forms or args.no_studies)
    eigen = eigen_study(w, torch, rpy) if studies else None
    if eigen:
        print(f"# eigen {eigen}", file=sys.stderr, flush=True)
    if studies:
        torch.cuda.empty_cache()
        eigen["scaling_with_N"] = eigen_scaling(torch, rpy, inputs)
        print(f"# eigen scaling {json.dumps(eigen['scaling_with_N']['fit'])}", file=sys.stderr,
              flush=True)
        forms["theta_statics"] = theta_statics(torch, rpy, inputs, steps=args.theta_steps)
        print(f"# theta statics {json.dumps(forms['theta_statics'])}", file=sys.stderr,
              flush=True)
        traj = trajectory_n1000(torch, rpy, inputs)
        print(f"# trajectory n1000 {traj}", file=sys.stderr, flush=True)
        forms["trajectory_n1000"] = traj
        batch = batch_study(torch, rpy, inputs)
        print(f"# batch {batch}", file=sys.stderr, flush=True)
        forms["batched_256_boxes"] = batch
        dstudy = diff_study(torch, rpy, inputs)
        print(f"# differentiation {dstudy}", file=sys.stderr, flush=True)
        forms["differentiation_n2000"] = dstudy
        forms["hma_lma_crossover"] = lma_study(torch, rpy, inputs)
    cpu = None if args.no_cpu else cpu_baseline(w, args.cpu_seconds)
    otab = oracle_table(args.oracle_table_seconds) if args.oracle_table else None
    line = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "n4000: 80 chains x 50 beads, c/c*=2, h*=0.28, narrow-Gaussian "
                               "excluded volume z*=1 d*=0.5, alpha L=6, alpha r_c=3.5, "
                               "k_c=2 alpha M (618 half-space k), dt=1e-3, device Philox noise; "
                               f"N_Ch by eq. nint raised until E_f < {TOL_EF:g} on an FP64 "
                               f"Lanczos interval ({LANCZOS_STEPS} steps, "
                               f"{LANCZOS_MARGIN:g} margin) refreshed every {REFRESH} steps",
                   "n_beads": w.n, "n_cheb_mean": head["n_cheb_mean"],
                   "E_f_tol": TOL_EF, "box_l": w.L, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_symv6<double,1> (packed symmetric tile product, FP64, m=1)",
                     "memory": "the 396 MB stored tile array is streamed from HBM with "
                               "non-temporal loads (larger than the 256 MB Infinity Cache)",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_us": sym["avg_us"], "launches": sym["launches"]},
        "step_configurations": configs,
        "kernels": prof,
        "forms": forms,
        "eigen": eigen,
        "cpu_baseline": cpu,
    }
    if otab is not None:
        line["oracle_table"] = otab
    print(json.dumps(line))


if __name__ == "__main__":
    main()
