"""Seeded synthetic workloads for the Ewald-RPY Brownian-dynamics path.

This module holds no arithmetic of the method itself: it only draws polymer
conformations and noise from seeds and turns a workload description (chains,
beads per chain, c/c*, h*, alpha*L, M) into the scalar inputs the method takes
(box length L, bead radius a, alpha, r_c, k_c and the integer wave-vector
cutoff).  Both the HIP path and the CPU oracle receive exactly these numbers.

Sources (arXiv:1203.6208):
  * a = sqrt(pi) h* (section "Governing equation");
  * c* = N_b / ((4 pi/3) R_g0^3) with the theta-solvent R_g0^2 = (N_b^2-1)/(2 N_b)
    (section "Optimisation of the evaluation of sum D.F" and eq. Rg2);
  * alpha = M / r_c (eq. rparameter) and K = 2 alpha M (eq. kparameter);
  * initial conformations: each chain starts uniform in [0, L)^3 and its bonds
    are N(0, I_3), the exact theta-equilibrium bond distribution of Hookean
    springs in these units (eq. Re2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

POSITION_SEED_BASE = 12036208


@dataclass
class Workload:
    name: str
    nchains: int
    bpc: int                 # beads per chain
    c_over_cstar: float
    hstar: float = 0.28
    alphaL: float = 6.0      # alpha * L
    M: float = 3.5           # alpha * r_c
    nch: int = 30            # Chebyshev terms N_Ch
    dt: float = 1e-3
    ev: dict | None = None   # {"zstar":..,"dstar":..,"rcut":..} or None
    seed: int = POSITION_SEED_BASE
    # derived
    n: int = field(init=False)
    L: float = field(init=False)
    a: float = field(init=False)
    alpha: float = field(init=False)
    rc: float = field(init=False)
    kc: float = field(init=False)
    n2max: int = field(init=False)

    def __post_init__(self):
        self.n = self.nchains * self.bpc
        self.L = box_length(self.n, self.bpc, self.c_over_cstar)
        self.a = math.sqrt(math.pi) * self.hstar
        self.alpha = self.alphaL / self.L
        self.rc = self.M / self.alpha
        self.kc = 2.0 * self.alpha * self.M
        self.n2max = wavevector_cutoff(self.kc, self.L)

    def params(self) -> dict:
        return {k: v for k, v in asdict(self).items()}

    def positions(self, seed: int | None = None) -> np.ndarray:
        return random_walks(self.nchains, self.bpc, self.L,
                            self.seed if seed is None else seed)

    def noise(self, m: int = 1, seed: int | None = None) -> np.ndarray:
        s = (self.seed + 1000) if seed is None else seed
        return gaussian_block(m, self.n, self.dt, s)


def theta_rg2(bpc: int) -> float:
    return (bpc * bpc - 1.0) / (2.0 * bpc)


def overlap_concentration(bpc: int) -> float:
    rg0 = math.sqrt(theta_rg2(bpc))
    return bpc / (4.0 * math.pi / 3.0 * rg0 ** 3)


def box_length(n: int, bpc: int, c_over_cstar: float) -> float:
    c = c_over_cstar * overlap_concentration(bpc)
    return (n / c) ** (1.0 / 3.0)


def wavevector_cutoff(kc: float, L: float) -> int:
    """Integer cutoff n2max = floor((kc L / 2 pi)^2) on |nvec|^2, decided once
    on the host so that both implementations use the same wave-vector set."""
    return int(math.floor((kc * L / (2.0 * math.pi)) ** 2))


def random_walks(nchains: int, bpc: int, L: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    starts = rng.uniform(0.0, L, size=(nchains, 1, 3))
    bonds = rng.standard_normal(size=(nchains, bpc - 1, 3))
    chains = np.concatenate([starts, starts + np.cumsum(bonds, axis=1)], axis=1)
    return np.ascontiguousarray(chains.reshape(nchains * bpc, 3))


def gaussian_block(m: int, n: int, dt: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal(size=(m, n, 3)) * math.sqrt(dt))


NG_EV = {"zstar": 1.0, "dstar": 0.5, "rcut": 4.0}


def workload(name: str) -> Workload:
    """The workloads: plain FP64 N=100 and N=1000, the precision form at
    N=4000, the differentiation form at N=2000, the theta-statics check
    (batching boxes: batch_boxes).

    N=1000 takes M = alpha r_c = 4.6 so that both truncations of the Ewald
    sum (section "Choice of Ewald parameters", eq. rparameter, kparameter)
    leave less than 1e-6: erfc(M) = 8e-11 for the real-space cut, and for the
    reciprocal cut the factor of eq. M2 at k = K = 2 alpha M,
    (1 + M^2 + 2 M^4) e^{-M^2} = 5.9e-7 (at M = 3.5 it is 1.5e-3)."""
    base = POSITION_SEED_BASE
    if name == "n100":
        return Workload("n100", 10, 10, 1.0, nch=20, seed=base + 0)
    if name == "n1000":
        return Workload("n1000", 40, 25, 1.0, M=4.6, nch=30, seed=base + 1)
    if name == "n4000":
        return Workload("n4000", 80, 50, 2.0, nch=30, ev=dict(NG_EV), seed=base + 2)
    if name == "n2000":
        return Workload("n2000", 40, 50, 1.0, nch=30, ev=dict(NG_EV), seed=base + 4)
    if name == "theta20":
        # theta-statics check: N_c = 20 chains of N_b = 20 beads, a = 0.5,
        # dt = 0.01, c/c* = 1, no excluded volume (section "Testing and
        # verification")
        return Workload("theta20", 20, 20, 1.0, hstar=0.5 / math.sqrt(math.pi), nch=0,
                        dt=0.01, seed=base + 5)
    raise KeyError(name)


def eigen_state(n: int, replica: int = 0) -> Workload:
    """A state of the eigenvalue study (section "Decomposition of the
    diffusion tensor", eq. fmax and fmin): chains of N_b = 10 beads at
    c = 4.44 c*, bead radius a = 0.5, N = 10 N_c beads, no excluded volume,
    the start conformation of `replica`."""
    if n % 10:
        raise ValueError("N must be a multiple of N_b = 10")
    return Workload(f"eigen{n}_{replica}", n // 10, 10, 4.44, hstar=0.5 / math.sqrt(math.pi),
                    nch=0, seed=POSITION_SEED_BASE + 100 + 97 * n + replica)


def theta_state(bpc: int, c_over_cstar: float, nchains: int = 20, replica: int = 0) -> Workload:
    """A state of the theta-statics grid (section "Testing and verification",
    theta solvents): N_c = 20 chains of N_b beads, a = 0.5, dt = 0.01, no
    excluded volume, c/c* set by the box length; `replica` picks an
    independent start."""
    return Workload(f"theta{bpc}_c{c_over_cstar:g}_{replica}", nchains, bpc, c_over_cstar,
                    hstar=0.5 / math.sqrt(math.pi), nch=0, dt=0.01,
                    seed=POSITION_SEED_BASE + 200 + 1009 * bpc + int(round(1e4 * c_over_cstar))
                    + 100003 * replica)


def batch_boxes(count: int = 256, seed: int = POSITION_SEED_BASE + 3, n_lo: int = 100,
                n_hi: int = 2000):
    """Ragged ensemble: N_b ~ U{10..50}, N in whole chains with n_lo <= N <= n_hi
    (100..2000 for the batching workload), c/c* ~ U[0.5, 3], no excluded
    volume."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        bpc = int(rng.integers(10, 51))
        lo = math.ceil(n_lo / bpc)
        hi = max(lo, n_hi // bpc)
        nchains = int(rng.integers(lo, hi + 1))
        cc = float(rng.uniform(0.5, 3.0))
        out.append(Workload(f"box{b}", nchains, bpc, cc, nch=30, seed=seed + 7919 * (b + 1)))
    return out
