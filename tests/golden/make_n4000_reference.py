"""Write tests/golden/n4000_oracle.npz: the CPU oracle's results for the
N = 4000 precision-form workload (80 chains x 50 beads, c/c* = 2, h* = 0.28,
narrow-Gaussian excluded volume z* = 1, d* = 0.5, alpha L = 6, M = 3.5), from
which the benchmark states the error of each product precision against the
FP64 oracle.  Calls only the oracle (and numpy's symmetric eigenvalue
routine for the extreme eigenvalues); nothing here comes from the GPU path.

Stored (block rows of every 8th bead, 500 of 4000):
  rows             bead indices of the stored rows
  drift            D.F, F = Hookean springs + excluded volume at the
                   initial positions (eq. sde, eq. DFmodified)
  dmin, dmax       the paper's bound rule at C = 60 (eq. lmax-lmin-dilute,
                   fmax, fmin) on this D
  ds1, ef1         the N_Ch = 30 Chebyshev sum p(D) dW (eq. cheb1-cheb3) for
                   the workload's first noise vector, and its E_f
  ds16             the same for the workload's 16-vector noise block
  lam_min, lam_max extreme eigenvalues of the dense D

Run: python tests/golden/make_n4000_reference.py   (a few minutes on 8
host threads; it needs about 4 GB of memory).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1203_6208_amd import inputs  # noqa: E402

NCH = 30
BOUNDS_C = 60.0
STRIDE = 8


def main(out=os.path.join(HERE, "n4000_oracle.npz")):
    oracle.build(force=False)
    w = inputs.workload("n4000")
    pos = w.positions()
    t0 = time.time()
    D = oracle.diffusion_matrix(pos, w.L, w.a, w.alpha, w.rc, w.n2max)
    print(f"dense D: {time.time() - t0:.1f} s", flush=True)
    F = oracle.spring_forces(pos, w.nchains, w.bpc) + oracle.ev_forces(
        pos, w.L, w.ev["zstar"], w.ev["dstar"], w.ev["rcut"])
    drift = oracle.matvec(D, F.reshape(1, -1)).reshape(w.n, 3)
    dmin, dmax = oracle.bounds_rule(D, w.n, BOUNDS_C)
    dw1 = w.noise()[0]
    ds1 = oracle.cheb_sqrt(D, dw1.reshape(1, -1), NCH, dmin, dmax).reshape(w.n, 3)
    ef1 = oracle.sqrt_error(D, dw1, ds1)
    dw16 = w.noise(m=16)
    t0 = time.time()
    ds16 = oracle.cheb_sqrt(D, dw16.reshape(16, -1), NCH, dmin, dmax).reshape(16, w.n, 3)
    print(f"16-vector Chebyshev sum: {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    lam = np.linalg.eigvalsh(D)
    print(f"eigenvalues: {time.time() - t0:.1f} s, [{lam[0]:.6f}, {lam[-1]:.4f}]", flush=True)
    rows = np.arange(0, w.n, STRIDE)
    np.savez(out, rows=rows, drift=drift[rows], dmin=dmin, dmax=dmax, n_cheb=NCH,
             bounds_C=BOUNDS_C, ds1=ds1[rows], ef1=ef1, ds16=ds16[:, rows],
             lam_min=lam[0], lam_max=lam[-1], n_beads=w.n, box_l=w.L, seed=w.seed)
    print(f"wrote {out}: E_f(m=1) = {ef1:.4f}, interval [{dmin:.5f}, {dmax:.3f}]")


if __name__ == "__main__":
    main()
