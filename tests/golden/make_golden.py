"""Writes the stored expected values under tests/golden/.

Calls only the CPU oracle (``oracle/``) and the seeded workload generator.
The paper prints no light-curve values, so every stored value here is the
oracle's, recomputed by running this script:

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import glo  # noqa: E402
from oracle import mcmc  # noqa: E402
from paper_2410_05408_amd import workloads  # noqa: E402

JWST_NOISE_SEED = 541


def make_jwst():
    """The simulated JWST visit of Section 5.3: the oracle's light curve of the
    injected planet plus seeded 20-ppm white noise."""
    times, t_exp, n_ss = workloads.jwst_grid()
    params = mcmc.params_from_walkers(workloads.jwst_truth())
    model = glo.flux_batch(params, times, n_ss=np.array([n_ss], np.int32), t_exp=np.array([t_exp]),
                           tol=1e-14)[0]
    rng = np.random.default_rng(JWST_NOISE_SEED)
    data = model + rng.normal(0.0, workloads.JWST_SIGMA, times.size)
    path = os.path.join(HERE, "jwst_injected.txt")
    with open(path, "w") as fh:
        fh.write("# Simulated JWST/NIRISS visit (Section 5.3): 2-min cadence, 20 ppm white noise,\n")
        fh.write("# K2 fit medians (Table of fit results) with injected f = 0.15, eta = 0, xi = 29 deg;\n")
        fh.write(f"# oracle flux (n_ss = {n_ss}, t_exp = one cadence, tol 1e-14) plus N(0, sigma) noise,\n")
        fh.write(f"# numpy default_rng({JWST_NOISE_SEED}).  columns: t_days data sigma model\n")
        for row in zip(times, data, np.full(times.size, workloads.JWST_SIGMA), model):
            fh.write(" ".join(f"{v:.17e}" for v in row) + "\n")
    print("wrote", path)


def main():
    w = workloads.single_transit()
    out = glo.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp, tol=1e-14)[0]
    path = os.path.join(HERE, "single_transit_oracle.txt")
    with open(path, "w") as fh:
        fh.write("# Oracle relative flux for the single oblate transit workload\n")
        fh.write("# (k=0.1 f=0.3 theta=60deg phi=30deg b=0.3 a/R*=200 P=500d u1=0.4 u2=0.25,\n")
        fh.write("#  1000 times uniform over +-T14), oracle tol 1e-14.  columns: t_days flux\n")
        for t, f in zip(w.times, out):
            fh.write(f"{t:.17e} {f:.17e}\n")
    print("wrote", path)
    make_jwst()


if __name__ == "__main__":
    main()
