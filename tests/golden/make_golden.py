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
from paper_2410_05408_amd import workloads  # noqa: E402


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


if __name__ == "__main__":
    main()
