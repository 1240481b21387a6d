"""Write the stored oracle outputs under tests/golden/.

Calls only the oracle (and the seeded input generator).  The paper prints no
correlator values, so these fixtures are oracle regressions: they fix the
oracle's output for the 4^3 x 8 plain-method workload (Haar links seed 1,
point source column 0, kappa = 0.25, N = 10) so that a later change to the
oracle's arithmetic shows up as a diff.

    python tests/golden/make_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1111_5596_amd import synth  # noqa: E402


def config1():
    dims = (4, 4, 4, 8)
    U = synth.su3_links(dims, 1)
    psi = oracle.smear(U, synth.point_source(dims, [0]), dims, 0.25, 10)[0]
    per_site = np.sum(np.abs(psi) ** 2, axis=(1, 2))
    corr = oracle.timeslice_sum(per_site, dims)[:, 0].real
    return {
        "workload": "4^3x8, Haar SU(3) links seed 1, point source column 0, kappa 0.25, N 10",
        "source": "oracle (FP64); regression fixture, not a paper value",
        "pion_correlator": [float(v) for v in corr],
        "psi_origin": [float(psi[0, 0, 0].real), float(psi[0, 0, 0].imag)],
        "norm2": float(np.sum(per_site)),
    }


def main():
    with open(os.path.join(HERE, "config1_fp64.json"), "w") as f:
        json.dump(config1(), f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
