"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

    python tests/golden/make_golden.py

he64_fp64.txt: the 64-atom jittered-lattice Fock build (4x4x4 lattice, spacing 2 bohr,
jitter 0.2, seed 1, tau 1e-12, STO-3G He basis), G as a 64x64 matrix with E2 and the number of
unique quartets kept in the header.

he128_grad.txt: the analytic nuclear gradient dE2/dR (128 x 3) of the 128-atom lattice
(8x4x4, seed 4, tau 1e-10), with E2 (as the sum over unique quartets of Gamma (ij|kl)) and
the number of quartets kept in the header.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from he_inputs import config_system  # noqa: E402


def main():
    s = config_system("he64_fp64")
    F, E2, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("64 He jittered lattice (4x4x4, spacing 2.0, jitter 0.2, seed 1), tau 1e-12, FP64 CPU oracle\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he64_fp64.txt"), F, fmt="%.17g", header=hdr)

    s = config_system("he128_grad")
    g, E2, ns = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("128 He jittered lattice (8x4x4, spacing 2.0, jitter 0.2, seed 4), tau 1e-10, FP64 CPU oracle, dE2/dR\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he128_grad.txt"), g, fmt="%.17g", header=hdr)


if __name__ == "__main__":
    main()
