"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

    python tests/golden/make_golden.py

he64_fp64.txt: the 64-atom jittered-lattice Fock build (4x4x4 lattice, spacing 2 bohr,
jitter 0.2, seed 1, tau 1e-12, STO-3G He basis), G as a 64x64 matrix with E2 and the number of
unique quartets kept in the header.

he512_fp64_sample.txt: the 512-atom lattice (8x8x8, seed 2, tau 1e-10): E2 and the number
of unique quartets kept in the header, and 64 elements (i, j, G_ij) of G at positions drawn
with numpy's PCG64 seeded 512 (always including (0, 0), (0, 511) and (511, 511)).

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


def he512():
    s = config_system("he512_fp64")
    F, E2, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    rng = np.random.default_rng(512)
    idx = [(0, 0), (0, 511), (511, 511)] + [tuple(int(v) for v in p) for p in rng.integers(0, 512, (61, 2))]
    rows = np.array([[i, j, F[i, j]] for i, j in idx])
    hdr = ("512 He jittered lattice (8x8x8, spacing 2.0, jitter 0.2, seed 2), tau 1e-10, FP64 CPU oracle;"
           " columns i j G_ij\nE2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he512_fp64_sample.txt"), rows, fmt=["%d", "%d", "%.17g"], header=hdr)


def main():
    only = sys.argv[1:]
    if only and "he512" in only:
        return he512()
    s = config_system("he64_fp64")
    F, E2, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("64 He jittered lattice (4x4x4, spacing 2.0, jitter 0.2, seed 1), tau 1e-12, FP64 CPU oracle\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he64_fp64.txt"), F, fmt="%.17g", header=hdr)

    he512()

    s = config_system("he128_grad")
    g, E2, ns = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("128 He jittered lattice (8x4x4, spacing 2.0, jitter 0.2, seed 4), tau 1e-10, FP64 CPU oracle, dE2/dR\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he128_grad.txt"), g, fmt="%.17g", header=hdr)


if __name__ == "__main__":
    main()
