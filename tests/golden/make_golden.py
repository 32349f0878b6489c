"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

    python tests/golden/make_golden.py [he64] [he512] [he128grad] [he1024] [batched]

With no argument every file is written (the 1024-atom build takes about 20 minutes on 8
cores; the others a few minutes together).

he64_fp64.txt: the 64-atom jittered-lattice Fock build (4x4x4 lattice, spacing 2 bohr,
jitter 0.2, seed 1, tau 1e-12, STO-3G He basis), G as a 64x64 matrix with E2 and the number of
unique quartets kept in the header.

he512_fp64.npz: the 512-atom lattice (8x8x8, seed 2, tau 1e-10): the whole G as its packed
lower triangle ``tri`` (row i holds G_i0 .. G_ii; the oracle's G is symmetric by
construction), ``e2`` and ``survivors`` (unique quartets kept).

he1024_fp64.npz: the same for the 1024-atom lattice (16x8x8, seed 3, tau 1e-10).

he128_grad.txt: the analytic nuclear gradient dE2/dR (128 x 3) of the 128-atom lattice
(8x4x4, seed 4, tau 1e-10), with E2 (as the sum over unique quartets of Gamma (ij|kl)) and
the number of quartets kept in the header.

batched_2000_sample.npz: 50 of the 2000 ragged He clusters (seed 5, tau 1e-10): the ten
largest and 40 more drawn with PCG64 seeded 2000 among the rest.  Per cluster ``mol`` (its
index in the batch), ``natoms``, ``e2``; ``tri`` concatenates the packed lower triangles of G
and ``grad`` the (n, 3) gradients, cluster after cluster in the order of ``mol``.

Every file is loaded with allow_pickle=False.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from he_inputs import cluster_batch, config_system  # noqa: E402


def packed_lower(F):
    return F[np.tril_indices(F.shape[0])]


def he64():
    s = config_system("he64_fp64")
    F, E2, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("64 He jittered lattice (4x4x4, spacing 2.0, jitter 0.2, seed 1), tau 1e-12, FP64 CPU oracle\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he64_fp64.txt"), F, fmt="%.17g", header=hdr)


def full_build(config, fname):
    s = config_system(config)
    F, E2, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert np.array_equal(F, F.T)
    np.savez(os.path.join(HERE, fname), tri=packed_lower(F), e2=np.float64(E2), survivors=np.int64(ns))


def he128grad():
    s = config_system("he128_grad")
    g, E2, ns = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    hdr = ("128 He jittered lattice (8x4x4, spacing 2.0, jitter 0.2, seed 4), tau 1e-10, FP64 CPU oracle, dE2/dR\n"
           "E2 %.17g\nsurvivors %d" % (E2, ns))
    np.savetxt(os.path.join(HERE, "he128_grad.txt"), g, fmt="%.17g", header=hdr)


def batched_picks(counts):
    """The ten largest clusters (ties to the lower index) and 40 more drawn among the rest."""
    order = np.argsort(-counts, kind="stable")
    big = [int(m) for m in order[:10]]
    rest = np.array(sorted(set(range(len(counts))) - set(big)))
    rng = np.random.Generator(np.random.PCG64(2000))
    more = [int(m) for m in rng.choice(rest, size=40, replace=False)]
    return sorted(big + more)


def batched():
    systems = cluster_batch()
    counts = np.array([s.natoms for s in systems])
    picks = batched_picks(counts)
    tri, grad, e2, nat = [], [], [], []
    for m in picks:
        s = systems[m]
        F, E2, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        g, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        tri.append(packed_lower(F))
        grad.append(g)
        e2.append(E2)
        nat.append(s.natoms)
    np.savez(os.path.join(HERE, "batched_2000_sample.npz"), mol=np.array(picks, dtype=np.int64),
             natoms=np.array(nat, dtype=np.int64), e2=np.array(e2), tri=np.concatenate(tri),
             grad=np.concatenate(grad, axis=0))


JOBS = {
    "he64": he64,
    "he512": lambda: full_build("he512_fp64", "he512_fp64.npz"),
    "he128grad": he128grad,
    "he1024": lambda: full_build("he1024_mixed", "he1024_fp64.npz"),
    "batched": batched,
}


def main():
    only = sys.argv[1:] or list(JOBS)
    for name in only:
        JOBS[name]()
        print("wrote", name, flush=True)


if __name__ == "__main__":
    main()
