"""Seeded synthetic He inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers: positions, densities and the basis constants.  It holds
none of the method's arithmetic (no integrals, no screening, no Fock build), so that the
CPU oracle and the HIP path can both consume the same inputs without sharing any code
that computes a result.

Recipe (stated once, used everywhere):
  * RNG: ``numpy.random.Generator(PCG64(seed))``.
  * Lattice points in C order over (ix, iy, iz), x slowest.  Position = spacing * (ix, iy, iz)
    plus one (n, 3) draw of U(-jitter, +jitter).  Units: bohr.
  * Density: M = U[0, 1) drawn as one (n, n) array after the positions;
    D = 0.1 * (M + M^T) / 2 with the diagonal then set to 1.0.
  * Basis: one contracted s function per atom with the STO-3G helium exponents and
    contraction coefficients below (the same three primitives on every atom).
  * Per-atom bases (mixed H/He systems): after positions and density, one (n,) draw of
    U[0, 1) marks atom i as hydrogen when below ``frac_h``; hydrogen carries the STO-3G
    hydrogen exponents with the same coefficients.  Random contractions for brute-force
    checks draw log-uniform exponents in [0.1, 10] and U(0.1, 1) coefficients.

The paper measures on helium test systems (up to 256 atoms with three Gaussians per atom,
and 1024 atoms with six; Methodology section and Table 4) whose input files are not
available; the jittered lattices below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# STO-3G helium: exponents (bohr^-2) and contraction coefficients of the single s function.
HE_STO3G_EXPS = np.array([6.36242139, 1.15892300, 0.31364979], dtype=np.float64)
HE_STO3G_COEFS = np.array([0.15432897, 0.53532814, 0.44463454], dtype=np.float64)
# STO-3G hydrogen: its own exponents, the same three contraction coefficients.
H_STO3G_EXPS = np.array([3.42525091, 0.62391373, 0.16885540], dtype=np.float64)


@dataclass
class System:
    """One molecule: atom positions, density and the shared basis."""
    xyz: np.ndarray                 # (n, 3) float64, bohr
    dens: np.ndarray                # (n, n) float64, symmetric
    exps: np.ndarray = field(default_factory=lambda: HE_STO3G_EXPS.copy())
    coefs: np.ndarray = field(default_factory=lambda: HE_STO3G_COEFS.copy())
    tau: float = 1e-10

    @property
    def natoms(self) -> int:
        return int(self.xyz.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_points(shape, spacing: float = 2.0) -> np.ndarray:
    nx, ny, nz = shape
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return spacing * idx


def density_from(rng: np.random.Generator, n: int) -> np.ndarray:
    m = rng.uniform(0.0, 1.0, size=(n, n))
    d = 0.1 * (m + m.T) / 2.0
    np.fill_diagonal(d, 1.0)
    return d


def jittered_lattice(shape, seed: int, tau: float, spacing: float = 2.0,
                     jitter: float = 0.2) -> System:
    rng = _rng(seed)
    pts = lattice_points(shape, spacing)
    n = pts.shape[0]
    xyz = pts + rng.uniform(-jitter, jitter, size=(n, 3))
    dens = density_from(rng, n)
    return System(xyz=xyz, dens=dens, tau=tau)


# The five workloads.  Config names describe what they are.
CONFIGS = {
    "he64_fp64":    dict(shape=(4, 4, 4), seed=1, tau=1e-12),
    "he512_fp64":   dict(shape=(8, 8, 8), seed=2, tau=1e-10),
    "he1024_mixed": dict(shape=(16, 8, 8), seed=3, tau=1e-10),
    "he128_grad":   dict(shape=(8, 4, 4), seed=4, tau=1e-10),
}


def config_system(name: str) -> System:
    c = CONFIGS[name]
    return jittered_lattice(c["shape"], c["seed"], c["tau"])


def cluster_batch(nmol: int = 2000, seed: int = 5, nmin: int = 4, nmax: int = 96,
                  tau: float = 1e-10, spacing: float = 2.0, jitter: float = 0.2):
    """Ragged batch of He clusters.

    The atom counts are drawn first (uniform integers in [nmin, nmax]); then, cluster by
    cluster, the jitter of its positions and its density M.  A cluster of n atoms is the
    first n points (C order) of an m^3 lattice with m = ceil(n^(1/3)).
    """
    rng = _rng(seed)
    counts = rng.integers(nmin, nmax + 1, size=nmol)
    systems = []
    for n in counts:
        n = int(n)
        m = int(math.ceil(round(n ** (1.0 / 3.0), 12)))
        while m ** 3 < n:
            m += 1
        pts = lattice_points((m, m, m), spacing)[:n]
        xyz = pts + rng.uniform(-jitter, jitter, size=(n, 3))
        dens = density_from(rng, n)
        systems.append(System(xyz=xyz, dens=dens, tau=tau))
    return systems


def pack_batch(systems):
    """CSR packing: atom offsets, stacked positions and the densities flattened one after another."""
    counts = np.array([s.natoms for s in systems], dtype=np.int64)
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    xyz = np.concatenate([s.xyz for s in systems], axis=0)
    dens = np.concatenate([s.dens.ravel() for s in systems])
    return off, xyz, dens


def random_cluster(n: int, seed: int, box: float = 4.0, tau: float = 0.0) -> System:
    """Tiny random cluster (uniform positions in a cube of side ``box``) for brute-force checks."""
    rng = _rng(seed)
    xyz = rng.uniform(0.0, box, size=(n, 3))
    dens = density_from(rng, n)
    return System(xyz=xyz, dens=dens, tau=tau)


def mixed_lattice(shape, seed: int, tau: float, frac_h: float = 0.5, spacing: float = 2.0,
                  jitter: float = 0.2) -> System:
    """Jittered lattice of H and He atoms with per-atom bases: ``exps`` and ``coefs`` are
    (n, 3), row i the contraction of atom i."""
    rng = _rng(seed)
    pts = lattice_points(shape, spacing)
    n = pts.shape[0]
    xyz = pts + rng.uniform(-jitter, jitter, size=(n, 3))
    dens = density_from(rng, n)
    is_h = rng.uniform(0.0, 1.0, size=n) < frac_h
    exps = np.where(is_h[:, None], H_STO3G_EXPS[None, :], HE_STO3G_EXPS[None, :])
    coefs = np.broadcast_to(HE_STO3G_COEFS, (n, 3)).copy()
    return System(xyz=xyz, dens=dens, exps=exps, coefs=coefs, tau=tau)


def random_basis_rows(n: int, g: int, seed: int):
    """(n, g) exponents (log-uniform in [0.1, 10]) and coefficients (U(0.1, 1)), one
    contraction per atom."""
    rng = _rng(seed)
    exps = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=(n, g)))
    coefs = rng.uniform(0.1, 1.0, size=(n, g))
    return exps, coefs


# A tight contraction whose Schwarz bounds reach above 2 (one-centre Q about 2.09), for the
# case of a bra pair whose threshold tau / Q_s lies above every bound below 2.
TIGHT_EXPS = np.array([40.0, 4.0, 0.6], dtype=np.float64)
TIGHT_COEFS = np.array([0.5, 0.5, 0.5], dtype=np.float64)


def tight_cluster() -> System:
    """60 atoms in a 10 bohr box with the tight contraction above and tau = 1e-3."""
    s = random_cluster(60, 2, box=10.0, tau=1e-3)
    s.exps = TIGHT_EXPS.copy()
    s.coefs = TIGHT_COEFS.copy()
    return s


def hhe_rows(n: int, seed: int, frac_h: float = 0.5):
    """(n, 3) per-atom rows for stacked atoms: one (n,) draw of U[0, 1) marks hydrogen when
    below ``frac_h`` (STO-3G hydrogen exponents), helium otherwise; both with the STO-3G
    coefficients."""
    rng = _rng(seed)
    is_h = rng.uniform(0.0, 1.0, size=n) < frac_h
    exps = np.where(is_h[:, None], H_STO3G_EXPS[None, :], HE_STO3G_EXPS[None, :])
    coefs = np.broadcast_to(HE_STO3G_COEFS, (n, 3)).copy()
    return exps, coefs
