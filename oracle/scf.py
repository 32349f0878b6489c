"""Plain self-consistent field around the oracle's two-electron build (TEST INFRASTRUCTURE
ONLY, like the rest of ``oracle/``).

The paper's kernel computes the electron-repulsion term of the Fock operator; this module is
the loop on either side of it for a closed-shell system: core Hamiltonian H = T + V from the
one-electron integrals, symmetric orthogonalisation X = S^(-1/2), F = H + G(D) with the
oracle's G, energy E = 1/2 sum D o (H + F) + E_nn, orbitals from the eigenproblem of
X^T F X, D = 2 C_occ C_occ^T (Aufbau), and DIIS on the commutator X^T (F D S - S D F) X.
Every step is numpy on the CPU in FP64.
"""
from __future__ import annotations

import numpy as np

from . import fock_atoms, one_electron_atoms


def nuclear_repulsion(xyz, charges) -> float:
    xyz = np.asarray(xyz, dtype=np.float64)
    Z = np.asarray(charges, dtype=np.float64)
    e = 0.0
    for a in range(len(Z)):
        for b in range(a):
            e += Z[a] * Z[b] / np.linalg.norm(xyz[a] - xyz[b])
    return e


def orthogonaliser(S):
    s, U = np.linalg.eigh(S)
    return (U / np.sqrt(s)) @ U.T


def density_from(F, X, nocc):
    eps, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    Co = C[:, :nocc]
    return 2.0 * Co @ Co.T, eps, C


def diis_extrapolate(Fs, errs):
    m = len(Fs)
    B = -np.ones((m + 1, m + 1))
    B[m, m] = 0.0
    for i in range(m):
        for j in range(m):
            B[i, j] = np.sum(errs[i] * errs[j])
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(B, rhs)[:m]
    return sum(ci * Fi for ci, Fi in zip(c, Fs))


def scf(xyz, charges, exps, coefs, nocc, tau, max_iter=100, e_tol=1e-10, d_tol=1e-7, diis=8, D0=None):
    """Returns dict(E, D, eps, C, iterations, converged, H, S, X, F)."""
    S, T, V = one_electron_atoms(xyz, charges, exps, coefs)
    H = T + V
    enn = nuclear_repulsion(xyz, charges)
    X = orthogonaliser(S)
    if D0 is None:
        D, eps, C = density_from(H, X, nocc)          # core-Hamiltonian guess
    else:
        D = np.array(D0, dtype=np.float64)
    Fs, errs = [], []
    e_old = None
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        G = fock_atoms(xyz, D, exps, coefs, tau)[0]
        F = H + G
        E = 0.5 * float(np.sum(D * (H + F))) + enn
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        Fs.append(F)
        errs.append(err)
        if len(Fs) > diis:
            Fs.pop(0)
            errs.pop(0)
        if e_old is not None and abs(E - e_old) < e_tol and np.abs(err).max() < d_tol:
            converged = True
            break
        Fx = diis_extrapolate(Fs, errs) if len(Fs) >= 2 else F
        D, eps, C = density_from(Fx, X, nocc)
        e_old = E
    _, eps, C = density_from(F, X, nocc)
    return dict(E=E, D=D, eps=eps, C=C, iterations=it, converged=converged, H=H, S=S, X=X, F=F, enn=enn)
