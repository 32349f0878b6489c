"""Helpers for the GPU tests (no arithmetic of the method here)."""
import os
import sys

import numpy as np


def announce(msg: str):
    """Names the case on stdout before a GPU step, flushed, so a failing run says where it was."""
    sys.stdout.write("[gpu-case] %s\n" % msg)
    sys.stdout.flush()


def rel_fro(a, b) -> float:
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b) -> float:
    """max |a - b| over max |b|: the element-wise companion of rel_fro (a bound on every
    element relative to the largest reference element)."""
    a = np.asarray(a); b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_close(a, ref, tol, what=""):
    """Both relative errors of a result against its reference within tol: Frobenius
    (||a - ref|| / ||ref||) and element-wise (max |a - ref| / max |ref|)."""
    fro, mx = rel_fro(a, ref), max_rel(a, ref)
    assert fro < tol and mx < tol, "%s rel_fro %.3e, max-abs/max|ref| %.3e, tol %.1e" % (what, fro, mx, tol)


def rel(a: float, b: float) -> float:
    return abs(a - b) / abs(b)


def load_golden(name: str):
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".txt")
    lines = open(path).read().split("\n")
    e2 = float([l for l in lines if l.startswith("# E2")][0].split()[2])
    ns = int([l for l in lines if l.startswith("# survivors")][0].split()[2])
    return np.loadtxt(path), e2, ns


def unpack_lower(tri, n):
    """Symmetric n x n matrix from its packed lower triangle (row i holds columns 0..i)."""
    G = np.zeros((n, n))
    G[np.tril_indices(n)] = tri
    return G + np.tril(G, -1).T


def load_full(name: str):
    """A stored whole-matrix build (tests/golden/<name>.npz): (G, E2, survivors)."""
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".npz")
    with np.load(path, allow_pickle=False) as z:
        tri = z["tri"]
        n = int(round((np.sqrt(8 * tri.size + 1) - 1) / 2))
        return unpack_lower(tri, n), float(z["e2"]), int(z["survivors"])


def load_batched_sample(name: str = "batched_2000_sample"):
    """Stored oracle results of sampled clusters: list of (molecule index, G, E2, gradient)."""
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".npz")
    out = []
    with np.load(path, allow_pickle=False) as z:
        t0 = g0 = 0
        for m, n, e2 in zip(z["mol"], z["natoms"], z["e2"]):
            n = int(n)
            nt = n * (n + 1) // 2
            out.append((int(m), unpack_lower(z["tri"][t0:t0 + nt], n), float(e2), z["grad"][g0:g0 + n].copy()))
            t0 += nt
            g0 += n
    return out
