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


def rel(a: float, b: float) -> float:
    return abs(a - b) / abs(b)


def load_golden(name: str):
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".txt")
    lines = open(path).read().split("\n")
    e2 = float([l for l in lines if l.startswith("# E2")][0].split()[2])
    ns = int([l for l in lines if l.startswith("# survivors")][0].split()[2])
    return np.loadtxt(path), e2, ns
