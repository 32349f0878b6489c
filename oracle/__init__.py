"""CPU oracle for the screened two-electron Fock build (FP64, plain C + OpenMP).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py``.  The product package never imports it and shares no code
with it.  See ``hf_oracle.c`` for what every function computes and which passage of the
paper it follows.

Parity status of each function (what pins it, in ``tests/test_oracle.py``):
  boys_series / boys0 / boys1   pinned: erf closed form, F(0) values, downward recursion
  eri                           pinned: Gaussian-charge self energy 2 sqrt(a/pi), two-centre
                                closed form erf(sqrt(rho) R)/R, far-field S_ij S_kl / R limit,
                                8-fold permutation symmetry, Schwarz inequality
  schwarz                       pinned: sqrt of eri(ij|ij), Cauchy-Schwarz bound on all quartets
  fock                          pinned: brute-force plain definition (n <= 6, tau = 0 and > 0),
                                invariances, E2(lambda D) = lambda^2 E2, dE2/dD = G
  fock_element                  pinned: the plain definition itself, equals brute force
  grad                          pinned: central finite differences of E2, zero net force and torque
  eri4                          pinned (per-centre contractions): two-centre Gaussian-charge closed
                                form with unequal exponents, coincident-centre value, scaling law
                                (exponents x l^2, lengths / l gives x l), 8-fold symmetry
  one_electron_atoms            pinned: 1-D quadrature of overlap and kinetic energy (the latter as
                                1/2 <g_a'|g_b'>), nucleus-on-centre closed form 2 sqrt(2a/pi), each
                                Gaussian product as a charge cloud erf(sqrt(p) R)/R away from a nucleus
  scf (scf.py)                  pinned: one-function closed form 2h/S + J/S^2, D S D = 2 D, the
                                commutator F D S - S D F at convergence, energy as a trace, orbitals
                                orthonormal, rotation invariance, the filled-shell case D = 2 S^-1
  *_atoms                       pinned: brute-force plain definition with per-atom bases, reduction
                                to the one-basis build when every row is equal, atom-permutation
                                equivariance, far-field S_ii S_kk / R, central differences of E2
                                and of the pairing W o G (grad_pair_atoms)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.hfo_boys_series.restype = ctypes.c_double
        lib.hfo_boys_series.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.hfo_boys0.restype = ctypes.c_double
        lib.hfo_boys0.argtypes = [ctypes.c_double]
        lib.hfo_boys1.restype = ctypes.c_double
        lib.hfo_boys1.argtypes = [ctypes.c_double]
        lib.hfo_overlap.restype = ctypes.c_double
        lib.hfo_overlap.argtypes = [_dp, _dp, ctypes.c_int, _dp, _dp]
        lib.hfo_eri.restype = ctypes.c_double
        lib.hfo_eri.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp]
        lib.hfo_schwarz.restype = None
        lib.hfo_schwarz.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
        lib.hfo_fock.restype = ctypes.c_int
        lib.hfo_fock.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                 _dp, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _dp, _dp, _i64p]
        lib.hfo_fock_element.restype = ctypes.c_double
        lib.hfo_fock_element.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp,
                                         ctypes.c_double, _dp, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int64]
        lib.hfo_fock_bruteforce.restype = ctypes.c_int
        lib.hfo_fock_bruteforce.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp,
                                            ctypes.c_double, _dp, _dp]
        lib.hfo_grad_pair.restype = ctypes.c_int
        lib.hfo_grad_pair.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double,
                                      _dp, ctypes.c_int, _dp]
        lib.hfo_grad.restype = ctypes.c_int
        lib.hfo_grad.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                 _dp, ctypes.c_int, _dp, _dp, _i64p]
        lib.hfo_eri4.restype = ctypes.c_double
        lib.hfo_eri4.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int] + [_dp] * 8
        lib.hfo_schwarz_atoms.restype = ctypes.c_int
        lib.hfo_schwarz_atoms.argtypes = lib.hfo_schwarz.argtypes
        lib.hfo_fock_atoms.restype = ctypes.c_int
        lib.hfo_fock_atoms.argtypes = lib.hfo_fock.argtypes
        lib.hfo_fock_element_atoms.restype = ctypes.c_double
        lib.hfo_fock_element_atoms.argtypes = lib.hfo_fock_element.argtypes
        lib.hfo_fock_bruteforce_atoms.restype = ctypes.c_int
        lib.hfo_fock_bruteforce_atoms.argtypes = lib.hfo_fock_bruteforce.argtypes
        lib.hfo_grad_pair_atoms.restype = ctypes.c_int
        lib.hfo_grad_pair_atoms.argtypes = lib.hfo_grad_pair.argtypes
        lib.hfo_grad_atoms.restype = ctypes.c_int
        lib.hfo_grad_atoms.argtypes = lib.hfo_grad.argtypes
        lib.hfo_one_electron_atoms.restype = ctypes.c_int
        lib.hfo_one_electron_atoms.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        lib.hfo_num_threads.restype = ctypes.c_int
        lib.hfo_num_threads.argtypes = []
        _lib = lib
    return _lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def boys_series(m: int, t: float) -> float:
    return _load().hfo_boys_series(int(m), float(t))


def boys0(t: float) -> float:
    return _load().hfo_boys0(float(t))


def boys1(t: float) -> float:
    return _load().hfo_boys1(float(t))


def overlap(A, B, exps, coefs) -> float:
    A, pa = _c(A); B, pb = _c(B); e, pe = _c(exps); c, pc = _c(coefs)
    return _load().hfo_overlap(pa, pb, len(e), pe, pc)


def eri(A, B, C, D, exps, coefs) -> float:
    A, pa = _c(A); B, pb = _c(B); C, pc_ = _c(C); D, pd = _c(D)
    e, pe = _c(exps); c, pc = _c(coefs)
    return _load().hfo_eri(pa, pb, pc_, pd, len(e), pe, pc)


def num_threads() -> int:
    return _load().hfo_num_threads()


def schwarz(xyz, exps, coefs, nthreads: int = 0) -> np.ndarray:
    """Q[i(i+1)/2 + j] = sqrt((ij|ij)) for i >= j."""
    xyz, px = _c(xyz); e, pe = _c(exps); c, pc = _c(coefs)
    n = xyz.shape[0]
    Q = np.zeros(n * (n + 1) // 2)
    _load().hfo_schwarz(n, px, len(e), pe, pc, int(nthreads), Q.ctypes.data_as(_dp))
    return Q


def fock(xyz, dens, exps, coefs, tau, Q=None, nthreads: int = 0, bra_range=None):
    """Unique-quartet Fock build.  Returns (G, E2, survivors)."""
    xyz, px = _c(xyz); d, pd = _c(dens); e, pe = _c(exps); c, pc = _c(coefs)
    n = xyz.shape[0]
    npair = n * (n + 1) // 2
    b0, b1 = (0, npair) if bra_range is None else bra_range
    F = np.zeros((n, n))
    e2 = ctypes.c_double(0.0)
    ns = ctypes.c_int64(0)
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_fock(n, px, len(e), pe, pc, pd, float(tau), qp, int(nthreads), int(b0), int(b1),
                          F.ctypes.data_as(_dp), ctypes.byref(e2), ctypes.byref(ns))
    if rc != 0:
        raise MemoryError("oracle fock: out of memory")
    return F, e2.value, ns.value


def fock_element(xyz, dens, exps, coefs, tau, Q, i, j, nthreads: int = 0) -> float:
    xyz, px = _c(xyz); d, pd = _c(dens); e, pe = _c(exps); c, pc = _c(coefs); Q, qp = _c(Q)
    return _load().hfo_fock_element(xyz.shape[0], px, len(e), pe, pc, pd, float(tau), qp,
                                    int(nthreads), int(i), int(j))


def fock_bruteforce(xyz, dens, exps, coefs, tau):
    xyz, px = _c(xyz); d, pd = _c(dens); e, pe = _c(exps); c, pc = _c(coefs)
    n = xyz.shape[0]
    F = np.zeros((n, n))
    e2 = ctypes.c_double(0.0)
    rc = _load().hfo_fock_bruteforce(n, px, len(e), pe, pc, pd, float(tau), F.ctypes.data_as(_dp),
                                     ctypes.byref(e2))
    if rc != 0:
        raise MemoryError("oracle brute force: out of memory")
    return F, e2.value


def grad(xyz, dens, exps, coefs, tau, Q=None, nthreads: int = 0):
    """dE2/dR (n, 3), E2 from the unique-quartet energy sum, survivors."""
    xyz, px = _c(xyz); d, pd = _c(dens); e, pe = _c(exps); c, pc = _c(coefs)
    n = xyz.shape[0]
    g = np.zeros((n, 3))
    e2 = ctypes.c_double(0.0)
    ns = ctypes.c_int64(0)
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_grad(n, px, len(e), pe, pc, pd, float(tau), qp, int(nthreads),
                          g.ctypes.data_as(_dp), ctypes.byref(e2), ctypes.byref(ns))
    if rc != 0:
        raise MemoryError("oracle grad: out of memory")
    return g, e2.value, ns.value


def grad_pair(xyz, dens, xdens, exps, coefs, tau, Q=None, nthreads: int = 0):
    """sum_unique B(X, D) d(ij|kl)/dR (n, 3): the gradient of sum_ij W_ij G_ij for X = W, of E2
    for X = D / 2."""
    xyz, px = _c(xyz); d, pd = _c(dens); x, pxd = _c(xdens); e, pe = _c(exps); c, pc = _c(coefs)
    n = xyz.shape[0]
    g = np.zeros((n, 3))
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_grad_pair(n, px, len(e), pe, pc, pd, pxd, float(tau), qp, int(nthreads), g.ctypes.data_as(_dp))
    if rc != 0:
        raise MemoryError("oracle grad_pair: out of memory")
    return g


# ---------------------------------------------------------------- per-atom bases
# exps and coefs are (n, g): row i is the contraction of atom i.

def _atoms(xyz, exps, coefs):
    xyz, px = _c(xyz)
    e, pe = _c(exps)
    c, pc = _c(coefs)
    n = xyz.shape[0]
    if e.shape != c.shape or e.ndim != 2 or e.shape[0] != n:
        raise ValueError("per-atom exps and coefs must both be (natoms, ngauss)")
    return xyz, px, e, pe, c, pc, n, e.shape[1]


def eri4(A, B, C, D, basis_a, basis_b, basis_c, basis_d) -> float:
    """(AB|CD) with a contraction (exps, coefs) of its own on each centre."""
    pts = [_c(x) for x in (A, B, C, D)]
    bs = []
    g = len(basis_a[0])
    for e, c in (basis_a, basis_b, basis_c, basis_d):
        e, pe = _c(e)
        c, pc = _c(c)
        if len(e) != g or len(c) != g:
            raise ValueError("every centre needs the same number of primitives")
        bs += [(e, pe), (c, pc)]
    return _load().hfo_eri4(*[p for _, p in pts], g, *[p for _, p in bs])


def schwarz_atoms(xyz, exps, coefs, nthreads: int = 0) -> np.ndarray:
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    Q = np.zeros(n * (n + 1) // 2)
    if _load().hfo_schwarz_atoms(n, px, g, pe, pc, int(nthreads), Q.ctypes.data_as(_dp)) != 0:
        raise MemoryError("oracle schwarz_atoms: out of memory")
    return Q


def fock_atoms(xyz, dens, exps, coefs, tau, Q=None, nthreads: int = 0, bra_range=None):
    """Unique-quartet Fock build with per-atom bases.  Returns (G, E2, survivors)."""
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    d, pd = _c(dens)
    npair = n * (n + 1) // 2
    b0, b1 = (0, npair) if bra_range is None else bra_range
    F = np.zeros((n, n))
    e2 = ctypes.c_double(0.0)
    ns = ctypes.c_int64(0)
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_fock_atoms(n, px, g, pe, pc, pd, float(tau), qp, int(nthreads), int(b0), int(b1),
                                F.ctypes.data_as(_dp), ctypes.byref(e2), ctypes.byref(ns))
    if rc != 0:
        raise MemoryError("oracle fock_atoms: out of memory")
    return F, e2.value, ns.value


def fock_element_atoms(xyz, dens, exps, coefs, tau, Q, i, j, nthreads: int = 0) -> float:
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    d, pd = _c(dens)
    Q, qp = _c(Q)
    v = _load().hfo_fock_element_atoms(n, px, g, pe, pc, pd, float(tau), qp, int(nthreads), int(i), int(j))
    if v != v:
        raise MemoryError("oracle fock_element_atoms: out of memory")
    return v


def fock_bruteforce_atoms(xyz, dens, exps, coefs, tau):
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    d, pd = _c(dens)
    F = np.zeros((n, n))
    e2 = ctypes.c_double(0.0)
    if _load().hfo_fock_bruteforce_atoms(n, px, g, pe, pc, pd, float(tau), F.ctypes.data_as(_dp),
                                         ctypes.byref(e2)) != 0:
        raise MemoryError("oracle fock_bruteforce_atoms: out of memory")
    return F, e2.value


def grad_atoms(xyz, dens, exps, coefs, tau, Q=None, nthreads: int = 0):
    """dE2/dR (n, 3) with per-atom bases, E2, survivors."""
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    d, pd = _c(dens)
    gr = np.zeros((n, 3))
    e2 = ctypes.c_double(0.0)
    ns = ctypes.c_int64(0)
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_grad_atoms(n, px, g, pe, pc, pd, float(tau), qp, int(nthreads),
                                gr.ctypes.data_as(_dp), ctypes.byref(e2), ctypes.byref(ns))
    if rc != 0:
        raise MemoryError("oracle grad_atoms: out of memory")
    return gr, e2.value, ns.value


def grad_pair_atoms(xyz, dens, xdens, exps, coefs, tau, Q=None, nthreads: int = 0):
    """grad_pair with per-atom bases."""
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    d, pd = _c(dens)
    x, pxd = _c(xdens)
    gr = np.zeros((n, 3))
    qp = None
    if Q is not None:
        Q, qp = _c(Q)
    rc = _load().hfo_grad_pair_atoms(n, px, g, pe, pc, pd, pxd, float(tau), qp, int(nthreads),
                                     gr.ctypes.data_as(_dp))
    if rc != 0:
        raise MemoryError("oracle grad_pair_atoms: out of memory")
    return gr


def one_electron_atoms(xyz, charges, exps, coefs):
    """(S, T, V), each (n, n), for per-atom rows and nuclear charges Z (n,)."""
    xyz, px, e, pe, c, pc, n, g = _atoms(xyz, exps, coefs)
    Z, pz = _c(charges)
    S = np.zeros((n, n)); T = np.zeros((n, n)); V = np.zeros((n, n))
    if _load().hfo_one_electron_atoms(n, px, pz, g, pe, pc, S.ctypes.data_as(_dp), T.ctypes.data_as(_dp),
                                      V.ctypes.data_as(_dp)) != 0:
        raise MemoryError("oracle one_electron_atoms: out of memory")
    return S, T, V
