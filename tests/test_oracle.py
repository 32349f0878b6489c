"""Pins for the CPU oracle: each check comes from mathematics or physics that the oracle's
own code does not restate (closed forms, quadrature, limits, invariances, brute force), so
that a dropped term, a wrong sign, a wrong index or a transposed operand fails one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

from he_inputs import HE_STO3G_COEFS as C3, HE_STO3G_EXPS as E3, random_cluster, config_system

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ------------------------------------------------------------------ Boys function

T_GRID = [0.0, 1e-12, 1e-8, 1e-3, 0.1, 0.5, 1.0, 2.5, 5.0, 10.0, 20.0, 33.0, 40.0, 60.0, 99.0, 150.0]


def _boys_quad(m, t):
    """F_m(t) = int_0^1 u^(2m) exp(-t u^2) du by adaptive quadrature."""
    v, _ = integrate.quad(lambda u: u ** (2 * m) * math.exp(-t * u * u), 0.0, 1.0,
                          epsabs=0.0, epsrel=2e-14, limit=200)
    return v


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_boys_series_matches_quadrature(oracle_lib, m):
    for t in T_GRID:
        ref = _boys_quad(m, t)
        got = oracle_lib.boys_series(m, t)
        assert abs(got - ref) <= 2e-14 * ref, (m, t, got, ref)


def test_boys_at_zero(oracle_lib):
    for m in range(6):
        assert oracle_lib.boys_series(m, 0.0) == pytest.approx(1.0 / (2 * m + 1), rel=1e-16)
    assert oracle_lib.boys0(0.0) == 1.0
    assert oracle_lib.boys1(0.0) == pytest.approx(1.0 / 3.0, rel=1e-16)


def test_boys0_closed_form_vs_series(oracle_lib):
    # F0(t) = (1/2) sqrt(pi/t) erf(sqrt t) against the positive series.
    for t in T_GRID[1:]:
        s = oracle_lib.boys_series(0, t)
        c = 0.5 * math.sqrt(math.pi / t) * math.erf(math.sqrt(t))
        assert abs(oracle_lib.boys0(t) - s) <= 3e-15 * s
        assert abs(c - s) <= 3e-15 * s


def test_boys_downward_recursion(oracle_lib):
    # (2m+1) F_m = 2 t F_{m+1} + exp(-t), from integrating u^(2m) exp(-t u^2) by parts.
    for t in T_GRID:
        for m in range(4):
            lhs = (2 * m + 1) * oracle_lib.boys_series(m, t)
            rhs = 2 * t * oracle_lib.boys_series(m + 1, t) + math.exp(-t)
            assert abs(lhs - rhs) <= 1e-14 * lhs, (t, m)


def test_boys1_hybrid_matches_series(oracle_lib):
    for t in T_GRID + [0.99999, 1.0, 1.00001, 3.7, 12.3]:
        s = oracle_lib.boys_series(1, t)
        assert abs(oracle_lib.boys1(t) - s) <= 5e-15 * s, t


def test_boys_large_t_limit(oracle_lib):
    for t in (50.0, 100.0, 200.0, 1e4):
        assert oracle_lib.boys0(t) == pytest.approx(0.5 * math.sqrt(math.pi / t), rel=1e-15)


# ------------------------------------------------------------------ integrals

def _norm_prim(a):
    return (2.0 * a / math.pi) ** 0.75


def test_overlap_matches_quadrature(oracle_lib):
    """<phi_A|phi_B> factorises into three 1-D Gaussian integrals; integrate them numerically."""
    rng = np.random.default_rng(11)
    for _ in range(3):
        A = rng.uniform(-2, 2, 3)
        B = A + rng.uniform(-2, 2, 3)
        ref = 0.0
        for a, ca in zip(E3, C3):
            for b, cb in zip(E3, C3):
                prod = ca * cb * _norm_prim(a) * _norm_prim(b)
                for x in range(3):
                    v, _ = integrate.quad(lambda s: math.exp(-a * (s - A[x]) ** 2 - b * (s - B[x]) ** 2),
                                          -40, 40, epsabs=0, epsrel=1e-13, limit=400,
                                          points=[A[x], B[x]])
                    prod *= v
                ref += prod
        assert oracle_lib.overlap(A, B, E3, C3) == pytest.approx(ref, rel=1e-12)


def test_he_sto3g_self_overlap(oracle_lib):
    # Normalised primitives, coefficients as given: S_ii is 1 to the basis' 8 printed digits.
    assert oracle_lib.overlap(np.zeros(3), np.zeros(3), E3, C3) == pytest.approx(1.0, abs=1e-8)


@pytest.mark.parametrize("alpha", [0.3, 1.0, 6.5])
def test_single_gaussian_self_repulsion(oracle_lib, alpha):
    """|g|^2 of a normalised s Gaussian is a unit Gaussian charge with exponent 2 alpha;
    its Coulomb self energy is sqrt(2 * 2alpha / pi) = 2 sqrt(alpha / pi)."""
    A = np.array([0.3, -1.2, 2.0])
    got = oracle_lib.eri(A, A, A, A, [alpha], [1.0])
    assert got == pytest.approx(2.0 * math.sqrt(alpha / math.pi), rel=1e-14)


@pytest.mark.parametrize("R", [0.0, 1e-4, 0.3, 1.0, 2.0, 5.0, 9.0])
@pytest.mark.parametrize("a", [0.4, 1.3])
def test_two_gaussian_charges(oracle_lib, R, a):
    """(AA|BB) for one normalised primitive of exponent a: g_a^2 is a unit Gaussian charge of
    exponent 2a, and two such charges R apart interact as erf(sqrt(a) R) / R (reduced
    exponent (2a)(2a)/(4a) = a), tending to 2 sqrt(a/pi) as R -> 0."""
    A = np.array([0.1, 0.2, -0.4])
    d = np.array([1.0, -2.0, 0.5])
    B = A + R * d / np.linalg.norm(d)
    ref = 2.0 * math.sqrt(a / math.pi) if R == 0 else erf(math.sqrt(a) * R) / R
    got = oracle_lib.eri(A, A, B, B, [a], [1.0])
    assert got == pytest.approx(ref, rel=1e-13, abs=1e-15)


def test_contracted_far_field_limit(oracle_lib):
    """Far apart, (ii|jj) -> S_ii S_jj / R (point charges)."""
    A = np.zeros(3)
    for R in (30.0, 60.0):
        B = np.array([0.0, 0.0, R])
        s = oracle_lib.overlap(A, A, E3, C3)
        assert oracle_lib.eri(A, A, B, B, E3, C3) == pytest.approx(s * s / R, rel=1e-14)


def test_contracted_coincident_value(oracle_lib):
    # STO-3G He (ii|ii): every primitive quartet at T = 0.
    ref = 0.0
    w = C3 * (2 * E3 / math.pi) ** 0.75
    for a in range(3):
        for b in range(3):
            for c in range(3):
                for d in range(3):
                    p = E3[a] + E3[b]
                    q = E3[c] + E3[d]
                    # charge of each Gaussian product times the self-energy kernel of two
                    # spherical Gaussian charges at the same centre: 2 sqrt(rho/pi)
                    sab = w[a] * w[b] * (math.pi / p) ** 1.5
                    scd = w[c] * w[d] * (math.pi / q) ** 1.5
                    rho = p * q / (p + q)
                    ref += sab * scd * 2.0 * math.sqrt(rho / math.pi)
    got = oracle_lib.eri(np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3), E3, C3)
    assert got == pytest.approx(ref, rel=1e-14)
    assert got == pytest.approx(1.0557129304699764, rel=1e-13)


def test_gaussian_charge_form_general_quartet(oracle_lib):
    """Each primitive (ab|cd) equals S_ab S_cd erf(sqrt(rho) |P-Q|) / |P-Q| (two spherical
    Gaussian charge clouds); the oracle goes through 2 pi^(5/2)/(pq sqrt(p+q)) K K F0(T)."""
    rng = np.random.default_rng(5)
    w = C3 * (2 * E3 / math.pi) ** 0.75
    for _ in range(5):
        X = rng.uniform(-2.5, 2.5, (4, 3))
        ref = 0.0
        for a in range(3):
            for b in range(3):
                p = E3[a] + E3[b]
                P = (E3[a] * X[0] + E3[b] * X[1]) / p
                sab = w[a] * w[b] * (math.pi / p) ** 1.5 * math.exp(-E3[a] * E3[b] / p * np.sum((X[0] - X[1]) ** 2))
                for c in range(3):
                    for d in range(3):
                        q = E3[c] + E3[d]
                        Q = (E3[c] * X[2] + E3[d] * X[3]) / q
                        scd = w[c] * w[d] * (math.pi / q) ** 1.5 * math.exp(-E3[c] * E3[d] / q * np.sum((X[2] - X[3]) ** 2))
                        rho = p * q / (p + q)
                        r = np.linalg.norm(P - Q)
                        ref += sab * scd * (2 * math.sqrt(rho / math.pi) if r < 1e-12 else erf(math.sqrt(rho) * r) / r)
        got = oracle_lib.eri(X[0], X[1], X[2], X[3], E3, C3)
        assert got == pytest.approx(ref, rel=1e-13)


def test_eightfold_symmetry(oracle_lib):
    rng = np.random.default_rng(3)
    A, B, C, D = rng.uniform(-2, 2, (4, 3))
    ref = oracle_lib.eri(A, B, C, D, E3, C3)
    for perm in [(B, A, C, D), (A, B, D, C), (B, A, D, C), (C, D, A, B), (D, C, A, B), (C, D, B, A), (D, C, B, A)]:
        assert oracle_lib.eri(*perm, E3, C3) == pytest.approx(ref, rel=1e-14)
    # and it is not symmetric under a swap across bra and ket (ik|jl)
    assert abs(oracle_lib.eri(A, C, B, D, E3, C3) - ref) > 1e-6 * ref


def test_schwarz_bounds_all_quartets(oracle_lib):
    s = random_cluster(5, 21, box=5.0)
    Q = oracle_lib.schwarz(s.xyz, E3, C3)
    n = s.natoms
    def q(i, j):
        i, j = max(i, j), min(i, j)
        return Q[i * (i + 1) // 2 + j]
    for i in range(n):
        for j in range(n):
            assert q(i, j) ** 2 == pytest.approx(oracle_lib.eri(s.xyz[i], s.xyz[j], s.xyz[i], s.xyz[j], E3, C3), rel=1e-14)
            for k in range(n):
                for l in range(n):
                    v = oracle_lib.eri(s.xyz[i], s.xyz[j], s.xyz[k], s.xyz[l], E3, C3)
                    assert abs(v) <= q(i, j) * q(k, l) * (1 + 1e-13)


# ------------------------------------------------------------------ Fock build

@pytest.mark.parametrize("n,seed,box,tau", [(1, 1, 1.0, 0.0), (2, 2, 3.0, 0.0), (4, 3, 4.0, 0.0),
                                            (5, 4, 4.0, 0.0), (6, 5, 9.0, 1e-4), (6, 6, 12.0, 1e-6)])
def test_unique_scatter_equals_plain_definition(oracle_lib, n, seed, box, tau):
    s = random_cluster(n, seed, box=box)
    Fb, Eb = oracle_lib.fock_bruteforce(s.xyz, s.dens, E3, C3, tau)
    Fu, Eu, ns = oracle_lib.fock(s.xyz, s.dens, E3, C3, tau)
    scale = np.abs(Fb).max()
    assert np.abs(Fu - Fb).max() <= 1e-14 * scale
    assert Eu == pytest.approx(Eb, rel=1e-14)
    assert np.array_equal(Fu, Fu.T)
    P = n * (n + 1) // 2
    Q = oracle_lib.schwarz(s.xyz, E3, C3)
    kept = sum(1 for a in range(P) for b in range(a + 1) if Q[a] * Q[b] >= tau)
    assert ns == kept
    if tau > 0:
        assert kept < P * (P + 1) // 2  # the screen removed something


def test_screening_changes_result_consistently(oracle_lib):
    s = random_cluster(6, 6, box=12.0)
    F0, _, n0 = oracle_lib.fock(s.xyz, s.dens, E3, C3, 0.0)
    F1, _, n1 = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-6)
    assert n1 < n0
    assert 0 < np.abs(F1 - F0).max() < 1e-5


def test_single_atom(oracle_lib):
    # G_11 = D_11 [(11|11) - 1/2 (11|11)]
    xyz = np.array([[0.2, 0.1, -0.3]])
    D = np.array([[0.8]])
    F, E2, _ = oracle_lib.fock(xyz, D, E3, C3, 0.0)
    j = 1.0557129304699764
    assert F[0, 0] == pytest.approx(0.5 * 0.8 * j, rel=1e-13)
    assert E2 == pytest.approx(0.5 * 0.8 * 0.5 * 0.8 * j, rel=1e-13)


def test_two_distant_atoms(oracle_lib):
    """Two atoms 40 bohr apart: the overlap pair is screened away, leaving Coulomb between
    the atoms as S^2/R point charges and the on-site halves."""
    R = 40.0
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, R, 0.0]])
    D = np.array([[1.0, 0.3], [0.3, 0.7]])
    F, E2, _ = oracle_lib.fock(xyz, D, E3, C3, 1e-12)
    j = 1.0557129304699764
    s = oracle_lib.overlap(xyz[0], xyz[0], E3, C3)
    jab = s * s / R
    assert F[0, 0] == pytest.approx(0.5 * D[0, 0] * j + D[1, 1] * jab, rel=1e-13)
    assert F[1, 1] == pytest.approx(0.5 * D[1, 1] * j + D[0, 0] * jab, rel=1e-13)
    # off-diagonal: (01|kl) screened for all kl; exchange -1/2 D_10 (00|11)
    assert F[0, 1] == pytest.approx(-0.5 * D[1, 0] * jab, rel=1e-12)


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q


def test_invariances(oracle_lib):
    s = random_cluster(5, 9, box=5.0)
    F, E2, _ = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-9)
    Ft, Et, _ = oracle_lib.fock(s.xyz + np.array([3.0, -7.0, 11.0]), s.dens, E3, C3, 1e-9)
    Fr, Er, _ = oracle_lib.fock(s.xyz @ _rot(1).T, s.dens, E3, C3, 1e-9)
    perm = np.array([3, 0, 4, 1, 2])
    Fp, Ep, _ = oracle_lib.fock(s.xyz[perm], s.dens[np.ix_(perm, perm)], E3, C3, 1e-9)
    sc = np.abs(F).max()
    assert np.abs(Ft - F).max() < 1e-12 * sc
    assert np.abs(Fr - F).max() < 1e-12 * sc
    assert np.abs(Fp - F[np.ix_(perm, perm)]).max() < 1e-13 * sc
    for e in (Et, Er, Ep):
        assert e == pytest.approx(E2, rel=1e-12)


def test_linearity_and_quadratic_energy(oracle_lib):
    s = random_cluster(5, 10, box=6.0)
    D2 = random_cluster(5, 99).dens
    F1, E1, _ = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-8)
    F2, _, _ = oracle_lib.fock(s.xyz, D2, E3, C3, 1e-8)
    F12, _, _ = oracle_lib.fock(s.xyz, s.dens + D2, E3, C3, 1e-8)
    assert np.abs(F12 - F1 - F2).max() < 1e-13 * np.abs(F12).max()
    for lam in (0.5, 2.0, -3.0):
        _, El, _ = oracle_lib.fock(s.xyz, lam * s.dens, E3, C3, 1e-8)
        assert El == pytest.approx(lam * lam * E1, rel=1e-13)


def test_energy_derivative_wrt_density_is_G(oracle_lib):
    s = random_cluster(4, 12, box=5.0)
    G, E, _ = oracle_lib.fock(s.xyz, s.dens, E3, C3, 0.0)
    h = 1e-3
    for (i, j) in [(0, 0), (1, 0), (3, 2), (2, 2)]:
        Dp = s.dens.copy(); Dm = s.dens.copy()
        Dp[i, j] += h; Dm[i, j] -= h
        if i != j:
            Dp[j, i] += h; Dm[j, i] -= h
        _, Ep, _ = oracle_lib.fock(s.xyz, Dp, E3, C3, 0.0)
        _, Em, _ = oracle_lib.fock(s.xyz, Dm, E3, C3, 0.0)
        fd = (Ep - Em) / (2 * h)
        expect = G[i, j] * (1 if i == j else 2)
        assert fd == pytest.approx(expect, rel=1e-10, abs=1e-12)


def test_fock_element_equals_bruteforce(oracle_lib):
    s = random_cluster(5, 13, box=7.0)
    tau = 1e-7
    Fb, _ = oracle_lib.fock_bruteforce(s.xyz, s.dens, E3, C3, tau)
    Q = oracle_lib.schwarz(s.xyz, E3, C3)
    for (i, j) in [(0, 0), (4, 1), (2, 3)]:
        assert oracle_lib.fock_element(s.xyz, s.dens, E3, C3, tau, Q, i, j) == pytest.approx(Fb[i, j], rel=1e-14, abs=1e-16)


def test_bra_range_partition_sums(oracle_lib):
    """Splitting the bra loop into ranges and summing gives the full build (used by the CPU
    baseline, which times a bounded bra range)."""
    s = random_cluster(6, 14, box=5.0)
    F, E, ns = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-10)
    Fa, _, na = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-10, bra_range=(0, 9))
    Fb, _, nb = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-10, bra_range=(9, 21))
    assert na + nb == ns
    assert np.abs(Fa + Fb - F).max() < 1e-14 * np.abs(F).max()


# ------------------------------------------------------------------ gradient

def test_gradient_vs_finite_differences(oracle_lib):
    s = random_cluster(4, 15, box=4.0)
    g, Eg, _ = oracle_lib.grad(s.xyz, s.dens, E3, C3, 0.0)
    _, E, _ = oracle_lib.fock(s.xyz, s.dens, E3, C3, 0.0)
    assert Eg == pytest.approx(E, rel=1e-13)
    h = 1e-4
    fd = np.zeros_like(g)
    for a in range(s.natoms):
        for x in range(3):
            xp = s.xyz.copy(); xm = s.xyz.copy()
            xp[a, x] += h; xm[a, x] -= h
            fd[a, x] = (oracle_lib.fock(xp, s.dens, E3, C3, 0.0)[1] - oracle_lib.fock(xm, s.dens, E3, C3, 0.0)[1]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max())


def test_gradient_net_force_and_torque(oracle_lib):
    s = random_cluster(6, 16, box=6.0)
    g, _, _ = oracle_lib.grad(s.xyz, s.dens, E3, C3, 1e-9)
    sc = np.abs(g).max()
    assert np.abs(g.sum(axis=0)).max() < 1e-13 * max(sc, 1)
    c = s.xyz - s.xyz.mean(axis=0)
    torque = np.cross(c, g).sum(axis=0)
    assert np.abs(torque).max() < 1e-12 * max(sc, 1)


def _sym_matrix(rng, n):
    m = rng.uniform(-1.0, 1.0, size=(n, n))
    return 0.5 * (m + m.T)


def test_grad_pair_vs_finite_differences(oracle_lib):
    """The pairing L(R) = sum W o G(R) with a fixed symmetric W: its gradient against
    central differences of the forward oracle (tau = 0 and tau > 0, screen held fixed by a
    geometry step far from any threshold)."""
    rng = np.random.default_rng(31)
    for tau in (0.0, 1e-9):
        s = random_cluster(5, 32, box=4.5)
        W = _sym_matrix(rng, s.natoms)
        g = oracle_lib.grad_pair(s.xyz, s.dens, W, E3, C3, tau)
        h = 1e-4
        Q = oracle_lib.schwarz(s.xyz, E3, C3)
        fd = np.zeros_like(g)
        for a in range(s.natoms):
            for x in range(3):
                xp = s.xyz.copy(); xm = s.xyz.copy()
                xp[a, x] += h; xm[a, x] -= h
                # the screen is a property of the base geometry: pass its Q to both steps
                Gp = oracle_lib.fock(xp, s.dens, E3, C3, tau, Q=Q)[0]
                Gm = oracle_lib.fock(xm, s.dens, E3, C3, tau, Q=Q)[0]
                fd[a, x] = (np.sum(W * Gp) - np.sum(W * Gm)) / (2 * h)
        assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max()), tau


def test_grad_pair_special_cases(oracle_lib):
    """X = D/2 reduces the pairing to E2 (same gradient as grad); linear in X; the pull-back
    of W through D -> G is G(W) (sum W o G(D) = sum D o G(W): the map is self-adjoint)."""
    rng = np.random.default_rng(33)
    s = random_cluster(6, 34, box=5.0)
    g, _, _ = oracle_lib.grad(s.xyz, s.dens, E3, C3, 1e-10)
    gp = oracle_lib.grad_pair(s.xyz, s.dens, 0.5 * s.dens, E3, C3, 1e-10)
    assert np.abs(gp - g).max() <= 1e-13 * np.abs(g).max()
    W1, W2 = _sym_matrix(rng, s.natoms), _sym_matrix(rng, s.natoms)
    a = oracle_lib.grad_pair(s.xyz, s.dens, W1, E3, C3, 1e-10)
    b = oracle_lib.grad_pair(s.xyz, s.dens, W2, E3, C3, 1e-10)
    c = oracle_lib.grad_pair(s.xyz, s.dens, 2.0 * W1 - 3.0 * W2, E3, C3, 1e-10)
    assert np.abs(c - (2.0 * a - 3.0 * b)).max() <= 1e-12 * np.abs(c).max()
    GD = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-10)[0]
    GW = oracle_lib.fock(s.xyz, W1, E3, C3, 1e-10)[0]
    assert np.sum(W1 * GD) == pytest.approx(np.sum(s.dens * GW), rel=1e-13)


def test_config_he64_matches_fixture(oracle_lib):
    """The 64-atom build against the stored fixture written by tests/golden/make_golden.py."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "he64_fp64.txt")
    lines = open(path).read().split("\n")
    e2_ref = float([l for l in lines if l.startswith("# E2")][0].split()[2])
    ns_ref = int([l for l in lines if l.startswith("# survivors")][0].split()[2])
    s = config_system("he64_fp64")
    F, E2, ns = oracle_lib.fock(s.xyz, s.dens, E3, C3, s.tau)
    assert ns == ns_ref
    assert E2 == pytest.approx(e2_ref, rel=1e-13)
    Fref = np.loadtxt(path)
    assert np.abs(F - Fref).max() <= 1e-13 * np.abs(Fref).max()


def test_he512_fixture_elements_match_element_definition(oracle_lib):
    """Entries of the stored 512-atom build (written by the unique-quartet oracle) against
    the element-wise plain definition, a separate code path; the stored matrix is symmetric
    and its energy is 1/2 sum D o G."""
    import os
    from gpu_util import load_full
    G, e2, _ = load_full("he512_fp64")
    s = config_system("he512_fp64")
    assert G.shape == (512, 512) and np.array_equal(G, G.T)
    assert 0.5 * float(np.sum(s.dens * G)) == pytest.approx(e2, rel=1e-13)
    Q = oracle_lib.schwarz(s.xyz, E3, C3)
    scale = np.abs(G).max()
    rng = np.random.default_rng(5120)
    idx = [(0, 0), (511, 0), (511, 511)] + [tuple(int(v) for v in p) for p in rng.integers(0, 512, (5, 2))]
    for i, j in idx:
        e = oracle_lib.fock_element(s.xyz, s.dens, E3, C3, s.tau, Q, i, j)
        assert abs(e - G[i, j]) <= 1e-12 * scale, (i, j)


# ------------------------------------------------------------------ per-atom bases

from he_inputs import H_STO3G_EXPS as EH, random_basis_rows  # noqa: E402


@pytest.mark.parametrize("R", [0.0, 1e-4, 0.7, 2.0, 6.0])
@pytest.mark.parametrize("a,b", [(0.4, 2.5), (3.0, 0.15)])
def test_eri4_two_gaussian_charges_unequal(oracle_lib, R, a, b):
    """One normalised primitive on A (exponent a) and one on B (exponent b): g_a^2 and g_b^2 are
    unit Gaussian charges of exponents 2a and 2b, interacting as erf(sqrt(r) R) / R with the
    reduced exponent r = (2a)(2b)/(2a + 2b), and 2 sqrt(r/pi) at R = 0."""
    A = np.array([0.2, -0.1, 0.3])
    d = np.array([0.3, 1.0, -0.7])
    B = A + R * d / np.linalg.norm(d)
    r = 4.0 * a * b / (2.0 * a + 2.0 * b)
    ref = 2.0 * math.sqrt(r / math.pi) if R == 0 else erf(math.sqrt(r) * R) / R
    ba, bb = ([a], [1.0]), ([b], [1.0])
    assert oracle_lib.eri4(A, A, B, B, ba, ba, bb, bb) == pytest.approx(ref, rel=1e-13, abs=1e-15)
    # the same pair of charges seen from the other side
    assert oracle_lib.eri4(B, B, A, A, bb, bb, ba, ba) == pytest.approx(ref, rel=1e-13, abs=1e-15)


def test_eri4_scaling_law(oracle_lib):
    """Exponents times l^2 and lengths divided by l map each normalised function to
    l^(3/2) phi(l r); the Coulomb integral then scales by l."""
    rng = np.random.default_rng(17)
    X = rng.uniform(-2, 2, (4, 3))
    e, c = random_basis_rows(4, 3, 18)
    basis = [(e[k], c[k]) for k in range(4)]
    ref = oracle_lib.eri4(*X, *basis)
    for lam in (0.5, 1.7, 3.0):
        scaled = [(e[k] * lam * lam, c[k]) for k in range(4)]
        got = oracle_lib.eri4(*(X / lam), *scaled)
        assert got == pytest.approx(lam * ref, rel=1e-13)


def test_eri4_eightfold_symmetry(oracle_lib):
    """Permuting the centres together with their own contractions leaves (ij|kl) unchanged;
    swapping only the contractions of two centres changes it."""
    rng = np.random.default_rng(19)
    A, B, C, D = rng.uniform(-2, 2, (4, 3))
    e, c = random_basis_rows(4, 3, 20)
    a, b, cc, d = [(e[k], c[k]) for k in range(4)]
    ref = oracle_lib.eri4(A, B, C, D, a, b, cc, d)
    for pts, bs in [((B, A, C, D), (b, a, cc, d)), ((A, B, D, C), (a, b, d, cc)), ((C, D, A, B), (cc, d, a, b)),
                    ((D, C, B, A), (d, cc, b, a)), ((B, A, D, C), (b, a, d, cc)), ((C, D, B, A), (cc, d, b, a)),
                    ((D, C, A, B), (d, cc, a, b))]:
        assert oracle_lib.eri4(*pts, *bs) == pytest.approx(ref, rel=1e-14)
    assert abs(oracle_lib.eri4(A, B, C, D, b, a, cc, d) - ref) > 1e-6 * abs(ref)


def test_eri4_gaussian_charge_form(oracle_lib):
    """Each primitive (ab|cd) with its own exponents on every centre is S_ab S_cd erf(sqrt(rho)
    |P-Q|) / |P-Q|: two spherical Gaussian charges of exponents p and q at the product centres."""
    rng = np.random.default_rng(23)
    e, c = random_basis_rows(4, 2, 24)
    w = c * (2 * e / math.pi) ** 0.75
    X = rng.uniform(-1.5, 1.5, (4, 3))
    ref = 0.0
    for a in range(2):
        for b in range(2):
            p = e[0, a] + e[1, b]
            P = (e[0, a] * X[0] + e[1, b] * X[1]) / p
            sab = w[0, a] * w[1, b] * (math.pi / p) ** 1.5 * math.exp(-e[0, a] * e[1, b] / p * np.sum((X[0] - X[1]) ** 2))
            for cc in range(2):
                for d in range(2):
                    q = e[2, cc] + e[3, d]
                    Q = (e[2, cc] * X[2] + e[3, d] * X[3]) / q
                    scd = w[2, cc] * w[3, d] * (math.pi / q) ** 1.5 * math.exp(-e[2, cc] * e[3, d] / q * np.sum((X[2] - X[3]) ** 2))
                    rho = p * q / (p + q)
                    r = np.linalg.norm(P - Q)
                    ref += sab * scd * erf(math.sqrt(rho) * r) / r
    got = oracle_lib.eri4(*X, *[(e[k], c[k]) for k in range(4)])
    assert got == pytest.approx(ref, rel=1e-13)


def _rows_cluster(n, seed, box, g=3):
    s = random_cluster(n, seed, box=box)
    e, c = random_basis_rows(n, g, seed + 100)
    return s, e, c


@pytest.mark.parametrize("n,seed,box,tau", [(1, 1, 1.0, 0.0), (2, 2, 3.0, 0.0), (4, 3, 4.0, 0.0),
                                            (5, 4, 5.0, 0.0), (6, 5, 9.0, 1e-4), (6, 6, 12.0, 1e-6)])
def test_fock_atoms_equals_plain_definition(oracle_lib, n, seed, box, tau):
    s, e, c = _rows_cluster(n, seed, box)
    Fb, Eb = oracle_lib.fock_bruteforce_atoms(s.xyz, s.dens, e, c, tau)
    Fu, Eu, ns = oracle_lib.fock_atoms(s.xyz, s.dens, e, c, tau)
    assert np.abs(Fu - Fb).max() <= 1e-14 * np.abs(Fb).max()
    assert Eu == pytest.approx(Eb, rel=1e-14)
    assert np.array_equal(Fu, Fu.T)
    P = n * (n + 1) // 2
    Q = oracle_lib.schwarz_atoms(s.xyz, e, c)
    assert ns == sum(1 for a in range(P) for b in range(a + 1) if Q[a] * Q[b] >= tau)


def test_schwarz_atoms_bounds_all_quartets(oracle_lib):
    s, e, c = _rows_cluster(4, 31, 4.0)
    Q = oracle_lib.schwarz_atoms(s.xyz, e, c)
    b = [(e[k], c[k]) for k in range(4)]

    def q(i, j):
        i, j = max(i, j), min(i, j)
        return Q[i * (i + 1) // 2 + j]
    for i in range(4):
        for j in range(4):
            assert q(i, j) ** 2 == pytest.approx(oracle_lib.eri4(s.xyz[i], s.xyz[j], s.xyz[i], s.xyz[j],
                                                                 b[i], b[j], b[i], b[j]), rel=1e-14)
            for k in range(4):
                for l in range(4):
                    v = oracle_lib.eri4(s.xyz[i], s.xyz[j], s.xyz[k], s.xyz[l], b[i], b[j], b[k], b[l])
                    assert abs(v) <= q(i, j) * q(k, l) * (1 + 1e-13)


def test_fock_atoms_with_identical_rows_is_the_one_basis_build(oracle_lib):
    s = random_cluster(7, 41, box=6.0)
    e = np.tile(E3, (7, 1))
    c = np.tile(C3, (7, 1))
    Fa, Ea, na = oracle_lib.fock_atoms(s.xyz, s.dens, e, c, 1e-8, nthreads=1)
    Fu, Eu, nu = oracle_lib.fock(s.xyz, s.dens, E3, C3, 1e-8, nthreads=1)
    assert np.array_equal(Fa, Fu) and Ea == Eu and na == nu


def test_fock_atoms_permutation_equivariance(oracle_lib):
    """Relabelling the atoms, each keeping its own contraction, permutes G and keeps E2."""
    s, e, c = _rows_cluster(6, 43, 6.0)
    perm = np.array([3, 0, 5, 1, 4, 2])
    F, E, _ = oracle_lib.fock_atoms(s.xyz, s.dens, e, c, 0.0)
    Fp, Ep, _ = oracle_lib.fock_atoms(s.xyz[perm], s.dens[np.ix_(perm, perm)], e[perm], c[perm], 0.0)
    assert np.abs(Fp - F[np.ix_(perm, perm)]).max() <= 1e-14 * np.abs(F).max()
    assert Ep == pytest.approx(E, rel=1e-14)
    # attaching the contractions to the wrong atoms changes the result
    Fw, _, _ = oracle_lib.fock_atoms(s.xyz, s.dens, e[perm], c[perm], 0.0)
    assert np.abs(Fw - F).max() > 1e-3 * np.abs(F).max()


def test_fock_atoms_h_and_he_far_apart(oracle_lib):
    """H at the origin and He 40 bohr away: on-site halves of each atom's own (ii|ii), Coulomb
    between them as point charges S_HH S_HeHe / R, and the exchange of the screened pair."""
    R = 40.0
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    D = np.array([[0.9, 0.2], [0.2, 1.1]])
    e = np.stack([EH, E3])
    c = np.stack([C3, C3])
    F, _, _ = oracle_lib.fock_atoms(xyz, D, e, c, 1e-12)
    jh = oracle_lib.eri(xyz[0], xyz[0], xyz[0], xyz[0], EH, C3)
    jhe = oracle_lib.eri(xyz[1], xyz[1], xyz[1], xyz[1], E3, C3)
    sh = oracle_lib.overlap(xyz[0], xyz[0], EH, C3)
    she = oracle_lib.overlap(xyz[1], xyz[1], E3, C3)
    jab = sh * she / R
    assert F[0, 0] == pytest.approx(0.5 * D[0, 0] * jh + D[1, 1] * jab, rel=1e-13)
    assert F[1, 1] == pytest.approx(0.5 * D[1, 1] * jhe + D[0, 0] * jab, rel=1e-13)
    assert F[0, 1] == pytest.approx(-0.5 * D[1, 0] * jab, rel=1e-12)
    # hydrogen is the more diffuse atom: its on-site repulsion is the smaller one
    assert jh < jhe


def test_grad_atoms_vs_finite_differences(oracle_lib):
    s, e, c = _rows_cluster(4, 47, 3.5)
    g, E, _ = oracle_lib.grad_atoms(s.xyz, s.dens, e, c, 0.0)
    _, E2, _ = oracle_lib.fock_atoms(s.xyz, s.dens, e, c, 0.0)
    assert E == pytest.approx(E2, rel=1e-13)
    h = 1e-4
    fd = np.zeros_like(g)
    for a in range(4):
        for x in range(3):
            xp = s.xyz.copy(); xp[a, x] += h
            xm = s.xyz.copy(); xm[a, x] -= h
            fd[a, x] = (oracle_lib.fock_atoms(xp, s.dens, e, c, 0.0)[1] -
                        oracle_lib.fock_atoms(xm, s.dens, e, c, 0.0)[1]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(g).max())
    assert np.abs(g.sum(axis=0)).max() <= 1e-12 * np.abs(g).max()


def test_grad_pair_atoms_vs_finite_differences(oracle_lib):
    """The pairing sum W o G(R) with per-atom bases: its position derivative (screen held
    fixed) against central differences, and X = D/2 reproduces the energy gradient."""
    s, e, c = _rows_cluster(4, 53, 3.5)
    rng = np.random.default_rng(54)
    W = rng.uniform(-1, 1, (4, 4))
    W = 0.5 * (W + W.T)
    g = oracle_lib.grad_pair_atoms(s.xyz, s.dens, W, e, c, 0.0)
    h = 1e-4
    fd = np.zeros_like(g)
    for a in range(4):
        for x in range(3):
            xp = s.xyz.copy(); xp[a, x] += h
            xm = s.xyz.copy(); xm[a, x] -= h
            Gp = oracle_lib.fock_atoms(xp, s.dens, e, c, 0.0)[0]
            Gm = oracle_lib.fock_atoms(xm, s.dens, e, c, 0.0)[0]
            fd[a, x] = np.sum(W * (Gp - Gm)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(g).max())
    ge, _, _ = oracle_lib.grad_atoms(s.xyz, s.dens, e, c, 0.0)
    gh = oracle_lib.grad_pair_atoms(s.xyz, s.dens, 0.5 * s.dens, e, c, 0.0)
    assert np.abs(gh - ge).max() <= 1e-12 * np.abs(ge).max()


# ------------------------------------------------------------------ one-electron integrals and SCF

def _quad1(f, lo=-40.0, hi=40.0, pts=None):
    v, _ = integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=400, points=pts)
    return v


def test_one_electron_overlap_and_kinetic_by_quadrature(oracle_lib):
    """S and T of two contracted functions with their own exponents, as sums of products of
    1-D integrals: S = prod_x <g|g>_x and T = sum_x 1/2 <g'|g'>_x prod_{y != x} <g|g>_y."""
    rng = np.random.default_rng(61)
    xyz = rng.uniform(-1.0, 1.0, (2, 3))
    e, c = random_basis_rows(2, 2, 62)
    S, T, V = oracle_lib.one_electron_atoms(xyz, [1.0, 2.0], e, c)
    w = c * (2 * e / math.pi) ** 0.75
    Sref = Tref = 0.0
    for a in range(2):
        for b in range(2):
            A, B, al, be = xyz[0], xyz[1], e[0, a], e[1, b]
            ov, ki = [], []
            for x in range(3):
                g1 = lambda s, x=x: math.exp(-al * (s - A[x]) ** 2)
                g2 = lambda s, x=x: math.exp(-be * (s - B[x]) ** 2)
                ov.append(_quad1(lambda s: g1(s) * g2(s), pts=[A[x], B[x]]))
                ki.append(0.5 * _quad1(lambda s: (-2 * al * (s - A[x]) * g1(s)) * (-2 * be * (s - B[x]) * g2(s)),
                                       pts=[A[x], B[x]]))
            pref = w[0, a] * w[1, b]
            Sref += pref * ov[0] * ov[1] * ov[2]
            Tref += pref * (ki[0] * ov[1] * ov[2] + ov[0] * ki[1] * ov[2] + ov[0] * ov[1] * ki[2])
    assert S[0, 1] == pytest.approx(Sref, rel=1e-12)
    assert T[0, 1] == pytest.approx(Tref, rel=1e-11)
    assert S[1, 0] == S[0, 1] and T[1, 0] == T[0, 1]


@pytest.mark.parametrize("alpha,Z", [(0.4, 1.0), (3.0, 2.0)])
def test_nuclear_attraction_on_centre(oracle_lib, alpha, Z):
    """|g|^2 of a normalised primitive is a unit Gaussian charge of exponent 2a; a nucleus at its
    centre feels -Z 2 sqrt(2a/pi)."""
    S, T, V = oracle_lib.one_electron_atoms(np.zeros((1, 3)), [Z], [[alpha]], [[1.0]])
    assert S[0, 0] == pytest.approx(1.0, rel=1e-14)
    assert V[0, 0] == pytest.approx(-Z * 2.0 * math.sqrt(2 * alpha / math.pi), rel=1e-13)
    # kinetic energy of a normalised s Gaussian: 3a/2 (virial of the harmonic form)
    assert T[0, 0] == pytest.approx(1.5 * alpha, rel=1e-13)


def test_nuclear_attraction_as_charge_cloud(oracle_lib):
    """Each primitive product is a Gaussian charge S_ab of exponent p at P: a nucleus C away
    adds -Z_C S_ab erf(sqrt(p) |P - C|) / |P - C| (the charge-cloud route, not F0)."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.9, -0.3, 0.4], [2.5, 1.0, -1.5]])
    Zs = [0.0, 0.0, 1.7]      # only the third atom carries a nucleus
    e = np.array([[1.3], [0.6], [2.0]])
    c = np.ones((3, 1))
    S, T, V = oracle_lib.one_electron_atoms(xyz, Zs, e, c)
    a, b = 1.3, 0.6
    p = a + b
    P = (a * xyz[0] + b * xyz[1]) / p
    r = np.linalg.norm(P - xyz[2])
    ref = -1.7 * S[0, 1] * erf(math.sqrt(p) * r) / r
    assert V[0, 1] == pytest.approx(ref, rel=1e-13)
    # far away the cloud is a point charge
    xyz_far = xyz.copy()
    xyz_far[2] = [0.0, 0.0, 80.0]
    S2, _, V2 = oracle_lib.one_electron_atoms(xyz_far, Zs, e, c)
    assert V2[0, 0] == pytest.approx(-1.7 * S2[0, 0] / np.linalg.norm(xyz_far[2]), rel=1e-12)


def _scf_system(shape, seed, tau=1e-12):
    from he_inputs import mixed_lattice
    s = mixed_lattice(shape, seed=seed, tau=tau)
    Z = np.where(s.exps[:, 0] < 5.0, 1.0, 2.0)
    return s, Z, int(Z.sum()) // 2


def test_scf_single_function_closed_form(oracle_lib):
    """One He atom, one basis function: D = 2/S, and E = 2 h / S + J / S^2 with h = T + V and
    J = (11|11), each pinned on its own above."""
    from oracle.scf import scf
    xyz = np.zeros((1, 3))
    r = scf(xyz, [2.0], [E3], [C3], 1, 0.0)
    S, T, V = oracle_lib.one_electron_atoms(xyz, [2.0], [E3], [C3])
    h = T[0, 0] + V[0, 0]
    J = oracle_lib.eri(xyz[0], xyz[0], xyz[0], xyz[0], E3, C3)
    assert r["converged"]
    assert r["D"][0, 0] == pytest.approx(2.0 / S[0, 0], rel=1e-14)
    assert r["E"] == pytest.approx(2 * h / S[0, 0] + J / S[0, 0] ** 2, rel=1e-13)
    assert r["E"] == pytest.approx(-2.807783957, abs=2e-9)   # minimal-basis helium


# STO-3G fit of a 1s Slater function of unit exponent; a Slater exponent zeta scales the
# Gaussian exponents by zeta^2 (the coefficients are C3).
STO3G_UNIT_EXPS = np.array([2.227660, 0.405771, 0.109818])


def test_scf_textbook_h2():
    """H2 at R = 1.4 bohr in STO-3G (zeta 1.24): the minimal-basis example of Szabo and Ostlund,
    Modern Quantum Chemistry (section 3.5), whose electronic energy is -1.8310 hartree
    (total -1.1167).  Pins the two-centre overlap, kinetic, nuclear-attraction and
    two-electron integrals and the SCF loop against numbers computed elsewhere."""
    from he_inputs import H_STO3G_EXPS
    from oracle.scf import scf
    R = 1.4
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    r = scf(xyz, [1.0, 1.0], np.tile(H_STO3G_EXPS, (2, 1)), np.tile(C3, (2, 1)), 1, 0.0)
    assert r["converged"]
    assert r["E"] - 1.0 / R == pytest.approx(-1.8310, abs=5e-5)
    assert r["E"] == pytest.approx(-1.1167, abs=5e-5)
    # the same exponents from the unit-exponent fit
    assert np.allclose(STO3G_UNIT_EXPS * 1.24 ** 2, H_STO3G_EXPS, rtol=5e-6)


def test_scf_textbook_heh_cation():
    """HeH+ at R = 1.4632 bohr, STO-3G with zeta 2.0925 (He) and 1.24 (H): the worked example of
    Szabo and Ostlund (section 3.5 and the SCF program of their appendix B): electronic energy
    -4.227529, total -2.860662 hartree, orbital energies -1.5974 and -0.0617.  Two different
    nuclei, per-atom bases and an asymmetric density."""
    from he_inputs import H_STO3G_EXPS
    from oracle.scf import scf
    R = 1.4632
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    exps = np.stack([STO3G_UNIT_EXPS * 2.0925 ** 2, H_STO3G_EXPS])
    r = scf(xyz, [2.0, 1.0], exps, np.tile(C3, (2, 1)), 1, 0.0)
    assert r["converged"]
    # the printed exponents carry six digits: 1e-5 hartree covers their rounding
    assert r["E"] - 2.0 / R == pytest.approx(-4.227529, abs=1e-5)
    assert r["E"] == pytest.approx(-2.860662, abs=1e-5)
    assert r["eps"] == pytest.approx([-1.5974, -0.0617], abs=1e-4)


def test_scf_filled_shell_is_inverse_overlap(oracle_lib):
    """Every orbital occupied (He only): D = 2 S^-1 whatever F is."""
    from oracle.scf import scf
    s = random_cluster(6, 71, box=5.0)
    r = scf(s.xyz, np.full(6, 2.0), np.tile(E3, (6, 1)), np.tile(C3, (6, 1)), 6, 1e-12)
    assert r["converged"] and r["iterations"] <= 3
    assert np.abs(r["D"] @ r["S"] - 2 * np.eye(6)).max() < 1e-10


def test_scf_converged_properties(oracle_lib):
    """H/He 32: converged; D S D = 2 D, tr(D S) = 2 nocc, the commutator vanishes, orbitals are
    S-orthonormal and ascending, and E is the trace formula for the returned D."""
    from oracle.scf import scf
    s, Z, nocc = _scf_system((4, 4, 2), 16)
    r = scf(s.xyz, Z, s.exps, s.coefs, nocc, s.tau)
    assert r["converged"]
    D, S, F, H = r["D"], r["S"], r["F"], r["H"]
    assert np.abs(D @ S @ D - 2 * D).max() < 1e-7
    assert np.trace(D @ S) == pytest.approx(2 * nocc, rel=1e-10)
    assert np.abs(F @ D @ S - S @ D @ F).max() < 1e-6
    C = r["C"]
    assert np.abs(C.T @ S @ C - np.eye(len(Z))).max() < 1e-10
    assert np.all(np.diff(r["eps"]) >= 0)
    G = oracle_lib.fock_atoms(s.xyz, D, s.exps, s.coefs, s.tau)[0]
    Eref = 0.5 * np.sum(D * (2 * H + G)) + r["enn"]
    assert r["E"] == pytest.approx(Eref, rel=1e-13)


def test_scf_rotation_invariance_and_variational(oracle_lib):
    """E is unchanged by a rigid rotation, and lies below the energy of the core-Hamiltonian
    guess density (both idempotent, the SCF one variationally optimal)."""
    from oracle.scf import scf, density_from, orthogonaliser, nuclear_repulsion
    s, Z, nocc = _scf_system((4, 2, 2), 18)
    r = scf(s.xyz, Z, s.exps, s.coefs, nocc, s.tau)
    R = _rot(3)
    r2 = scf(s.xyz @ R.T, Z, s.exps, s.coefs, nocc, s.tau)
    assert r2["E"] == pytest.approx(r["E"], rel=1e-11)
    S, T, V = oracle_lib.one_electron_atoms(s.xyz, Z, s.exps, s.coefs)
    H = T + V
    D0, _, _ = density_from(H, orthogonaliser(S), nocc)
    G0 = oracle_lib.fock_atoms(s.xyz, D0, s.exps, s.coefs, s.tau)[0]
    E0 = 0.5 * np.sum(D0 * (2 * H + G0)) + nuclear_repulsion(s.xyz, Z)
    assert r["E"] < E0
