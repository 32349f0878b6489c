"""GPU parity of the Fock build with per-atom bases (every atom its own contraction) against
the CPU oracle's per-atom functions, through the C ABI."""
import numpy as np
import pytest

import oracle
from he_inputs import mixed_lattice, random_basis_rows, random_cluster, config_system
from gpu_util import announce, assert_close, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _run(torch_dev, xyz, dens, exps, coefs, tau, precision="fp64", strategy=0):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    n, g = exps.shape
    X = torch.tensor(xyz, device=dev)
    D = torch.tensor(dens, device=dev)
    ws = hfk.new_workspace(hfk.workspace_bytes_atoms(n, g, precision), dev)
    G, E2 = hfk.fock_atoms(X, D, exps, coefs, tau, precision=precision, strategy=strategy, workspace=ws)
    st = hfk.read_stats(ws)
    return G.cpu().numpy(), float(E2.item()), st


def _kept_quartets(Q, tau):
    """Unique quartets {ab, cd} (ab >= cd) with Q_ab Q_cd >= tau, counted from the sorted bounds."""
    q = np.sort(Q[Q > 0])
    k = len(q) - np.searchsorted(q, tau / q, side="left")   # partners b with q_b >= tau / q_a
    diag = int(np.sum(q * q >= tau))
    return (int(k.sum()) + diag) // 2


@pytest.mark.parametrize("n,seed,box,tau", [(1, 1, 1.0, 0.0), (2, 2, 3.0, 0.0), (3, 3, 3.0, 0.0),
                                            (5, 4, 4.0, 0.0), (7, 5, 6.0, 1e-6), (8, 6, 12.0, 1e-8)])
def test_atoms_tiny_vs_bruteforce(torch_dev, n, seed, box, tau):
    s = random_cluster(n, seed, box=box)
    e, c = random_basis_rows(n, 3, seed + 50)
    announce("atoms tiny n=%d seed=%d tau=%g" % (n, seed, tau))
    G, E2, _ = _run(torch_dev, s.xyz, s.dens, e, c, tau)
    Gb, Eb = oracle.fock_bruteforce_atoms(s.xyz, s.dens, e, c, tau)
    assert_close(G, Gb, FP64_TOL)
    assert rel(E2, Eb) < FP64_TOL
    assert np.array_equal(G, G.T)


@pytest.fixture(scope="module")
def hhe64():
    s = mixed_lattice((4, 4, 4), seed=12, tau=1e-12)
    Gr, Er, nr = oracle.fock_atoms(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    return s, Gr, Er, nr


@pytest.mark.parametrize("strategy", [1, 2])
def test_atoms_hhe64_fp64_vs_oracle(torch_dev, hhe64, strategy):
    s, Gr, Er, nr = hhe64
    assert 0 < int(np.sum(s.exps[:, 0] < 5.0)) < s.natoms   # both elements present
    announce("atoms H/He 64 fp64 strategy=%d" % strategy)
    G, E2, st = _run(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau, strategy=strategy)
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    assert np.abs(G - Gr).max() < FP64_TOL * np.abs(Gr).max()
    assert abs(st["quartets"] - nr) <= 4
    assert st["strategy"] == strategy and st["variant"] == 1


def test_atoms_hhe64_mixed_vs_oracle(torch_dev, hhe64):
    s, Gr, Er, nr = hhe64
    announce("atoms H/He 64 mixed")
    G, E2, st = _run(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau, precision="mixed")
    assert_close(G, Gr, MIXED_TOL)
    assert rel(E2, Er) < MIXED_TOL
    assert abs(st["quartets"] - nr) <= 4


@pytest.mark.parametrize("g", [1, 2, 3, 4, 5, 6])
def test_atoms_random_contractions(torch_dev, g):
    """Random exponents (0.1 .. 10) and coefficients on every atom, 1 to 6 primitives, FP64
    and mixed; 30 atoms in a 7 bohr box, so near and far primitive quartets mix."""
    s = random_cluster(30, 60 + g, box=7.0)
    e, c = random_basis_rows(30, g, 70 + g)
    tau = 1e-10
    announce("atoms random contractions g=%d" % g)
    Gr, Er, nr = oracle.fock_atoms(s.xyz, s.dens, e, c, tau)
    G, E2, st = _run(torch_dev, s.xyz, s.dens, e, c, tau)
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    assert abs(st["quartets"] - nr) <= 4
    Gm, Em, _ = _run(torch_dev, s.xyz, s.dens, e, c, tau, precision="mixed")
    assert_close(Gm, Gr, MIXED_TOL)
    assert rel(Em, Er) < MIXED_TOL


@pytest.mark.parametrize("n,seed", [(33, 7), (70, 8)])
def test_atoms_ragged_sizes(torch_dev, n, seed):
    """Sizes that leave partial 64-ket chunks and partial items."""
    s = random_cluster(n, seed, box=9.0)
    e, c = random_basis_rows(n, 3, seed + 80)
    announce("atoms ragged n=%d" % n)
    Gr, Er, _ = oracle.fock_atoms(s.xyz, s.dens, e, c, 1e-9)
    G, E2, _ = _run(torch_dev, s.xyz, s.dens, e, c, 1e-9)
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL


def test_atoms_identical_rows_match_one_basis_build(torch_dev):
    """With the same contraction on every atom the per-atom kernel (rho per quartet) and the
    one-basis kernel (rho from its table) agree to rounding."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = config_system("he64_fp64")
    e = np.tile(s.exps, (s.natoms, 1))
    c = np.tile(s.coefs, (s.natoms, 1))
    announce("atoms identical rows vs one basis")
    G, E2, st = _run(torch_dev, s.xyz, s.dens, e, c, s.tau)
    X = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    G1, E1 = hfk.fock(X, D, s.exps, s.coefs, s.tau)
    G1 = G1.cpu().numpy()
    assert_close(G, G1, 1e-13)
    assert rel(E2, float(E1.item())) < 1e-13


def test_atoms_permutation_equivariance(torch_dev):
    s = random_cluster(40, 91, box=8.0)
    e, c = random_basis_rows(40, 3, 92)
    perm = np.random.default_rng(93).permutation(40)
    announce("atoms permutation")
    G, E2, _ = _run(torch_dev, s.xyz, s.dens, e, c, 1e-10)
    Gp, Ep, _ = _run(torch_dev, s.xyz[perm], s.dens[np.ix_(perm, perm)], e[perm], c[perm], 1e-10)
    assert_close(Gp, G[np.ix_(perm, perm)], 1e-12)
    assert rel(Ep, E2) < 1e-12


def test_atoms_everything_screened(torch_dev):
    s = random_cluster(6, 51, box=4.0)
    e, c = random_basis_rows(6, 3, 52)
    announce("atoms everything screened")
    G, E2, st = _run(torch_dev, s.xyz, s.dens, e, c, 1e6)
    assert st["quartets"] == 0 and st["sig_pairs"] == 0
    assert not np.any(G) and E2 == 0.0


def test_atoms_hhe512_sampled(torch_dev):
    """512 H/He atoms (8x8x8 lattice, tau 1e-10), FP64 and mixed: sampled elements against the
    oracle's element-wise definition, survivors against the count from the oracle's bounds,
    E2 against 1/2 sum D o G, mixed against FP64."""
    s = mixed_lattice((8, 8, 8), seed=13, tau=1e-10)
    announce("atoms H/He 512 fp64 + mixed sampled")
    G, E2, st = _run(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau)
    Gm, Em, _ = _run(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau, precision="mixed")
    Q = oracle.schwarz_atoms(s.xyz, s.exps, s.coefs)
    sig = Q[Q * Q.max() >= s.tau]
    nk = _kept_quartets(sig, s.tau)
    assert abs(st["quartets"] - nk) <= 1e-7 * nk + 8, (st["quartets"], nk)
    rng = np.random.default_rng(512)
    idx = [(0, 0), (511, 3)] + [tuple(int(v) for v in p) for p in rng.integers(0, 512, (6, 2))]
    ref = [oracle.fock_element_atoms(s.xyz, s.dens, s.exps, s.coefs, s.tau, Q, i, j) for i, j in idx]
    scale = max(abs(r) for r in ref)
    for (i, j), r in zip(idx, ref):
        assert abs(G[i, j] - r) <= FP64_TOL * scale, (i, j, G[i, j], r)
        assert abs(Gm[i, j] - r) <= MIXED_TOL * scale, (i, j)
    assert rel(E2, 0.5 * float(np.sum(s.dens * G))) < 1e-12
    assert rel(Em, E2) < MIXED_TOL
    assert_close(Gm, G, MIXED_TOL)


def test_atoms_workspace_too_small_is_rejected(torch_dev):
    """The one-basis workspace lacks the per-atom tables: HFK_ENOMEM before any launch."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(20, 3, box=5.0)
    e, c = random_basis_rows(20, 3, 4)
    announce("atoms workspace too small")
    ws = hfk.new_workspace(hfk.workspace_bytes(20, 3, "fp64"), dev)
    X = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock_atoms(X, D, e, c, 1e-10, workspace=ws)
    assert ei.value.status == hfk.HFK_ENOMEM


def test_atoms_bounds_above_two(torch_dev):
    """Per-atom rows of a tight contraction (bounds above 2) on half the atoms, helium on the
    rest: bras with tau / Q_s above 2 keep their kets."""
    from he_inputs import tight_cluster, HE_STO3G_EXPS, HE_STO3G_COEFS
    s = tight_cluster()
    n = s.natoms
    e = np.tile(s.exps, (n, 1))
    c = np.tile(s.coefs, (n, 1))
    e[1::2] = HE_STO3G_EXPS
    c[1::2] = HE_STO3G_COEFS
    Q = oracle.schwarz_atoms(s.xyz, e, c)
    small = Q[(Q < s.tau / 2) & (Q * Q.max() >= s.tau)]
    assert sum(int(np.sum(Q * q >= s.tau)) for q in small) > 0
    announce("atoms bounds above two")
    G, E2, st = _run(torch_dev, s.xyz, s.dens, e, c, s.tau)
    Gr, Er, nr = oracle.fock_atoms(s.xyz, s.dens, e, c, s.tau)
    assert st["quartets"] == nr
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL


# ------------------------------------------------------------------ gradient with per-atom bases

def _grad_atoms(torch_dev, xyz, dens, e, c, tau, precision="fp64", g_e2=None, GF=None):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    X = torch.tensor(xyz, device=dev)
    D = torch.tensor(dens, device=dev)
    G, _ = hfk.fock_atoms(X, D, e, c, tau, precision=precision)
    ge = None if g_e2 is None else torch.tensor([g_e2], dtype=torch.float64, device=dev)
    gf = None if GF is None else torch.tensor(GF, device=dev)
    d_xyz, d_dens, E2 = hfk.fock_grad(X, D, e, c, tau, precision, g_e2=ge, fock_in=G, g_fock=gf)
    return d_xyz.cpu().numpy(), d_dens.cpu().numpy(), float(E2.item()), G.cpu().numpy()


@pytest.mark.parametrize("g", [1, 2, 3, 4, 5, 6])
def test_atoms_grad_vs_oracle(torch_dev, g):
    """dE2/dR with random per-atom contractions against the oracle (screen held fixed);
    dE2/dD = G and the recomputed E2."""
    s = random_cluster(24, 110 + g, box=6.0)
    e, c = random_basis_rows(24, g, 120 + g)
    tau = 1e-10
    announce("atoms grad g=%d" % g)
    dx, dd, E2g, G = _grad_atoms(torch_dev, s.xyz, s.dens, e, c, tau)
    gr, Er, _ = oracle.grad_atoms(s.xyz, s.dens, e, c, tau)
    assert_close(dx, gr, FP64_TOL)
    assert rel(E2g, Er) < FP64_TOL
    assert np.array_equal(dd, G)


def test_atoms_grad_hhe128(torch_dev):
    """The 128-atom gradient workload with hydrogen on about half the atoms, FP64 and mixed."""
    s = mixed_lattice((8, 4, 4), seed=14, tau=1e-10)
    announce("atoms grad H/He 128 fp64 + mixed")
    gr, Er, _ = oracle.grad_atoms(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    dx, _, E2g, _ = _grad_atoms(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(dx, gr, FP64_TOL)
    assert rel(E2g, Er) < FP64_TOL
    dm, _, Em, _ = _grad_atoms(torch_dev, s.xyz, s.dens, s.exps, s.coefs, s.tau, precision="mixed")
    assert_close(dm, gr, MIXED_TOL)
    assert rel(Em, Er) < MIXED_TOL


@pytest.mark.parametrize("n,seed,ge2", [(5, 131, 0.0), (30, 132, -0.8)])
def test_atoms_vjp_through_G(torch_dev, n, seed, ge2):
    """An upstream dL/dG (not symmetric) and dL/dE2 with per-atom bases: positions through the
    two-density contraction, density through ge2 G + G(sym(dL/dG))."""
    s = random_cluster(n, seed, box=6.0)
    e, c = random_basis_rows(n, 3, seed + 1)
    tau = 1e-10
    GF = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))
    announce("atoms vjp through G n=%d" % n)
    dx, dd, _, _ = _grad_atoms(torch_dev, s.xyz, s.dens, e, c, tau, g_e2=ge2, GF=GF)
    W = 0.5 * (GF + GF.T)
    gx = oracle.grad_pair_atoms(s.xyz, s.dens, W + 0.5 * ge2 * s.dens, e, c, tau)
    G = oracle.fock_atoms(s.xyz, s.dens, e, c, tau)[0]
    GW = oracle.fock_atoms(s.xyz, W, e, c, tau)[0]
    assert_close(dx, gx, FP64_TOL)
    assert_close(dd, ge2 * G + GW, FP64_TOL)


def test_atoms_gradcheck(torch_dev):
    """torch.autograd.gradcheck through FockEnergy with per-atom rows (both outputs)."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(4, 141, box=3.0)
    e, c = random_basis_rows(4, 3, 142)
    announce("atoms gradcheck n=4")
    xyz = torch.tensor(s.xyz, device=dev, requires_grad=True)
    D = torch.tensor(s.dens, device=dev, requires_grad=True)

    def f(x, d):
        dd = 0.5 * (d + d.transpose(0, 1))
        return hfk.FockEnergy.apply(x, dd.contiguous(), e, c, 0.0, "fp64")

    # dynamic work distribution: the last bits differ between calls
    assert torch.autograd.gradcheck(f, (xyz, D), eps=1e-6, atol=1e-7, rtol=1e-6, nondet_tol=1e-12)
