"""GPU SCF (one-electron kernels, the two-electron build, rocBLAS/rocSOLVER products and
eigenproblems, DIIS) against the oracle's plain numpy SCF."""
import numpy as np
import pytest

import oracle
from oracle.scf import scf as oracle_scf
from he_inputs import HE_STO3G_COEFS as C3, HE_STO3G_EXPS as E3, mixed_lattice, random_cluster
from gpu_util import announce, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _system(shape, seed, tau=1e-12):
    s = mixed_lattice(shape, seed=seed, tau=tau)
    Z = np.where(s.exps[:, 0] < 5.0, 1.0, 2.0)
    return s, Z, int(Z.sum()) // 2


def _gpu_scf(torch_dev, xyz, Z, e, c, nocc, tau, **kw):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    r = hfk.scf(torch.tensor(xyz, device=dev), Z, e, c, nocc, tau, **kw)
    return r, r["D"].cpu().numpy(), r["eps"].cpu().numpy()


def test_scf_single_helium(torch_dev):
    announce("scf single helium")
    xyz = np.zeros((1, 3))
    r, D, eps = _gpu_scf(torch_dev, xyz, [2.0], np.array([E3]), np.array([C3]), 1, 0.0)
    ref = oracle_scf(xyz, [2.0], [E3], [C3], 1, 0.0)
    assert r["converged"]
    assert rel(r["E"], ref["E"]) < 1e-12
    assert abs(D[0, 0] - ref["D"][0, 0]) < 1e-12


@pytest.mark.parametrize("name", ["H2", "HeH+"])
def test_scf_textbook_diatomics(torch_dev, name):
    """The minimal-basis H2 (R = 1.4 bohr) and HeH+ (R = 1.4632 bohr, helium zeta 2.0925) of
    Szabo and Ostlund (section 3.5): total energies -1.1167 and -2.860662 hartree, and the
    oracle's energy, density and orbital energies."""
    from he_inputs import H_STO3G_EXPS
    announce("scf textbook %s" % name)
    if name == "H2":
        R, Z, expect, tol = 1.4, [1.0, 1.0], -1.1167, 5e-5
        e = np.tile(H_STO3G_EXPS, (2, 1))
    else:
        R, Z, expect, tol = 1.4632, [2.0, 1.0], -2.860662, 1e-5
        e = np.stack([np.array([2.227660, 0.405771, 0.109818]) * 2.0925 ** 2, H_STO3G_EXPS])
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    c = np.tile(C3, (2, 1))
    r, D, eps = _gpu_scf(torch_dev, xyz, Z, e, c, 1, 0.0)
    ref = oracle_scf(xyz, Z, e, c, 1, 0.0)
    assert r["converged"]
    assert r["E"] == pytest.approx(expect, abs=tol)
    # both loops stop at |dE| < 1e-10 and max |FDS - SDF| < 1e-7
    assert rel(r["E"], ref["E"]) < 1e-10
    assert np.abs(D - ref["D"]).max() < 1e-6
    assert np.abs(eps - ref["eps"]).max() < 1e-6


@pytest.mark.parametrize("shape,seed", [((4, 4, 2), 16), ((4, 4, 4), 15)])
def test_scf_hhe_vs_oracle(torch_dev, shape, seed):
    """H/He lattices (32 and 64 atoms; the 64-atom one is a cation): converged energy, density
    and orbital energies against the oracle's SCF, and the converged-state properties of the
    GPU density."""
    s, Z, nocc = _system(shape, seed)
    announce("scf H/He n=%d" % s.natoms)
    r, D, eps = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau)
    ref = oracle_scf(s.xyz, Z, s.exps, s.coefs, nocc, s.tau)
    assert r["converged"] and ref["converged"]
    assert abs(r["E"] - ref["E"]) < 1e-8 * abs(ref["E"])
    assert np.abs(D - ref["D"]).max() < 1e-5
    assert np.abs(eps - ref["eps"]).max() < 1e-5
    S = ref["S"]
    assert np.abs(D @ S @ D - 2 * D).max() < 1e-6
    assert np.trace(D @ S) == pytest.approx(2 * nocc, rel=1e-9)
    assert np.all(np.diff(eps) >= -1e-12)


def test_scf_mixed_precision(torch_dev):
    """FP32 two-electron integrals inside the loop: energy within 1e-6 of the FP64 SCF."""
    s, Z, nocc = _system((4, 4, 2), 16)
    announce("scf mixed")
    r64, _, _ = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau)
    rm, Dm, _ = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau, precision="mixed", d_tol=1e-5,
                         e_tol=1e-8)
    assert rm["converged"]
    assert rel(rm["E"], r64["E"]) < 1e-6


def test_scf_deterministic_and_restart(torch_dev):
    """With the deterministic strategy two runs agree bit for bit; restarting from the
    converged density converges at once."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s, Z, nocc = _system((4, 4, 2), 16)
    announce("scf deterministic + restart")
    a, Da, _ = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau, strategy=hfk.STRATEGY_DETERMINISTIC)
    b, Db, _ = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau, strategy=hfk.STRATEGY_DETERMINISTIC)
    assert a["E"] == b["E"] and np.array_equal(Da, Db) and a["iterations"] == b["iterations"]
    c, Dc, _ = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau, dens0=torch.tensor(Da, device=dev))
    assert c["converged"] and c["iterations"] <= 3
    assert abs(c["E"] - a["E"]) < 1e-9 * abs(a["E"])


def test_scf_filled_shell(torch_dev):
    """Helium only, every orbital occupied: D = 2 S^-1."""
    s = random_cluster(20, 73, box=8.0)
    announce("scf filled shell")
    r, D, _ = _gpu_scf(torch_dev, s.xyz, np.full(20, 2.0), np.tile(E3, (20, 1)), np.tile(C3, (20, 1)), 20, 1e-12)
    S, _, _ = oracle.one_electron_atoms(s.xyz, np.full(20, 2.0), np.tile(E3, (20, 1)), np.tile(C3, (20, 1)))
    assert r["converged"]
    assert np.abs(D @ S - 2 * np.eye(20)).max() < 1e-9


def test_scf_singular_overlap_is_refused(torch_dev):
    """Two atoms on one spot with the same contraction make S singular: HFK_EUNSUPPORTED."""
    import paper_2509_21039_amd as hfk
    announce("scf singular overlap")
    xyz = np.zeros((2, 3))
    with pytest.raises(hfk.HfkError) as ei:
        _gpu_scf(torch_dev, xyz, [2.0, 2.0], np.tile(E3, (2, 1)), np.tile(C3, (2, 1)), 2, 0.0)
    assert ei.value.status == hfk.HFK_EUNSUPPORTED


@pytest.mark.parametrize("max_iter", [1, 3])
def test_scf_unconverged_returns_the_density_of_its_energy(torch_dev, max_iter):
    """A loop cut off by max_iter returns the density whose Fock matrix gave the returned
    energy: E = 1/2 sum D o (2H + G(D)) + E_nn recomputed from the oracle (one-electron
    integrals, the two-electron build and the nuclear repulsion) for the returned D.
    Regression: the last iteration once diagonalised again and returned the next density."""
    s, Z, nocc = _system((4, 4, 2), 16)
    announce("scf unconverged max_iter=%d" % max_iter)
    r, D, eps = _gpu_scf(torch_dev, s.xyz, Z, s.exps, s.coefs, nocc, s.tau, max_iter=max_iter)
    assert not r["converged"] and r["iterations"] == max_iter
    S, T, V = oracle.one_electron_atoms(s.xyz, Z, s.exps, s.coefs)
    H = T + V
    G, _, _ = oracle.fock_atoms(s.xyz, D, s.exps, s.coefs, s.tau)
    n = len(Z)
    enn = sum(Z[a] * Z[b] / np.linalg.norm(s.xyz[a] - s.xyz[b]) for a in range(n) for b in range(a))
    E = 0.5 * float(np.sum(D * (2.0 * H + G))) + enn
    assert rel(r["E"], E) < 1e-10, (r["E"], E)
    assert np.isfinite(D).all() and np.isfinite(eps).all()
