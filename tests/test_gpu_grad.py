"""GPU parity of the backward kernel (dE2/dR, dE2/dD, and the pull-back of dL/dG) against
the CPU oracle and finite differences, through the C ABI and the autograd Function."""
import numpy as np
import pytest

import oracle
from he_inputs import config_system, random_cluster
from gpu_util import announce, assert_close, load_golden, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _grad(torch_dev, s, precision="fp64"):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    G, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, precision=precision)
    d_xyz, d_dens, E2g = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, precision=precision, fock_in=G)
    torch.cuda.synchronize()
    return d_xyz.cpu().numpy(), d_dens.cpu().numpy(), float(E2g.item()), G.cpu().numpy(), float(E2.item())


@pytest.mark.parametrize("n,seed,box,tau", [(2, 1, 2.0, 0.0), (4, 2, 4.0, 0.0), (6, 3, 5.0, 0.0),
                                            (8, 4, 9.0, 1e-8), (37, 5, 9.0, 1e-10)])
def test_grad_vs_oracle(torch_dev, n, seed, box, tau):
    s = random_cluster(n, seed, box=box, tau=tau)
    announce("grad n=%d seed=%d tau=%g" % (n, seed, tau))
    g, dD, E2g, G, E2 = _grad(torch_dev, s)
    gr, Er, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, tau)
    assert_close(g, gr, FP64_TOL)
    assert rel(E2g, Er) < FP64_TOL
    assert rel(E2, Er) < FP64_TOL
    assert np.abs(dD - G).max() == 0.0        # g_e2 = 1: dE2/dD is G itself
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * max(1.0, np.abs(g).max())


def test_he128_grad_vs_oracle(torch_dev):
    s = config_system("he128_grad")
    announce("he128 grad fp64")
    g, _, E2g, _, E2 = _grad(torch_dev, s)
    gr, Er, _ = load_golden("he128_grad")
    assert_close(g, gr, FP64_TOL)
    assert rel(E2g, Er) < FP64_TOL
    assert rel(E2, Er) < FP64_TOL


def test_he128_grad_mixed(torch_dev):
    s = config_system("he128_grad")
    announce("he128 grad mixed")
    g, _, E2g, _, _ = _grad(torch_dev, s, precision="mixed")
    gr, Er, _ = load_golden("he128_grad")
    assert_close(g, gr, MIXED_TOL)
    assert rel(E2g, Er) < MIXED_TOL


def test_grad_vs_central_differences(torch_dev):
    """Central differences (h = 1e-4 bohr) of the GPU energy against the GPU gradient, tau = 0."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(10, 6, box=6.0, tau=0.0)
    announce("grad fd n=10")
    g, _, _, _, _ = _grad(torch_dev, s)
    D = torch.tensor(s.dens, device=dev)
    h = 1e-4
    fd = np.zeros_like(g)
    for a in range(s.natoms):
        for c in range(3):
            xp = s.xyz.copy(); xm = s.xyz.copy()
            xp[a, c] += h; xm[a, c] -= h
            ep = hfk.fock(torch.tensor(xp, device=dev), D, s.exps, s.coefs, 0.0)[1].item()
            em = hfk.fock(torch.tensor(xm, device=dev), D, s.exps, s.coefs, 0.0)[1].item()
            fd[a, c] = (ep - em) / (2 * h)
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_autograd_function(torch_dev):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(7, 7, box=5.0, tau=1e-10)
    announce("autograd n=7")
    xyz = torch.tensor(s.xyz, device=dev, requires_grad=True)
    D = torch.tensor(s.dens, device=dev, requires_grad=True)
    G, E2 = hfk.FockEnergy.apply(xyz, D, s.exps, s.coefs, s.tau, "fp64")
    (3.0 * E2.sum()).backward()
    gr, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(xyz.grad.cpu().numpy(), 3.0 * gr, FP64_TOL)
    assert np.abs(D.grad.cpu().numpy() - 3.0 * G.detach().cpu().numpy()).max() < 1e-13 * np.abs(G.detach().cpu().numpy()).max()


def _vjp_reference(s, GF, ge2):
    """Oracle pull-back of (dL/dG = GF, dL/dE2 = ge2): positions through the two-density
    contraction with X = sym(GF) + (ge2/2) D, density through ge2 G + G(sym(GF))."""
    W = 0.5 * (GF + GF.T)
    gx = oracle.grad_pair(s.xyz, s.dens, W + 0.5 * ge2 * s.dens, s.exps, s.coefs, s.tau)
    G = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)[0]
    GW = oracle.fock(s.xyz, W, s.exps, s.coefs, s.tau)[0]
    return gx, ge2 * G + GW


@pytest.mark.parametrize("n,seed,box,tau,ge2", [(3, 21, 3.0, 0.0, 0.0), (8, 22, 7.0, 1e-10, 0.7),
                                                (37, 23, 9.0, 1e-10, -1.3)])
def test_fock_output_vjp_vs_oracle(torch_dev, n, seed, box, tau, ge2):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(n, seed, box=box, tau=tau)
    announce("vjp through G n=%d seed=%d ge2=%g" % (n, seed, ge2))
    GF = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))   # not symmetric on purpose
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    G, _ = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    g_e2 = torch.tensor([ge2], dtype=torch.float64, device=dev)
    d_xyz, d_dens, _ = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, g_e2=g_e2, fock_in=G,
                                     g_fock=torch.tensor(GF, device=dev))
    gx, gd = _vjp_reference(s, GF, ge2)
    assert_close(d_xyz.cpu().numpy(), gx, FP64_TOL)
    assert_close(d_dens.cpu().numpy(), gd, FP64_TOL)


def test_fock_output_vjp_mixed(torch_dev):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(20, 24, box=8.0, tau=1e-10)
    announce("vjp through G mixed n=20")
    GF = np.random.default_rng(24).uniform(-1.0, 1.0, size=(20, 20))
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    G, _ = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, precision="mixed")
    g_e2 = torch.tensor([0.5], dtype=torch.float64, device=dev)
    d_xyz, d_dens, _ = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, precision="mixed", g_e2=g_e2, fock_in=G,
                                     g_fock=torch.tensor(GF, device=dev))
    gx, gd = _vjp_reference(s, GF, 0.5)
    assert_close(d_xyz.cpu().numpy(), gx, MIXED_TOL)
    assert_close(d_dens.cpu().numpy(), gd, MIXED_TOL)


def test_autograd_through_both_outputs(torch_dev):
    """A loss on G and E2 together, through the autograd Function."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(9, 25, box=6.0, tau=1e-10)
    announce("autograd through G and E2 n=9")
    M = np.random.default_rng(25).uniform(-1.0, 1.0, size=(9, 9))
    xyz = torch.tensor(s.xyz, device=dev, requires_grad=True)
    D = torch.tensor(s.dens, device=dev, requires_grad=True)
    G, E2 = hfk.FockEnergy.apply(xyz, D, s.exps, s.coefs, s.tau, "fp64")
    ((G * torch.tensor(M, device=dev)).sum() + 2.5 * E2.sum()).backward()
    gx, gd = _vjp_reference(s, M, 2.5)
    assert_close(xyz.grad.cpu().numpy(), gx, FP64_TOL)
    assert_close(D.grad.cpu().numpy(), gd, FP64_TOL)


def test_gradcheck_small(torch_dev):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(4, 8, box=3.0, tau=0.0)
    announce("gradcheck n=4")
    xyz = torch.tensor(s.xyz, device=dev, requires_grad=True)
    D = torch.tensor(s.dens, device=dev, requires_grad=True)

    def f(x, d):
        dd = 0.5 * (d + d.transpose(0, 1))
        return hfk.FockEnergy.apply(x, dd.contiguous(), s.exps, s.coefs, 0.0, "fp64")

    # work is handed out dynamically, so per-workgroup partial sums, and with them the last
    # bits of the FP64 result, differ between calls: allow that much nondeterminism
    assert torch.autograd.gradcheck(f, (xyz, D), eps=1e-6, atol=1e-7, rtol=1e-6, nondet_tol=1e-12)


@pytest.mark.parametrize("exps,coefs", [([0.8], [1.0]), ([3.0, 0.45], [0.4, 0.7]),
                                        ([9.0, 2.1, 0.6, 0.19], [0.05, 0.25, 0.5, 0.3]),
                                        ([24.0, 6.5, 2.0, 0.7, 0.25], [0.03, 0.12, 0.35, 0.45, 0.2]),
                                        ([30.0, 8.0, 2.5, 0.9, 0.35, 0.14], [0.02, 0.08, 0.25, 0.4, 0.3, 0.1])])
def test_grad_other_basis_sizes(torch_dev, exps, coefs):
    s = random_cluster(9, 41, box=5.0, tau=1e-10)
    s.exps = np.array(exps)
    s.coefs = np.array(coefs)
    announce("grad ngauss=%d" % len(exps))
    g, _, E2g, _, _ = _grad(torch_dev, s)
    gr, Er, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(g, gr, FP64_TOL)
    assert rel(E2g, Er) < FP64_TOL


def test_grad_max_atoms_sparse_lattice(torch_dev):
    """The largest system the gradient accepts (4096 atoms) on a sparse lattice, where the
    LDS gradient copy (3n doubles) and both tables are at their largest: sampled components
    against central differences of the GPU energy, and zero net force."""
    import paper_2509_21039_amd as hfk
    from he_inputs import jittered_lattice
    torch, dev = torch_dev
    s = jittered_lattice((16, 16, 16), seed=12, tau=1e-10, spacing=14.0, jitter=0.5)
    assert s.natoms == 4096
    announce("grad max atoms 4096 sparse")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, 3, "fp64", True), dev)
    d_xyz, _, E2g = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, want_dens=False, workspace=ws)
    g = d_xyz.cpu().numpy()
    _, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, workspace=ws)
    assert rel(E2g.item(), E2.item()) < FP64_TOL
    assert np.abs(g.sum(axis=0)).max() < 1e-10 * max(1.0, np.abs(g).max())
    h = 1e-3
    for a, c in [(0, 0), (1234, 1), (4095, 2)]:
        xp = s.xyz.copy(); xm = s.xyz.copy()
        xp[a, c] += h; xm[a, c] -= h
        ep = hfk.fock(torch.tensor(xp, device=dev), D, s.exps, s.coefs, s.tau, workspace=ws)[1].item()
        em = hfk.fock(torch.tensor(xm, device=dev), D, s.exps, s.coefs, s.tau, workspace=ws)[1].item()
        assert abs((ep - em) / (2 * h) - g[a, c]) < 1e-6 * max(1.0, np.abs(g).max()), (a, c)
