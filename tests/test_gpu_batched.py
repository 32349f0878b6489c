"""GPU parity of the ragged batched path (one persistent launch, forward + gradient)."""
import numpy as np
import pytest

import oracle
from he_inputs import cluster_batch, pack_batch, random_cluster
from gpu_util import announce, assert_close, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _run(torch_dev, systems, precision, with_grad=True):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    off, xyz, dens = pack_batch(systems)
    X = torch.tensor(xyz, device=dev)
    Dp = torch.tensor(dens, device=dev)
    F, E2, g = hfk.fock_batched(off, X, Dp, systems[0].exps, systems[0].coefs, systems[0].tau,
                                precision=precision, with_grad=with_grad)
    torch.cuda.synchronize()
    return off, F.cpu().numpy(), E2.cpu().numpy(), (g.cpu().numpy() if g is not None else None)


def _mol(off, F, g, m, n):
    d0 = int(sum(int(off[k + 1] - off[k]) ** 2 for k in range(m)))
    Fm = F[d0:d0 + n * n].reshape(n, n)
    gm = g[off[m]:off[m + 1]] if g is not None else None
    return Fm, gm


def _small_batch(tau):
    sizes = [1, 2, 5, 17, 3, 30, 9, 1, 24, 12, 40, 7]
    return [random_cluster(n, 100 + i, box=1.2 * n ** (1 / 3) * 2.0, tau=tau) for i, n in enumerate(sizes)]


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_small_batch_vs_oracle(torch_dev, precision, tol):
    systems = _small_batch(1e-10)
    announce("batched small %s" % precision)
    off, F, E2, g = _run(torch_dev, systems, precision)
    for m, s in enumerate(systems):
        n = s.natoms
        Fm, gm = _mol(off, F, g, m, n)
        Fr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        gr, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        assert_close(Fm, Fr, tol, str((m, n)))
        assert rel(E2[m], Er) < tol, (m, n)
        # a one-atom molecule has zero gradient (translation invariance): absolute floor
        assert np.linalg.norm(gm - gr) <= tol * max(np.linalg.norm(gr), 1e-6), (m, n)


def test_forward_only_matches_fused(torch_dev):
    systems = _small_batch(1e-10)
    announce("batched forward-only")
    off, F1, E1, _ = _run(torch_dev, systems, "fp64", with_grad=False)
    _, F2, E2, g2 = _run(torch_dev, systems, "fp64", with_grad=True)
    assert np.abs(F1 - F2).max() <= 1e-13 * np.abs(F2).max()
    assert np.abs(E1 - E2).max() <= 1e-12 * np.abs(E2).max()


def test_cluster_batch_2000_sampled(torch_dev):
    """The 2000-cluster workload (mixed precision + gradient, one launch); sampled molecules
    are checked one by one against the FP64 oracle."""
    systems = cluster_batch()
    announce("batched 2000 clusters mixed+grad")
    off, F, E2, g = _run(torch_dev, systems, "mixed")
    counts = np.array([s.natoms for s in systems])
    picks = [int(np.argmin(counts))]
    for target in (20, 40, 60):
        picks.append(int(np.argmin(np.abs(counts - target))))
    for m in picks:
        s = systems[m]
        n = s.natoms
        Fm, gm = _mol(off, F, g, m, n)
        Fr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        gr, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        assert_close(Fm, Fr, MIXED_TOL, str((m, n)))
        assert rel(E2[m], Er) < MIXED_TOL, (m, n)
        assert_close(gm, gr, MIXED_TOL, str((m, n)))
    # properties over the whole batch: finite results, zero net force per molecule
    assert np.isfinite(F).all() and np.isfinite(E2).all() and np.isfinite(g).all()
    for m in range(len(systems)):
        gm = g[off[m]:off[m + 1]]
        assert np.abs(gm.sum(axis=0)).max() < 1e-5 * max(1.0, np.abs(gm).max())


def test_six_primitive_batch(torch_dev):
    """Six primitives per function in the batched launch, FP64 and mixed."""
    systems = [random_cluster(n, 200 + i, box=1.2 * n ** (1 / 3) * 2.0, tau=1e-10) for i, n in enumerate([3, 11, 1, 19])]
    for s in systems:
        s.exps = np.array([30.0, 8.0, 2.5, 0.9, 0.35, 0.14])
        s.coefs = np.array([0.02, 0.08, 0.25, 0.4, 0.3, 0.1])
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        announce("batched six primitives %s" % precision)
        off, F, E2, g = _run(torch_dev, systems, precision)
        for m, s in enumerate(systems):
            Fm, gm = _mol(off, F, g, m, s.natoms)
            Fr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
            gr, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
            assert_close(Fm, Fr, tol, str((precision, m)))
            assert rel(E2[m], Er) < tol, (precision, m)
            assert np.linalg.norm(gm - gr) <= tol * max(np.linalg.norm(gr), 1e-6), (precision, m)


def test_batch_with_bounds_above_two(torch_dev):
    """A molecule whose Schwarz bounds reach above 2 inside a batch (see the single-molecule
    regression): its bras with tau / Q_s above 2 keep their kets."""
    from he_inputs import tight_cluster
    t = tight_cluster()
    others = [random_cluster(n, 300 + n, box=4.0, tau=t.tau) for n in (5, 12)]
    for o in others:
        o.exps, o.coefs = t.exps.copy(), t.coefs.copy()
    systems = [others[0], t, others[1]]
    announce("batched bounds above two")
    off, F, E2, g = _run(torch_dev, systems, "fp64")
    for m, s in enumerate(systems):
        Fm, gm = _mol(off, F, g, m, s.natoms)
        Fr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        gr, _, _ = oracle.grad(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        assert_close(Fm, Fr, FP64_TOL, str(m))
        assert rel(E2[m], Er) < FP64_TOL, m
        assert np.linalg.norm(gm - gr) <= FP64_TOL * max(np.linalg.norm(gr), 1e-6), m


# ------------------------------------------------------------------ per-atom bases

def _run_atoms(torch_dev, systems, rows, precision, with_grad=True):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    off, xyz, dens = pack_batch(systems)
    X = torch.tensor(xyz, device=dev)
    Dp = torch.tensor(dens, device=dev)
    e, c = rows
    F, E2, g = hfk.fock_batched(off, X, Dp, e, c, systems[0].tau, precision=precision, with_grad=with_grad)
    torch.cuda.synchronize()
    return off, F.cpu().numpy(), E2.cpu().numpy(), (g.cpu().numpy() if g is not None else None)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_small_batch_atoms_vs_oracle(torch_dev, precision, tol):
    """Random per-atom contractions over a ragged batch: every molecule's G, E2 and gradient
    against the oracle's per-atom functions."""
    from he_inputs import random_basis_rows
    systems = _small_batch(1e-10)
    ntot = sum(s.natoms for s in systems)
    e, c = random_basis_rows(ntot, 3, 401)
    announce("batched per-atom small %s" % precision)
    off, F, E2, g = _run_atoms(torch_dev, systems, (e, c), precision)
    for m, s in enumerate(systems):
        n = s.natoms
        a0, a1 = int(off[m]), int(off[m + 1])
        Fm, gm = _mol(off, F, g, m, n)
        Fr, Er, _ = oracle.fock_atoms(s.xyz, s.dens, e[a0:a1], c[a0:a1], s.tau)
        gr, _, _ = oracle.grad_atoms(s.xyz, s.dens, e[a0:a1], c[a0:a1], s.tau)
        assert_close(Fm, Fr, tol, str((m, n)))
        assert rel(E2[m], Er) < tol, (m, n)
        assert np.linalg.norm(gm - gr) <= tol * max(np.linalg.norm(gr), 1e-6), (m, n)


def test_batch_atoms_forward_only_and_identical_rows(torch_dev):
    """Forward-only equals the fused forward; identical rows equal the one-basis batch."""
    systems = _small_batch(1e-10)
    ntot = sum(s.natoms for s in systems)
    e = np.tile(systems[0].exps, (ntot, 1))
    c = np.tile(systems[0].coefs, (ntot, 1))
    announce("batched per-atom forward-only and identical rows")
    _, F1, E1, _ = _run_atoms(torch_dev, systems, (e, c), "fp64", with_grad=False)
    _, F2, E2, g2 = _run_atoms(torch_dev, systems, (e, c), "fp64", with_grad=True)
    _, F0, E0, g0 = _run(torch_dev, systems, "fp64")
    assert np.abs(F1 - F2).max() <= 1e-13 * np.abs(F2).max()
    assert np.abs(F2 - F0).max() <= 1e-13 * np.abs(F0).max()
    assert np.abs(E2 - E0).max() <= 1e-12 * np.abs(E0).max()
    assert np.abs(g2 - g0).max() <= 1e-12 * np.abs(g0).max()


def test_hhe_cluster_batch_sampled(torch_dev):
    """500 H/He clusters (the cluster recipe with per-atom rows), mixed precision + gradient
    in one launch; sampled molecules against the FP64 oracle, net force per molecule."""
    from he_inputs import hhe_rows
    systems = cluster_batch(nmol=500, seed=6)
    ntot = sum(s.natoms for s in systems)
    e, c = hhe_rows(ntot, 7)
    announce("batched 500 H/He clusters mixed+grad")
    off, F, E2, g = _run_atoms(torch_dev, systems, (e, c), "mixed")
    counts = np.array([s.natoms for s in systems])
    picks = [int(np.argmin(counts))] + [int(np.argmin(np.abs(counts - t))) for t in (30, 60)]
    for m in picks:
        s = systems[m]
        a0, a1 = int(off[m]), int(off[m + 1])
        Fm, gm = _mol(off, F, g, m, s.natoms)
        Fr, Er, _ = oracle.fock_atoms(s.xyz, s.dens, e[a0:a1], c[a0:a1], s.tau)
        gr, _, _ = oracle.grad_atoms(s.xyz, s.dens, e[a0:a1], c[a0:a1], s.tau)
        assert_close(Fm, Fr, MIXED_TOL, str((m, s.natoms)))
        assert rel(E2[m], Er) < MIXED_TOL, m
        assert_close(gm, gr, MIXED_TOL, str(m))
    assert np.isfinite(F).all() and np.isfinite(E2).all() and np.isfinite(g).all()
    for m in range(len(systems)):
        gm = g[off[m]:off[m + 1]]
        assert np.abs(gm.sum(axis=0)).max() < 1e-5 * max(1.0, np.abs(gm).max())
