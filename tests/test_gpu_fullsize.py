"""Full-size parity: every element of the GPU results against the stored FP64 oracle builds of
the measured workloads (written by tests/golden/make_golden.py, which calls only the
oracle), in the launch configurations the bench times.

  512 He atoms (8x8x8, tau 1e-10), FP64: the tuned configuration, both accumulation
      strategies and non-default tile shapes; max |dG| <= 1e-10 max |G|, Frobenius, E2 and
      the kept-quartet count.
  1024 He atoms (16x8x8, tau 1e-10): FP64 at 1e-10 and mixed at 1e-6, element-wise.
  2000 ragged clusters, mixed + gradient in one launch (tuned), and FP64: 50 clusters (the
      ten largest and 40 drawn) element by element, G, E2 and every gradient component.
"""
import numpy as np
import pytest

from he_inputs import cluster_batch, config_system, pack_batch
from gpu_util import announce, assert_close, load_batched_sample, load_full, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def he512_ref():
    return load_full("he512_fp64")


def _build(torch_dev, s, precision="fp64", strategy=0):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, len(s.exps), precision), dev)
    G, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, precision=precision, strategy=strategy, workspace=ws)
    st = hfk.read_stats(ws)
    return G.cpu().numpy(), float(E2.item()), st


def _check_full(G, E2, st, ref, tol, what):
    Gr, Er, nr = ref
    assert np.array_equal(G, G.T), what
    assert_close(G, Gr, tol, what)
    assert rel(E2, Er) < tol, (what, E2, Er)
    assert st["quartets"] == nr, (what, st["quartets"], nr)


def test_he512_tuned_every_element(torch_dev, he512_ref):
    """The configuration bench.py times: tuned first, then the default strategy."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = config_system("he512_fp64")
    announce("he512 fp64 tuned, every element")
    hfk.tune(torch.tensor(s.xyz, device=dev), torch.tensor(s.dens, device=dev), s.exps, s.coefs, s.tau,
             precision="fp64")
    G, E2, st = _build(torch_dev, s)
    _check_full(G, E2, st, he512_ref, FP64_TOL, "tuned %s" % st)
    hfk.clear_tuning()


@pytest.mark.parametrize("strategy", [1, 2])
def test_he512_strategies_every_element(torch_dev, he512_ref, strategy):
    s = config_system("he512_fp64")
    announce("he512 fp64 strategy=%d, every element" % strategy)
    G, E2, st = _build(torch_dev, s, strategy=strategy)
    assert st["strategy"] == strategy
    _check_full(G, E2, st, he512_ref, FP64_TOL, "strategy %d" % strategy)


@pytest.mark.parametrize("tile,gbras,kcopies", [(1, 256, 8), (16, 4096, 0), (2, 512, 32), (8, 2048, 1)])
def test_he512_tile_shapes_every_element(torch_dev, he512_ref, tile, gbras, kcopies):
    """Quartet-tile shapes the tuner may pick: items per block, bras per group and shared
    ket-vector copies (atomics) all give the oracle's G."""
    import paper_2509_21039_amd as hfk
    s = config_system("he512_fp64")
    announce("he512 fp64 tile=%d gbras=%d kcopies=%d" % (tile, gbras, kcopies))
    hfk.set_shape(tile, gbras, kcopies)
    try:
        G, E2, st = _build(torch_dev, s)
    finally:
        hfk.set_shape(0, 0, -1)
    assert st["tile_items"] == tile and st["group_bras"] == gbras
    if kcopies:
        assert st["ket_copies"] == kcopies
    _check_full(G, E2, st, he512_ref, FP64_TOL, "shape %s" % ((tile, gbras, kcopies),))


def test_he1024_fp64_and_mixed_every_element(torch_dev):
    """The 1024-atom workload (the mixed-precision configuration): FP64 at 1e-10 and mixed at
    1e-6 against the oracle, element by element, tuned as the bench runs them."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    ref = load_full("he1024_fp64")
    s = config_system("he1024_mixed")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    announce("he1024 fp64 tuned, every element")
    hfk.tune(xyz, D, s.exps, s.coefs, s.tau, precision="fp64")
    G, E2, st = _build(torch_dev, s)
    _check_full(G, E2, st, ref, FP64_TOL, "fp64")
    announce("he1024 mixed tuned, every element")
    hfk.tune(xyz, D, s.exps, s.coefs, s.tau, precision="mixed")
    Gm, Em, stm = _build(torch_dev, s, precision="mixed")
    _check_full(Gm, Em, stm, ref, MIXED_TOL, "mixed")
    hfk.clear_tuning()


def _batched(torch_dev, systems, precision, tune):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    off, xyz, dens = pack_batch(systems)
    X = torch.tensor(xyz, device=dev)
    Dp = torch.tensor(dens, device=dev)
    s0 = systems[0]
    if tune:
        hfk.tune_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision=precision, with_grad=True)
    F, E2, g = hfk.fock_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision=precision, with_grad=True)
    torch.cuda.synchronize()
    return off, F.cpu().numpy(), E2.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("precision,tol,tune", [("mixed", MIXED_TOL, True), ("fp64", FP64_TOL, False)])
def test_batched_2000_sampled_clusters_every_element(torch_dev, precision, tol, tune):
    """50 of the 2000 clusters (the ten largest among them) against the stored oracle, every
    element of G and every gradient component; the whole batch stays finite with zero net
    force per molecule."""
    import paper_2509_21039_amd as hfk
    systems = cluster_batch()
    sample = load_batched_sample()
    counts = np.array([s.natoms for s in systems])
    assert sorted(counts, reverse=True)[:10] == sorted([counts[m] for m, *_ in sample], reverse=True)[:10]
    announce("batched 2000 clusters %s+grad tune=%s, 50 clusters every element" % (precision, tune))
    off, F, E2, g = _batched(torch_dev, systems, precision, tune)
    doff = np.concatenate([[0], np.cumsum(counts.astype(np.int64) ** 2)])
    for m, Gr, Er, gr in sample:
        n = counts[m]
        Fm = F[doff[m]:doff[m] + n * n].reshape(n, n)
        gm = g[off[m]:off[m + 1]]
        assert_close(Fm, Gr, tol, "cluster %d (n=%d) G" % (m, n))
        assert rel(E2[m], Er) < tol, (m, n, E2[m], Er)
        assert_close(gm, gr, tol, "cluster %d (n=%d) gradient" % (m, n))
    assert np.isfinite(F).all() and np.isfinite(E2).all() and np.isfinite(g).all()
    for m in range(len(systems)):
        gm = g[off[m]:off[m + 1]]
        assert np.abs(gm.sum(axis=0)).max() < 1e-5 * max(1.0, np.abs(gm).max())
    if tune:
        hfk.clear_tuning()
