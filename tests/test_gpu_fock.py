"""GPU parity of the forward Fock build against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from he_inputs import config_system, random_cluster
from gpu_util import announce, assert_close, load_full, load_golden, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10      # relative, Frobenius for G and absolute-relative for E2
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _run(torch_dev, s, precision="fp64", strategy=0, variant=-1):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    hfk.set_config(variant, 0)
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, len(s.exps), precision), dev)
    G, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, precision=precision, strategy=strategy, workspace=ws)
    st = hfk.read_stats(ws)
    hfk.set_config(-1, 0)
    if variant >= 0:
        assert st["variant"] == variant
    return G.cpu().numpy(), float(E2.item()), st


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n,seed,box,tau", [(1, 1, 1.0, 0.0), (2, 2, 3.0, 0.0), (3, 3, 3.0, 0.0),
                                            (5, 4, 4.0, 0.0), (7, 5, 6.0, 1e-6), (8, 6, 12.0, 1e-8)])
def test_tiny_vs_bruteforce(torch_dev, n, seed, box, tau, variant):
    s = random_cluster(n, seed, box=box, tau=tau)
    announce("tiny n=%d seed=%d tau=%g variant=%d" % (n, seed, tau, variant))
    G, E2, st = _run(torch_dev, s, variant=variant)
    Gb, Eb = oracle.fock_bruteforce(s.xyz, s.dens, s.exps, s.coefs, tau)
    assert_close(G, Gb, FP64_TOL)
    assert rel(E2, Eb) < FP64_TOL
    assert np.array_equal(G, G.T)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("strategy", [1, 2])
def test_he64_fp64_vs_oracle(torch_dev, strategy, variant):
    s = config_system("he64_fp64")
    announce("he64 fp64 strategy=%d variant=%d" % (strategy, variant))
    G, E2, st = _run(torch_dev, s, strategy=strategy, variant=variant)
    Gr, Er, nsr = load_golden("he64_fp64")
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    assert np.abs(G - Gr).max() < FP64_TOL * np.abs(Gr).max()
    # screening decisions taken in FP64 on both sides: the kept count matches up to
    # quartets whose Q product sits within rounding of tau
    assert abs(st["quartets"] - nsr) <= 4, (st["quartets"], nsr)
    assert st["strategy"] == strategy


@pytest.mark.parametrize("variant", [0, 1])
def test_he64_mixed_vs_oracle(torch_dev, variant):
    s = config_system("he64_fp64")
    announce("he64 mixed variant=%d" % variant)
    G, E2, st = _run(torch_dev, s, precision="mixed", variant=variant)
    Gr, Er, nsr = load_golden("he64_fp64")
    assert_close(G, Gr, MIXED_TOL)
    assert rel(E2, Er) < MIXED_TOL
    assert abs(st["quartets"] - nsr) <= 4


@pytest.mark.parametrize("n,seed", [(33, 7), (70, 8)])
def test_ragged_sizes_vs_oracle(torch_dev, n, seed):
    """Sizes that leave partial 64-ket chunks and partial items."""
    s = random_cluster(n, seed, box=9.0, tau=1e-9)
    announce("ragged n=%d" % n)
    G, E2, st = _run(torch_dev, s)
    Gr, Er, nsr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    assert abs(st["quartets"] - nsr) <= 2


@pytest.mark.parametrize("exps,coefs", [
    ([0.8], [1.0]),
    ([3.0, 0.45], [0.4, 0.7]),
    ([9.0, 2.1, 0.6, 0.19], [0.05, 0.25, 0.5, 0.3]),
])
@pytest.mark.parametrize("variant", [0, 1])
def test_other_basis_sizes(torch_dev, exps, coefs, variant):
    """1..4 primitives per function, both forms of the quartet kernel."""
    s = random_cluster(23, 31, box=8.0, tau=1e-10)
    s.exps = np.array(exps)
    s.coefs = np.array(coefs)
    announce("ngauss=%d variant=%d" % (len(exps), variant))
    G, E2, st = _run(torch_dev, s, variant=variant)
    Gr, Er, nsr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    Gm, Em, _ = _run(torch_dev, s, precision="mixed", variant=variant)
    assert_close(Gm, Gr, MIXED_TOL)


# Five and six primitives per function (the paper's 1024-atom case uses six); made-up
# exponents spanning the same range as a six-term He contraction.
G5 = ([24.0, 6.5, 2.0, 0.7, 0.25], [0.03, 0.12, 0.35, 0.45, 0.2])
G6 = ([30.0, 8.0, 2.5, 0.9, 0.35, 0.14], [0.02, 0.08, 0.25, 0.4, 0.3, 0.1])


@pytest.mark.parametrize("exps,coefs", [G5, G6])
def test_five_and_six_primitives(torch_dev, exps, coefs):
    """g = 5, 6 run the hybrid form only (the direct form is built for g <= 4)."""
    s = random_cluster(17, 33, box=7.0, tau=1e-10)
    s.exps = np.array(exps)
    s.coefs = np.array(coefs)
    announce("ngauss=%d" % len(exps))
    G, E2, st = _run(torch_dev, s)
    assert st["variant"] == 1
    Gr, Er, nsr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert st["quartets"] == nsr
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL
    Gm, Em, _ = _run(torch_dev, s, precision="mixed")
    assert_close(Gm, Gr, MIXED_TOL)


def test_unsupported_ngauss_raises(torch_dev):
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(4, 1)
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock(xyz, D, [1.0] * 7, [0.2] * 7, 0.0)
    assert ei.value.status == hfk.HFK_EUNSUPPORTED


def test_max_atoms_sparse_lattice(torch_dev):
    """The largest accepted system (6144 atoms) on a sparse lattice (14 bohr spacing): only
    the one-centre pairs pass the screen, so the kept quartets are the S(S+1)/2 pairs of
    them, while the LDS rows (> 64 KiB), the shared ket vectors and the workspace run at
    their maximum sizes.  Sampled elements against the oracle's element-wise definition;
    E2 against 1/2 sum D o G of the returned G."""
    from he_inputs import jittered_lattice
    s = jittered_lattice((16, 16, 24), seed=11, tau=1e-10, spacing=14.0, jitter=0.5)
    n = s.natoms
    assert n == 6144
    announce("max atoms 6144 sparse fp64")
    G, E2, st = _run(torch_dev, s)
    Q = oracle.schwarz(s.xyz, s.exps, s.coefs)
    S = int((Q * Q.max() >= s.tau).sum())
    assert S == n
    assert st["quartets"] == S * (S + 1) // 2
    rng = np.random.default_rng(3)
    idx = [(int(i), int(i)) for i in rng.integers(0, n, 6)] + \
          [(int(i), int(j)) for i, j in rng.integers(0, n, (6, 2))] + [(0, n - 1), (n - 1, n - 1)]
    ref = [oracle.fock_element(s.xyz, s.dens, s.exps, s.coefs, s.tau, Q, i, j) for i, j in idx]
    scale = max(abs(r) for r in ref)
    for (i, j), r in zip(idx, ref):
        assert abs(G[i, j] - r) <= FP64_TOL * scale, (i, j, G[i, j], r)
    assert np.array_equal(G, G.T)
    assert rel(E2, 0.5 * float(np.sum(s.dens * G))) < 1e-12


def test_everything_screened(torch_dev):
    """A threshold no pair product reaches: no quartet survives, G and E2 are exactly zero,
    and the gradient is zero too."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(6, 51, box=4.0, tau=1e6)
    announce("everything screened")
    G, E2, st = _run(torch_dev, s)
    assert st["quartets"] == 0 and st["sig_pairs"] == 0
    assert not np.any(G) and E2 == 0.0
    Gr, Er, nr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert nr == 0 and not np.any(Gr)
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    d_xyz, _, E2g = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, want_dens=False)
    assert not torch.any(d_xyz).item() and E2g.item() == 0.0


def test_workspace_too_small_is_rejected(torch_dev):
    """A workspace below hfk_workspace_bytes gives HFK_ENOMEM before any launch, for the
    forward, gradient and batched calls."""
    import paper_2509_21039_amd as hfk
    from he_inputs import pack_batch
    torch, dev = torch_dev
    s = random_cluster(12, 61, box=5.0, tau=1e-10)
    announce("workspace too small")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    small = hfk.new_workspace(4096, dev)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock(xyz, D, s.exps, s.coefs, s.tau, workspace=small)
    assert ei.value.status == hfk.HFK_ENOMEM
    G, _ = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    # a forward-sized workspace is too small for the gradient
    fwd_ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, 3, "fp64"), dev)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, fock_in=G, workspace=fwd_ws)
    assert ei.value.status == hfk.HFK_ENOMEM
    off, bx, bd = pack_batch([s, random_cluster(3, 62)])
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock_batched(off, torch.tensor(bx, device=dev), torch.tensor(bd, device=dev), s.exps, s.coefs, s.tau,
                         precision="fp64", with_grad=True, workspace=small)
    assert ei.value.status == hfk.HFK_ENOMEM


def _crossing_quartets(s):
    """Quartets kept by the screen whose bra bound Q_s is below tau / 2 (their partner Q_t
    lies above 2)."""
    Q = oracle.schwarz(s.xyz, s.exps, s.coefs)
    small = Q[(Q < s.tau / 2) & (Q * Q.max() >= s.tau)]
    return sum(int(np.sum(Q * q >= s.tau)) for q in small)


@pytest.mark.parametrize("variant", [0, 1])
def test_bounds_above_two(torch_dev, variant):
    """Schwarz bounds above 2 (a tight contraction): a bra with tau / Q_s above 2 still has
    kets, in the open-ended top band.  Regression: such bras once got an empty ket range,
    which dropped quartets worth ~1e-3 each here."""
    from he_inputs import tight_cluster
    s = tight_cluster()
    assert _crossing_quartets(s) > 100
    announce("bounds above two variant=%d" % variant)
    G, E2, st = _run(torch_dev, s, variant=variant)
    Gr, Er, nr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert st["quartets"] == nr
    assert_close(G, Gr, FP64_TOL)
    assert rel(E2, Er) < FP64_TOL


# ------------------------------------------------------------------ deterministic strategy

def _det_builds(torch_dev, s, precision="fp64", reps=3, atoms=False):
    """reps builds with the deterministic strategy, each on a freshly allocated workspace."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    g = s.exps.shape[-1]
    out = []
    for r in range(reps):
        nb = hfk.workspace_bytes_atoms(s.natoms, g, precision) if atoms else hfk.workspace_bytes(s.natoms, g, precision)
        ws = hfk.new_workspace(nb, dev)
        ws.fill_(r * 37 % 251)   # contents on entry must not matter
        build = hfk.fock_atoms if atoms else hfk.fock
        G, E2 = build(xyz, D, s.exps, s.coefs, s.tau, precision=precision, strategy=hfk.STRATEGY_DETERMINISTIC,
                      workspace=ws)
        st = hfk.read_stats(ws)
        assert st["strategy"] == hfk.STRATEGY_DETERMINISTIC
        out.append((G.cpu().numpy(), float(E2.item()), st["quartets"]))
        del ws
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_deterministic_repeats_bitwise_he64(torch_dev, precision, tol):
    s = config_system("he64_fp64")
    announce("deterministic he64 %s" % precision)
    runs = _det_builds(torch_dev, s, precision)
    G0, E0, n0 = runs[0]
    for G, E, nq in runs[1:]:
        assert np.array_equal(G, G0) and E == E0 and nq == n0
    Gr, Er, nr = load_golden("he64_fp64")
    assert_close(G0, Gr, tol)
    assert rel(E0, Er) < tol
    assert np.array_equal(G0, G0.T)


def test_deterministic_repeats_bitwise_ragged_and_atoms(torch_dev):
    """A ragged random cluster (one basis) and an H/He lattice (per-atom bases)."""
    from he_inputs import mixed_lattice
    s = random_cluster(70, 8, box=9.0, tau=1e-9)
    announce("deterministic ragged 70")
    runs = _det_builds(torch_dev, s)
    for G, E, _ in runs[1:]:
        assert np.array_equal(G, runs[0][0]) and E == runs[0][1]
    Gr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(runs[0][0], Gr, FP64_TOL)
    m = mixed_lattice((4, 4, 4), seed=12, tau=1e-12)
    announce("deterministic H/He 64 per-atom")
    runs = _det_builds(torch_dev, m, atoms=True)
    for G, E, _ in runs[1:]:
        assert np.array_equal(G, runs[0][0]) and E == runs[0][1]
    Gr, Er, _ = oracle.fock_atoms(m.xyz, m.dens, m.exps, m.coefs, m.tau)
    assert_close(runs[0][0], Gr, FP64_TOL)
    assert rel(runs[0][1], Er) < FP64_TOL


def test_deterministic_he512_full_size(torch_dev):
    """The 512-atom workload with the deterministic strategy: two builds agree bit for bit,
    and every element, E2 and the survivors match the stored oracle build."""
    s = config_system("he512_fp64")
    announce("deterministic he512")
    Gr, e2_ref, ns_ref = load_full("he512_fp64")
    runs = _det_builds(torch_dev, s, reps=2)
    assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]
    G, E2, nq = runs[0]
    assert nq == ns_ref
    assert rel(E2, e2_ref) < FP64_TOL
    assert_close(G, Gr, FP64_TOL)


def test_deterministic_refuses_a_crowded_bucket(torch_dev):
    """100 coincident atoms put all 5050 pairs in one (Q band, cell) bucket: the deterministic
    strategy refuses (its per-bucket sort is sized for realistic buckets), before any sort."""
    import paper_2509_21039_amd as hfk
    torch, dev = torch_dev
    s = random_cluster(100, 3, box=1.0, tau=1e-10)
    s.xyz[:] = 0.0
    announce("deterministic crowded bucket")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock(xyz, D, s.exps, s.coefs, s.tau, strategy=hfk.STRATEGY_DETERMINISTIC)
    assert ei.value.status == hfk.HFK_EUNSUPPORTED
    assert "bucket" in str(ei.value)
