"""Debug mode: densities are checked on the device before a build (HFK_ENOTSYM, HFK_EINVAL)."""
import numpy as np
import pytest

import oracle
from he_inputs import pack_batch, random_cluster
from gpu_util import announce, assert_close, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture
def debug_on():
    import paper_2509_21039_amd as hfk
    hfk.set_debug(True, 1e-12)
    yield hfk
    hfk.set_debug(False, 0.0)


def _tensors(torch_dev, s, D=None):
    torch, dev = torch_dev
    return torch.tensor(s.xyz, device=dev), torch.tensor(s.dens if D is None else D, device=dev)


def test_symmetric_density_builds_as_without_debug(torch_dev, debug_on):
    hfk = debug_on
    s = random_cluster(20, 71, box=6.0, tau=1e-10)
    xyz, D = _tensors(torch_dev, s)
    announce("debug symmetric build")
    G, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    Gr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert_close(G.cpu().numpy(), Gr, 1e-10)
    assert rel(E2.item(), Er) < 1e-10
    # the gradient call checks its density too, and accepts this one
    d_xyz, _, _ = hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, want_dens=False)
    assert np.isfinite(d_xyz.cpu().numpy()).all()


def test_asymmetric_density_is_refused(torch_dev, debug_on):
    hfk = debug_on
    s = random_cluster(20, 72, box=6.0, tau=1e-10)
    Dbad = s.dens.copy()
    Dbad[3, 7] += 1e-6
    xyz, D = _tensors(torch_dev, s, Dbad)
    announce("debug asymmetric density")
    for call in (lambda: hfk.fock(xyz, D, s.exps, s.coefs, s.tau),
                 lambda: hfk.fock_atoms(xyz, D, np.tile(s.exps, (20, 1)), np.tile(s.coefs, (20, 1)), s.tau),
                 lambda: hfk.fock_grad(xyz, D, s.exps, s.coefs, s.tau, want_dens=False)):
        with pytest.raises(hfk.HfkError) as ei:
            call()
        assert ei.value.status == hfk.HFK_ENOTSYM
        assert "not symmetric" in str(ei.value)


def test_tolerance_and_exact_mode(torch_dev, debug_on):
    """An asymmetry of 1e-14 relative passes a 1e-12 tolerance and fails an exact check."""
    hfk = debug_on
    s = random_cluster(12, 73, box=5.0, tau=1e-10)
    Dnear = s.dens.copy()
    Dnear[1, 4] *= 1.0 + 1e-14
    xyz, D = _tensors(torch_dev, s, Dnear)
    announce("debug tolerance")
    hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    hfk.set_debug(True, 0.0)
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    assert ei.value.status == hfk.HFK_ENOTSYM


def test_non_finite_density_is_refused(torch_dev, debug_on):
    hfk = debug_on
    s = random_cluster(9, 74, box=5.0, tau=1e-10)
    Dnan = s.dens.copy()
    Dnan[2, 2] = np.nan
    xyz, D = _tensors(torch_dev, s, Dnan)
    announce("debug NaN density")
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    assert ei.value.status == hfk.HFK_EINVAL and "non-finite" in str(ei.value)


def test_batched_names_the_asymmetric_molecule(torch_dev, debug_on):
    hfk = debug_on
    torch, dev = torch_dev
    systems = [random_cluster(n, 80 + n, box=5.0, tau=1e-10) for n in (4, 9, 6, 11)]
    systems[2].dens[0, 5] += 1e-5
    off, xyz, dens = pack_batch(systems)
    announce("debug batched asymmetric molecule")
    with pytest.raises(hfk.HfkError) as ei:
        hfk.fock_batched(off, torch.tensor(xyz, device=dev), torch.tensor(dens, device=dev), systems[0].exps,
                         systems[0].coefs, 1e-10, precision="fp64", with_grad=False)
    assert ei.value.status == hfk.HFK_ENOTSYM and "molecule 2" in str(ei.value)
    systems[2].dens[0, 5] -= 1e-5
    off, xyz, dens = pack_batch(systems)
    F, E2, _ = hfk.fock_batched(off, torch.tensor(xyz, device=dev), torch.tensor(dens, device=dev), systems[0].exps,
                                systems[0].coefs, 1e-10, precision="fp64", with_grad=False)
    assert np.isfinite(E2.cpu().numpy()).all()


def test_without_debug_the_density_is_not_checked(torch_dev):
    """Debug mode off (the default): an asymmetric density is not refused (the build reads it
    as the kernel listing does; the result is then not the plain definition's G)."""
    import paper_2509_21039_amd as hfk
    s = random_cluster(10, 75, box=5.0, tau=1e-10)
    Dbad = s.dens.copy()
    Dbad[0, 1] += 0.5
    xyz, D = _tensors(torch_dev, s, Dbad)
    announce("no debug, asymmetric density")
    G, E2 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    assert np.isfinite(G.cpu().numpy()).all()


def test_last_stats_follows_the_last_build(torch_dev):
    import paper_2509_21039_amd as hfk
    s = random_cluster(16, 76, box=6.0, tau=1e-10)
    xyz, D = _tensors(torch_dev, s)
    announce("last stats")
    torch, dev = torch_dev
    ws = hfk.new_workspace(hfk.workspace_bytes(16, 3, "fp64"), dev)   # alive while the stats are read
    hfk.fock(xyz, D, s.exps, s.coefs, s.tau, workspace=ws)
    st = hfk.last_stats()
    _, _, nr = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
    assert st["natoms"] == 16 and st["quartets"] == nr and st["tile_items"] >= 1 and st["group_bras"] >= 256
