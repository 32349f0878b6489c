"""The allocation-free entry point (hfk_fock_noalloc, static scratch) against the workspace
entry point (hfk_fock) and the oracle: two calls in a row, the second on a smaller system,
and the refusal of a system beyond the scratch."""
import ctypes

import numpy as np
import pytest

import oracle
from he_inputs import random_cluster
from gpu_util import announce, assert_close, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6


def _noalloc_raw(hfk, torch, xyz, D, s, precision):
    """hfk_fock_noalloc called through the C ABI with caller-allocated outputs."""
    n = s.natoms
    F = torch.full((n, n), float("nan"), dtype=torch.float64, device=xyz.device)
    E2 = torch.full((1,), float("nan"), dtype=torch.float64, device=xyz.device)
    e = np.ascontiguousarray(s.exps, dtype=np.float64)
    c = np.ascontiguousarray(s.coefs, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    st = hfk.lib().hfk_fock_noalloc(n, xyz.data_ptr(), len(e), e.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                    D.data_ptr(), float(s.tau), 0 if precision == "fp64" else 1, F.data_ptr(),
                                    E2.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, F, E2


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_noalloc_matches_workspace_entry_two_calls(precision, tol):
    import torch
    import paper_2509_21039_amd as hfk
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    # the largest system of the scratch first, then a smaller ragged one: the second call
    # must not see the first call's leftovers
    for n, seed, box in ((256, 301, 16.0), (37, 302, 7.0)):
        s = random_cluster(n, seed, box=box, tau=1e-10)
        xyz = torch.tensor(s.xyz, device=dev)
        D = torch.tensor(s.dens, device=dev)
        announce("noalloc %s n=%d" % (precision, n))
        st, G, E2 = _noalloc_raw(hfk, torch, xyz, D, s, precision)
        assert st == hfk.HFK_OK, hfk.lib().hfk_last_error()
        torch.cuda.synchronize()
        Gw, E2w = hfk.fock(xyz, D, s.exps, s.coefs, s.tau, precision=precision)
        Gn, Gwn = G.cpu().numpy(), Gw.cpu().numpy()
        assert_close(Gn, Gwn, tol, "noalloc vs hfk_fock n=%d" % n)
        assert rel(E2.item(), E2w.item()) < tol
        Gr, Er, _ = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau)
        assert_close(Gn, Gr, tol, "noalloc vs oracle n=%d" % n)
        assert rel(E2.item(), Er) < tol


def test_noalloc_refuses_a_system_beyond_the_scratch():
    import torch
    import paper_2509_21039_amd as hfk
    dev = torch.device("cuda:0")
    s = random_cluster(320, 303, box=18.0, tau=1e-10)
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    announce("noalloc beyond the scratch")
    st, G, E2 = _noalloc_raw(hfk, torch, xyz, D, s, "fp64")
    assert st == hfk.HFK_EUNSUPPORTED
    assert "scratch" in hfk.lib().hfk_last_error().decode()
    torch.cuda.synchronize()
    assert torch.isnan(E2).all().item()   # nothing was written
