"""The autotuners run, keep a valid choice and round-trip their cache file."""
import json

import numpy as np
import pytest

from he_inputs import cluster_batch, config_system, pack_batch
from gpu_util import announce, rel

pytestmark = pytest.mark.gpu


def test_tune_single_molecule(tmp_path):
    import torch
    import paper_2509_21039_amd as hfk
    dev = torch.device("cuda:0")
    s = config_system("he64_fp64")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    announce("tune he64")
    G0, E0 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    path = str(tmp_path / "tune.json")
    best = hfk.tune(xyz, D, s.exps, s.coefs, s.tau, cache_path=path)
    assert best in (hfk.STRATEGY_PRIVATE, hfk.STRATEGY_ATOMIC)
    table = json.load(open(path))
    assert table["format"] == "hfk-tuning-1" and len(table["entries"]) >= 1
    hfk.load_tuning(path)
    G1, E1 = hfk.fock(xyz, D, s.exps, s.coefs, s.tau)
    assert rel(E1.item(), E0.item()) < 1e-12


def test_tune_batched(tmp_path):
    import torch
    import paper_2509_21039_amd as hfk
    dev = torch.device("cuda:0")
    systems = cluster_batch(nmol=60, seed=9)
    off, xyz, dens = pack_batch(systems)
    X = torch.tensor(xyz, device=dev)
    Dp = torch.tensor(dens, device=dev)
    announce("tune batched 60")
    gpc = hfk.tune_batched(off, X, Dp, systems[0].exps, systems[0].coefs, systems[0].tau,
                           cache_path=str(tmp_path / "tb.json"))
    assert 1 <= gpc <= 3
    F, E2, g = hfk.fock_batched(off, X, Dp, systems[0].exps, systems[0].coefs, systems[0].tau)
    assert np.isfinite(E2.cpu().numpy()).all()
