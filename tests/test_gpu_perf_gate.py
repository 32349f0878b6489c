"""Performance gate of the headline workload: the 512-atom FP64 build, tuned, must keep at
least 50% of the FP64 vector peak in nominal flops (2,525 per kept quartet) in its quartet
kernel, the target the build is held to.  Measured: 66-70% across boxes (the engine clock
under load differs by a few percent between them)."""
import pytest

from he_inputs import config_system
from gpu_util import announce

pytestmark = pytest.mark.gpu

FP64_PEAK_TFLOPS = 78.6
FLOP_PER_QUARTET = 81 * 31 + 14


def test_he512_fp64_peak_fraction():
    import torch
    import paper_2509_21039_amd as hfk
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    s = config_system("he512_fp64")
    announce("perf gate he512 fp64")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    hfk.tune(xyz, D, s.exps, s.coefs, s.tau, precision="fp64")
    ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, 3, "fp64"), dev)
    hfk.fock(xyz, D, s.exps, s.coefs, s.tau, workspace=ws)
    torch.cuda.synchronize()
    hfk.profile_read()
    hfk.profile_enable(True)
    for _ in range(3):
        hfk.fock(xyz, D, s.exps, s.coefs, s.tau, workspace=ws)
    torch.cuda.synchronize()
    hfk.profile_enable(False)
    kms, launches = hfk.profile_read()
    q = hfk.read_stats(ws)["quartets"]
    frac = q * FLOP_PER_QUARTET / (kms / launches * 1e-3) / (FP64_PEAK_TFLOPS * 1e12)
    print("he512 fp64 nominal peak fraction %.3f" % frac)
    assert frac >= 0.50, frac
