"""Benchmark of the two-electron Fock build on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one whole Fock build (pair preparation, Schwarz screen, quartet kernel,
reduction, symmetrisation, E2) of the 512-atom He lattice (8x8x8, spacing 2 bohr, jitter
0.2, STO-3G, tau 1e-10) in FP64, inputs resident in HBM.  Prints one JSON line with the
throughput in surviving unique quartets per second, the roofline of the quartet kernel
(FP64 vector ALU), the CPU oracle timed on a bounded sample of the same workload, and the
mixed-precision and forward+gradient comparisons on their own workloads.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ERI quartets/s & % FP64 VALU peak; mixed-prec and fwd+grad vs plain FP64"
FP64_VALU_PEAK_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, FP64 vector
FP32_VALU_PEAK_TFLOPS = 157.3
FLOP_PER_PRIM_QUARTET = 31        # nominal flops per primitive quartet: the algorithmic work unit
FLOP_SCATTER_PER_QUARTET = 14


# Hardware-counter summary of the quartet kernel (FETCH_SIZE / WRITE_SIZE, scaled by the
# same counters read on a plain copy of known size).  Used only while the kernel sources
# and the launch configuration are the ones the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fock_he512_fp64_traffic.json")
KERNEL_SOURCES = ["paper_2509_21039_amd/csrc/hfk_fock.hip", "paper_2509_21039_amd/csrc/hfk_device.hpp",
                  "paper_2509_21039_amd/csrc/hfk_internal.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stats):
    """HBM bytes per launch from the committed counter summary, or None if it is stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    for e in t.get("entries", []):
        cfg = e.get("config", {})
        if all(cfg.get(k) == stats.get(k) for k in ("strategy", "variant", "groups", "tile_items", "group_bras",
                                                   "ket_copies")):
            return e.get("bytes_per_launch")
    return None


GOLDEN = os.path.join(ROOT, "tests", "golden")
# Nominal flops of the forward + gradient contraction per kept quartet: 31 (integral) + 45
# (F1, nine derivative components, Gamma contraction) per primitive quartet, plus 14.
FLOP_GRAD_PER_PRIM_QUARTET = 31 + 45
# FP32 vector rates: the published 157.3 TFLOP/s counts packed FP32 (two lanes per
# instruction); packed FP32 instructions are disabled in this build, so 78.6 TFLOP/s
# (256 CU x 64 lanes x 2 flop x 2.4 GHz, one FP32 FMA per lane per cycle) is its ceiling.
FP32_VALU_NONPACKED_TFLOPS = 78.6


def stored_oracle(name):
    """A whole matrix written by tests/golden/make_golden.py (oracle only): (G, E2, survivors)."""
    with np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False) as z:
        tri = z["tri"]
        n = int(round((math.sqrt(8 * tri.size + 1) - 1) / 2))
        G = np.zeros((n, n))
        G[np.tril_indices(n)] = tri
        return G + np.tril(G, -1).T, float(z["e2"]), int(z["survivors"])


def stored_grad(name="he128_grad"):
    path = os.path.join(GOLDEN, name + ".txt")
    return np.loadtxt(path)


def err_vs(x, ref):
    """Errors of a result against the FP64 oracle: element-wise (max |dx| / max |ref|) and Frobenius."""
    x = np.asarray(x); ref = np.asarray(ref)
    return {"max_abs_over_max_ref": float(np.abs(x - ref).max() / np.abs(ref).max()),
            "fro_rel": float(np.linalg.norm(x - ref) / np.linalg.norm(ref))}


# Counter-based FP64 flops of the quartet kernel (rocprofv3 VALU instruction counts), used
# only while the kernel sources and the launch configuration match the counted run.
VALU_FILE = os.path.join(ROOT, "profiles", "k_fock_he512_fp64_valu.json")


def counted_fp64_flop(stats):
    try:
        with open(VALU_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    for e in t.get("entries", []):
        cfg = e.get("config", {})
        if all(cfg.get(k) == stats.get(k) for k in ("strategy", "variant", "groups", "tile_items", "group_bras",
                                                   "ket_copies")):
            return e.get("fp64_flop_per_launch")
    return None


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def sample_sclk(delay_s: float, out: dict):
    """Reads the shader clock once with rocm-smi, delay_s into the timed run (None if the tool
    is missing or its output has no sclk figure)."""
    import re
    import subprocess
    time.sleep(delay_s)
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        d = json.loads(r.stdout)
        for card in d.values():
            for k, v in card.items():
                if "sclk" in k.lower():
                    m = re.search(r"(\d+)\s*Mhz", str(v), re.I)
                    if m:
                        out["sclk_mhz"] = int(m.group(1))
                        return
    except Exception:
        pass


def flop_per_quartet(g: int) -> int:
    return g ** 4 * FLOP_PER_PRIM_QUARTET + FLOP_SCATTER_PER_QUARTET


def time_builds(hfk, torch, s, precision, steps, warmup, ws, atoms=False):
    dev = torch.device("cuda:0")
    build = hfk.fock_atoms if atoms else hfk.fock
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    n = s.natoms
    F = torch.empty((n, n), dtype=torch.float64, device=dev)
    E2 = torch.empty((1,), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        build(xyz, D, s.exps, s.coefs, s.tau, precision=precision, workspace=ws, out=(F, E2))
    torch.cuda.synchronize()
    stats = hfk.read_stats(ws)
    hfk.profile_read()                      # drop anything recorded so far
    hfk.profile_enable(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    clock = {}
    import threading
    sampler = threading.Thread(target=sample_sclk, args=(0.3, clock), daemon=True)
    sampler.start()
    e0.record(stream)
    marks[0].record(stream)
    for k in range(steps):
        build(xyz, D, s.exps, s.coefs, s.tau, precision=precision, workspace=ws, out=(F, E2))
        marks[k + 1].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sampler.join(timeout=30)
    hfk.profile_enable(False)
    kern_ms, launches = hfk.profile_read()
    total_ms = e0.elapsed_time(e1)
    per = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))

    def pct(q):
        return per[min(len(per) - 1, int(round(q * (len(per) - 1))))]

    return {"ms_per_step": total_ms / steps, "kernel_ms": kern_ms / max(launches, 1), "stats": stats,
            "e2": float(E2.item()), "F": F, "step_ms": {"median": pct(0.5), "p10": pct(0.1), "p90": pct(0.9)},
            "sclk_mhz": clock.get("sclk_mhz")}


def time_grad(hfk, torch, s, steps, warmup, precision="fp64"):
    """Forward build followed by the backward (dE2/dR, dE2/dD) per step; the gradient
    kernel's own duration from the library's HIP events around it."""
    dev = torch.device("cuda:0")
    xyz = torch.tensor(s.xyz, device=dev)
    D = torch.tensor(s.dens, device=dev)
    atoms = np.ndim(s.exps) == 2
    g = s.exps.shape[-1]
    nb = (hfk.workspace_bytes_atoms(s.natoms, g, precision, True) if atoms
          else hfk.workspace_bytes(s.natoms, g, precision, True))
    ws = hfk.new_workspace(nb, dev)
    g_e2 = torch.ones((1,), dtype=torch.float64, device=dev)
    build = hfk.fock_atoms if atoms else hfk.fock
    grad = hfk.fock_grad
    out = {}

    def step(prof):
        G, E2 = build(xyz, D, s.exps, s.coefs, s.tau, precision=precision, workspace=ws)
        if prof:
            hfk.profile_enable(True)     # events are recorded when the launch is enqueued
        r = grad(xyz, D, s.exps, s.coefs, s.tau, precision=precision, g_e2=g_e2, fock_in=G, workspace=ws)
        if prof:
            hfk.profile_enable(False)
        out["d_xyz"] = r[0]
        return r

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    hfk.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step(True)
    e1.record()
    torch.cuda.synchronize()
    kms, nl = hfk.profile_read()
    return {"ms_per_step": e0.elapsed_time(e1) / steps, "grad_kernel_ms": kms / max(nl, 1),
            "d_xyz": out["d_xyz"].cpu().numpy(), "quartets": hfk.read_stats(ws)["quartets"]}


def time_batched(hfk, torch, systems, steps, warmup):
    """The ragged batch, mixed + gradient in one launch, tuned first; errors of the sampled
    clusters against the stored oracle results."""
    from he_inputs import pack_batch
    dev = torch.device("cuda:0")
    off, xyz, dens = pack_batch(systems)
    X = torch.tensor(xyz, device=dev)
    Dp = torch.tensor(dens, device=dev)
    s0 = systems[0]
    gpc = hfk.tune_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision="mixed", with_grad=True)
    ws = hfk.new_workspace(hfk.batched_workspace_bytes(off, len(s0.exps), "mixed", True), dev)
    for _ in range(warmup):
        hfk.fock_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision="mixed", with_grad=True, workspace=ws)
    torch.cuda.synchronize()
    stats = hfk.read_stats(ws)
    hfk.profile_read()
    hfk.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        F, E2, g = hfk.fock_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision="mixed", with_grad=True,
                                    workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    hfk.profile_enable(False)
    kms, nl = hfk.profile_read()
    ms = e0.elapsed_time(e1) / steps
    kernel_ms = kms / max(nl, 1)
    q = stats["quartets"]
    g_ = len(s0.exps)
    achieved = q * (g_ ** 4 * FLOP_GRAD_PER_PRIM_QUARTET + FLOP_SCATTER_PER_QUARTET) / (kernel_ms / 1e3) / 1e12
    res = {"molecules": len(systems), "atoms": int(off[-1]), "quartets": q,
           "ms_per_batch": ms, "kernel_ms": kernel_ms, "quartets_per_s": q / (ms / 1e3),
           "config": {"groups_per_cu": gpc, "workgroups": stats["groups"], "items_per_block": stats["tile_items"]},
           "roofline": {"bound": "alu", "kernel": "k_batched<3,float,grad>", "achieved": achieved,
                        "unit": "TFLOP/s", "flop_per_quartet": g_ ** 4 * FLOP_GRAD_PER_PRIM_QUARTET
                        + FLOP_SCATTER_PER_QUARTET,
                        "peak_fp32_packed": FP32_VALU_PEAK_TFLOPS, "frac_fp32_packed": achieved / FP32_VALU_PEAK_TFLOPS,
                        "peak_fp32_nonpacked": FP32_VALU_NONPACKED_TFLOPS,
                        "frac_fp32_nonpacked": achieved / FP32_VALU_NONPACKED_TFLOPS}}
    try:
        with np.load(os.path.join(GOLDEN, "batched_2000_sample.npz"), allow_pickle=False) as z:
            counts = np.array([s.natoms for s in systems], dtype=np.int64)
            doff = np.concatenate([[0], np.cumsum(counts ** 2)])
            Fh, Eh, gh = F.cpu().numpy(), E2.cpu().numpy(), g.cpu().numpy()
            worst = {"G_max_abs_over_max_ref": 0.0, "E2_rel": 0.0, "grad_max_abs_over_max_ref": 0.0}
            t0 = g0 = 0
            for m, n, e2r in zip(z["mol"], z["natoms"], z["e2"]):
                n = int(n)
                nt = n * (n + 1) // 2
                Gr = np.zeros((n, n))
                Gr[np.tril_indices(n)] = z["tri"][t0:t0 + nt]
                Gr = Gr + np.tril(Gr, -1).T
                gr = z["grad"][g0:g0 + n]
                t0 += nt
                g0 += n
                Fm = Fh[doff[m]:doff[m] + n * n].reshape(n, n)
                worst["G_max_abs_over_max_ref"] = max(worst["G_max_abs_over_max_ref"],
                                                      err_vs(Fm, Gr)["max_abs_over_max_ref"])
                worst["E2_rel"] = max(worst["E2_rel"], abs(Eh[m] - e2r) / abs(e2r))
                worst["grad_max_abs_over_max_ref"] = max(worst["grad_max_abs_over_max_ref"],
                                                         err_vs(gh[off[m]:off[m + 1]], gr)["max_abs_over_max_ref"])
            res["errors_vs_oracle"] = dict(worst, clusters=int(len(z["mol"])),
                                           note="largest over the stored 50 clusters (the ten largest and 40 drawn)")
    except OSError:
        res["errors_vs_oracle"] = None
    return res


def cpu_baseline(s, target_s=12.0):
    """Oracle on a bounded bra range of the same system, scaled to quartets/s."""
    import oracle
    oracle.build(force=False)
    Q = oracle.schwarz(s.xyz, s.exps, s.coefs)
    npair = s.natoms * (s.natoms + 1) // 2
    nb = 8
    while True:
        t0 = time.perf_counter()
        _, _, ns = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau, Q=Q, bra_range=(npair - nb, npair))
        dt = time.perf_counter() - t0
        if dt >= target_s or nb >= npair:
            break
        grow = max(2.0, min(8.0, target_s / max(dt, 1e-3)))
        nb = min(npair, int(nb * grow) + 1)
    cores = oracle.num_threads()
    # one thread on the last 1/64 of the same bra range (a few seconds)
    nb1 = max(1, nb // 64)
    t0 = time.perf_counter()
    _, _, ns1 = oracle.fock(s.xyz, s.dens, s.exps, s.coefs, s.tau, Q=Q, nthreads=1, bra_range=(npair - nb1, npair))
    dt1 = time.perf_counter() - t0
    oracle.fock(s.xyz[:2], s.dens[:2, :2], s.exps, s.coefs, s.tau, nthreads=cores)   # restore the thread count
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": ns / dt, "unit": "quartets/s", "cores": cores, "kind": "oracle",
            "sample": "last %d bra pairs (canonical order) of the 512-atom build: %d quartets in %.1f s; "
                      "Schwarz bounds precomputed outside the timing" % (nb, ns, dt),
            "single_thread": {"value": ns1 / dt1, "unit": "quartets/s", "cores": 1,
                              "sample": "last %d bra pairs: %d quartets in %.1f s" % (nb1, ns1, dt1)},
            "cpu_model": model, "host_cpus": os.cpu_count()}


def plain_copy(torch, dev, nbytes=512 << 20):
    """A device copy of known size: the reference that scales the traffic counters."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return nbytes


def run_probe(hfk, torch, dev, which):
    """One warm-up and one timed call of the batched or gradient workload in the untuned
    default configuration, then a plain copy; prints what ran."""
    from he_inputs import cluster_batch, config_system, pack_batch
    info = {"probe": which}
    if which == "batched":
        systems = cluster_batch()
        off, xyz, dens = pack_batch(systems)
        X = torch.tensor(xyz, device=dev)
        Dp = torch.tensor(dens, device=dev)
        s0 = systems[0]
        ws = hfk.new_workspace(hfk.batched_workspace_bytes(off, len(s0.exps), "mixed", True), dev)
        for _ in range(2):
            t0 = time.perf_counter()
            hfk.fock_batched(off, X, Dp, s0.exps, s0.coefs, s0.tau, precision="mixed", with_grad=True, workspace=ws)
            torch.cuda.synchronize()
            info.setdefault("call_ms", []).append((time.perf_counter() - t0) * 1e3)
        st = hfk.read_stats(ws)
    else:
        s = config_system("he128_grad")
        X = torch.tensor(s.xyz, device=dev)
        D = torch.tensor(s.dens, device=dev)
        ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, len(s.exps), "fp64", True), dev)
        g_e2 = torch.ones((1,), dtype=torch.float64, device=dev)
        for _ in range(2):
            t0 = time.perf_counter()
            G, _ = hfk.fock(X, D, s.exps, s.coefs, s.tau, workspace=ws)
            hfk.fock_grad(X, D, s.exps, s.coefs, s.tau, g_e2=g_e2, fock_in=G, workspace=ws)
            torch.cuda.synchronize()
            info.setdefault("call_ms", []).append((time.perf_counter() - t0) * 1e3)
        st = hfk.read_stats(ws)
    info.update({"quartets": st["quartets"], "groups": st["groups"], "tile_items": st.get("tile_items"),
                 "copy_bytes": plain_copy(torch, dev)})
    print(json.dumps(info), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip mixed / fwd+grad / batched comparisons")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one he512 FP64 build (hybrid kernel, default workgroups, --probe-strategy) and one plain "
                         "512 MiB device copy, for hardware-counter runs; prints the configuration")
    ap.add_argument("--probe-strategy", type=int, default=2, choices=[1, 2],
                    help="accumulation strategy of the traffic probe (1 private copies, 2 atomics)")
    ap.add_argument("--probe-shape", default="",
                    help="launch shape of the traffic probe: gpc,tile_items,group_bras,ket_copies "
                         "(default: the untuned default)")
    ap.add_argument("--probe-mixed", action="store_true",
                    help="the traffic probe on the 1024-atom lattice in mixed precision instead of he512 FP64")
    ap.add_argument("--batched-probe", action="store_true",
                    help="one warm-up and one timed call of the 2000-cluster batch (mixed + gradient, default "
                         "configuration, no tuning) and one plain 512 MiB device copy, for counter runs")
    ap.add_argument("--valu-probe", action="store_true",
                    help="run the VALU throughput probe (built next to the library) and print its JSON line")
    ap.add_argument("--grad-probe", action="store_true",
                    help="one warm-up and one timed forward + backward of the 128-atom lattice (FP64, default "
                         "configuration) and one plain 512 MiB device copy, for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the Fock build here is single-GPU (the multi-GPU "
              "design is an all-reduce of F over a cost-balanced split of the tile list, not built). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.valu_probe:
        import subprocess
        probe = os.path.join(ROOT, "paper_2509_21039_amd", "valu_probe")
        if not os.path.exists(probe):
            sys.exit("valu_probe is not built: run python -m paper_2509_21039_amd.build")
        sys.exit(subprocess.run([probe]).returncode)

    import torch
    import paper_2509_21039_amd as hfk
    from he_inputs import config_system

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    s = config_system("he512_fp64")
    g = len(s.exps)
    if args.batched_probe or args.grad_probe:
        return run_probe(hfk, torch, dev, "batched" if args.batched_probe else "grad")
    if args.traffic_probe:
        # one build in a fixed configuration (hybrid kernel, default workgroups), then a copy
        prec = "mixed" if args.probe_mixed else "fp64"
        if args.probe_mixed:
            s = config_system("he1024_mixed")
        ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, g, prec), dev)
        xyz_t = torch.tensor(s.xyz, device=dev)
        D_t = torch.tensor(s.dens, device=dev)
        if args.probe_shape:
            gpc, tile, gbras, kcop = (int(v) for v in args.probe_shape.split(","))
            hfk.set_config(1, gpc)
            hfk.set_shape(tile, gbras, kcop)
        else:
            hfk.set_config(1, 0)
        hfk.fock(xyz_t, D_t, s.exps, s.coefs, s.tau, precision=prec, strategy=args.probe_strategy, workspace=ws)
        torch.cuda.synchronize()
        st = hfk.read_stats(ws)
        nbytes = plain_copy(torch, dev)
        print(json.dumps({"copy_bytes": nbytes, "precision": prec, "natoms": s.natoms, "quartets": st["quartets"],
                          "strategy": st["strategy"], "variant": st["variant"],
                          "groups": st["groups"], "tile_items": st["tile_items"], "group_bras": st["group_bras"],
                          "ket_copies": st["ket_copies"], "source_sha256": kernel_source_hash()}), flush=True)
        return
    ws = hfk.new_workspace(hfk.workspace_bytes(s.natoms, g, "fp64"), dev)
    log("he512 fp64: autotune")
    xyz_t = torch.tensor(s.xyz, device=dev)
    D_t = torch.tensor(s.dens, device=dev)
    hfk.tune(xyz_t, D_t, s.exps, s.coefs, s.tau, precision="fp64")
    del xyz_t, D_t
    log("he512 fp64: warmup %d, steps %d" % (args.warmup, args.steps))
    r = time_builds(hfk, torch, s, "fp64", args.steps, args.warmup, ws)
    q = r["stats"]["quartets"]
    value = q / (r["ms_per_step"] / 1e3)
    achieved = q * flop_per_quartet(g) / (r["kernel_ms"] / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "he512_fp64: 512 He atoms, jittered 8x8x8 lattice (spacing 2.0 bohr, jitter 0.2, "
                               "seed 2), STO-3G (3 primitives), density 0.1*(M+M^T)/2 with unit diagonal, "
                               "Schwarz tau 1e-10, FP64",
                   "natoms": s.natoms, "ngauss": g, "tau": s.tau, "quartets": q,
                   "primitive_quartets": q * g ** 4, "sig_pairs": r["stats"]["sig_pairs"],
                   "kernel_variant": r["stats"]["variant"], "accumulation": r["stats"]["strategy"],
                   "workgroups": r["stats"]["groups"], "tile_items": r["stats"]["tile_items"],
                   "group_bras": r["stats"]["group_bras"], "ket_copies": r["stats"]["ket_copies"],
                   "parallelism": "single GPU"},
        "pct_fp64_valu_peak_nominal": 100.0 * achieved / FP64_VALU_PEAK_TFLOPS,
        "step_ms": r["step_ms"],
        "sclk_mhz_sampled": r["sclk_mhz"],
        "pct_fp64_valu_peak_at_sampled_clock": (100.0 * achieved / (FP64_VALU_PEAK_TFLOPS * r["sclk_mhz"] / 2400.0)
                                                if r["sclk_mhz"] else None),
        "primitive_quartets_per_s": q * g ** 4 / (r["ms_per_step"] / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": measured_traffic(r["stats"]),
                     "kernel": "k_fock<3,double>", "kernel_ms": r["kernel_ms"],
                     "flop_per_quartet": flop_per_quartet(g)},
        "e2": r["e2"],
    }
    try:
        Gr, Er, nr = stored_oracle("he512_fp64")
        out["errors_vs_oracle"] = {"G": err_vs(r["F"].cpu().numpy(), Gr), "E2_rel": abs(r["e2"] - Er) / abs(Er),
                                   "quartets_equal": q == nr, "oracle": "tests/golden/he512_fp64.npz"}
    except OSError:
        out["errors_vs_oracle"] = None
    counted = counted_fp64_flop(r["stats"])
    if counted is not None:
        out["roofline"]["counted_flop_per_launch"] = counted
        out["roofline"]["counted_frac"] = counted / (r["kernel_ms"] / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS
    else:
        out["roofline"]["counted_frac"] = None
    del r
    if not args.no_extras:
        extras = {}
        try:
            s3 = config_system("he1024_mixed")
            ws3 = hfk.new_workspace(hfk.workspace_bytes(s3.natoms, g, "fp64"), dev)
            log("he1024: autotune fp64 and mixed, then time")
            x3 = torch.tensor(s3.xyz, device=dev)
            d3 = torch.tensor(s3.dens, device=dev)
            hfk.tune(x3, d3, s3.exps, s3.coefs, s3.tau, precision="fp64")
            hfk.tune(x3, d3, s3.exps, s3.coefs, s3.tau, precision="mixed")
            del x3, d3
            a = time_builds(hfk, torch, s3, "fp64", 3, 1, ws3)
            b = time_builds(hfk, torch, s3, "mixed", 3, 1, ws3)
            qa = a["stats"]["quartets"]
            Fa, Fb = a["F"], b["F"]
            mixed_tflops = b["stats"]["quartets"] * flop_per_quartet(g) / (b["kernel_ms"] / 1e3) / 1e12
            extras["mixed_he1024"] = {
                "quartets": qa,
                "fp64_quartets_per_s": qa / (a["ms_per_step"] / 1e3),
                "mixed_quartets_per_s": b["stats"]["quartets"] / (b["ms_per_step"] / 1e3),
                "speedup_vs_fp64": a["ms_per_step"] / b["ms_per_step"],
                "fp64_kernel_ms": a["kernel_ms"], "mixed_kernel_ms": b["kernel_ms"],
                "rel_err_F_vs_fp64": float(torch.linalg.norm(Fb - Fa) / torch.linalg.norm(Fa)),
                "rel_err_E2_vs_fp64": abs(b["e2"] - a["e2"]) / abs(a["e2"]),
                "mixed_tflops_nominal": mixed_tflops,
                "pct_fp32_packed_peak_nominal": 100.0 * mixed_tflops / FP32_VALU_PEAK_TFLOPS,
                "pct_fp32_nonpacked_peak_nominal": 100.0 * mixed_tflops / FP32_VALU_NONPACKED_TFLOPS,
                "fp32_peaks_tflops": {"packed": FP32_VALU_PEAK_TFLOPS, "nonpacked": FP32_VALU_NONPACKED_TFLOPS,
                                      "note": "packed FP32 is disabled in this build"},
            }
            try:
                Gr3, Er3, nr3 = stored_oracle("he1024_fp64")
                extras["mixed_he1024"]["errors_vs_oracle"] = {
                    "fp64": {"G": err_vs(Fa.cpu().numpy(), Gr3), "E2_rel": abs(a["e2"] - Er3) / abs(Er3)},
                    "mixed": {"G": err_vs(Fb.cpu().numpy(), Gr3), "E2_rel": abs(b["e2"] - Er3) / abs(Er3)},
                    "quartets_equal": qa == nr3 and b["stats"]["quartets"] == nr3}
            except OSError:
                extras["mixed_he1024"]["errors_vs_oracle"] = None
            del ws3, a, b, Fa, Fb
            torch.cuda.empty_cache()
        except hfk.HfkError as e:
            extras["mixed_he1024"] = {"error": str(e)}
        try:
            s4 = config_system("he128_grad")
            log("he128: forward vs forward+gradient")
            ws4 = hfk.new_workspace(hfk.workspace_bytes(s4.natoms, g, "fp64"), dev)
            f4 = time_builds(hfk, torch, s4, "fp64", 10, 2, ws4)
            fg = time_grad(hfk, torch, s4, 10, 2)
            fgm = time_grad(hfk, torch, s4, 10, 2, precision="mixed")
            q4 = f4["stats"]["quartets"]
            gtf = q4 * (g ** 4 * FLOP_GRAD_PER_PRIM_QUARTET + FLOP_SCATTER_PER_QUARTET) / (fg["grad_kernel_ms"] / 1e3) / 1e12
            extras["fwd_grad_he128"] = {
                "quartets": q4,
                "fwd_ms": f4["ms_per_step"], "fwd_grad_ms": fg["ms_per_step"],
                "fwd_quartets_per_s": q4 / (f4["ms_per_step"] / 1e3),
                "fwd_grad_quartets_per_s": q4 / (fg["ms_per_step"] / 1e3),
                "fwd_grad_over_fwd_time": fg["ms_per_step"] / f4["ms_per_step"],
                "mixed_fwd_grad_ms": fgm["ms_per_step"],
                "grad_kernel_ms": fg["grad_kernel_ms"], "mixed_grad_kernel_ms": fgm["grad_kernel_ms"],
                "grad_roofline": {"bound": "alu", "kernel": "k_grad<3,double>", "achieved": gtf, "unit": "TFLOP/s",
                                  "peak": FP64_VALU_PEAK_TFLOPS, "frac": gtf / FP64_VALU_PEAK_TFLOPS,
                                  "flop_per_quartet": g ** 4 * FLOP_GRAD_PER_PRIM_QUARTET + FLOP_SCATTER_PER_QUARTET},
            }
            try:
                gr = stored_grad("he128_grad")
                extras["fwd_grad_he128"]["errors_vs_oracle"] = {"fp64": err_vs(fg["d_xyz"], gr),
                                                                "mixed": err_vs(fgm["d_xyz"], gr)}
            except OSError:
                extras["fwd_grad_he128"]["errors_vs_oracle"] = None
        except hfk.HfkError as e:
            extras["fwd_grad_he128"] = {"error": str(e)}
        try:
            from he_inputs import mixed_lattice
            s5 = mixed_lattice((8, 8, 8), seed=13, tau=1e-10)
            log("512 H/He atoms, per-atom bases: fp64 and mixed")
            ws5 = hfk.new_workspace(hfk.workspace_bytes_atoms(s5.natoms, g, "fp64"), dev)
            a = time_builds(hfk, torch, s5, "fp64", 5, 1, ws5, atoms=True)
            b = time_builds(hfk, torch, s5, "mixed", 5, 1, ws5, atoms=True)
            qa = a["stats"]["quartets"]
            s6 = mixed_lattice((8, 4, 4), seed=14, tau=1e-10)
            ws6 = hfk.new_workspace(hfk.workspace_bytes_atoms(s6.natoms, g, "fp64"), dev)
            f6 = time_builds(hfk, torch, s6, "fp64", 10, 2, ws6, atoms=True)
            fg6 = time_grad(hfk, torch, s6, 10, 2)
            extras["atoms_hhe128_fwd_grad"] = {
                "quartets": f6["stats"]["quartets"], "fwd_ms": f6["ms_per_step"], "fwd_grad_ms": fg6["ms_per_step"],
                "fwd_grad_over_fwd_time": fg6["ms_per_step"] / f6["ms_per_step"],
            }
            extras["atoms_hhe512"] = {
                "quartets": qa,
                "fp64_ms": a["ms_per_step"], "fp64_kernel_ms": a["kernel_ms"],
                "fp64_quartets_per_s": qa / (a["ms_per_step"] / 1e3),
                "pct_fp64_valu_peak_nominal": 100.0 * qa * flop_per_quartet(g) / (a["kernel_ms"] / 1e3) / 1e12
                / FP64_VALU_PEAK_TFLOPS,
                "mixed_ms": b["ms_per_step"],
                "mixed_quartets_per_s": b["stats"]["quartets"] / (b["ms_per_step"] / 1e3),
                "mixed_speedup_vs_fp64": a["ms_per_step"] / b["ms_per_step"],
                "rel_err_F_mixed_vs_fp64": float(torch.linalg.norm(b["F"] - a["F"]) / torch.linalg.norm(a["F"])),
            }
            del ws5, a, b
            torch.cuda.empty_cache()
        except hfk.HfkError as e:
            extras["atoms_hhe512"] = {"error": str(e)}
        try:
            from he_inputs import mixed_lattice
            s7 = mixed_lattice((4, 4, 8), seed=17, tau=1e-12)
            Z7 = np.where(s7.exps[:, 0] < 5.0, 1.0, 2.0)
            nocc7 = int(Z7.sum()) // 2
            log("SCF, 128 H/He atoms (per-atom bases)")
            x7 = torch.tensor(s7.xyz, device=dev)
            ws7 = hfk.new_workspace(hfk.scf_workspace_bytes(s7.natoms, g, "fp64"), dev)
            hfk.scf(x7, Z7, s7.exps, s7.coefs, nocc7, s7.tau, max_iter=3, workspace=ws7)   # warm-up
            torch.cuda.synchronize()
            hfk.profile_read()
            hfk.profile_enable(True)
            t0 = time.time()
            r7 = hfk.scf(x7, Z7, s7.exps, s7.coefs, nocc7, s7.tau, workspace=ws7)
            torch.cuda.synchronize()
            wall7 = (time.time() - t0) * 1e3
            hfk.profile_enable(False)
            k7, _ = hfk.profile_read()
            extras["scf_hhe128"] = {
                "energy": r7["E"], "iterations": r7["iterations"], "converged": r7["converged"],
                "total_ms": wall7, "ms_per_iteration": wall7 / max(r7["iterations"], 1),
                "quartet_kernel_share": k7 / wall7,
            }
            del ws7, x7
        except hfk.HfkError as e:
            extras["scf_hhe128"] = {"error": str(e)}
        try:
            from he_inputs import cluster_batch
            log("2000-cluster batch: mixed + gradient, one launch")
            extras["batched_2000_mixed_grad"] = time_batched(hfk, torch, cluster_batch(), 5, 1)
        except hfk.HfkError as e:
            extras["batched_2000_mixed_grad"] = {"error": str(e)}
        out["extras"] = extras
    if not args.no_cpu:
        log("cpu oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
