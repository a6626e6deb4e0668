"""Benchmark: one non-local application step on one MI355X.

A step is the whole hot path over the benchmark workload with inputs resident
in HBM:  c = projection(psi)  then  out += expansion(c)  (the paper's prj and
add, sec. 3.2 steps 1 and 3; "prj+add" in sec. 6), through the library's
plan API.  Plans are built once (the per-geometry setup), outside the timed
region.

Workload: periodic 128^3 grid, h = 0.2 Bohr, 512 atoms (random sequential
placement, 2 Bohr minimum separation), sigma = 0.6 Bohr, nu_max = 5 (56
functions), 32 real FP64 bands psi ~ N(0,1) (synthetic, seeded).

Metric: projected gridpoint*bands per second = sum_a |S_a| * B per step / time.
The JSON line also carries the roofline of the dominant kernel (algorithmic
HBM bytes per launch / its mean event-timed duration vs 8 TB/s) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB elementwise copy kernel (reads 1 GiB, "
                         "writes 1 GiB) so that profiler byte counters can be scaled")
    return ap.parse_args()


def cpu_baseline(s, psi, c, target_s):
    """Oracle projection + expansion timed on a sample of atoms (all bands,
    the full grid), scaled to gridpoint*bands per second."""
    import oracle
    from paper_1905_00480_amd import workloads as wl
    off = wl.coeff_offsets(s)
    rng = np.random.default_rng(99)
    order = rng.permutation(s.natoms)

    def run(k):
        atoms = np.sort(order[:k])
        sub = s.subset(atoms)
        csub = np.concatenate([c[off[a]:off[a + 1]] for a in atoms])
        out = np.zeros_like(psi)
        t0 = time.perf_counter()
        oracle.project(*sub.geometry(), psi)
        oracle.expand(*sub.geometry(), csub, out)
        return time.perf_counter() - t0, atoms

    t, atoms = run(2)
    k = int(np.clip(2 * target_s / max(t, 1e-3), 2, s.natoms))
    t, atoms = run(k)
    pts = sum(len(oracle.support(s.n, s.h, s.periodic, s.pos[a],
                                 oracle.box_radius(s.sigma[a], s.numax[a], s.h))[1])
              for a in atoms)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": pts * s.nbands / t, "unit": "gridpoint*bands/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d of %d atoms (all %d bands, full grid), projection + expansion, "
                      "%.1f s" % (len(atoms), s.natoms, s.nbands, t)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); the path "
              "shards over bands or z-slabs as described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_00480_amd import binding as bd
    from paper_1905_00480_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    bd.load_library()
    dev = torch.device("cuda:0")
    s = wl.scale()
    psi_h = wl.psi_for(s)
    c_h = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    psi = torch.from_numpy(psi_h).to(dev)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device=dev)
    out = torch.zeros_like(psi)
    B = s.nbands
    S = plan.support_points
    units = S * B  # gridpoint*bands per step
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.project(psi, c)
        if ev is not None:
            ev[1].record(stream)
        plan.expand(c, out)
        if ev is not None:
            ev[2].record(stream)

    if args.copy_calib:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
           for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = t_start.elapsed_time(t_end)
    prj_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    add_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_per_step = total_ms / args.steps

    coeff_bytes = plan.coeff_doubles * 8
    prj_bytes = S * B * 8 + coeff_bytes          # psi box reads + c write
    add_bytes = 2 * S * B * 8 + coeff_bytes      # psi box read+write + c read
    prj_gbs = prj_bytes / (prj_ms * 1e-3) / 1e9
    add_gbs = add_bytes / (add_ms * 1e-3) / 1e9
    dom = ("expand", add_bytes, add_ms, add_gbs) if add_ms >= prj_ms else \
          ("project", prj_bytes, prj_ms, prj_gbs)

    rec = {
        "metric": "projected gridpoint*bands/s",
        "value": units / (ms_per_step * 1e-3),
        "unit": "gridpoint*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "scale: periodic 128^3, h=0.2 Bohr, 512 atoms (RSA 2 Bohr), "
                               "sigma=0.6, nu_max=5 (56 functions), 32 FP64 bands; "
                               "step = projection + expansion",
                   "global_batch": B, "support_points": S, "grid": list(s.n),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": dom[3],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom[3] / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_launch": dom[1],
                     "launch_ms": dom[2]},
        "kernels": {"project": {"ms": prj_ms, "GB/s": prj_gbs, "bytes": prj_bytes},
                    "expand": {"ms": add_ms, "GB/s": add_gbs, "bytes": add_bytes}},
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(s, psi_h, c_h, args.cpu_seconds)
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
