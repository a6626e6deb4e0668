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

Kernels of a step and their algorithmic HBM bytes per launch:
  project        box reads sum_a |S_a| B 8 + coefficient writes
  expand_z       coefficient reads + plane-partial writes (U2, z pass)
  expand_xy      read + write of every grid value some support covers
                 (2 * union points * B * 8) + plane-partial reads (y and x
                 passes; the blocks it moves also hold a few uncovered values)
The roofline object is the dominant (longest) kernel's bytes over its mean
duration, both measured in this run with HIP events that the library records
around its own launches on the launch stream, against 8 TB/s.  `traffic` is
the dominant kernel's HBM bytes per launch from rocprofv3 FETCH_SIZE /
WRITE_SIZE counters (profiles/traffic.json), reported only while the kernel
source is the one the counters were taken with.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
KERNEL_SRC = os.path.join(ROOT, "paper_1905_00480_amd", "csrc", "sho_kernels.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stored", action="store_true",
                    help="skip timing the stored-projector baseline")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the uneven-atom batching workload")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the request-stream (serving) workload")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper-geometry table (SHO vs stored, nu_max 0..5)")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the differentiation (forward + backward) workload")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the single-precision scale step")
    ap.add_argument("--no-per-atom", action="store_true",
                    help="batching workload: skip timing the per-atom launch reference")
    ap.add_argument("--no-bloch", action="store_true",
                    help="skip the complex Bloch-band scale step")
    ap.add_argument("--no-det", action="store_true",
                    help="skip the SHO_FLAG_DETERMINISTIC scale step")
    ap.add_argument("--by-cutoff", action="store_true",
                    help="only time the batching workload's projection on atom subsets "
                         "by cut-off, print one JSON line and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the plan's default schedule (no autotuning)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--digest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE) "
                         "into profiles/traffic.json and exit")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB elementwise copy kernel (reads 1 GiB, "
                         "writes 1 GiB) so that profiler byte counters can be scaled")
    return ap.parse_args()


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kind, workload="scale"):
    """HBM bytes per launch of kernel kind `kind` (project, expand_z,
    expand_xy) of `workload` from the committed counter runs, if they were
    taken with the current kernel source."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    rec = t.get("kinds", {}).get(workload, {}).get(kind)
    return rec.get("hbm_bytes_per_launch") if rec else None


# Kernel kinds of the counter runs: (workload, kind) -> regexes of the
# kernels that make up one launch of the kind; the first names the main
# kernel, whose dispatch count is the number of launches.
COUNTER_KINDS = {
    "scale": {"project": [r"k_project(_any|_blocks)?<5\b", r"k_zpass<5>"],
              "expand_z": [r"k_u2<5>"],
              "expand_xy": [r"k_expand_blocks<5, false>"]},
    "batching": {"project": [r"k_project(_any|_blocks)?<9\b", r"k_zpass<[0-9]>"],
                 "expand_z": [r"k_u2<9>", r"k_u2<[0-8]>"],
                 "expand_xy": [r"k_expand_blocks<9, false>"]},
}


def digest_counters(fetch_csv, write_csv, out=TRAFFIC):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of `bench.py --copy-calib`: each counter is
    scaled by what it reads for the plain 1 GiB elementwise copy kernel
    (reads 1 GiB, writes 1 GiB) of the same run.  Dispatches from the first
    kernel of cut-off 9 on belong to the batching workload (which runs after
    the scale step).  Writes `out`."""
    import csv
    import re

    def per_kernel(path, counter):
        rows = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"],
                                 float(r["Counter_Value"]) * 1024.0))
        first9 = min([d for d, k, _ in rows if re.search(r"k_(project\w*|expand_blocks)<9", k)]
                     or [1 << 62])
        tot, cnt = {}, {}
        for d, k, v in rows:
            key = ("batching" if d >= first9 else "scale", k.split("(")[0])
            tot[key] = tot.get(key, 0.0) + v
            cnt[key] = cnt.get(key, 0) + 1
        return tot, cnt

    ft, fc = per_kernel(fetch_csv, "FETCH_SIZE")
    wt, wc = per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in ft if "elementwise_kernel" in k[1] and "AUnaryFunctor" in k[1]]
    if not copy:
        raise SystemExit("no copy-calibration kernel in the counter runs (--copy-calib)")
    gib = float(1 << 30)
    fscale = gib / (ft[copy[0]] / fc[copy[0]])
    wscale = gib / (wt[copy[0]] / wc[copy[0]])
    kernels = {}
    for (ph, k) in ft:
        if "sho::" not in k:
            continue
        fb = ft[(ph, k)] / fc[(ph, k)] * fscale
        wb = wt.get((ph, k), 0.0) / max(wc.get((ph, k), 1), 1) * wscale
        kernels.setdefault(ph, {})[k] = {"dispatches": fc[(ph, k)], "fetch_bytes": fb,
                                        "write_bytes": wb, "hbm_bytes_per_launch": fb + wb}
    kinds = {}
    for wname, ks in COUNTER_KINDS.items():
        kk = kernels.get(wname, {})
        for kind, pats in ks.items():
            main = [k for k in kk if re.search(pats[0], k)]
            if not main:
                continue
            n = sum(kk[k]["dispatches"] for k in main)
            names = [k for k in kk if any(re.search(p, k) for p in pats)]
            fb = sum(kk[k]["fetch_bytes"] * kk[k]["dispatches"] for k in names) / n
            wb = sum(kk[k]["write_bytes"] * kk[k]["dispatches"] for k in names) / n
            kinds.setdefault(wname, {})[kind] = {"kernels": sorted(names), "launches": n,
                                                 "fetch_bytes": fb, "write_bytes": wb,
                                                 "hbm_bytes_per_launch": fb + wb}
    rec = {"workload": "scale and batching steps of bench.py (default schedules, --no-tune)",
           "kernel_source_sha": kernel_source_sha(), "fetch_scale": fscale,
           "write_scale": wscale, "kinds": kinds, "kernels": kernels}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def cpu_baseline(s, psi, c, target_s):
    """CPU reference points on the host cores of this machine:
    * the oracle (plain triple sums, long double) timed on a sample of atoms
      (all bands, the full grid), scaled to gridpoint*bands per second;
    * the factorised CPU path (x, y, z passes, double, OpenMP), the whole
      step on the whole workload, median of 3 runs."""
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

    k = 16
    t, atoms = run(k)
    while t < target_s / 3 and k < s.natoms:
        k = int(min(s.natoms, max(2 * k, k * target_s / max(t, 1e-3) * 0.9)))
        t, atoms = run(k)
    pts = sum(len(oracle.support(s.n, s.h, s.periodic, s.pos[a],
                                 oracle.box_radius(s.sigma[a], s.numax[a], s.h))[1])
              for a in atoms)
    threads = oracle.threads()
    rec = {"value": pts * s.nbands / t, "unit": "gridpoint*bands/s", "cores": threads,
           "kind": "oracle",
           "sample": "%d of %d atoms (all %d bands, full grid), projection + expansion, "
                     "%.1f s" % (len(atoms), s.natoms, s.nbands, t)}
    all_pts = sum(len(oracle.support(s.n, s.h, s.periodic, s.pos[a],
                                     oracle.box_radius(s.sigma[a], s.numax[a], s.h))[1])
                  for a in range(s.natoms))
    out = np.zeros_like(psi)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.factorised_project(*s.geometry(), psi)
        oracle.factorised_expand(*s.geometry(), c, out)
        times.append(time.perf_counter() - t0)
    tf = float(np.median(times))
    rec["factorised"] = {"value": all_pts * s.nbands / tf, "unit": "gridpoint*bands/s",
                         "cores": threads, "s_per_step": tf,
                         "sample": "the whole step (all %d atoms, %d bands), median of 3"
                                   % (s.natoms, s.nbands),
                         "nproc": os.cpu_count(),
                         "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    return rec


def _best_stored_form(plan, c, out, reps=3):
    """Stored plans have two expansion forms (block form with matrix-core
    products, atom-owner form with global atomics); the faster one for this
    plan is kept, so that the baseline is measured at its best."""
    import torch
    best = None
    for form in (1, 0):
        plan.set_expand(form)
        plan.expand(c, out)
        torch.cuda.synchronize()
        plan.profile(True)
        for _ in range(reps):
            plan.expand(c, out)
        torch.cuda.synchronize()
        ms = plan.profile_read()["expand_xy"][1]
        plan.profile(False)
        if best is None or ms < best[1]:
            best = (form, ms)
    plan.set_expand(best[0])
    return best


def stored_baseline(bd, s, psi, c, out, args):
    """The same step with the projector values sampled once into HBM and read
    back (SHO_FLAG_STORED), timed like the main step."""
    import torch
    plan = bd.Plan.from_system(s, flags=bd.FLAG_STORED)
    form = _best_stored_form(plan, c, out)

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    ms, _ = _time_steps(step, args.steps, args.warmup)
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.close()
    S = plan.support_points
    return {"value": S * s.nbands / (ms * 1e-3), "unit": "gridpoint*bands/s",
            "ms_per_step": ms, "stored_bytes": plan.info["stored_bytes"],
            "expand_form": form[0],
            "project_ms": prof["project"][1], "expand_ms": prof["expand_xy"][1]}


def _log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def _time_steps(step, steps, warmup):
    """Mean ms per step over `steps` back-to-back steps after `warmup`, and the
    per-step distribution (events between steps)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return ev[0].elapsed_time(ev[-1]) / steps, per


def _paper_protocol(step, runs=15, reps=10):
    """The paper's timing protocol (sec. 6): one warm-up, then `runs` runs of
    `reps` back-to-back steps each; median and p10/p90 of the per-step time
    of the runs."""
    import torch
    step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    per_run = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        per_run.append(e0.elapsed_time(e1) / reps)
    return {"runs": runs, "reps": reps,
            "ms_per_step_median": float(np.median(per_run)),
            "ms_per_step_p10_p90": [float(np.percentile(per_run, q)) for q in (10, 90)]}


def ceilings():
    """In-run memory ceilings: a plain 1 GiB copy (read + write) and a 1 GiB
    read (sum), timed with events, as achieved GB/s."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 2 << 30),
                             ("read", lambda: x.sum(), 1 << 30)):
        ms, _ = _time_steps(fn, 10, 2)
        out[name + "_GB/s"] = nbytes / (ms * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return out


def apply_step(bd, wl, plan, s, psi, args):
    """The whole non-local application on the scale workload: project, the
    per-atom product with random atomic matrices (FP64 matrix cores), expand;
    once through the API calls and once as a captured graph."""
    import torch
    off = plan.matrix_offsets()
    D = torch.from_numpy(np.random.default_rng(11).standard_normal(int(off[-1]))).cuda()
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    d = torch.empty_like(c)
    out = torch.zeros_like(psi)
    ms, _ = _time_steps(lambda: plan.apply(psi, D, out, c, d), args.steps, args.warmup)
    g = plan.apply_graph(psi, D, c, d, out)
    ms_graph, _ = _time_steps(g.launch, args.steps, args.warmup)
    g.close()
    # the product alone
    ms_mul, _ = _time_steps(lambda: plan.multiply(D, c, d), args.steps, args.warmup)
    nsho = (s.numax + 1) * (s.numax + 2) * (s.numax + 3) // 6
    flops = float(np.sum(2.0 * nsho.astype(np.float64) ** 2 * s.nbands))
    return {"ms_per_step": ms, "graph_ms_per_step": ms_graph, "multiply_ms": ms_mul,
            "multiply_TFLOP/s": flops / (ms_mul * 1e-3) / 1e12,
            "value": plan.support_points * s.nbands / (ms * 1e-3)}


def fp32_step(bd, wl, args, ms_fp64):
    """The scale workload with single-precision bands (SHO_FLAG_FP32, the
    paper's float kernels): the same 32 bands, tuned, step = projection +
    expansion; per-kernel times and the expansion's achieved bandwidth."""
    import torch
    s = wl.scale()
    psi = torch.from_numpy(wl.psi_for(s, dtype=np.float32)).cuda()
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float32, device="cuda")
    out = torch.zeros_like(psi)
    tune = None if args.no_tune else plan.tune(psi, c, reps=3)

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    ms, _ = _time_steps(step, args.steps, args.warmup)
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    info = plan.info
    B = s.nbands
    xy_bytes = 2 * info["union_points"] * B * 4 + info["expand_scratch_doubles"] * 8
    xy_ms = prof["expand_xy"][1]
    units = plan.support_points * B
    plan.close()
    return {"workload": "scale: periodic 128^3, h=0.2 Bohr, 512 atoms, sigma=0.6, nu_max=5, "
                        "32 FP32 bands; step = projection + expansion",
            "dtype": "f32", "ms_per_step": ms, "gridpoint*bands/s": units / (ms * 1e-3),
            "speedup_vs_fp64": ms_fp64 / ms, "tune": tune,
            "kernel_ms": {k: round(v[1], 4) for k, v in prof.items() if v[0]},
            "expand_xy_GB/s": xy_bytes / (xy_ms * 1e-3) / 1e9 if xy_ms > 0 else None}


def bloch_step(bd, wl, args, ms_fp64):
    """The scale workload with 32 complex Bloch bands at k = (0.31, -0.17,
    0.52) Bohr^-1 (SHO_FLAG_BLOCH, sec. 2.5: every periodic image carries its
    phase), FP64, tuned; step = projection + expansion.  Twice the bytes of
    the 32 real bands of the headline step."""
    import torch
    s = wl.scale()
    rng = np.random.default_rng(21)
    psi_h = rng.standard_normal(s.psi_shape + (2,))
    psi = torch.view_as_complex(torch.from_numpy(psi_h).cuda())
    plan = bd.Plan.from_system(s, flags=bd.FLAG_BLOCH)
    plan.set_kpoint((0.31, -0.17, 0.52))
    c = torch.empty(plan.coeff_doubles // 2, dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(psi)
    tune = None if args.no_tune else plan.tune(psi, c, reps=3)

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    ms, _ = _time_steps(step, args.steps, args.warmup)
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    S = plan.support_points
    prj_ms = prof["project"][1]
    units = S * s.nbands
    plan.close()
    return {"workload": "scale: periodic 128^3, h=0.2 Bohr, 512 atoms, sigma=0.6, nu_max=5, "
                        "32 complex FP64 bands at k = (0.31, -0.17, 0.52) Bohr^-1; "
                        "step = projection + expansion",
            "dtype": "c128", "ms_per_step": ms,
            "gridpoint*complex_bands/s": units / (ms * 1e-3),
            "ms_vs_real_32_bands": ms / ms_fp64, "tune": tune,
            "kernel_ms": {k: round(v[1], 4) for k, v in prof.items() if v[0]},
            "project_per_atom_GB/s": S * s.nbands * 16 / (prj_ms * 1e-3) / 1e9
            if prj_ms > 0 else None}


def deterministic_step(bd, wl, args, ms_default):
    """The scale workload with SHO_FLAG_DETERMINISTIC (every sum in an order
    fixed by the plan: per-wave coefficient tiles added in wave order, one
    work item per atom, the owner form of the expansion); step = projection
    + expansion, FP64, default schedule.  Also checks that two steps on the
    same inputs give identical bits."""
    import torch
    s = wl.scale()
    psi = torch.from_numpy(wl.psi_for(s)).cuda()
    plan = bd.Plan.from_system(s, flags=bd.FLAG_DETERMINISTIC)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(psi)

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    ms, _ = _time_steps(step, args.steps, args.warmup)
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    out.zero_()
    step()
    c1, o1 = c.clone(), out.clone()
    out.zero_()
    step()
    torch.cuda.synchronize()
    same = bool(torch.equal(c1.view(torch.int64), c.view(torch.int64)) and
                torch.equal(o1.view(torch.int64), out.view(torch.int64)))
    plan.close()
    return {"workload": "scale: periodic 128^3, h=0.2 Bohr, 512 atoms, sigma=0.6, nu_max=5, "
                        "32 FP64 bands, SHO_FLAG_DETERMINISTIC; step = projection + expansion",
            "ms_per_step": ms, "ms_vs_default": ms / ms_default,
            "kernel_ms": {k: round(v[1], 4) for k, v in prof.items() if v[0]},
            "bitwise_repeat": same}


def by_cutoff(bd, wl, reps=10):
    """The batching workload's projection on subsets of its atoms by cut-off
    (each subset a plan of its own over the same psi, default schedule,
    64-band tiles): mean ms per launch over `reps` launches and the per-atom
    box bytes per second.  Shows which cut-offs stream below the rest."""
    import torch
    s = wl.batching()
    psi = torch.from_numpy(wl.psi_for(s)).cuda()
    nus = np.asarray(s.numax)
    rows = []
    subsets = [("3-9", None), ("3-6", (3, 6)), ("7-9", (7, 9))] + \
        [(str(n), (n, n)) for n in range(3, 10)]
    for name, rng in subsets:
        sub = s if rng is None else s.subset(np.nonzero((nus >= rng[0]) & (nus <= rng[1]))[0])
        plan = bd.Plan.from_system(sub)
        sched = plan.schedule()
        plan.set_schedule(sched[0], 64, sched[2])
        c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
        for _ in range(3):
            plan.project(psi, c)
        torch.cuda.synchronize()
        plan.profile(True)
        for _ in range(reps):
            plan.project(psi, c)
        torch.cuda.synchronize()
        ms = plan.profile_read()["project"][1]
        plan.profile(False)
        gbytes = plan.support_points * s.nbands * 8 / 1e9
        rows.append({"nu": name, "atoms": int(sub.natoms), "schedule": list(plan.schedule()),
                     "support_points": int(plan.support_points), "project_ms": round(ms, 4),
                     "per_atom_box_TB/s": round(gbytes / ms, 3)})
        _log("cut-offs %s: %.3f ms" % (name, ms))
        plan.close()
        del c
    return {"workload": "batching: periodic 160^3, h=0.18 Bohr, 2048 atoms, nu_max 3..9, "
                        "64 FP64 bands; projection of atom subsets by cut-off", "rows": rows}


def setup_step(bd):
    """Host-side set-up of the basis (once per SCF cycle, sec. 3.5): the
    atomic matrix of 18 synthetic radial projectors (two each for s, p, d) in
    the Cartesian SHO basis, on a 2001-point radial quadrature."""
    r = np.linspace(0.0, 10.0, 2001)
    w = np.full(r.size, r[1] - r[0])
    w[1:-1:2] *= 4.0 / 3.0
    w[2:-1:2] *= 2.0 / 3.0
    w[[0, -1]] /= 3.0
    ell = [0, 0, 1, 1, 2, 2]
    P = np.array([r ** l * (1.0 + 0.3 * k * r) * np.exp(-r * r / 1.2)
                  for k, l in enumerate(ell)])
    D = np.eye(18)
    out = {}
    bd.setup_matrix(4, 0.6, ell, r, w, P, D)  # warm-up (library load)
    for nu_max in (4, 5, 10):
        t0 = time.perf_counter()
        reps = 0
        while True:
            bd.setup_matrix(nu_max, 0.6, ell, r, w, P, D)
            reps += 1
            if time.perf_counter() - t0 > 0.2:
                break
        out["nu_max=%d ms" % nu_max] = (time.perf_counter() - t0) / reps * 1e3
    return {"workload": "18 radial projectors (s, p, d x 2), 2001-point radial grid, "
                        "script-D = U^T F^T D F U on the host", **out}


def diff_step(bd, wl, args):
    """Differentiation workload (isolated 96^3, 256 atoms, nu 6, 16 bands):
    forward projection and the backward pair (expansion of h^3 dL/dc for
    dL/dpsi, derivative kernel for dL/dR), as the autograd wrapper runs them."""
    import torch
    s = wl.diff()
    psi = torch.from_numpy(wl.psi_for(s)).cuda()
    w = torch.from_numpy(wl.coeffs_for(s)).cuda()
    plan = bd.Plan.from_system(s)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    gpsi = torch.zeros_like(psi)
    grad = torch.empty((s.natoms, 3), dtype=torch.float64, device="cuda")
    # plan set-up, untimed: the schedule tuner (its work items serve the
    # projection and the derivative kernel)
    tune = None if args.no_tune else plan.tune(psi, c, reps=3)

    def step():
        plan.project(psi, c)
        gpsi.zero_()
        plan.expand(w, gpsi, alpha=s.h ** 3)
        plan.force(psi, w, grad)

    ms, _ = _time_steps(step, args.steps, args.warmup)
    plan.profile(True)
    step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    units = plan.support_points * s.nbands
    plan.close()
    return {"workload": "diff: isolated 96^3, h=0.2 Bohr, 256 atoms, sigma=0.6, nu_max=6, "
                        "16 FP64 bands; step = forward projection + backward (expansion "
                        "of h^3 dL/dc, derivative kernel at nu+1)",
            "ms_per_step": ms, "gridpoint*bands/s (forward units)": units / (ms * 1e-3),
            "tune": tune,
            "kernel_ms": {k: round(v[1], 4) for k, v in prof.items() if v[0]}}


def paper_table(bd, wl, args):
    """The paper's benchmark geometry (sec. 6: fcc, 64^3 at h = 0.25 A, 650
    atoms whose 3.55 A spheres reach the grid, 1024 bands) for nu_max 0..5,
    projection (prj) and expansion (add), with functions generated on the fly
    (SHO) and read from stored tables (USU), as in the paper's table 1."""
    import torch
    s5 = wl.paper_fcc(numax=5)
    psi = torch.from_numpy(wl.psi_for(s5)).cuda()
    out = torch.zeros_like(psi)
    rows = []
    for nu in range(6):
        s = wl.paper_fcc(numax=nu)
        row = {"nu_max": nu, "functions": (nu + 1) * (nu + 2) * (nu + 3) // 6}
        for tag, flags in (("SHO", 0), ("USU", bd.FLAG_STORED)):
            plan = bd.Plan.from_system(s, flags=flags)
            c = torch.zeros(plan.coeff_doubles, dtype=torch.float64, device="cuda")
            plan.project(psi, c)
            if flags:
                row["USU_expand_form"] = _best_stored_form(plan, c, out, reps=2)[0]
            plan.expand(c, out)
            torch.cuda.synchronize()
            plan.profile(True)
            for _ in range(3):
                plan.project(psi, c)
            for _ in range(3):
                plan.expand(c, out)
            torch.cuda.synchronize()
            prof = plan.profile_read()
            plan.profile(False)
            row[tag + "prj_ms"] = prof["project"][1]
            row[tag + "add_ms"] = prof["expand_z"][1] + prof["expand_xy"][1]
            row["support_points"] = plan.support_points
            plan.close()
            del c
        row["S_prj"] = row["USUprj_ms"] / row["SHOprj_ms"]
        row["S_add"] = row["USUadd_ms"] / row["SHOadd_ms"]
        rows.append(row)
        _log("paper geometry nu_max %d: SHO prj %.2f add %.2f ms, USU prj %.2f add %.2f ms"
             % (nu, row["SHOprj_ms"], row["SHOadd_ms"], row["USUprj_ms"], row["USUadd_ms"]))
    # table 2 of the paper: 18 stored numerical projectors (two radial
    # functions each for s, p, d) against the 35 SHO functions of nu_max = 4
    # that span them, on the same spheres
    s = wl.paper_fcc(numax=0)
    rc = float(s.rbox[0])
    ell, dr, tab = wl.radial_set(rc)
    plan = bd.Plan.radial(s.n, s.h, s.periodic, s.pos, np.full(s.natoms, rc), ell, dr, tab,
                          s.nbands)
    c = torch.zeros(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    plan.project(psi, c)
    form = _best_stored_form(plan, c, out, reps=2)[0]
    plan.expand(c, out)
    torch.cuda.synchronize()
    plan.profile(True)
    for _ in range(3):
        plan.project(psi, c)
    for _ in range(3):
        plan.expand(c, out)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    usu = {"projectors": int(plan.coeff_doubles // (s.natoms * s.nbands)),
           "prj_ms": prof["project"][1],
           "add_ms": prof["expand_z"][1] + prof["expand_xy"][1],
           "expand_form": form, "stored_bytes": plan.info["device_bytes"]}
    plan.close()
    del c
    sho35 = rows[4]
    table2 = {"USU18_prj_ms": usu["prj_ms"], "USU18_add_ms": usu["add_ms"],
              "SHO35_prj_ms": sho35["SHOprj_ms"], "SHO35_add_ms": sho35["SHOadd_ms"],
              "S_prj": usu["prj_ms"] / sho35["SHOprj_ms"],
              "S_add": usu["add_ms"] / sho35["SHOadd_ms"],
              "S_both": (usu["prj_ms"] + usu["add_ms"]) /
                        (sho35["SHOprj_ms"] + sho35["SHOadd_ms"]),
              "USU18": usu,
              "paper_double_P100_V100": {"prj": [2.2, 1.4], "add": [3.1, 2.5],
                                         "both": [2.6, 2.0]}}
    _log("paper geometry USU18 vs SHO35: prj %.2f / %.2f ms, add %.2f / %.2f ms"
         % (usu["prj_ms"], sho35["SHOprj_ms"], usu["add_ms"], sho35["SHOadd_ms"]))
    del psi, out
    torch.cuda.empty_cache()
    return {"workload": "fcc a=4.08 A, isolated 64^3 at h=0.25 A, 650 atoms with 3.55 A "
                        "projection spheres (11 projections per grid value), sigma=1.6 Bohr, "
                        "1024 FP64 bands; times per kernel call",
            "rows": rows, "table2_usu18_vs_sho35": table2}


def batching(bd, wl, args):
    """Uneven atoms (periodic 160^3, h = 0.18, 2048 atoms, nu 3..9, sigma
    0.4..1.2, 64 bands): the batched single launch (default, then tuned), its
    captured graph, and the per-atom launch schedule it must beat."""
    import torch
    dev = torch.device("cuda:0")
    s = wl.batching()
    psi = torch.from_numpy(wl.psi_for(s)).to(dev)
    out = torch.zeros_like(psi)
    plan = bd.Plan.from_system(s)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device=dev)
    units = plan.support_points * s.nbands
    steps = max(3, args.steps // 4)
    res = {"workload": "batching: periodic 160^3, h=0.18 Bohr, 2048 atoms uniform, "
                       "nu_max 3..9, sigma 0.4..1.2 Bohr, 64 FP64 bands; step = "
                       "projection + expansion",
           "support_points": plan.support_points, "union_points": plan.info["union_points"],
           "steps": steps}

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    ms, _ = _time_steps(step, steps, 1)
    res["default"] = {"schedule": plan.schedule(), "ms_per_step": ms,
                      "value": units / (ms * 1e-3)}
    tune = None if args.no_tune else plan.tune(psi, c, reps=2)
    ms, per = _time_steps(step, steps, 1)
    plan.profile(True)
    step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    res["tuned"] = {"schedule": plan.schedule(), "tune": tune, "ms_per_step": ms,
                    "value": units / (ms * 1e-3),
                    "project_ms": prof["project"][1],
                    "expand_z_ms": prof["expand_z"][1],
                    "expand_xy_ms": prof["expand_xy"][1],
                    "project_per_atom_box_GB/s":
                        (units * 8 + plan.coeff_doubles * 8) / (prof["project"][1] * 1e-3) / 1e9,
                    "hbm_bytes_counters": {k: measured_traffic(k, "batching")
                                           for k in ("project", "expand_z", "expand_xy")}}
    g = plan.graph(psi, c, out)
    ms, _ = _time_steps(g.launch, steps, 1)
    res["graph"] = {"ms_per_step": ms, "value": units / (ms * 1e-3)}
    g.close()
    plan.close()
    if args.no_per_atom:
        del psi, out, c
        torch.cuda.empty_cache()
        return res
    ref = bd.Plan.from_system(s, flags=bd.FLAG_PER_ATOM)

    def ref_step():
        ref.project(psi, c)
        ref.expand(c, out)

    _log("batching: batched %.2f ms, graph %.2f ms per step; timing per-atom launches"
         % (res["tuned"]["ms_per_step"], res["graph"]["ms_per_step"]))
    ms, _ = _time_steps(ref_step, max(2, steps // 2), 1)
    ref.close()
    res["per_atom_launches"] = {"ms_per_step": ms, "value": units / (ms * 1e-3),
                                "launches_per_step": 2 * s.natoms}
    res["speedup_vs_per_atom"] = res["per_atom_launches"]["ms_per_step"] / min(
        res["tuned"]["ms_per_step"], res["graph"]["ms_per_step"])
    del psi, out, c
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.digest_counters:
        rec = digest_counters(*args.digest_counters)
        print(json.dumps(rec["kinds"], indent=1))
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (--gpus 1); sharding the "
              "path over bands or z-slabs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_00480_amd import binding as bd
    from paper_1905_00480_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    bd.load_library()
    if args.by_cutoff:
        print(json.dumps(by_cutoff(bd, wl)))
        return
    dev = torch.device("cuda:0")
    s = wl.scale()
    psi_h = wl.psi_for(s)
    c_h = wl.coeffs_for(s)
    t0 = time.perf_counter()
    plan = bd.Plan.from_system(s)
    plan_s = time.perf_counter() - t0
    psi = torch.from_numpy(psi_h).to(dev)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device=dev)
    out = torch.zeros_like(psi)
    B = s.nbands
    info = plan.info
    S = info["support_points"]
    units = S * B  # gridpoint*bands per step
    stream = torch.cuda.current_stream()

    def step():
        plan.project(psi, c)
        plan.expand(c, out)

    if args.copy_calib:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    # plan set-up: the autotuner picks the projection schedule (untimed)
    tune = None if args.no_tune else plan.tune(psi, c, reps=3)
    # timed region: exactly `steps` steps, events between the steps
    w0 = time.perf_counter()
    ms_per_step, per_step = _time_steps(step, args.steps, args.warmup)
    wall = time.perf_counter() - w0

    # per-kernel durations: a second pass with the library's launch events
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)

    coeff_bytes = plan.coeff_doubles * 8
    u2_bytes = info["expand_scratch_doubles"] * 8
    # per-atom box accounting (every atom's support counted once per atom,
    # as the paper counts each grid value once per projection it enters)
    kbytes = {
        "project": S * B * 8 + coeff_bytes,
        "expand_z": coeff_bytes + u2_bytes,
        "expand_xy": 2 * S * B * 8 + u2_bytes,
    }
    kernels = {}
    for k, nbytes in kbytes.items():
        n, ms = prof[k]
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
        hbm = measured_traffic(k)
        kernels[k] = {"launches": n, "ms": ms, "bytes_per_atom_accounting": nbytes,
                      "GB/s": gbs, "frac_per_atom": gbs / HBM_PEAK_GBS if gbs else None,
                      "hbm_bytes_counters": hbm,
                      "frac_counters": (hbm / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                        if hbm and ms > 0 else None)}
    # the expansion writes each covered value once: its unique bytes
    kernels["expand_xy"]["bytes_unique_points"] = (2 * info["union_points"] * B * 8
                                                   + u2_bytes)
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    d = kernels["project"]
    ceil = ceilings()
    # unique-psi floor of the step: every covered value read once by the
    # projection and read + written once by the expansion, or the x-pass flops
    union_bytes = info["union_points"] * B * 8
    xflops = 2 * 6 * S * B * 2  # x passes of projection and expansion, nu = 5
    floor_ms = max(3 * union_bytes / (HBM_PEAK_GBS * 1e9), xflops / 78.6e12) * 1e3
    protocol = _paper_protocol(step)
    # the same step replayed as one captured graph (sho_graph_create), for
    # comparison: the headline stays the plain calls
    g = plan.graph(psi, c, out)
    ms_graph, _ = _time_steps(g.launch, args.steps, args.warmup)
    g.close()

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
                   "bands": B, "support_points": S,
                   "union_points": info["union_points"], "grid": list(s.n)},
        "roofline": {"bound": "hbm", "kernel": "project", "achieved": d["GB/s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": d["frac_per_atom"], "traffic": d["hbm_bytes_counters"],
                     "frac_counters": d["frac_counters"],
                     "algorithmic_bytes_per_launch": d["bytes_per_atom_accounting"],
                     "launch_ms": d["ms"],
                     "frac_of_read_ceiling": d["GB/s"] / ceil["read_GB/s"],
                     "dominant_kernel": dom,
                     "dominant_frac_per_atom": kernels[dom]["frac_per_atom"]},
        "ceilings": ceil,
        "unique_psi_floor_ms_per_step": floor_ms,
        "kernels": kernels,
        "per_atom_box_GB/s": 3 * S * B * 8 / (ms_per_step * 1e-3) / 1e9,
        "plan_build_s": plan_s,
        "tune": tune,
        "schedule": plan.schedule(),
        "wall_s_incl_warmup": wall,
        "step_ms_p10_p50_p90": [float(np.percentile(per_step, q)) for q in (10, 50, 90)],
        "paper_protocol": protocol,
        "graph_ms_per_step": ms_graph,
    }
    _log("scale workload: %.3f ms per step" % ms_per_step)
    rec["apply"] = apply_step(bd, wl, plan, s, psi, args)
    _log("non-local application: %.3f ms per step" % rec["apply"]["ms_per_step"])
    rec["setup"] = setup_step(bd)
    if not args.no_fp32:
        rec["fp32"] = fp32_step(bd, wl, args, ms_per_step)
        _log("fp32 scale step: %.3f ms" % rec["fp32"]["ms_per_step"])
    if not args.no_det:
        rec["deterministic"] = deterministic_step(bd, wl, args, ms_per_step)
        _log("deterministic scale step: %.3f ms" % rec["deterministic"]["ms_per_step"])
    if not args.no_bloch:
        rec["bloch"] = bloch_step(bd, wl, args, ms_per_step)
        _log("bloch scale step: %.3f ms" % rec["bloch"]["ms_per_step"])
    if not args.no_stored:
        rec["stored_baseline"] = stored_baseline(bd, s, psi, c, out, args)
    if not args.no_stored:
        _log("stored baseline: %.3f ms per step" % rec["stored_baseline"]["ms_per_step"])
    if not args.no_diff:
        rec["diff"] = diff_step(bd, wl, args)
        _log("diff workload: %.3f ms per step" % rec["diff"]["ms_per_step"])
    if not args.no_paper:
        rec["paper_geometry"] = paper_table(bd, wl, args)
    if not args.no_batching:
        rec["batching"] = batching(bd, wl, args)
        _log("batching workload done")
    if not args.no_serving:
        from paper_1905_00480_amd import serve
        rec["serving"] = serve.compare(requests=args.serve_requests, warmup=args.serve_warmup)
        _log("serving workload done")
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle")
        rec["cpu_baseline"] = cpu_baseline(s, psi_h, c_h, args.cpu_seconds)
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
