"""Request-stream driver of the library's server (sho_server_*).

A pool of systems is registered once; requests (project, expand or force on
one system of the pool) arrive as a Poisson stream and are submitted at their
arrival times.  The server keeps systems resident under an HBM byte budget
(least recently used ones are evicted), runs the requests of one system in
order on one stream and overlaps different systems over several streams.
Latency of a request = completion (taken by the server when the request's
event fires) - arrival.  The per-request reference is the same server with
one stream (FIFO) and per-atom launches (SHO_FLAG_PER_ATOM).

Inputs are synthetic: psi and the expansion / derivative weights w are a
seeded block of 2^20 standard normal values tiled over each buffer.
"""
import sys
import time

import numpy as np

from . import binding as bd
from . import workloads as wl

BLOCK = 1 << 20


def _log(msg):
    print("serve: " + msg, file=sys.stderr, flush=True)


def _tile_fill(dst, seed):
    block = np.random.default_rng(seed).standard_normal(BLOCK)
    n = dst.shape[0]
    k = n // BLOCK
    if k:
        dst[:k * BLOCK].reshape(k, BLOCK)[:] = block
    dst[k * BLOCK:] = block[:n - k * BLOCK]


def register(server, pool, seed=4):
    """Add every system of the pool and fill its inputs in place."""
    sids = []
    for k, s in enumerate(pool):
        sid = server.add(s)
        psi, w = server.inputs(sid)
        if psi is not None:
            _tile_fill(psi, seed * 7919 + 2 * k)
            _tile_fill(w, seed * 7919 + 2 * k + 1)
        sids.append(sid)
        if (k + 1) % 8 == 0:
            _log("%d of %d systems registered" % (k + 1, len(pool)))
    return sids


def units_of(pool):
    """sum_a |S_a| * B of every system (gridpoint*bands of one request)."""
    out = []
    for s in pool:
        p = bd.Plan(s.n, s.h, s.periodic, s.pos, s.sigma, s.numax, s.nbands,
                    flags=bd.FLAG_HOST_ONLY)
        out.append(p.support_points * s.nbands)
        p.close()
    return np.array(out, dtype=np.float64)


def alone_ms(server, sids, which, reps=3):
    """Latency (ms) of each job of the systems `which` on an otherwise idle
    device, one request at a time: the least time a request to them can
    take in the stream (median of reps)."""
    out = {}
    for k in which:
        row = []
        for job in (0, 1, 2):
            t = []
            for _ in range(reps):
                rid = server.submit(sids[k], job)
                server.drain()
                _, _, t_sub, t_done = server.request_info(rid)
                t.append(1e3 * (t_done - t_sub))
            row.append(float(np.median(t)))
        out[int(k)] = row
    return out


def run(server, sids, units, rate_hz=200.0, warmup=200, requests=2000, seed=4,
        preload=True, alone_largest=False):
    """Submit a Poisson stream (warm-up requests first, not measured) and
    return throughput and latency percentiles of the measured requests.  With
    preload, every system that fits the budget is made resident first (as a
    service loads its systems before it takes requests)."""
    count = warmup + requests
    if preload:
        t0 = time.perf_counter()
        for sid in sids:
            try:
                server.prefetch(sid)
            except bd.ShoError as e:
                if e.code != bd.SHO_E_BUDGET:
                    raise
        _log("preloaded %d systems in %.1f s" % (len(sids), time.perf_counter() - t0))
    arrivals, kinds, rng = wl.poisson_arrivals(rate_hz, count, seed)
    which = rng.integers(0, len(sids), size=count)
    base_srv = server.clock()
    base = time.perf_counter()
    rids = []
    for i in range(count):
        target = base + arrivals[i]
        while True:
            d = target - time.perf_counter()
            if d <= 0:
                break
            time.sleep(d if d > 2e-3 else 0)
        rids.append(server.submit(sids[which[i]], int(kinds[i])))
        if (i + 1) % 500 == 0:
            _log("%d of %d requests submitted (%.1f s behind schedule)"
                 % (i + 1, count, time.perf_counter() - target))
    server.drain()
    lat, done, jobs = [], [], []
    for i in range(warmup, count):
        _, job, _, t_done = server.request_info(rids[i])
        lat.append(t_done - (base_srv + arrivals[i]))
        done.append(t_done)
        jobs.append(job)
    lat = np.array(lat)
    span = max(done) - (base_srv + arrivals[warmup])
    # where the tail comes from: requests to the three largest systems (by
    # support points x bands) against the rest
    big = set(np.argsort(units)[::-1][:3].tolist())
    sel = np.array([int(which[i]) in big for i in range(warmup, count)])
    work = float(units[which[warmup:]].sum())
    st = server.stats()
    alone = alone_ms(server, sids, sorted(big)) if alone_largest else None
    return {"requests": requests, "warmup": warmup, "rate_hz": rate_hz,
            "span_s": span, "req_per_s": requests / span,
            "gridpoint*bands/s": work / span,
            "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
            "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
            "latency_ms_mean": 1e3 * float(lat.mean()),
            "largest3_share_of_work": float(units[sorted(big)].sum() / units.sum()),
            "latency_ms_p50_p99_largest3": [1e3 * float(np.percentile(lat[sel], q))
                                            for q in (50, 99)] if sel.any() else None,
            "latency_ms_p50_p99_others": [1e3 * float(np.percentile(lat[~sel], q))
                                          for q in (50, 99)] if (~sel).any() else None,
            "jobs": {j: int(np.sum(np.array(jobs) == k))
                     for k, j in enumerate(("project", "expand", "force"))},
            "short_requests": st["short_requests"],
            "alone_ms_largest3": alone,
            "admissions": st["admissions"], "evictions": st["evictions"],
            "peak_resident_GB": st["peak_resident_bytes"] / 1e9}


def compare(budget_bytes=64 << 30, nstreams=4, rate_hz=200.0, warmup=200, requests=2000,
            seed=4, nsystems=32, plain_requests=200, plain_warmup=20,
            tight_budget_bytes=40 << 30, tight_requests=300, tight_warmup=30):
    """The batched server and the per-request reference on the same stream of
    requests over the same pool (the reference on its first plain_warmup +
    plain_requests requests only: it serves a few requests per second, so a
    full stream would queue for many minutes), and the batched server again
    under a budget below the pool's resident size, so that systems are
    evicted and admitted again during the stream."""
    pool = wl.serving_pool(seed=seed, nsystems=nsystems)
    units = units_of(pool)
    _log("pool of %d systems sized" % len(pool))
    res = {"pool": {"systems": len(pool),
                    "psi_GB": float(sum(np.prod(s.n) * s.nbands * 8 for s in pool)) / 1e9},
           "budget_GB": budget_bytes / 1e9}
    for name, streams, flags, nw, nr, budget in (
            ("batched", nstreams, 0, warmup, requests, budget_bytes),
            ("batched_tight_budget", nstreams, 0, tight_warmup, tight_requests,
             tight_budget_bytes),
            ("per_request_plain", 1, bd.FLAG_PER_ATOM, plain_warmup, plain_requests,
             budget_bytes)):
        srv = bd.Server(budget, streams, flags)
        t0 = time.perf_counter()
        sids = register(srv, pool, seed)
        reg_s = time.perf_counter() - t0
        _log("%s: registered in %.1f s" % (name, reg_s))
        r = run(srv, sids, units, rate_hz, nw, nr, seed, alone_largest=(name == "batched"))
        _log("%s: %d requests, p50 %.2f ms, p99 %.2f ms, %.1f req/s"
             % (name, nr, r["latency_ms_p50"], r["latency_ms_p99"], r["req_per_s"]))
        r["streams"] = streams
        r["register_s"] = reg_s
        r["budget_GB"] = budget / 1e9
        srv.close()
        res[name] = r
    res["p99_ratio_plain_over_batched"] = (res["per_request_plain"]["latency_ms_p99"] /
                                           res["batched"]["latency_ms_p99"])
    return res


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--systems", type=int, default=32)
    ap.add_argument("--plain-requests", type=int, default=200)
    a = ap.parse_args()
    bd.load_library()
    print(json.dumps(compare(int(a.budget_gb * (1 << 30)), a.streams, a.rate, a.warmup,
                             a.requests, nsystems=a.systems,
                             plain_requests=a.plain_requests,
                             plain_warmup=max(1, a.plain_requests // 10))), flush=True)


if __name__ == "__main__":
    main()
