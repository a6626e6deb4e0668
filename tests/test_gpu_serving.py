"""Request server on the GPU: results of requests served in a mix (four
streams, interleaved systems, evictions and re-admissions) equal those of
the same request served alone and the oracle's, to the abs-sum-scaled 1e-12
bound of the other parity tests."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
JOBS = (0, 1, 2)


def _bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00480_amd import binding
    binding.load_library()
    return binding


def _pool():
    return [wl.small_periodic(seed=40, natoms=4, nbands=8),
            wl.small_mixed(seed=41, nbands=5),
            wl.make_system("srv_iso", (24, 20, 28), 0.2, (False, False, False), 5, None,
                           None, 16, 42, sigma_range=(0.5, 0.9), numax_range=(3, 9)),
            wl.small_periodic(seed=43, natoms=3, nbands=33, numax=7, n=24)]


def _register(bd, srv, pool):
    from paper_1905_00480_amd import serve
    sids = serve.register(srv, pool, seed=9)
    inputs = [tuple(x.copy() for x in srv.inputs(sid)) for sid in sids]
    return sids, inputs


@pytest.fixture(scope="module")
def reference():
    """Oracle results (with abs-sums) of every job on every pool system."""
    bd = _bd()
    pool = _pool()
    srv = bd.Server(1 << 34, 1, 0)
    _, inputs = _register(bd, srv, pool)
    srv.close()
    ref = []
    for s, (psi, w) in zip(pool, inputs):
        psi = psi.reshape(s.psi_shape)
        ref.append({0: oracle.project(*s.geometry(), psi, with_abs=True),
                    1: oracle.expand(*s.geometry(), w, np.zeros(s.psi_shape), with_abs=True),
                    2: oracle.force(*s.geometry(), psi, w, with_abs=True)})
    return pool, ref


def _check(got, ref_abs, what, slack=1.0):
    ref, absum = ref_abs
    err = np.abs(np.ravel(got) - np.ravel(ref))
    bound = slack * RTOL * np.ravel(absum) + 1e-300
    assert np.all(err <= bound), (what, float(np.max(err / bound)))


def test_mix_equals_alone_and_oracle(reference):
    bd = _bd()
    pool, ref = reference
    alone = []
    for k, s in enumerate(pool):
        srv = bd.Server(1 << 34, 1, 0)
        sids, _ = _register(bd, srv, pool)
        out = {}
        for j in JOBS:
            srv.submit(sids[k], j)
            out[j] = srv.read(sids[k], j)
        srv.close()
        alone.append(out)
    srv = bd.Server(1 << 34, 4, 0)
    sids, _ = _register(bd, srv, pool)
    rng = np.random.default_rng(5)
    for _ in range(40):
        srv.submit(sids[rng.integers(len(pool))], int(rng.integers(3)))
    final = [(k, j) for k in range(len(pool)) for j in JOBS]
    for i in rng.permutation(len(final)):
        k, j = final[i]
        srv.submit(sids[k], j)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == st["requests"] == 40 + len(final)
    for k in range(len(pool)):
        for j in JOBS:
            mix = srv.read(sids[k], j)
            _check(mix, ref[k][j], "mix system %d job %d vs oracle" % (k, j))
            _check(alone[k][j], ref[k][j], "alone system %d job %d vs oracle" % (k, j))
            _check(mix, (alone[k][j], ref[k][j][1]), "mix vs alone %d %d" % (k, j), slack=2.0)
    for r in range(st["requests"]):
        _, _, ts, td = srv.request_info(r)
        assert td >= ts >= 0
    srv.close()


def _tables(bd, s):
    p = bd.Plan(s.n, s.h, s.periodic, s.pos, s.sigma, s.numax, s.nbands,
                flags=bd.FLAG_HOST_ONLY)
    b = p.info["device_bytes"] - max(p.info["expand_scratch_doubles"], 1) * 8
    p.close()
    return (b + 4095) // 4096 * 4096


@pytest.mark.parametrize("keep_plans", [False, True])
def test_eviction_and_readmission(reference, keep_plans):
    """Evicted systems admitted again give the same results, whether their
    plans had to be freed (budget of the two largest systems) or were kept
    (room for every plan's tables besides)."""
    bd = _bd()
    pool, ref = reference
    probe = bd.Server(1 << 34, 1, bd.FLAG_HOST_ONLY)
    charges = [probe.system_info(probe.add(s))[0] for s in pool]
    probe.close()
    budget = sorted(charges)[-1] + sorted(charges)[-2]
    if keep_plans:
        budget += sum(_tables(bd, s) for s in pool)
    srv = bd.Server(budget, 2, 0)
    sids, _ = _register(bd, srv, pool)
    for rnd in range(3):
        for k in range(len(pool)):
            srv.submit(sids[k], (rnd + k) % 3)
    # the last system touched gets all jobs after its latest admission
    last = len(pool) - 1
    for j in JOBS:
        srv.submit(sids[last], j)
    srv.drain()
    st = srv.stats()
    assert st["evictions"] > 0 and st["admissions"] > len(pool)
    assert st["peak_resident_bytes"] <= budget
    if keep_plans:
        assert st["plan_reuses"] > 0 and st["plan_drops"] == 0
    for j in JOBS:
        _check(srv.read(sids[last], j), ref[last][j], "after re-admission job %d" % j)
    srv.close()


def test_request_stream_small():
    """A short Poisson stream through serve.run: every request completes and
    the latencies are sane."""
    bd = _bd()
    from paper_1905_00480_amd import serve
    pool = _pool()
    srv = bd.Server(1 << 34, 4, 0)
    sids = serve.register(srv, pool, seed=4)
    r = serve.run(srv, sids, serve.units_of(pool), rate_hz=200.0, warmup=10,
                  requests=60, seed=4)
    assert r["requests"] == 60 and sum(r["jobs"].values()) == 60
    assert 0 < r["latency_ms_p50"] <= r["latency_ms_p99"] < 5e3
    assert r["req_per_s"] > 0
    srv.close()
