"""Batched work decomposition: every projection schedule, band tile and work
item size, the per-atom reference schedule, the autotuner and the captured
project -> expand graph give the oracle's results (same abs-sum-scaled
1e-12 bound as the other parity tests)."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00480_amd import binding
    binding.load_library()
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _check(got, ref, absum, what):
    got, ref, absum = (np.asarray(x).ravel() for x in (got, ref, absum))
    assert got.shape == ref.shape, what
    err = np.abs(got - ref)
    bad = err > RTOL * absum + 1e-300
    assert not bad.any(), (what, int(bad.sum()), float(np.max(err / (absum + 1e-300))))


@pytest.fixture(scope="module")
def mixed():
    s = wl.small_mixed()
    s.numax = np.array([0, 3, 6, 9, 10, 7, 4, 8])  # every kernel family
    psi = wl.psi_for(s)
    cin = wl.coeffs_for(s)
    c_ref = oracle.project(*s.geometry(), psi, with_abs=True)
    e_ref = oracle.expand(*s.geometry(), cin, psi, with_abs=True)
    g_ref = oracle.force(*s.geometry(), psi, cin, with_abs=True)
    return s, psi, cin, c_ref, e_ref, g_ref


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("tile_half", [False, True])
@pytest.mark.parametrize("target", [256, 16384])
def test_schedules_match_oracle(mixed, sched, tile_half, target):
    """Uneven atoms (nu 0..10, sigma 0.4..1.2), mixed periodicity, 20 bands."""
    bd = _bd()
    s, psi, cin, (c_ref, c_abs), (e_ref, e_abs), (g_ref, g_abs) = mixed
    plan = bd.Plan.from_system(s)
    tile = plan.schedule()[1] // (2 if tile_half else 1)
    plan.set_schedule(sched, tile, target)
    assert plan.schedule() == (sched, tile, target)
    d_psi = _dev(psi)
    _check(_host(plan.project(d_psi)), c_ref, c_abs, "project %s" % ((sched, tile, target),))
    d_acc = d_psi.clone()
    plan.expand(_dev(cin), d_acc)
    _check(_host(d_acc), e_ref, e_abs, "expand")
    _check(_host(plan.force(d_psi, _dev(cin))), g_ref, g_abs, "force")
    plan.close()


def test_per_atom_reference_schedule(mixed):
    """One launch per atom, atom-owner expansion with atomics."""
    bd = _bd()
    s, psi, cin, (c_ref, c_abs), (e_ref, e_abs), (g_ref, g_abs) = mixed
    plan = bd.Plan.from_system(s, flags=bd.FLAG_PER_ATOM)
    d_psi = _dev(psi)
    _check(_host(plan.project(d_psi)), c_ref, c_abs, "per-atom project")
    d_acc = d_psi.clone()
    plan.expand(_dev(cin), d_acc)
    _check(_host(d_acc), e_ref, e_abs, "per-atom expand")
    _check(_host(plan.force(d_psi, _dev(cin))), g_ref, g_abs, "per-atom force")
    with pytest.raises(bd.ShoError):
        plan.tune(d_psi, torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda"))
    plan.close()


def test_graph_replays_match_oracle(mixed):
    """The captured project -> expand, replayed three times with eager work
    and synchronisations in between; every replay checked."""
    bd = _bd()
    s, psi, cin, (c_ref, c_abs), _, _ = mixed
    plan = bd.Plan.from_system(s)
    side = torch.cuda.Stream()
    d_psi = _dev(psi)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    out = torch.empty_like(d_psi)
    g = plan.graph(d_psi, c, out)
    for rep in range(3):
        with torch.cuda.stream(side):
            out.zero_()
            c.fill_(np.nan)
            junk = torch.randn(1 << 16, dtype=torch.float64, device="cuda").sum()
            g.launch()
        side.synchronize()
        assert np.isfinite(float(junk))
        c_h = _host(c)
        _check(c_h, c_ref, c_abs, "graph project, replay %d" % rep)
        # the expansion of the coefficients this replay produced
        e_ref, e_abs = oracle.expand(*s.geometry(), c_h, np.zeros(s.psi_shape), with_abs=True)
        _check(_host(out), e_ref, e_abs, "graph expand, replay %d" % rep)
    # a schedule change invalidates the graph
    plan.set_schedule(bd.SCHED_BY_NU)
    with pytest.raises(bd.ShoError):
        g.launch()
    g.close()
    plan.close()


def test_release_scratch(mixed):
    """sho_plan_release_scratch: the plane partials are freed and allocated
    again by the next expansion (results unchanged, twice), the block
    projection's plane sums likewise, and a graph captured before is
    refused instead of replaying on the freed address."""
    bd = _bd()
    s, psi, cin, (c_ref, c_abs), (e_ref, e_abs), _ = mixed
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    d_c = _dev(cin)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    out = torch.empty_like(d_psi)
    g = plan.graph(d_psi, c, out)  # allocates the scratch
    scratch = plan.info["expand_scratch_doubles"] * 8
    held = plan_info(plan)["device_bytes"]
    plan.release_scratch()
    assert plan_info(plan)["device_bytes"] == held - scratch
    plan.release_scratch()  # nothing held: no-op
    with pytest.raises(bd.ShoError):
        g.launch()
    for rep in range(2):
        e = _dev(psi)
        plan.expand(d_c, e)
        _check(_host(e), e_ref, e_abs, "expand after release, %d" % rep)
        assert plan_info(plan)["device_bytes"] == held
        plan.release_scratch()
    plan.set_project(bd.PROJECT_BLOCKS)
    _check(_host(plan.project(d_psi, c)), c_ref, c_abs, "block projection after release")
    plan.release_scratch()
    _check(_host(plan.project(d_psi, c)), c_ref, c_abs, "block projection, released again")
    g.close()
    plan.close()


def plan_info(plan):
    from paper_1905_00480_amd import binding as bd
    info = bd.sho_plan_info()
    bd._check(plan._lib.sho_plan_get_info(plan._h, bd.ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in bd.sho_plan_info._fields_}


def test_tuner_keeps_results(mixed):
    bd = _bd()
    s, psi, cin, (c_ref, c_abs), _, _ = mixed
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    r = plan.tune(d_psi, c, reps=2)
    assert r["schedule"] in bd.SCHEDULES and r["candidates"] >= 10
    assert r["ms"] <= r["ms_before"] and r["ms"] > 0
    assert plan.schedule() == (r["schedule"], r["band_tile"], r["target_points"])
    _check(_host(plan.project(d_psi)), c_ref, c_abs, "tuned project")
    plan.close()


def test_batching_config_sampled():
    """Periodic 160^3, h = 0.18, 2048 atoms, nu 3..9, sigma 0.4..1.2, 64
    bands, at full size: the single-launch schedule (tuned) and the graph;
    coefficients of sampled atoms and expanded values at sampled points
    against the oracle."""
    bd = _bd()
    s = wl.batching()
    psi = wl.psi_for(s)
    w = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    plan.tune(d_psi, c, reps=1)
    c = _host(plan.project(d_psi, c))
    rng = np.random.default_rng(2)
    off = oracle.coeff_offsets(s.numax, s.nbands)
    # the smallest, the largest and a few random atoms
    sizes = s.sigma * np.sqrt(2 * s.numax + 3)
    atoms = np.unique(np.concatenate([[np.argmin(sizes), np.argmax(sizes)],
                                      rng.choice(s.natoms, 4, replace=False)]))
    sub = s.subset(atoms)
    c_ref, c_abs = oracle.project(*sub.geometry(), psi, with_abs=True)
    _check(np.concatenate([c[off[a]:off[a + 1]] for a in atoms]), c_ref, c_abs,
           "batching project (sampled atoms)")
    d_out = d_psi.clone()
    plan.expand(_dev(w), d_out)
    out = _host(d_out).reshape(-1, s.nbands)
    pts = rng.choice(out.shape[0], 24, replace=False)
    e_ref, e_abs = oracle.expand_at(*s.geometry(), w, pts, psi.reshape(-1, s.nbands)[pts],
                                    with_abs=True)
    _check(out[pts], e_ref, e_abs, "batching expand (sampled points)")
    plan.close()


@pytest.mark.parametrize("form", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (1, 2, 16), (1, 16, 8),
                                  (1, 3, 12), (1, 5, 10), (1, 2, 7)])
def test_expansion_forms_match_oracle(mixed, form):
    """Row form, block form at the default shape and at extreme shapes (one
    point per block; wide and tall blocks), and widths that are not powers of
    two (the tile row is padded to the next one; blocks at the grid's x edge
    are partial), accumulating into random psi."""
    bd = _bd()
    s, psi, cin, _, (e_ref, e_abs), _ = mixed
    plan = bd.Plan.from_system(s)
    plan.set_expand(*form)
    assert plan.expand_form()[0] == form[0]
    d_acc = _dev(psi)
    plan.expand(_dev(cin), d_acc)
    _check(_host(d_acc), e_ref, e_abs, "expand form %s" % (form,))
    plan.close()


def test_expansion_forms_wide_boxes():
    """Boxes wider than a small periodic cell (several images of one atom in
    one row and one block)."""
    bd = _bd()
    s = wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 2, 41)
    c = wl.coeffs_for(s)
    e_ref, e_abs = oracle.expand(*s.geometry(), c, np.zeros(s.psi_shape), with_abs=True)
    for form in ((0, 0, 0), (1, 0, 0), (1, 4, 4), (1, 1, 8), (1, 3, 5), (1, 2, 3)):
        plan = bd.Plan.from_system(s)
        plan.set_expand(*form)
        out = torch.zeros(s.psi_shape, dtype=torch.float64, device="cuda")
        plan.expand(_dev(c), out)
        _check(_host(out), e_ref, e_abs, "wide boxes, form %s" % (form,))
        plan.close()


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_expand_tile_matches_oracle(mixed, tile):
    """The expansion's block form with narrower band tiles (more, larger
    blocks), into zeros and accumulating."""
    bd = _bd()
    s, psi, cin, _, (e_ref, e_abs), _ = mixed
    plan = bd.Plan.from_system(s)
    plan.set_expand_tile(tile)
    assert plan.expand_tile() == tile
    d_acc = _dev(psi)
    plan.expand(_dev(cin), d_acc)
    _check(_host(d_acc), e_ref, e_abs, "expand, band tile %d" % tile)
    plan.set_expand_tile(0)
    plan.close()


def test_expand_tuner_keeps_results(mixed):
    bd = _bd()
    s, psi, cin, _, (e_ref, e_abs), _ = mixed
    plan = bd.Plan.from_system(s)
    scratch = torch.zeros(s.psi_shape, dtype=torch.float64, device="cuda")
    r = plan.tune_expand(_dev(cin), scratch, reps=2)
    assert r["candidates"] >= 4 and 0 < r["ms"] <= r["ms_before"]
    assert plan.expand_form()[0] == r["mode"]
    d_acc = _dev(psi)
    plan.expand(_dev(cin), d_acc)
    _check(_host(d_acc), e_ref, e_abs, "expand after tuning %s" % (r,))
    plan.close()
