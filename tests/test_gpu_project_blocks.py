"""The block form of the projection (SHO_PROJECT_BLOCKS): each block of psi
read once, every atom plane touching it adding its plane sums, then the z
pass.  Against the oracle at the bound of the other parity tests,
|c - c_oracle| <= 1e-12 A (A: the oracle's abs-sum of the coefficient).

Cases: uneven cut-offs 0..10 with mixed periodicity, boxes wider than the
cell, one band and 70 bands (ragged tiles), every band tile and several block
shapes (narrow and wide blocks, few rows, rows that do not divide the grid),
atoms whose support misses an isolated grid, the scale workload (every
coefficient) and the batching workload (sampled atoms), the tuner's choice,
and a graph replay."""
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


def _check(got, ref, ab, what):
    err = np.abs(np.ravel(got) - np.ravel(ref))
    bound = RTOL * np.ravel(ab) + 1e-300
    assert np.all(err <= bound), "%s: %d entries off, max |d| %.3e" % (
        what, int((err > bound).sum()), float(err.max()) if err.size else 0.0)


def _mixed():
    s = wl.small_mixed()
    s.numax = np.array([0, 3, 6, 9, 10, 7, 4, 8])
    return s


def _far():
    s = wl.make_system("far", (20, 18, 16), 0.2, (False,) * 3, 4, 0.5, 4, 12, 121)
    s.pos[1] = (-3.0, 1.0, 1.0)  # sphere outside the isolated grid
    return s


SYSTEMS = {
    "mixed": _mixed,
    "wide": lambda: wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 4, 41),
    "bands1": lambda: wl.make_system("b1", (24, 20, 22), 0.2, (True, True, False), 5, 0.6, 4,
                                     1, 61),
    "bands70": lambda: wl.make_system("b70", (20, 18, 16), 0.2, (True, True, True), 4, 0.6, 3,
                                      70, 63),
    "far": _far,
}

SHAPES = [(0, 0, 0), (0, 32, 8), (0, 16, 32), (0, 64, 8), (5, 24, 16), (3, 40, 32),
          (255, 1, 16)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_block_projection_matches_oracle(name, shape):
    bd = _bd()
    s = SYSTEMS[name]()
    R, X, TB = shape
    psi = wl.psi_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    plan = bd.Plan.from_system(s)
    plan.set_project(bd.PROJECT_BLOCKS, R, X, TB)
    form = plan.project_form()
    assert form[0] == bd.PROJECT_BLOCKS
    if X:
        assert form[2] == X
    d_psi = _dev(psi)
    c = torch.full((plan.coeff_doubles,), np.nan, dtype=torch.float64, device="cuda")
    plan.project(d_psi, c)
    _check(_host(c), c_ref, c_abs, "%s blocks %s" % (name, shape))
    # twice in a row: the plane sums start from zero again
    plan.project(d_psi, c)
    _check(_host(c), c_ref, c_abs, "%s blocks %s (again)" % (name, shape))
    # back to work items
    plan.set_project(bd.PROJECT_ITEMS)
    _check(_host(plan.project(d_psi)), c_ref, c_abs, "%s items after blocks" % name)
    plan.close()


def test_block_projection_scale_every_coefficient():
    bd = _bd()
    s = wl.scale()
    psi = wl.psi_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    plan = bd.Plan.from_system(s)
    plan.set_project(bd.PROJECT_BLOCKS)
    _check(_host(plan.project(_dev(psi))), c_ref, c_abs, "scale, block projection")
    plan.close()


def test_block_projection_batching_sampled_and_tuned():
    bd = _bd()
    s = wl.batching()
    psi = wl.psi_for(s)
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    plan.set_project(bd.PROJECT_BLOCKS)
    cb = _host(plan.project(d_psi, c))
    r = plan.tune(d_psi, c, reps=1)
    assert r["project_form"] in (bd.PROJECT_ITEMS, bd.PROJECT_BLOCKS)
    assert plan.project_form()[0] == r["project_form"]
    ct = _host(plan.project(d_psi, c))
    rng = np.random.default_rng(2)
    sizes = s.sigma * np.sqrt(2 * s.numax + 3)
    atoms = np.unique(np.concatenate([[np.argmin(sizes), np.argmax(sizes)],
                                      rng.choice(s.natoms, 4, replace=False)]))
    off = oracle.coeff_offsets(s.numax, s.nbands)
    sub = s.subset(atoms)
    c_ref, c_abs = oracle.project(*sub.geometry(), psi, with_abs=True)
    for tag, cc in (("block form", cb), ("tuned", ct)):
        _check(np.concatenate([cc[off[a]:off[a + 1]] for a in atoms]), c_ref, c_abs,
               "batching %s (sampled atoms)" % tag)
    plan.close()


def test_block_projection_graph_and_expand():
    """A captured project -> expand graph with the block projection (the plane
    sums and the expansion's plane partials share the plan's scratch),
    replayed with eager work in between."""
    bd = _bd()
    s = _mixed()
    psi = wl.psi_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    plan = bd.Plan.from_system(s)
    plan.set_project(bd.PROJECT_BLOCKS, 0, 16, 16)
    d_psi = _dev(psi)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    out = torch.empty_like(d_psi)
    g = plan.graph(d_psi, c, out)
    for rep in range(3):
        out.zero_()
        c.fill_(np.nan)
        junk = torch.randn(1 << 16, dtype=torch.float64, device="cuda").sum()
        g.launch()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        c_h = _host(c)
        _check(c_h, c_ref, c_abs, "graph block projection, replay %d" % rep)
        e_ref, e_abs = oracle.expand(*s.geometry(), c_h, np.zeros(s.psi_shape), with_abs=True)
        _check(_host(out), e_ref, e_abs, "graph expand, replay %d" % rep)
    g.close()
    plan.close()


def test_block_projection_refusals():
    bd = _bd()
    s = wl.small_periodic(natoms=2, nbands=4)
    for flags in (bd.FLAG_DETERMINISTIC, bd.FLAG_FP32, bd.FLAG_STORED, bd.FLAG_BLOCH):
        plan = bd.Plan.from_system(s, flags=flags)
        with pytest.raises(bd.ShoError):
            plan.set_project(bd.PROJECT_BLOCKS)
        plan.close()
    plan = bd.Plan.from_system(s)
    for bad in ((0, 0, 12), (0, 300, 0), (300, 0, 0), (64, 64, 64)):
        with pytest.raises(bd.ShoError):
            plan.set_project(bd.PROJECT_BLOCKS, *bad)
    plan.close()
