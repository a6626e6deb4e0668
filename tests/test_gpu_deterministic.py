"""The owner form of the expansion and SHO_FLAG_DETERMINISTIC plans.

Parity against the CPU oracle uses the bound of the other GPU tests,
|x - x_oracle| <= 1e-12 * A (A: the oracle's abs-sum of the entry).
Determinism is checked bitwise: the same call on the same inputs, repeated,
must give identical bits for the projection, the expansion (into zeros and
accumulating) and the derivative."""
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


def _parity(got, ref, absum, what):
    err = np.abs(np.ravel(got) - np.ravel(ref))
    bound = RTOL * np.ravel(absum) + 1e-300
    assert np.all(err <= bound), "%s: %d entries off, max |d| %.3e" % (
        what, int((err > bound).sum()), float(err.max()) if err.size else 0.0)


SYSTEMS = {
    "small_periodic": lambda: wl.small_periodic(),
    "small_mixed": lambda: wl.small_mixed(),
    "bands1": lambda: wl.make_system("b1", (24, 20, 22), 0.2, (True, True, False), 5, 0.6, 4,
                                     1, 61),
    "bands20": lambda: wl.make_system("b20", (24, 20, 22), 0.2, (True, False, True), 5, 0.6, 5,
                                      20, 62),
    "bands70": lambda: wl.make_system("b70", (20, 18, 16), 0.2, (True, True, True), 4, 0.6, 3,
                                      70, 63),
    "wide": lambda: wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 4, 41),
    "nu10": lambda: wl.make_system("nu10", (30, 28, 26), 0.15, (True, False, True), 3, 0.8, 10,
                                   9, 64),
}


@pytest.mark.parametrize("width", [16, 32])
@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_owner_expansion_parity(name, width):
    bd = _bd()
    s = SYSTEMS[name]()
    plan = bd.Plan.from_system(s)
    plan.set_expand(bd.EXPAND_OWNER, 0, width)
    assert plan.expand_form()[0] == bd.EXPAND_OWNER
    c_in = wl.coeffs_for(s)
    psi = wl.psi_for(s)
    out = torch.zeros(s.psi_shape, dtype=torch.float64, device="cuda")
    plan.expand(_dev(c_in), out)
    ref, ab = oracle.expand(*s.geometry(), c_in, np.zeros(s.psi_shape), with_abs=True)
    _parity(_host(out), ref, ab, name + " owner expand")
    acc = _dev(psi)
    plan.expand(_dev(c_in), acc)
    ref, ab = oracle.expand(*s.geometry(), c_in, psi, with_abs=True)
    _parity(_host(acc), ref, ab, name + " owner expand (accumulate)")
    plan.close()


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_deterministic_plan_parity(name):
    bd = _bd()
    s = SYSTEMS[name]()
    plan = bd.Plan.from_system(s, flags=bd.FLAG_DETERMINISTIC)
    psi = wl.psi_for(s)
    w = wl.coeffs_for(s)
    d_psi = _dev(psi)
    c = _host(plan.project(d_psi))
    ref, ab = oracle.project(*s.geometry(), psi, with_abs=True)
    _parity(c, ref, ab, name + " det project")
    out = _dev(psi)
    plan.expand(_dev(w), out)
    ref, ab = oracle.expand(*s.geometry(), w, psi, with_abs=True)
    _parity(_host(out), ref, ab, name + " det expand")
    g = _host(plan.force(d_psi, _dev(w)))
    ref, ab = oracle.force(*s.geometry(), psi, w, with_abs=True)
    _parity(g, ref, ab, name + " det force")
    plan.close()


def _repeat_bitwise(bd, s, reps=3):
    plan = bd.Plan.from_system(s, flags=bd.FLAG_DETERMINISTIC)
    psi = _dev(wl.psi_for(s))
    w = _dev(wl.coeffs_for(s))
    outs = []
    for _ in range(reps):
        c = plan.project(psi)
        e0 = torch.zeros_like(psi)
        plan.expand(w, e0)
        e1 = psi.clone()
        plan.expand(w, e1)
        g = plan.force(psi, w)
        torch.cuda.synchronize()
        outs.append([t.cpu() for t in (c, e0, e1, g)])
    for r in range(1, reps):
        for k, name in enumerate(("project", "expand", "expand(accumulate)", "force")):
            assert torch.equal(outs[0][k], outs[r][k]), "%s differs between runs" % name
    plan.close()
    return outs[0]


def test_deterministic_repeat_small_mixed():
    _repeat_bitwise(_bd(), wl.small_mixed())


def test_deterministic_repeat_scale_config():
    """The scale workload (periodic 128^3, 512 atoms, nu 5, 32 bands): three
    runs bitwise equal, and sampled atoms and points against the oracle."""
    bd = _bd()
    s = wl.scale()
    c, e0, _, g = _repeat_bitwise(bd, s, reps=2)
    psi = wl.psi_for(s)
    w = wl.coeffs_for(s)
    off = oracle.coeff_offsets(s.numax, s.nbands)
    atoms = np.array([0, 137, 511])
    sub = s.subset(atoms)
    ref, ab = oracle.project(*sub.geometry(), psi, with_abs=True)
    got = np.concatenate([c.numpy()[off[a]:off[a + 1]] for a in atoms])
    _parity(got, ref, ab, "scale det project (sampled)")
    wsub = np.concatenate([w[off[a]:off[a + 1]] for a in atoms])
    ref, ab = oracle.force(*sub.geometry(), psi, wsub, with_abs=True)
    _parity(g.numpy()[atoms], ref, ab, "scale det force (sampled)")
    pts = np.random.default_rng(7).choice(int(np.prod(s.n)), 64, replace=False)
    ref, ab = oracle.expand_at(*s.geometry(), w, pts, nbands=s.nbands, with_abs=True)
    _parity(e0.numpy().reshape(-1, s.nbands)[pts], ref, ab, "scale det expand (sampled)")
