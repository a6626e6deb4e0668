"""Non-local application on the GPU (project, per-atom matrix product on the
matrix cores, expand), its captured graph, and the product alone, against
the oracle (abs-sum-scaled 1e-12 bound, the abs-sum carried through the
chain)."""
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


def _matrices(s, seed):
    rng = np.random.default_rng(seed)
    off = oracle.matrix_offsets(s.numax)
    return rng.standard_normal(int(off[-1])), off


def _systems():
    mixed = wl.small_mixed()
    mixed.numax = np.array([0, 3, 6, 9, 10, 7, 4, 8])
    return {"periodic": wl.small_periodic(), "mixed": mixed,
            "bands70": wl.small_periodic(natoms=4, nbands=70, numax=4)}


@pytest.mark.parametrize("which", ["periodic", "mixed", "bands70"])
def test_multiply_matches_matmul(which):
    bd = _bd()
    s = _systems()[which]
    plan = bd.Plan.from_system(s)
    D, off = _matrices(s, 3)
    assert np.array_equal(plan.matrix_offsets(), off)
    c = wl.coeffs_for(s)
    d = _host(plan.multiply(_dev(D), _dev(c)))
    coff = oracle.coeff_offsets(s.numax, s.nbands)
    for a in range(s.natoms):
        N = oracle.nsho(int(s.numax[a]))
        Da = D[off[a]:off[a + 1]].reshape(N, N)
        ca = c[coff[a]:coff[a + 1]].reshape(N, s.nbands)
        _check(d[coff[a]:coff[a + 1]], (Da @ ca).ravel(), (np.abs(Da) @ np.abs(ca)).ravel(),
               "%s atom %d" % (which, a))
    plan.close()


@pytest.mark.parametrize("which", ["periodic", "mixed", "bands70"])
def test_apply_matches_oracle(which):
    bd = _bd()
    s = _systems()[which]
    plan = bd.Plan.from_system(s)
    D, _ = _matrices(s, 4)
    psi = wl.psi_for(s)
    psi_in = np.random.default_rng(6).standard_normal(s.psi_shape)
    ref, ref_abs = oracle.apply(*s.geometry(), psi, D, psi_in, with_abs=True)
    out = _dev(psi_in)
    plan.apply(_dev(psi), _dev(D), out)
    _check(_host(out), ref, ref_abs, "apply " + which)
    plan.close()


def test_apply_graph_replays():
    """The captured apply, replayed three times with eager work in between;
    every replay against the oracle."""
    bd = _bd()
    s = _systems()["mixed"]
    plan = bd.Plan.from_system(s)
    D, _ = _matrices(s, 5)
    psi = wl.psi_for(s)
    ref, ref_abs = oracle.apply(*s.geometry(), psi, D, np.zeros(s.psi_shape), with_abs=True)
    d_psi, d_D = _dev(psi), _dev(D)
    c = torch.empty(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    d = torch.empty_like(c)
    out = torch.empty_like(d_psi)
    g = plan.apply_graph(d_psi, d_D, c, d, out)
    side = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(side):
            out.zero_()
            c.fill_(np.nan)
            d.fill_(np.nan)
            _ = torch.randn(1 << 16, dtype=torch.float64, device="cuda").sum()
            g.launch()
        side.synchronize()
        _check(_host(out), ref, ref_abs, "apply graph replay %d" % rep)
    g.close()
    plan.close()


def test_apply_scale_full():
    """Periodic 128^3, 512 atoms, nu = 5, 32 bands, random atomic matrices:
    every grid value of the application against the oracle."""
    bd = _bd()
    s = wl.scale()
    plan = bd.Plan.from_system(s)
    D, _ = _matrices(s, 7)
    psi = wl.psi_for(s)
    ref, ref_abs = oracle.apply(*s.geometry(), psi, D, np.zeros(s.psi_shape), with_abs=True)
    out = torch.zeros(s.psi_shape, dtype=torch.float64, device="cuda")
    plan.apply(_dev(psi), _dev(D), out)
    _check(_host(out), ref, ref_abs, "apply scale")
    plan.close()
