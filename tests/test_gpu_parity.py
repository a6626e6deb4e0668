"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance (FP64): every entry must satisfy
    |x_gpu - x_oracle| <= 1e-12 * A
where A is the oracle's abs-sum of the same entry (h^3 sum |P psi| for a
coefficient, |psi_in| + sum |c P| for an expanded value, sum |w| h^3 sum
|dP psi| for a derivative).  The two sides sum the same terms in different
orders; rounding then differs by a few ulp of A, never by 1e-12 A, while a
dropped term or a wrong factor changes an entry by O(A).
"""
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


def assert_parity(got, ref, absum, what):
    got = np.asarray(got).ravel()
    ref = np.asarray(ref).ravel()
    absum = np.asarray(absum).ravel()
    assert got.shape == ref.shape, what
    err = np.abs(got - ref)
    bound = RTOL * absum + 1e-300
    worst = int(np.argmax(err / bound)) if err.size else 0
    assert np.all(err <= bound), (
        "%s: %d entries off, worst |d|=%.3e vs abs-sum %.3e (got %.17g ref %.17g)"
        % (what, int((err > bound).sum()), err[worst], absum[worst], got[worst], ref[worst]))


def run_all(bd, s, psi_in=True, force=True):
    """Project, expand (into zero and into random psi) and force on the GPU
    and compare with the oracle."""
    psi = wl.psi_for(s)
    c_in = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    # projection
    c = _host(plan.project(d_psi))
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    assert_parity(c, c_ref, c_abs, s.name + " project")
    # expansion into zeros
    d_out = torch.zeros_like(d_psi)
    plan.expand(_dev(c_in), d_out)
    e_ref, e_abs = oracle.expand(*s.geometry(), c_in, np.zeros(s.psi_shape), with_abs=True)
    assert_parity(_host(d_out), e_ref, e_abs, s.name + " expand")
    if psi_in:
        d_acc = d_psi.clone()
        plan.expand(_dev(c_in), d_acc)
        a_ref, a_abs = oracle.expand(*s.geometry(), c_in, psi, with_abs=True)
        assert_parity(_host(d_acc), a_ref, a_abs, s.name + " expand(accumulate)")
    if force:
        g = _host(plan.force(d_psi, _dev(c_in)))
        g_ref, g_abs = oracle.force(*s.geometry(), psi, c_in, with_abs=True)
        assert_parity(g, g_ref, g_abs, s.name + " force")
    plan.close()


def test_scaled_expansion():
    """sho_plan_expand_scaled: psi += alpha * expansion of c, against the
    oracle's expansion of alpha * c."""
    bd = _bd()
    s = wl.small_periodic()
    plan = bd.Plan.from_system(s)
    c_in = wl.coeffs_for(s)
    psi = wl.psi_for(s)
    alpha = 0.2 ** 3 * 1.7
    d_out = _dev(psi)
    plan.expand(_dev(c_in), d_out, alpha=alpha)
    ref, ab = oracle.expand(*s.geometry(), alpha * c_in, psi, with_abs=True)
    assert_parity(_host(d_out), ref, ab, "expand_scaled")
    with pytest.raises(bd.ShoError):
        plan.expand(_dev(c_in), d_out, alpha=float("nan"))
    plan.close()


def test_tiny_config():
    bd = _bd()
    run_all(bd, wl.tiny())


def test_small_periodic_scale_shape():
    """nu = 5, sigma = 0.6, h = 0.2, 32 bands: the scale workload's shape on a
    small periodic cell whose supports wrap across the faces."""
    bd = _bd()
    run_all(bd, wl.small_periodic())


def test_small_mixed_uneven_atoms():
    """nu 0..9, sigma 0.4..1.2, 20 bands (ragged tile), non-cubic grid with
    mixed periodic and isolated axes."""
    bd = _bd()
    run_all(bd, wl.small_mixed())


@pytest.mark.parametrize("nbands", [1, 3, 64, 70, 130])
def test_band_counts(nbands):
    bd = _bd()
    s = wl.make_system("bands%d" % nbands, (24, 20, 22), 0.2, (True, True, False), 5,
                       0.6, 4, nbands, 50 + nbands)
    run_all(bd, s, psi_in=nbands < 100, force=True)


def test_boxes_wider_than_cell():
    """Supports wider than a small periodic cell: every image contributes."""
    bd = _bd()
    s = wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 4, 41)
    run_all(bd, s)


def test_isolated_edges_and_empty_support():
    bd = _bd()
    s = wl.make_system("edge", (20, 16, 12), 0.25, (False,) * 3, 6, 0.5, 4, 3, 42)
    s.pos[0] = [-0.3, 1.0, 1.0]
    s.pos[1] = [5.2, 4.1, 3.2]
    s.pos[2] = [-9.0, 1.0, 1.0]   # no support point inside the grid
    run_all(bd, s)


def test_all_nu_values_one_launch_each():
    """Every nu in 0..10 (the force runs at nu+1, up to 11 functions)."""
    bd = _bd()
    s = wl.make_system("allnu", (30, 28, 26), 0.16, (True,) * 3, 11, None, 0, 5,
                       60, sigma_range=(0.7, 0.9))
    s.numax[:] = np.arange(11)
    run_all(bd, s, psi_in=False)


def test_zero_atoms():
    bd = _bd()
    p = bd.Plan((8, 8, 8), 0.2, (True,) * 3, np.zeros((0, 3)), [], [], 4)
    psi = torch.randn(8, 8, 8, 4, dtype=torch.float64, device="cuda")
    keep = psi.clone()
    c = torch.empty(0, dtype=torch.float64, device="cuda")
    p.project(psi, c)
    p.expand(c, psi)
    torch.cuda.synchronize()
    assert torch.equal(psi, keep)
    p.close()


def test_stateless_calls_match_plan():
    bd = _bd()
    s = wl.small_periodic(natoms=4, nbands=8)
    psi = _dev(wl.psi_for(s))
    c1 = bd.project(*s.geometry(), psi)
    plan = bd.Plan.from_system(s)
    c2 = plan.project(psi)
    ref, ab = oracle.project(*s.geometry(), wl.psi_for(s), with_abs=True)
    assert_parity(_host(c1), ref, ab, "stateless project")
    assert_parity(_host(c2), ref, ab, "plan project")
    w = _dev(wl.coeffs_for(s))
    g1 = _host(bd.force(*s.geometry(), psi, w))
    g2 = _host(plan.force(psi, w))
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))
    o = torch.zeros_like(psi)
    bd.expand(*s.geometry(), w, o)
    o2 = torch.zeros_like(psi)
    plan.expand(w, o2)
    assert torch.allclose(o, o2, rtol=0, atol=1e-12 * float(o2.abs().max()))
    bd.cache_clear()
    plan.close()


def test_argument_errors_on_device():
    bd = _bd()
    import ctypes
    s = wl.small_periodic(natoms=2, nbands=4)
    p = bd.Plan.from_system(s)
    psi = torch.zeros(s.psi_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        p.project(psi.cpu())
    with pytest.raises(ValueError):
        p.project(psi[..., :2].contiguous())
    # raw calls: host pointers, NULL and overlapping buffers are refused
    # before any launch (the library checks against the runtime's allocation
    # records; the binding checks exact element counts)
    host = np.zeros(p.coeff_doubles)
    lib = bd.load_library()
    code = lib.sho_plan_project(p._h, ctypes.c_void_p(psi.data_ptr()),
                                ctypes.c_void_p(host.ctypes.data), None)
    assert code == bd.SHO_E_INVALID
    code = lib.sho_plan_project(p._h, ctypes.c_void_p(psi.data_ptr()), None, None)
    assert code == bd.SHO_E_INVALID
    code = lib.sho_plan_project(p._h, ctypes.c_void_p(psi.data_ptr()),
                                ctypes.c_void_p(psi.data_ptr() + 64), None)
    assert code == bd.SHO_E_INVALID
    p.close()


# ---------------------------------------------------------- full sizes ----

def _scale_inputs():
    s = wl.scale()
    psi = wl.psi_for(s)
    return s, psi


def test_scale_full_size_sampled():
    """Periodic 128^3, 512 atoms, nu = 5, 32 bands -- the benchmarked launch
    configuration.  Coefficients and derivatives of sampled atoms, expanded
    values at sampled grid points, all against the oracle."""
    bd = _bd()
    s, psi = _scale_inputs()
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    c = _host(plan.project(d_psi))
    off = oracle.coeff_offsets(s.numax, s.nbands)
    rng = np.random.default_rng(123)
    atoms = np.sort(rng.choice(s.natoms, 10, replace=False))
    sub = s.subset(atoms)
    c_ref, c_abs = oracle.project(*sub.geometry(), psi, with_abs=True)
    got = np.concatenate([c[off[a]:off[a + 1]] for a in atoms])
    assert_parity(got, c_ref, c_abs, "scale project (sampled atoms)")

    w = wl.coeffs_for(s)
    g = _host(plan.force(d_psi, _dev(w)))
    wsub = np.concatenate([w[off[a]:off[a + 1]] for a in atoms])
    g_ref, g_abs = oracle.force(*sub.geometry(), psi, wsub, with_abs=True)
    assert_parity(g[atoms], g_ref, g_abs, "scale force (sampled atoms)")

    d_out = d_psi.clone()
    plan.expand(_dev(w), d_out)
    out = _host(d_out).reshape(-1, s.nbands)
    pts = rng.choice(out.shape[0], 48, replace=False)
    e_ref, e_abs = oracle.expand_at(*s.geometry(), w, pts, psi.reshape(-1, s.nbands)[pts],
                                    with_abs=True)
    assert_parity(out[pts], e_ref, e_abs, "scale expand (sampled points)")
    plan.close()


def test_scale_adjoint_identity_full():
    """<project psi, w> = h^3 <psi, expand w> over the whole scale workload."""
    bd = _bd()
    s, psi = _scale_inputs()
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    w = _dev(wl.coeffs_for(s))
    c = plan.project(d_psi)
    e = torch.zeros_like(d_psi)
    plan.expand(w, e)
    lhs = float(torch.dot(c, w))
    rhs = s.h ** 3 * float(torch.sum(d_psi * e))
    scale = float(torch.sum(torch.abs(c) * torch.abs(w)))
    assert abs(lhs - rhs) <= 1e-12 * scale
    plan.close()


def test_diff_config_force_finite_differences():
    """Isolated 96^3, 256 atoms, nu = 6, 16 bands.  Sampled derivatives
    against the oracle, and against central differences (delta = 1e-5 Bohr)
    of the GPU projection with the supports frozen (set_centres)."""
    bd = _bd()
    s = wl.diff()
    psi = wl.psi_for(s)
    w = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    d_psi = _dev(psi)
    d_w = _dev(w)
    g = _host(plan.force(d_psi, d_w))
    rng = np.random.default_rng(7)
    atoms = np.sort(rng.choice(s.natoms, 6, replace=False))
    off = oracle.coeff_offsets(s.numax, s.nbands)
    sub = s.subset(atoms)
    wsub = np.concatenate([w[off[a]:off[a + 1]] for a in atoms])
    g_ref, g_abs = oracle.force(*sub.geometry(), psi, wsub, with_abs=True)
    assert_parity(g[atoms], g_ref, g_abs, "diff force (sampled atoms)")
    delta = 1e-5
    for a in atoms[:3]:
        for d in range(3):
            pp = s.pos.copy()
            pp[a, d] += delta
            plan.set_centres(pp)
            lp = float(torch.dot(plan.project(d_psi), d_w))
            pp[a, d] -= 2 * delta
            plan.set_centres(pp)
            lm = float(torch.dot(plan.project(d_psi), d_w))
            fd = (lp - lm) / (2 * delta)
            assert abs(fd - g[a, d]) <= 1e-7 * max(1.0, abs(g[a, d])), (a, d, fd, g[a, d])
    plan.set_centres(s.pos)
    plan.close()
