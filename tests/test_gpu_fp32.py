"""Single-precision bands (SHO_FLAG_FP32) and complex bands, through the C ABI,
against the FP64 oracle evaluated on the same (float-valued) inputs.

Tolerance.  The FP32 path rounds the 1D functions to float once (relative
error <= u = 2^-24 each) and accumulates every sum in float.  For a sum of
terms evaluated with k roundings along any term's path, the computed value
differs from the exact one by at most gamma_k * (sum of |terms|),
gamma_k = k u / (1 - k u) (recursive summation in any order, products
carrying their own rounding).  Along one term of a coefficient there are
<= m_x + m_y + m_z roundings for the x, y and z accumulations (m_d: table
extent of the atom's box per axis), <= 6 for folding the lane slots, 3 for
the rounded functions, and 3 for the products and the h^3 factor; so
    |c_gpu - c_exact| <= gamma_k * A,   k = m_x + m_y + m_z + 12,
with A = h^3 sum |P psi| the oracle's abs-sum.  An expanded value passes
3 (nu_max + 1) accumulations over the basis, 3 rounded functions, one
product, and one addition per contribution that lands on the point
(overlapping atoms and images), so k = 3 (nu_max + 1) + 4 + overlaps and
A = |psi_in| + sum |c P|.  The tests use k from the geometry (overlaps
counted from the supports) and a factor 2 for gamma_k's denominator and
the FP64 oracle's own rounding; a dropped term or a wrong factor changes an
entry by O(A), far above k u A.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


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


def _extent(s):
    """Largest table extent per axis over the atoms (points)."""
    m = 0
    for a in range(s.natoms):
        R = s.rbox[a] if s.rbox is not None else oracle.box_radius(s.sigma[a], s.numax[a], s.h)
        m = max(m, int(np.ceil(2.0 * R / s.h)) + 2)
    return m


def _overlaps(s):
    """Number of (atom, image) supports containing each grid point, [npoints]."""
    cnt = np.zeros(int(np.prod(s.n)), dtype=np.int64)
    for a in range(s.natoms):
        R = s.rbox[a] if s.rbox is not None else oracle.box_radius(s.sigma[a], s.numax[a], s.h)
        _, mem = oracle.support(s.n, s.h, s.periodic, s.pos[a], R)
        cnt += np.bincount(mem, minlength=cnt.size)
    return cnt


def _assert_close(got, ref, absum, k, what):
    absum = np.asarray(absum, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    if k.ndim and k.size == absum.size:
        k = k.reshape(absum.shape)
    bound = (2.0 * k * U32 * absum + 1e-30).ravel()
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref).ravel()
    assert got.shape == ref.shape == bound.shape, what
    err = np.abs(got - ref)
    worst = int(np.argmax(err / bound)) if err.size else 0
    assert np.all(err <= bound), (
        "%s: %d entries off, worst |d|=%.3e bound %.3e (got %.9g ref %.17g)"
        % (what, int((err > bound).sum()), err[worst], bound[worst], got[worst], ref[worst]))
    return float(np.max(err / bound)) if err.size else 0.0


def _run_fp32(bd, s, accumulate=True):
    psi = wl.psi_for(s, dtype=np.float32)
    c_in = wl.coeffs_for(s).astype(np.float32)
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    assert plan.info["nbands"] == s.nbands
    assert plan.coeff_doubles == c_in.size
    assert np.array_equal(plan.coeff_offsets(), wl.coeff_offsets(s))
    d_psi = _dev(psi)
    c = _host(plan.project(d_psi))
    assert c.dtype == np.float32
    c_ref, c_abs = oracle.project(*s.geometry(), psi.astype(np.float64), rbox=s.rbox,
                                  with_abs=True)
    _assert_close(c, c_ref, c_abs, 3 * _extent(s) + 12, s.name + " fp32 project")
    kexp = 3 * (int(s.numax.max()) + 1) + 4 + _overlaps(s)
    kexp = np.repeat(kexp, s.nbands)
    d_out = torch.zeros_like(d_psi)
    plan.expand(_dev(c_in), d_out)
    e_ref, e_abs = oracle.expand(*s.geometry(), c_in.astype(np.float64),
                                 np.zeros(s.psi_shape), rbox=s.rbox, with_abs=True)
    _assert_close(_host(d_out), e_ref, e_abs, kexp, s.name + " fp32 expand")
    if accumulate:
        d_acc = d_psi.clone()
        plan.expand(_dev(c_in), d_acc)
        a_ref, a_abs = oracle.expand(*s.geometry(), c_in.astype(np.float64),
                                     psi.astype(np.float64), rbox=s.rbox, with_abs=True)
        _assert_close(_host(d_acc), a_ref, a_abs, kexp, s.name + " fp32 expand(accumulate)")
    plan.close()


def test_fp32_small_periodic():
    """The scale workload's shape (nu 5, sigma 0.6, h 0.2) on a periodic 32^3
    cell whose supports wrap across the faces; 32 bands = 16 pairs."""
    _run_fp32(_bd(), wl.small_periodic())


def test_fp32_small_mixed():
    """nu 0..9, sigma 0.4..1.2, 20 bands, mixed periodic / isolated axes."""
    _run_fp32(_bd(), wl.small_mixed())


@pytest.mark.parametrize("nbands", [2, 6, 66, 130])
def test_fp32_band_counts(nbands):
    """Pair counts 1, 3, 33 and 65: a single pair, ragged pair tiles."""
    bd = _bd()
    s = wl.make_system("f32bands%d" % nbands, (24, 20, 22), 0.2, (True, True, False), 5,
                       0.6, 4, nbands, 70 + nbands)
    _run_fp32(bd, s, accumulate=nbands < 100)


def test_fp32_boxes_wider_than_cell():
    """Supports wider than a small periodic cell: every image contributes."""
    _run_fp32(_bd(), wl.make_system("f32wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 4, 41))


def test_fp32_isolated_edges_and_empty_support():
    s = wl.make_system("f32edge", (20, 16, 12), 0.25, (False,) * 3, 6, 0.5, 4, 4, 42)
    s.pos[0] = [-0.3, 1.0, 1.0]
    s.pos[1] = [5.2, 4.1, 3.2]
    s.pos[2] = [-9.0, 1.0, 1.0]   # no support point inside the grid
    _run_fp32(_bd(), s)


def test_fp32_all_nu_values():
    """Every nu in 0..10 in one FP32 plan."""
    s = wl.make_system("f32allnu", (30, 28, 26), 0.16, (True,) * 3, 11, None, 0, 6,
                       60, sigma_range=(0.7, 0.9))
    s.numax[:] = np.arange(11)
    _run_fp32(_bd(), s, accumulate=False)


def test_fp32_zero_atoms():
    bd = _bd()
    p = bd.Plan((8, 8, 8), 0.2, (True,) * 3, np.zeros((0, 3)), [], [], 4, flags=bd.FLAG_FP32)
    psi = torch.randn(8 * 8 * 8 * 4, dtype=torch.float32, device="cuda")
    keep = psi.clone()
    c = torch.empty(0, dtype=torch.float32, device="cuda")
    p.project(psi, c)
    p.expand(c, psi)
    torch.cuda.synchronize()
    assert torch.equal(psi, keep)
    p.close()


def test_fp32_paper_geometry_sampled():
    """The paper's fcc geometry (11 projections per grid value) at 64 bands:
    sampled atoms and points against the oracle."""
    bd = _bd()
    s = wl.paper_fcc(numax=3, nbands=64)
    psi = wl.psi_for(s, dtype=np.float32)
    w = wl.coeffs_for(s).astype(np.float32)
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    d_psi = _dev(psi)
    c = _host(plan.project(d_psi))
    off = wl.coeff_offsets(s)
    rng = np.random.default_rng(321)
    atoms = np.sort(rng.choice(s.natoms, 8, replace=False))
    sub = s.subset(atoms)
    c_ref, c_abs = oracle.project(*sub.geometry(), psi.astype(np.float64), rbox=sub.rbox,
                                  with_abs=True)
    got = np.concatenate([c[off[a]:off[a + 1]] for a in atoms])
    _assert_close(got, c_ref, c_abs, 3 * _extent(s) + 12, "paper fcc fp32 project")
    d_out = d_psi.clone()
    plan.expand(_dev(w), d_out)
    out = _host(d_out).reshape(-1, s.nbands)
    pts = rng.choice(out.shape[0], 64, replace=False)
    e_ref, e_abs = oracle.expand_at(*s.geometry(), w.astype(np.float64), pts,
                                    psi.reshape(-1, s.nbands)[pts].astype(np.float64),
                                    rbox=s.rbox, with_abs=True)
    k = 3 * 4 + 4 + _overlaps(s)[pts]
    _assert_close(out[pts], e_ref, e_abs, k[:, None], "paper fcc fp32 expand")
    plan.close()


def test_fp32_scale_full_size_sampled():
    """The benchmarked scale workload (periodic 128^3, 512 atoms, nu 5) in FP32
    with 32 bands: sampled atoms and points against the oracle."""
    bd = _bd()
    s = wl.scale()
    psi = wl.psi_for(s, dtype=np.float32)
    w = wl.coeffs_for(s).astype(np.float32)
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    d_psi = _dev(psi)
    c = _host(plan.project(d_psi))
    off = wl.coeff_offsets(s)
    rng = np.random.default_rng(123)
    atoms = np.sort(rng.choice(s.natoms, 10, replace=False))
    sub = s.subset(atoms)
    c_ref, c_abs = oracle.project(*sub.geometry(), psi.astype(np.float64), with_abs=True)
    got = np.concatenate([c[off[a]:off[a + 1]] for a in atoms])
    _assert_close(got, c_ref, c_abs, 3 * _extent(s) + 12, "scale fp32 project")
    d_out = d_psi.clone()
    plan.expand(_dev(w), d_out)
    out = _host(d_out).reshape(-1, s.nbands)
    pts = rng.choice(out.shape[0], 48, replace=False)
    e_ref, e_abs = oracle.expand_at(*s.geometry(), w.astype(np.float64), pts,
                                    psi.reshape(-1, s.nbands)[pts].astype(np.float64),
                                    with_abs=True)
    k = 3 * 6 + 4 + _overlaps(s)[pts]
    _assert_close(out[pts], e_ref, e_abs, k[:, None], "scale fp32 expand")
    plan.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_complex_bands(precision):
    """Complex bands as interleaved (real, imaginary) pairs: c of a complex
    psi is c(Re psi) + i c(Im psi), and the expansion likewise, because the
    SHO functions are real."""
    bd = _bd()
    nb = 5 if precision == "f64" else 6
    s = wl.make_system("complex", (28, 24, 26), 0.2, (True, False, True), 5, 0.6, 4,
                       nb, 91)
    rng = np.random.default_rng(92)
    re = rng.standard_normal(s.psi_shape)
    im = rng.standard_normal(s.psi_shape)
    ctype, rtype = (np.complex128, np.float64) if precision == "f64" else (np.complex64,
                                                                           np.float32)
    psi = (re + 1j * im).astype(ctype)
    s2 = wl.System("complex2", s.n, s.h, s.periodic, s.pos, s.sigma, s.numax, 2 * nb)
    flags = bd.FLAG_FP32 if precision == "f32" else 0
    plan = bd.Plan.from_system(s2, flags=flags)
    d_psi = torch.view_as_real(torch.from_numpy(psi).to("cuda")).reshape(-1)
    c = _host(plan.project(d_psi)).reshape(-1, nb, 2)
    c = c[..., 0].astype(np.float64) + 1j * c[..., 1]
    rre = re.astype(rtype).astype(np.float64)
    rim = im.astype(rtype).astype(np.float64)
    ref_re, abs_re = oracle.project(*s.geometry(), rre, with_abs=True)
    ref_im, abs_im = oracle.project(*s.geometry(), rim, with_abs=True)
    ref_re = ref_re.reshape(-1, nb)
    ref_im = ref_im.reshape(-1, nb)
    if precision == "f64":
        tol_re = 1e-12 * abs_re.reshape(-1, nb)
        tol_im = 1e-12 * abs_im.reshape(-1, nb)
        assert np.all(np.abs(c.real - ref_re) <= tol_re)
        assert np.all(np.abs(c.imag - ref_im) <= tol_im)
    else:
        k = 3 * _extent(s) + 12
        _assert_close(c.real, ref_re, abs_re, k, "complex64 project (real)")
        _assert_close(c.imag, ref_im, abs_im, k, "complex64 project (imag)")
    # expansion of complex coefficients into zeros
    cre = rng.standard_normal(ref_re.shape)
    cim = rng.standard_normal(ref_re.shape)
    cc = (cre + 1j * cim).astype(ctype)
    d_c = torch.view_as_real(torch.from_numpy(cc).to("cuda")).reshape(-1)
    d_out = torch.zeros_like(d_psi)
    plan.expand(d_c, d_out)
    out = _host(d_out).reshape(s.psi_shape + (2,))
    z = np.zeros(s.psi_shape)
    for part, coef in ((0, cc.real), (1, cc.imag)):
        e_ref, e_abs = oracle.expand(*s.geometry(), coef.astype(np.float64).ravel(), z,
                                     with_abs=True)
        if precision == "f64":
            assert np.all(np.abs(out[..., part] - e_ref) <= 1e-12 * e_abs)
        else:
            k = np.repeat(3 * 6 + 4 + _overlaps(s), nb).reshape(s.psi_shape)
            _assert_close(out[..., part], e_ref, e_abs, k, "complex64 expand part %d" % part)
    plan.close()


@pytest.mark.parametrize("form", [(1, 3, 12), (1, 1, 5), (1, 8, 8)])
def test_fp32_block_shapes(form):
    """FP32 expansion with block widths that are not powers of two and with
    partial blocks at the grid's x edge."""
    bd = _bd()
    s = wl.small_mixed()
    c_in = wl.coeffs_for(s).astype(np.float32)
    psi = wl.psi_for(s, dtype=np.float32)
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    plan.set_expand(*form)
    d_acc = _dev(psi)
    plan.expand(_dev(c_in), d_acc)
    a_ref, a_abs = oracle.expand(*s.geometry(), c_in.astype(np.float64),
                                 psi.astype(np.float64), with_abs=True)
    k = np.repeat(3 * (int(s.numax.max()) + 1) + 4 + _overlaps(s), s.nbands)
    _assert_close(_host(d_acc), a_ref, a_abs, k, "fp32 expand form %s" % (form,))
    plan.close()


def test_fp32_tune_keeps_results():
    """The schedule tuner runs on FP32 plans; results stay within the bound."""
    bd = _bd()
    s = wl.small_periodic(nbands=64, natoms=10)
    psi = wl.psi_for(s, dtype=np.float32)
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    d_psi = _dev(psi)
    c0 = _host(plan.project(d_psi))
    d_c = torch.empty(plan.coeff_doubles, dtype=torch.float32, device="cuda")
    r = plan.tune(d_psi, d_c, reps=1)
    assert r["candidates"] >= 2
    c1 = _host(plan.project(d_psi))
    c_ref, c_abs = oracle.project(*s.geometry(), psi.astype(np.float64), with_abs=True)
    for c in (c0, c1):
        _assert_close(c, c_ref, c_abs, 3 * _extent(s) + 12, "tuned fp32 project")
    plan.close()


def test_fp32_argument_errors():
    bd = _bd()
    s = wl.small_periodic(nbands=8, natoms=2)
    with pytest.raises(bd.ShoError) as e:
        bd.Plan.from_system(wl.small_periodic(nbands=7, natoms=2), flags=bd.FLAG_FP32)
    assert e.value.code == bd.SHO_E_INVALID
    for extra in (bd.FLAG_STORED, bd.FLAG_PER_ATOM):
        with pytest.raises(bd.ShoError) as e:
            bd.Plan.from_system(s, flags=bd.FLAG_FP32 | extra)
        assert e.value.code == bd.SHO_E_INVALID
    plan = bd.Plan.from_system(s, flags=bd.FLAG_FP32)
    lib = plan._lib
    psi = torch.zeros(plan.psi_numel, dtype=torch.float32, device="cuda")
    c = torch.zeros(plan.coeff_doubles, dtype=torch.float32, device="cuda")
    vp = ctypes.c_void_p
    # double-precision entry points refuse an FP32 plan (and the reverse)
    assert lib.sho_plan_project(plan._h, vp(psi.data_ptr()), vp(c.data_ptr()),
                                None) == bd.SHO_E_INVALID
    assert lib.sho_plan_expand(plan._h, vp(c.data_ptr()), vp(psi.data_ptr()),
                               None) == bd.SHO_E_INVALID
    g = torch.zeros(3 * s.natoms, dtype=torch.float64, device="cuda")
    assert lib.sho_plan_force(plan._h, vp(psi.data_ptr()), vp(c.data_ptr()),
                              vp(g.data_ptr()), None) == bd.SHO_E_INVALID
    assert lib.sho_plan_set_expand(plan._h, bd.EXPAND_ROWS, 0, 0) == bd.SHO_E_INVALID
    with pytest.raises(TypeError):
        plan.project(psi.double())
    p64 = bd.Plan.from_system(s)
    assert lib.sho_plan_project_f32(p64._h, vp(psi.data_ptr()), vp(c.data_ptr()),
                                    None) == bd.SHO_E_INVALID
    p64.close()
    plan.close()
