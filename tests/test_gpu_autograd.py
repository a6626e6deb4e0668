"""Autograd wrapper: backward through the expansion and derivative kernels,
checked against the CPU oracle, central finite differences with frozen
supports, and torch.autograd.gradcheck on small systems."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00480_amd import autograd, binding
    binding.load_library()
    return binding, autograd


def test_backward_matches_oracle_diff_workload():
    """Isolated 96^3, 256 atoms, nu = 6, 16 bands; L = sum w c."""
    bd, ag = _mods()
    s = wl.diff()
    psi_h = wl.psi_for(s)
    w_h = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    psi = torch.from_numpy(psi_h).cuda().requires_grad_(True)
    pos = torch.from_numpy(s.pos.copy()).requires_grad_(True)
    w = torch.from_numpy(w_h).cuda()
    c = ag.project(psi, pos, plan)
    loss = torch.dot(c, w)
    loss.backward()
    # dL/dR on sampled atoms
    off = oracle.coeff_offsets(s.numax, s.nbands)
    atoms = np.array([3, 77, 200])
    sub = s.subset(atoms)
    wsub = np.concatenate([w_h[off[a]:off[a + 1]] for a in atoms])
    g_ref, g_abs = oracle.force(*sub.geometry(), psi_h, wsub, with_abs=True)
    g = pos.grad.numpy()[atoms]
    assert np.all(np.abs(g - g_ref) <= 1e-12 * g_abs + 1e-300)
    # dL/dpsi at sampled points = h^3 * expansion of w
    gp = psi.grad.detach().cpu().numpy().reshape(-1, s.nbands)
    pts = np.random.default_rng(5).choice(gp.shape[0], 40, replace=False)
    e_ref, e_abs = oracle.expand_at(*s.geometry(), w_h * s.h ** 3, pts, nbands=s.nbands,
                                    with_abs=True)
    assert np.all(np.abs(gp[pts] - e_ref) <= 1e-12 * e_abs + 1e-300)
    plan.close()


def test_position_gradient_finite_differences():
    bd, ag = _mods()
    s = wl.make_system("fdag", (28, 26, 24), 0.2, (True, True, False), 4, 0.6, 5, 8, 81)
    psi = torch.from_numpy(wl.psi_for(s)).cuda()
    w = torch.from_numpy(wl.coeffs_for(s)).cuda()
    plan = bd.Plan.from_system(s)
    pos = torch.from_numpy(s.pos.copy()).requires_grad_(True)
    torch.dot(ag.project(psi, pos, plan), w).backward()
    g = pos.grad.numpy()
    delta = 1e-5
    for a in range(s.natoms):
        for d in range(3):
            pp = s.pos.copy()
            pp[a, d] += delta
            lp = float(torch.dot(ag.project(psi, torch.from_numpy(pp), plan), w))
            pp[a, d] -= 2 * delta
            lm = float(torch.dot(ag.project(psi, torch.from_numpy(pp), plan), w))
            fd = (lp - lm) / (2 * delta)
            assert abs(fd - g[a, d]) <= 1e-7 * max(1.0, abs(g[a, d])), (a, d)
    plan.close()


def test_gradcheck_small():
    """torch.autograd.gradcheck (numerical Jacobians in float64) for psi and
    the centres on a tiny periodic system."""
    bd, ag = _mods()
    s = wl.make_system("gc", (10, 9, 8), 0.25, (True,) * 3, 2, 0.7, 2, 2, 82)
    plan = bd.Plan.from_system(s)
    psi = torch.from_numpy(wl.psi_for(s)).cuda().requires_grad_(True)
    pos = torch.from_numpy(s.pos.copy()).requires_grad_(True)
    f = lambda p, r: ag.project(p, r, plan)
    assert torch.autograd.gradcheck(f, (psi, pos), eps=1e-6, atol=1e-7, rtol=1e-6,
                                    nondet_tol=1e-12)
    plan.close()


def test_direct_set_centres_between_autograd_calls():
    """A direct Plan.set_centres between two autograd projections at the same
    positions: the second must move the centres back (the plan tracks the
    centres it holds), so both equal the oracle at those positions."""
    bd, ag = _mods()
    s = wl.make_system("setc", (24, 22, 20), 0.2, (True,) * 3, 3, 0.6, 4, 4, 83)
    psi_h = wl.psi_for(s)
    plan = bd.Plan.from_system(s)
    psi = torch.from_numpy(psi_h).cuda()
    pos = torch.from_numpy(s.pos.copy())
    c0 = ag.project(psi, pos, plan).cpu().numpy()
    plan.set_centres(s.pos + 0.05)
    c1 = ag.project(psi, pos, plan).cpu().numpy()
    ref, ab = oracle.project(*s.geometry(), psi_h, with_abs=True)
    for c in (c0, c1):
        assert np.all(np.abs(c - ref) <= 1e-12 * ab + 1e-300)
    plan.close()
