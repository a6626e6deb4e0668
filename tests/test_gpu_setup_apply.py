"""End to end: the atomic matrix built by the set-up side (sho_setup_matrix)
drives the non-local application on the GPU (sho_plan_apply), and the result
equals the direct grid evaluation sum_ij |p_i> D_ij <p_j | psi> with the
projectors p_j = P_k(r) Y_lm sampled on the same support.

The radial projectors are chosen inside the span of the SHO basis, so each
sampled p_j equals sum_c M[j][c] Phi_c point by point and both sides are the
same sums up to rounding and the radial quadrature of F (relative 1e-12);
the tolerance is 1e-9 of the abs chain of the direct evaluation.
"""
import numpy as np
import pytest
from scipy import special as sp

import oracle
from oracle import setup as st

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00480_amd import binding
    binding.load_library()
    return binding


def _grid(rmax, n=8001):
    r = np.linspace(0.0, rmax, n)
    w = np.full(n, r[1] - r[0])
    w[1:-1:2] *= 4.0 / 3.0
    w[2:-1:2] *= 2.0 / 3.0
    w[0] *= 1.0 / 3.0
    w[-1] *= 1.0 / 3.0
    return r, w


def _real_ylm(l, m, polar, azim):
    if m == 0:
        return sp.sph_harm_y(l, 0, polar, azim).real
    y = sp.sph_harm_y(l, abs(m), polar, azim) * (-1) ** abs(m)
    return np.sqrt(2.0) * (y.real if m > 0 else y.imag)


# radial projectors in the span of the basis (nu_max = 4): (l, [(nr, weight)])
PROJ = [(0, [(0, 1.0), (1, 0.3)]), (1, [(0, 1.0), (1, -0.5)]), (2, [(0, 1.0), (1, 0.2)])]


def _radial_proj(l, terms, sigma, r):
    return sum(c * st.radial(nr, l, sigma, r) for nr, c in terms)


def test_setup_matrix_drives_apply():
    bd = _bd()
    n, h, nu_max, sigma = (40, 36, 44), 0.2, 4, 0.6
    periodic = (False, False, False)
    pos = np.array([[3.9, 3.5, 4.3], [4.6, 3.8, 4.9]])
    natoms = pos.shape[0]
    rng = np.random.default_rng(17)
    nb = 6
    psi = rng.standard_normal((n[2], n[1], n[0], nb))
    r, w = _grid(8.0)
    ell = [l for l, _ in PROJ]
    P = np.array([_radial_proj(l, t, sigma, r) for l, t in PROJ])
    nproj = sum(2 * l + 1 for l in ell)
    Ds = []
    for a in range(natoms):
        D = rng.normal(size=(nproj, nproj))
        Ds.append(D + D.T)
    Dcal = [bd.setup_matrix(nu_max, sigma, ell, r, w, P, D) for D in Ds]
    # GPU: project, multiply by script-D, expand
    plan = bd.Plan(n, h, periodic, pos, [sigma] * natoms, [nu_max] * natoms, nb)
    off = plan.matrix_offsets()
    Dall = np.zeros(int(off[-1]))
    for a in range(natoms):
        Dall[off[a]:off[a + 1]] = Dcal[a].ravel()
    d_psi = torch.from_numpy(psi).cuda()
    out = torch.zeros_like(d_psi)
    plan.apply(d_psi, torch.from_numpy(Dall).cuda(), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(-1, nb)
    plan.close()
    # direct: sample every projector on the atom's support
    ref = np.zeros_like(got)
    chain = np.zeros_like(got)
    flat = psi.reshape(-1, nb)
    for a in range(natoms):
        R = oracle.box_radius(sigma, nu_max, h)
        idx, mem = oracle.support(n, h, periodic, pos[a], R)
        d = idx * h - pos[a]
        rr = np.linalg.norm(d, axis=1)
        rs = np.where(rr > 0, rr, 1.0)
        polar = np.arccos(np.clip(d[:, 2] / rs, -1, 1))
        azim = np.arctan2(d[:, 1], d[:, 0])
        pj = []
        for l, t in PROJ:
            rad = _radial_proj(l, t, sigma, rr)
            for m in range(-l, l + 1):
                pj.append(rad * _real_ylm(l, m, polar, azim))
        pj = np.array(pj)                       # [nproj][points]
        c = h ** 3 * pj @ flat[mem]             # [nproj][nb]
        ca = h ** 3 * np.abs(pj) @ np.abs(flat[mem])
        np.add.at(ref, mem, pj.T @ (Ds[a] @ c))
        np.add.at(chain, mem, np.abs(pj).T @ (np.abs(Ds[a]) @ ca))
    assert np.all(np.abs(got - ref) <= 1e-9 * chain + 1e-300), np.max(np.abs(got - ref))
    assert np.abs(ref).max() > 1e-3  # the check is not vacuous
