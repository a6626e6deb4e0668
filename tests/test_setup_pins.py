"""Pins of the set-up oracle (oracle/setup.py): the Cartesian-to-radial map U
of sec. 2.5, the radial SHO functions of sec. 2.3, the transformed atomic
matrix of sec. 3.5 and the representation quality Q of sec. 4.

Each pin is fixed by something other than the oracle's own arithmetic:
orthogonality (both bases are orthonormal), the l = 1 shell by inspection,
pointwise reconstruction against scipy's Hermite, Laguerre and spherical
harmonic routines, closed forms of Q for Gaussian projectors, the identity
for a complete set of projectors, and the grid projection oracle (pinned in
test_oracle_pins.py) for the Cartesian coefficients of a radial projector.
"""
import numpy as np
import pytest
from scipy import special as sp

import oracle
from oracle import setup as st


def _grid(rmax, n=20001):
    r = np.linspace(0.0, rmax, n)
    w = np.full(n, r[1] - r[0])
    w[1:-1:2] *= 4.0 / 3.0
    w[2:-1:2] *= 2.0 / 3.0
    w[0] *= 1.0 / 3.0
    w[-1] *= 1.0 / 3.0
    return r, w


def _real_ylm(l, m, polar, azim):
    """Real harmonics without the Condon-Shortley sign from scipy's complex ones."""
    if m == 0:
        return sp.sph_harm_y(l, 0, polar, azim).real
    y = sp.sph_harm_y(l, abs(m), polar, azim) * (-1) ** abs(m)
    return np.sqrt(2.0) * (y.real if m > 0 else y.imag)


def _phi1d(n, x):
    return sp.eval_hermite(n, x) * np.exp(-0.5 * x * x) / np.sqrt(
        2.0 ** n * sp.factorial(n) * np.sqrt(np.pi))


def test_unitary_is_orthogonal():
    U = st.unitary(8)
    assert np.abs(U @ U.T - np.eye(U.shape[0])).max() < 1e-13


def test_unitary_block_diagonal_in_nu():
    U = st.unitary(6)
    cart = st.cartesian_states(6)
    rad = st.radial_states(6)
    for c, (x, y, z) in enumerate(cart):
        for s, (nu, l, m, nr) in enumerate(rad):
            if x + y + z != nu:
                assert U[c, s] == 0.0


def test_p_shell_by_inspection():
    """phi_1(x) phi_0 phi_0 is the x-type p function = +Y_11 (no CS sign)."""
    U = st.unitary(1)
    # coefficient order: 000, 100 (x), 010 (y), 001 (z); radial: s, m=-1 (y), 0 (z), +1 (x)
    expect = np.zeros((4, 4))
    expect[0, 0] = 1.0
    expect[1, 3] = 1.0
    expect[2, 1] = 1.0
    expect[3, 2] = 1.0
    assert np.allclose(U, expect, atol=1e-15)


def test_pointwise_reconstruction_against_scipy():
    """Phi_c(r) = sum_s U[c][s] Psi_s(r) at random points, both sides from scipy."""
    nu_max = 6
    U = st.unitary(nu_max)
    rng = np.random.default_rng(5)
    pts = rng.normal(scale=1.2, size=(12, 3))
    cart = st.cartesian_states(nu_max)
    rad = st.radial_states(nu_max)
    for p in pts:
        x, y, z = p
        r = np.linalg.norm(p)
        polar = np.arccos(z / r)
        azim = np.arctan2(y, x)
        phi = np.array([_phi1d(a, x) * _phi1d(b, y) * _phi1d(c, z) for a, b, c in cart])
        psi = np.array([st.radial(nr, l, 1.0, r) * _real_ylm(l, m, polar, azim)
                        for nu, l, m, nr in rad])
        assert np.abs(phi - U @ psi).max() < 1e-12


def test_radial_normalisation_and_orthogonality():
    r, w = _grid(20.0)
    for l in range(4):
        R = [st.radial(nr, l, 0.8, r) for nr in range(4)]
        G = np.array([[np.sum(w * r * r * a * b) for b in R] for a in R])
        assert np.abs(G - np.eye(4)).max() < 1e-10


def test_quality_of_a_basis_function_is_a_step():
    r, w = _grid(15.0)
    for nr, l in ((0, 0), (1, 2), (2, 1)):
        P = st.radial(nr, l, 0.7, r)
        Q = st.quality(8, 0.7, l, r, w, P)
        nu0 = l + 2 * nr
        assert np.all(np.abs(Q[:nu0]) < 1e-12)
        assert np.all(np.abs(Q[nu0:] - 1.0) < 1e-10)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_quality_gaussian_closed_form(l):
    """P = r^l exp(-r^2/(2 s'^2)): Q_l = (2 s s' / (s^2 + s'^2))^(2l+3), Q grows
    with nu and approaches 1 (completeness of the radial SHO set)."""
    sig, sig2 = 1.0, 1.4
    r, w = _grid(25.0, 40001)
    P = r ** l * np.exp(-r * r / (2 * sig2 ** 2))
    Q = st.quality(l + 40, sig, l, r, w, P)
    assert abs(Q[l] - (2 * sig * sig2 / (sig ** 2 + sig2 ** 2)) ** (2 * l + 3)) < 1e-10
    assert np.all(np.diff(Q[l:]) >= -1e-14)
    assert Q[-1] > 1.0 - 1e-5


def test_setup_matrix_identity_for_a_complete_projector_set():
    """Projectors = every radial SHO state up to nu_max, D = I: the operator
    sum_j |p_j><p_j| is the identity on the basis, so script-D = I."""
    nu_max, sig = 4, 0.9
    r, w = _grid(15.0)
    ell, P = [], []
    for nu in range(nu_max + 1):
        for l in range(nu % 2, nu + 1, 2):
            ell.append(l)
            P.append(st.radial((nu - l) // 2, l, sig, r))
    nproj = sum(2 * l + 1 for l in ell)
    Dc = st.setup_matrix(nu_max, sig, ell, r, w, np.array(P), np.eye(nproj))
    assert np.abs(Dc - np.eye(st.nsho(nu_max))).max() < 1e-10


def test_cartesian_coefficients_match_the_grid_projection():
    """M[j][c] = <p_j | Phi_c> equals the projection of p_j sampled on a fine
    grid (the pinned projection oracle) -- ties U, the radial functions, the
    harmonics' signs and the coefficient order to the projection kernel's."""
    nu_max, sig = 4, 0.6
    h, n = 0.075, 96
    centre = np.full(3, (n // 2) * h)
    r, w = _grid(12.0)
    sig_p = 0.45
    ell = [1, 2]
    P = np.array([r * np.exp(-r * r / (2 * sig_p ** 2)),
                  r * r * (1.0 - 0.3 * r) * np.exp(-r * r / (2 * sig_p ** 2))])
    F = st.F_matrix(nu_max, sig, ell, r, w, P)
    M = F @ st.unitary(nu_max).T
    # sample every projector on the grid: p_j = P_k(r) Y_lm
    idx = np.arange(n) * h - centre[0]
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    R = np.sqrt(X * X + Y * Y + Z * Z)
    Rs = np.where(R > 0, R, 1.0)
    polar = np.arccos(np.clip(Z / Rs, -1, 1))
    azim = np.arctan2(Y, X)
    cols = []
    for k, l, m in st.projector_list(ell):
        Pk = (R * np.exp(-R * R / (2 * sig_p ** 2)) if k == 0 else
              R * R * (1.0 - 0.3 * R) * np.exp(-R * R / (2 * sig_p ** 2)))
        cols.append(Pk * _real_ylm(l, m, polar, azim))
    psi = np.stack(cols, axis=-1)
    c = oracle.project((n, n, n), h, (False,) * 3, centre[None, :], [sig], [nu_max], psi,
                       rbox=[(n // 2 - 1) * h])
    c = c.reshape(st.nsho(nu_max), -1).T  # [j][c]
    scale = np.abs(M).max()
    assert np.abs(c - M).max() < 1e-9 * scale
