"""Set-up side (host code of libsho.so, no GPU) against the pinned set-up
oracle: the Cartesian-to-radial map U, the radial functions, the atomic
matrix in the Cartesian basis and the representation quality.

Tolerances: U entries are bounded by 1 and both sides are exact up to
rounding (exact rational sums on the oracle side, an exact Gauss-Hermite rule
with (nu+1)^3 nodes on the library side), so 1e-13 absolute.  Radial values
and Q are single sums of at most ~10^4 terms: 1e-12 relative to the largest
value.  The atomic matrix is compared per entry with 1e-12 times the abs
chain (|M|^T |D| |M|)(a, b), which bounds every rounding of the products
and sums of both sides, plus 1e-13 times the largest chain entry: the
library's quadrature leaves entries of U that are exactly zero at ~1e-16
instead of 0, which moves entries whose exact chain vanishes by that much
relative to the matrix scale.
"""
import ctypes

import numpy as np
import pytest

from oracle import setup as st
from paper_1905_00480_amd import binding as bd


def _grid(rmax, n=4001):
    r = np.linspace(0.0, rmax, n)
    w = np.full(n, r[1] - r[0])
    w[1:-1:2] *= 4.0 / 3.0
    w[2:-1:2] *= 2.0 / 3.0
    w[0] *= 1.0 / 3.0
    w[-1] *= 1.0 / 3.0
    return r, w


def _transition_metal_like(r, seed=3):
    """18 projectors: two radial functions each for s, p and d (the count the
    paper quotes per transition metal), smooth synthetic shapes."""
    rng = np.random.default_rng(seed)
    ell = [0, 0, 1, 1, 2, 2]
    P = []
    for l in ell:
        a = rng.uniform(0.5, 0.9)
        c1, c2 = rng.normal(size=2)
        P.append(r ** l * (1.0 + c1 * r + 0.2 * c2 * r * r) * np.exp(-r * r / (2 * a * a)))
    return ell, np.array(P)


@pytest.mark.parametrize("nu_max", list(range(11)))
def test_unitary_matches_oracle(nu_max):
    U = bd.setup_unitary(nu_max)
    assert np.abs(U - st.unitary(nu_max)).max() < 1e-13


def test_radial_matches_oracle():
    r, _ = _grid(12.0, 501)
    for sig in (0.4, 1.3):
        R = bd.setup_radial(10, sig, r)
        k = 0
        for nu in range(11):
            for l in range(nu % 2, nu + 1, 2):
                ref = st.radial((nu - l) // 2, l, sig, r)
                assert np.abs(R[k] - ref).max() <= 1e-12 * np.abs(ref).max(), (nu, l)
                k += 1


@pytest.mark.parametrize("nu_max,sigma", [(4, 0.6), (5, 0.7), (8, 0.55)])
def test_atomic_matrix_matches_oracle(nu_max, sigma):
    r, w = _grid(10.0)
    ell, P = _transition_metal_like(r)
    nproj = sum(2 * l + 1 for l in ell)
    assert nproj == 18
    rng = np.random.default_rng(nu_max)
    D = rng.normal(size=(nproj, nproj))
    D = D + D.T
    got = bd.setup_matrix(nu_max, sigma, ell, r, w, P, D)
    ref = st.setup_matrix(nu_max, sigma, ell, r, w, P, D)
    M = st.F_matrix(nu_max, sigma, ell, r, w, P) @ st.unitary(nu_max).T
    chain = np.abs(M).T @ np.abs(D) @ np.abs(M)
    assert np.all(np.abs(got - ref) <= 1e-12 * chain + 1e-13 * chain.max())
    assert np.abs(got - got.T).max() <= 1e-12 * chain.max()


def test_quality_matches_oracle():
    r, w = _grid(25.0, 20001)
    for l in (0, 1, 2, 3):
        P = r ** l * (1.0 - 0.2 * r) * np.exp(-r * r / 2.2)
        got = bd.setup_quality(30 + l, 0.9, l, r, w, P)
        ref = st.quality(30 + l, 0.9, l, r, w, P)
        assert np.abs(got - ref).max() < 1e-12


def test_setup_argument_errors():
    lib = bd.load_library()
    U = np.empty(4)
    assert lib.sho_setup_unitary(-1, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) \
        == bd.SHO_E_NU_RANGE
    assert lib.sho_setup_unitary(bd.SHO_NU_MAX + 1, U.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double))) == bd.SHO_E_NU_RANGE
    assert lib.sho_setup_unitary(1, None) == bd.SHO_E_INVALID
    r, w = _grid(5.0, 11)
    with pytest.raises(bd.ShoError) as e:
        bd.setup_quality(4, -1.0, 0, r, w, np.exp(-r * r))
    assert e.value.code == bd.SHO_E_INVALID
    with pytest.raises(bd.ShoError) as e:
        bd.setup_quality(4, 1.0, 0, r, w, np.zeros_like(r))
    assert e.value.code == bd.SHO_E_INVALID
    with pytest.raises(bd.ShoError) as e:
        bd.setup_matrix(4, 1.0, [-1], r, w, np.exp(-r * r)[None, :], np.eye(1))
    assert e.value.code == bd.SHO_E_INVALID
    with pytest.raises(bd.ShoError) as e:
        bd.setup_radial(bd.SHO_SETUP_NU_MAX + 1, 1.0, r)
    assert e.value.code == bd.SHO_E_NU_RANGE
