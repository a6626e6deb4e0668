"""The factorised CPU path (the benchmark's CPU reference point) against the
plain triple-sum oracle, on the CPU.

Both compute the projection and expansion of sec. 3.2 in the SHO basis; the
factorised path reorders the sums into x, y and z passes (sec. 3.4), so the
two agree to rounding: |x_fact - x_oracle| <= 1e-12 * A per entry, A the
oracle's abs-sum of the entry.  The systems cover periodic, isolated and mixed
axes, boxes wider than the cell (images that add), several cut-offs, a caller
radius and an atom whose support misses an isolated grid."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

RTOL = 1e-12


def _systems():
    out = {
        "tiny": wl.tiny(),
        "small_periodic": wl.small_periodic(natoms=4, nbands=5),
        "mixed": wl.make_system("mixed", (20, 18, 16), 0.2, (True, False, True), 5, 0.5, 4, 3,
                                 81, numax_range=(0, 6), sigma_range=(0.4, 0.7)),
        "wide": wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 2, 82),
    }
    far = wl.make_system("far", (12, 12, 12), 0.2, (False,) * 3, 2, 0.4, 2, 2, 83)
    far.pos[1] = (-3.0, 1.0, 1.0)  # sphere entirely outside the isolated grid
    out["far"] = far
    return out


@pytest.mark.parametrize("name", sorted(_systems()))
def test_factorised_matches_oracle(name):
    s = _systems()[name]
    psi = wl.psi_for(s)
    c_in = wl.coeffs_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    c_fact = oracle.factorised_project(*s.geometry(), psi)
    assert np.all(np.abs(c_fact - c_ref) <= RTOL * c_abs + 1e-300)
    e_ref, e_abs = oracle.expand(*s.geometry(), c_in, psi, with_abs=True)
    e_fact = oracle.factorised_expand(*s.geometry(), c_in, psi.copy())
    assert np.all(np.abs(e_fact - e_ref) <= RTOL * e_abs + 1e-300)


def test_factorised_caller_radius():
    s = wl.small_periodic(natoms=3, nbands=4)
    rbox = np.full(s.natoms, 1.7)
    psi = wl.psi_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, rbox=rbox, with_abs=True)
    c_fact = oracle.factorised_project(*s.geometry(), psi, rbox=rbox)
    assert np.all(np.abs(c_fact - c_ref) <= RTOL * c_abs + 1e-300)
    c_in = wl.coeffs_for(s)
    e_ref, e_abs = oracle.expand(*s.geometry(), c_in, psi, rbox=rbox, with_abs=True)
    e_fact = oracle.factorised_expand(*s.geometry(), c_in, psi.copy(), rbox=rbox)
    assert np.all(np.abs(e_fact - e_ref) <= RTOL * e_abs + 1e-300)


def test_factorised_detects_a_planted_mistake():
    """A dropped plane in the factorised sums (here: psi zeroed on one plane
    the support crosses) moves coefficients by O(A): the bound above is tight
    enough to see it."""
    s = wl.small_periodic(natoms=2, nbands=3)
    psi = wl.psi_for(s)
    c_ref, c_abs = oracle.project(*s.geometry(), psi, with_abs=True)
    z = int(round(s.pos[0][2] / s.h)) % s.n[2]
    bad = psi.copy()
    bad[z] = 0.0
    c_fact = oracle.factorised_project(*s.geometry(), bad)
    assert np.any(np.abs(c_fact - c_ref) > RTOL * c_abs)
