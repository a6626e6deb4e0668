"""Host side of stored numerical-projector plans (sho_plan_create_radial),
without a GPU: coefficient layout [nproj][B] per atom, supports equal to the
oracle's sphere of radius rcut, and argument refusals."""
import numpy as np
import pytest

import oracle
from oracle import radial
from paper_1905_00480_amd import binding as bd
from paper_1905_00480_amd import workloads as wl


def _lib():
    try:
        return bd.load_library()
    except RuntimeError as e:
        pytest.fail(str(e))


def test_layout_and_supports():
    _lib()
    s = wl.make_system("rh", (20, 18, 16), 0.2, (True, False, True), 5, 0.6, 0, 12, 95)
    rcut = np.array([1.2, 1.5, 1.9, 2.2, 0.9])
    ell, dr, tab = wl.radial_set(2.2, nr=100)
    npj = radial.nproj(ell)
    assert npj == 18
    p = bd.Plan.radial(s.n, s.h, s.periodic, s.pos, rcut, ell, dr, tab, s.nbands,
                       flags=bd.FLAG_HOST_ONLY)
    assert p.coeff_doubles == s.natoms * npj * s.nbands
    assert np.array_equal(p.coeff_offsets(), np.arange(s.natoms + 1) * npj * s.nbands)
    cnt = p.support_counts()
    for a in range(s.natoms):
        assert cnt[a] == len(oracle.support(s.n, s.h, s.periodic, s.pos[a], rcut[a])[1])
    p.close()


@pytest.mark.parametrize("what", ["l4", "too_many", "short_table", "bad_dr", "bad_rcut",
                                  "nan_table", "flags"])
def test_refusals(what):
    _lib()
    s = wl.make_system("rr", (12, 12, 12), 0.2, (True,) * 3, 2, 0.6, 0, 4, 96)
    rcut = np.full(s.natoms, 1.5)
    ell, dr, tab = wl.radial_set(1.5, nr=40)
    flags = bd.FLAG_HOST_ONLY
    if what == "l4":
        ell = np.array([0, 4])
        tab = tab[:2]
    elif what == "too_many":
        ell = np.full(8, 3)  # 56 + 7 > 56
        ell = np.concatenate([ell, [3]])
        tab = np.tile(tab[:1], (ell.size, 1))
    elif what == "short_table":
        tab = tab[:, :3]
    elif what == "bad_dr":
        dr = 0.0
    elif what == "bad_rcut":
        rcut[1] = -1.0
    elif what == "nan_table":
        tab = tab.copy()
        tab[2, 5] = np.nan
    elif what == "flags":
        flags |= bd.FLAG_STORED
    with pytest.raises(bd.ShoError) as err:
        bd.Plan.radial(s.n, s.h, s.periodic, s.pos, rcut, ell, dr, tab, s.nbands, flags=flags)
    assert err.value.code == bd.SHO_E_INVALID
