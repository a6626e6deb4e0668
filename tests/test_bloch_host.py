"""Host side of Bloch plans (SHO_FLAG_BLOCH), without a GPU: complex band
count and real-element sizes, flag combinations and arguments refused."""
import numpy as np
import pytest

from paper_1905_00480_amd import binding as bd
from paper_1905_00480_amd import workloads as wl


def _lib():
    try:
        return bd.load_library()
    except RuntimeError as e:
        pytest.fail(str(e))


@pytest.mark.parametrize("f32", [False, True])
def test_sizes(f32):
    _lib()
    s = wl.make_system("bh", (16, 14, 12), 0.2, (True, False, True), 4, 0.6, 3, 5, 111)
    flags = bd.FLAG_BLOCH | bd.FLAG_HOST_ONLY | (bd.FLAG_FP32 if f32 else 0)
    p = bd.Plan.from_system(s, flags=flags)
    assert p.info["nbands"] == s.nbands
    rows = int(wl.nsho_count(s.numax).sum())
    assert p.coeff_doubles == 2 * rows * s.nbands   # real and imaginary parts
    assert p.psi_numel == 2 * int(np.prod(s.n)) * s.nbands
    assert p.schedule()[0] == bd.SCHED_SINGLE      # single-launch schedules only
    with pytest.raises(bd.ShoError):
        p.set_schedule(bd.SCHED_BY_NU)
    with pytest.raises(bd.ShoError):
        p.set_expand(bd.EXPAND_OWNER)
    p.set_kpoint((0.3, -0.2, 1.0))
    with pytest.raises(bd.ShoError):
        p.set_kpoint((np.inf, 0.0, 0.0))
    p.close()


def test_refused_combinations_and_wide_supports():
    _lib()
    s = wl.make_system("bh2", (12, 12, 12), 0.2, (True,) * 3, 2, 0.6, 3, 4, 112)
    for extra in (bd.FLAG_STORED, bd.FLAG_PER_ATOM, bd.FLAG_DETERMINISTIC):
        with pytest.raises(bd.ShoError) as err:
            bd.Plan.from_system(s, flags=bd.FLAG_BLOCH | bd.FLAG_HOST_ONLY | extra)
        assert err.value.code == bd.SHO_E_INVALID
    # a support reaching more than 127 images along an axis: 4-point cell,
    # radius of 120 points
    tiny = wl.make_system("bh3", (4, 4, 4), 0.2, (True,) * 3, 1, 0.6, 0, 1, 113)
    with pytest.raises(bd.ShoError) as err:
        bd.Plan.from_system(tiny, flags=bd.FLAG_BLOCH | bd.FLAG_HOST_ONLY,
                            rbox=np.array([0.2 * 4 * 130]))
    assert err.value.code == bd.SHO_E_BOX
    plain = bd.Plan.from_system(s, flags=bd.FLAG_HOST_ONLY)
    with pytest.raises(bd.ShoError):
        plain.set_kpoint((0.1, 0.0, 0.0))
    plain.close()
