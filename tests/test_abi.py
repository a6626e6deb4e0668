"""C ABI of libsho.so checked without a GPU: exported symbols, argument
validation and the host-side support tables (bit-exact against the oracle's
support, which decides membership in the same IEEE double operation order).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import binding as bd
from paper_1905_00480_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sho.h")


def _lib():
    try:
        return bd.load_library()
    except RuntimeError as e:  # library not built
        pytest.fail(str(e))


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sho_[a-z0-9_]+)\s*\(", txt)))


def test_header_declarations_are_exported():
    lib = _lib()
    names = _declared()
    assert set(names) == set(bd.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_nsho():
    _lib()
    for nu in range(12):
        assert bd.nsho(nu) == oracle.nsho(nu)
    assert bd.nsho(-1) == -1


def _host_plan(s, flags=0, rbox=None):
    return bd.Plan(s.n, s.h, s.periodic, s.pos, s.sigma, s.numax, s.nbands,
                   rbox=rbox, flags=flags | bd.FLAG_HOST_ONLY)


def _expect(code, fn):
    with pytest.raises(bd.ShoError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_argument_errors():
    _lib()
    s = wl.small_periodic(natoms=2)
    mk = lambda **kw: bd.Plan(**{**dict(n=s.n, h=s.h, periodic=s.periodic, pos=s.pos,
                                        sigma=s.sigma, numax=s.numax, nbands=4,
                                        flags=bd.FLAG_HOST_ONLY), **kw})
    _expect(bd.SHO_E_INVALID, lambda: mk(nbands=0))
    _expect(bd.SHO_E_INVALID, lambda: mk(h=-0.2))
    _expect(bd.SHO_E_INVALID, lambda: mk(n=(0, 4, 4)))
    _expect(bd.SHO_E_INVALID, lambda: mk(sigma=[0.6, 0.0]))
    _expect(bd.SHO_E_INVALID, lambda: mk(pos=np.array([[np.nan, 0, 0], [1, 1, 1]])))
    _expect(bd.SHO_E_INVALID, lambda: mk(flags=bd.FLAG_HOST_ONLY | 0x100))
    _expect(bd.SHO_E_NU_RANGE, lambda: mk(numax=[5, 11]))
    _expect(bd.SHO_E_NU_RANGE, lambda: mk(numax=[-1, 3]))
    # h > pi sigma / sqrt(2 nu + 1): sigma = 0.1, nu = 5 gives h_max = 0.095
    _expect(bd.SHO_E_UNDERSAMPLED, lambda: mk(sigma=[0.1, 0.6]))
    mk(sigma=[0.1, 0.6], flags=bd.FLAG_HOST_ONLY | bd.FLAG_ALLOW_UNDERSAMPLED).close()
    # box wider than the on-chip tables allow
    _expect(bd.SHO_E_BOX, lambda: bd.Plan((2000, 8, 8), 0.2, (False,) * 3,
                                          [[200.0, 0.8, 0.8]], [0.6], [3], 1,
                                          rbox=[120.0], flags=bd.FLAG_HOST_ONLY))
    _expect(bd.SHO_E_INVALID, lambda: mk(rbox=[1.0, -1.0]))
    # the kernels address a grid line (n[0] * nbands values) in 32-bit integers
    _expect(bd.SHO_E_INVALID, lambda: mk(n=(1 << 16, 4, 4), nbands=1 << 15))
    _expect(bd.SHO_E_INVALID, lambda: mk(nbands=1 << 24))
    # deterministic sums are FP64, on-the-fly, batched only
    for other in (bd.FLAG_STORED, bd.FLAG_PER_ATOM, bd.FLAG_FP32):
        _expect(bd.SHO_E_INVALID,
                lambda: mk(flags=bd.FLAG_HOST_ONLY | bd.FLAG_DETERMINISTIC | other))
    # stored projector tables are offered up to nu = 5 only
    _expect(bd.SHO_E_NU_RANGE, lambda: mk(numax=[5, 6],
                                          flags=bd.FLAG_HOST_ONLY | bd.FLAG_STORED))
    mk(numax=[5, 4], flags=bd.FLAG_HOST_ONLY | bd.FLAG_STORED).close()


def test_schedule_arguments_host_only():
    """Schedules can be set on host-only plans (sizing); bad values refused."""
    _lib()
    s = wl.small_mixed()
    s.numax = np.array([0, 3, 6, 9, 10, 7, 4, 8])
    p = _host_plan(s, flags=bd.FLAG_PER_ATOM)
    sc, tile, tp = p.schedule()
    assert sc == bd.SCHED_SINGLE and tp == 16384 and tile & (tile - 1) == 0
    for sched in bd.SCHEDULES:
        p.set_schedule(sched, tile // 2, 4096)
        assert p.schedule() == (sched, tile // 2, 4096)
    _expect(bd.SHO_E_INVALID, lambda: p.set_schedule(-1, 0, 4096))
    _expect(bd.SHO_E_INVALID, lambda: p.set_schedule(8, 0, 4096))
    _expect(bd.SHO_E_INVALID, lambda: p.set_schedule(12, 0, 4096))
    _expect(bd.SHO_E_INVALID, lambda: p.set_schedule(0, 3, 4096))
    _expect(bd.SHO_E_INVALID, lambda: p.set_schedule(0, 0, 10))
    # nu_max + 1 = 11 coefficients tile (364 functions) at twice the widest
    # tile no longer fits 63 KiB of LDS
    _expect(bd.SHO_E_BOX, lambda: p.set_schedule(0, 2 * tile, 4096))
    p.close()
    one = _host_plan(wl.small_periodic(natoms=3))
    assert one.schedule()[0] == bd.SCHED_BY_NU
    one.close()


def test_expand_form_arguments_host_only():
    _lib()
    s = wl.scale()
    p = _host_plan(s)
    mode, R, X = p.expand_form()
    assert mode == bd.EXPAND_BLOCKS and R * X * 32 <= 4096 and X * 8 <= 256
    p.set_expand(bd.EXPAND_ROWS)
    assert p.expand_form()[0] == bd.EXPAND_ROWS
    p.set_expand(bd.EXPAND_BLOCKS, 8, 16)
    assert p.expand_form() == (bd.EXPAND_BLOCKS, 8, 16)
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(3))
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(bd.EXPAND_BLOCKS, 16, 16))   # 8192 doubles
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(bd.EXPAND_BLOCKS, 1, 64))    # staging
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(bd.EXPAND_BLOCKS, 0, 4))
    p.close()


def test_host_only_plan_refuses_compute():
    lib = _lib()
    s = wl.small_periodic(natoms=2)
    p = _host_plan(s)
    code = lib.sho_plan_project(p._h, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert code == bd.SHO_E_INVALID
    p.close()


@pytest.mark.parametrize("case", ["periodic", "mixed", "wide", "isolated_edge"])
def test_support_tables_match_oracle(case):
    """Per-atom support sizes and coefficient offsets equal the oracle's
    exactly (integer work: bit-exact)."""
    _lib()
    if case == "periodic":
        s = wl.small_periodic(natoms=12, nbands=3)
    elif case == "mixed":
        s = wl.small_mixed()
    elif case == "wide":  # boxes wider than the cell: several images
        s = wl.make_system("wide", (8, 9, 7), 0.2, (True,) * 3, 3, 0.6, 3, 2, 41)
    else:  # atoms near and beyond the faces of an isolated grid
        s = wl.make_system("edge", (20, 16, 12), 0.25, (False,) * 3, 6, 0.5, 4, 2, 42)
        s.pos[0] = [-0.3, 1.0, 1.0]
        s.pos[1] = [5.2, 4.1, 3.2]
        s.pos[2] = [-9.0, 1.0, 1.0]   # support misses the grid entirely
    p = _host_plan(s)
    cnt = p.support_counts()
    for a in range(s.natoms):
        R = oracle.box_radius(s.sigma[a], s.numax[a], s.h)
        idx, mem = oracle.support(s.n, s.h, s.periodic, s.pos[a], R)
        assert cnt[a] == len(mem), (case, a)
    assert np.array_equal(p.coeff_offsets(), oracle.coeff_offsets(s.numax, s.nbands))
    assert p.support_points == int(cnt.sum())
    p.close()


def test_workload_scale_geometry_counts():
    """The scale workload's support sizes (used by the throughput metric)."""
    _lib()
    s = wl.scale()
    p = _host_plan(s)
    cnt = p.support_counts()
    R = oracle.box_radius(0.6, 5, 0.2)
    for a in (0, 17, 511):
        assert cnt[a] == len(oracle.support(s.n, s.h, s.periodic, s.pos[a], R)[1])
    # sphere of radius 2.563 Bohr at h = 0.2: about (4/3) pi (R/h)^3 points
    assert abs(cnt.mean() / (4 / 3 * np.pi * (R / 0.2) ** 3) - 1) < 0.02
    p.close()


def test_paper_fcc_geometry():
    """The benchmark geometry of sec. 6: 64^3 points at h = 0.25 Angstrom,
    fcc a = 4.08 Angstrom, projection spheres of 3.55 Angstrom.  The paper
    states that each grid value enters about eleven projections (figure of
    the test system) and that 241 atoms lie inside the 16 Angstrom domain
    (four per 4.08^3 cell); both follow from this construction."""
    _lib()
    s = wl.paper_fcc(nbands=4)
    p = _host_plan(s, rbox=s.rbox)
    per_point = p.support_points / np.prod(s.n)
    assert round(per_point) == 11, per_point
    # 4 atoms per cubic cell of 4.08 A in a (16 A)^3 domain
    assert round(4 * (16.0 / 4.08) ** 3) == 241
    R = float(s.rbox[0])
    assert abs(R - 3.55 / 0.529177210903) < 1e-12
    cnt = p.support_counts()
    assert cnt.max() == len(oracle.support(s.n, s.h, s.periodic, s.pos[int(np.argmax(cnt))], R)[1])
    assert 600 <= s.natoms <= 700   # the paper counts 665 with its own boundary rule
    p.close()


def test_device_plan_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _lib()
    s = wl.small_periodic(natoms=2)
    _expect(bd.SHO_E_DEVICE, lambda: bd.Plan.from_system(s))


def test_deterministic_host_plan_tables():
    """A deterministic plan takes the owner form of the expansion (strips of
    64 / T rows, T = 16 bands, or 8 for at most 8 bands), one work item per
    atom, and refuses the other expansion forms."""
    _lib()
    s = wl.small_mixed()
    p = _host_plan(s, flags=bd.FLAG_DETERMINISTIC)
    mode, rows, width = p.expand_form()
    assert mode == bd.EXPAND_OWNER and rows == (4 if s.nbands > 8 else 8) and width == 32
    p.set_expand(bd.EXPAND_OWNER, 0, 16)
    assert p.expand_form() == (bd.EXPAND_OWNER, rows, 16)
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(bd.EXPAND_BLOCKS))
    _expect(bd.SHO_E_INVALID, lambda: p.set_expand(bd.EXPAND_OWNER, 0, 24))
    p.set_schedule(bd.SCHED_SINGLE, 0, 256)   # would split large atoms
    p.close()
    q = _host_plan(s)
    q.set_expand(bd.EXPAND_OWNER)
    assert q.expand_form()[0] == bd.EXPAND_OWNER
    _expect(bd.SHO_E_INVALID, lambda: q.set_expand(bd.EXPAND_OWNER, 3, 32))
    q.close()
