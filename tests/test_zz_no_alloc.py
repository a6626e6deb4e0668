"""The allocation-free expansion (sho_plan_expand_noalloc) against the
expansion with the plan's own scratch (sho_plan_expand).

Both run the same kernels; only where the plane partials live differs.  The
bar is that of every expansion parity test: per grid value
|x - x_oracle| <= 1e-12 * A (A: the oracle's abs-sum of the value), for both
entry points, and the two agree within the sum of their bounds.  A
deterministic plan (fixed summation order) must give identical bits.  Two
calls run in a row on one device, the second with a smaller plan, so the
second reads plane partials that the first left in the shared array only if
it fails to overwrite them.  A plan whose plane partials exceed the array is
refused without touching psi."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
CAPACITY = 4194304  # SHO_STATIC_SCRATCH_DOUBLES


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


def _systems():
    big = wl.make_system("noalloc-big", (40, 36, 32), 0.2, (True, True, False), 10, 0.6, 6,
                         24, 71)
    small = wl.make_system("noalloc-small", (20, 18, 16), 0.2, (True, False, True), 3, 0.5, 3,
                           8, 72)
    return big, small


def _check_pair(bd, s, flags):
    plan = bd.Plan.from_system(s, flags=flags)
    assert 0 < plan.info["expand_scratch_doubles"] <= CAPACITY
    c_in = wl.coeffs_for(s)
    psi = wl.psi_for(s)
    ref, ab = oracle.expand(*s.geometry(), c_in, psi, with_abs=True)
    d_c = _dev(c_in)
    own = _dev(psi)
    plan.expand(d_c, own)
    static = _dev(psi)
    plan.expand_noalloc(d_c, static)
    got_own, got_static = _host(own).ravel(), _host(static).ravel()
    bound = RTOL * ab.ravel() + 1e-300
    for name, got in (("own scratch", got_own), ("static scratch", got_static)):
        err = np.abs(got - ref.ravel())
        assert np.all(err <= bound), "%s %s: %d values off, max |d| %.3e" % (
            s.name, name, int((err > bound).sum()), float(err.max()))
    assert np.all(np.abs(got_static - got_own) <= 2 * bound)
    if flags & bd.FLAG_DETERMINISTIC:
        assert np.array_equal(got_static, got_own), s.name + ": deterministic plan, bits differ"
    plan.close()


@pytest.mark.parametrize("det", [False, True])
def test_noalloc_matches_expand_two_calls(det):
    bd = _bd()
    flags = bd.FLAG_DETERMINISTIC if det else 0
    big, small = _systems()
    _check_pair(bd, big, flags)     # first call: the larger plan
    _check_pair(bd, small, flags)   # second call: a smaller one, same array


def test_noalloc_refuses_oversized_plan():
    bd = _bd()
    s = wl.make_system("noalloc-over", (40, 40, 40), 0.2, (True,) * 3, 24, 0.6, 9, 128, 73)
    plan = bd.Plan.from_system(s)
    need = plan.info["expand_scratch_doubles"]
    assert need > CAPACITY
    psi = torch.ones(s.psi_shape, dtype=torch.float64, device="cuda")
    c = torch.ones(plan.coeff_doubles, dtype=torch.float64, device="cuda")
    with pytest.raises(bd.ShoError) as err:
        plan.expand_noalloc(c, psi)
    assert err.value.code == bd.SHO_E_INVALID
    assert "static scratch" in str(err.value)
    assert bool(torch.all(psi == 1.0))
    plan.close()
