"""The named workloads at full size, checked on what their configurations
claim.

* Differentiation (isolated 96^3, h 0.2, 256 atoms, sigma 0.6, nu 6, 16 bands,
  L = sum w c): central differences (delta = 1e-5 Bohr, supports frozen) of
  the GPU projection for all 768 coordinates against the derivative kernel,
  and 1000 random entries of dL/dpsi (through the autograd Function) against
  central differences of L in psi.  Each c_a depends on R_a only, so one
  projection with every atom shifted along the same axis gives the
  differences of all atoms at once (6 projections for 768 coordinates).
  Bounds: the truncation error of the central difference is O(delta^2) and
  its rounding ~ eps A / delta (A = sum |w| |c| / sigma of the atom), far
  below 1e-7 A; L is linear in psi, so its differences are exact up to the
  rounding of the dot products (<= 1e-13 sum |w c|).
* Batching (periodic 160^3, 2048 atoms, nu 3..9, 64 bands): the derivative of
  sampled atoms (the smallest, the largest, random ones) against the oracle.
* Serving: eight systems of the request-stream pool (grids up to 160^3,
  up to 128 bands, cut-offs up to 9), every job of every system submitted
  interleaved over four streams; coefficients and derivatives of sampled
  atoms and expanded values at sampled points against the oracle.
All oracle comparisons use the abs-sum bound of the other parity tests,
|x - x_oracle| <= 1e-12 A."""
import numpy as np
import pytest

import oracle
from paper_1905_00480_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00480_amd import binding
    binding.load_library()
    return binding


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _parity(got, ref, ab, what):
    err = np.abs(np.ravel(got) - np.ravel(ref))
    bound = RTOL * np.ravel(ab) + 1e-300
    assert np.all(err <= bound), "%s: %d entries off, max |d| %.3e" % (
        what, int((err > bound).sum()), float(err.max()) if err.size else 0.0)


def test_diff_config_all_coordinates():
    bd = _bd()
    s = wl.diff()
    psi = torch.from_numpy(wl.psi_for(s)).cuda()
    w = wl.coeffs_for(s)
    d_w = torch.from_numpy(w).cuda()
    plan = bd.Plan.from_system(s)
    g = _host(plan.force(psi, d_w))
    off = wl.coeff_offsets(s)
    delta = 1e-5
    fd = np.zeros((s.natoms, 3))
    mag = np.zeros((s.natoms, 3))
    for d in range(3):
        pp = s.pos.copy()
        pp[:, d] += delta
        plan.set_centres(pp)
        cp = _host(plan.project(psi))
        pp[:, d] -= 2 * delta
        plan.set_centres(pp)
        cm = _host(plan.project(psi))
        for a in range(s.natoms):
            sl = slice(off[a], off[a + 1])
            fd[a, d] = np.dot(w[sl], cp[sl] - cm[sl]) / (2 * delta)
            mag[a, d] = np.dot(np.abs(w[sl]), np.abs(cp[sl]) + np.abs(cm[sl])) / (2 * s.sigma[a])
    plan.set_centres(s.pos)
    err = np.abs(fd - g)
    bound = 1e-7 * np.maximum(mag, np.abs(g))
    assert np.all(err <= bound), (int((err > bound).sum()), float(np.max(err / bound)))
    # the differences see the derivative, not noise: typical |g| far above the bound
    assert np.median(np.abs(g) / bound) > 1e3
    plan.close()


def test_diff_config_dpsi_finite_differences():
    bd = _bd()
    from paper_1905_00480_amd import autograd
    s = wl.diff()
    psi = torch.from_numpy(wl.psi_for(s)).cuda().requires_grad_(True)
    w = torch.from_numpy(wl.coeffs_for(s)).cuda()
    plan = bd.Plan.from_system(s)
    pos = torch.from_numpy(s.pos.copy())
    c = autograd.project(psi, pos, plan)
    loss = torch.dot(c, w)
    loss.backward()
    gpsi = psi.grad.detach().reshape(-1)
    x = psi.detach().clone()
    flat = x.view(-1)
    rng = np.random.default_rng(31)
    idx = rng.choice(flat.numel(), 1000, replace=False)
    # only entries inside some support have a nonzero derivative: draw half of
    # them from the support points
    cnt = plan.support_counts()
    inside = []
    for a in rng.choice(s.natoms, 50, replace=False):
        R = oracle.box_radius(s.sigma[a], s.numax[a], s.h)
        mem = oracle.support(s.n, s.h, s.periodic, s.pos[a], R)[1]
        inside.append(mem[rng.integers(mem.size, size=10)] * s.nbands +
                      rng.integers(s.nbands, size=10))
    idx[:500] = np.concatenate(inside)[:500]
    assert cnt.sum() > 0
    wabs = torch.abs(w)
    fd = np.zeros(idx.size)
    scale = np.zeros(idx.size)
    for k, i in enumerate(idx):
        i = int(i)
        v = float(flat[i])
        flat[i] = v + 1.0
        cp = plan.project(x)
        lp = float(torch.dot(cp, w))
        flat[i] = v - 1.0
        cm = plan.project(x)
        lm = float(torch.dot(cm, w))
        flat[i] = v
        fd[k] = (lp - lm) / 2.0
        scale[k] = float(torch.dot(torch.abs(cp), wabs))
    got = _host(gpsi)[idx]
    err = np.abs(fd - got)
    bound = 1e-13 * scale
    assert np.all(err <= bound), (int((err > bound).sum()), float(np.max(err / bound)))
    assert np.count_nonzero(got[:500]) > 400
    plan.close()


def test_batching_config_force_sampled():
    bd = _bd()
    s = wl.batching()
    psi_h = wl.psi_for(s)
    w = wl.coeffs_for(s)
    plan = bd.Plan.from_system(s)
    g = _host(plan.force(torch.from_numpy(psi_h).cuda(), torch.from_numpy(w).cuda()))
    rng = np.random.default_rng(3)
    sizes = s.sigma * np.sqrt(2 * s.numax + 3)
    atoms = np.unique(np.concatenate([[np.argmin(sizes), np.argmax(sizes)],
                                      rng.choice(s.natoms, 4, replace=False)]))
    off = wl.coeff_offsets(s)
    sub = s.subset(atoms)
    wsub = np.concatenate([w[off[a]:off[a + 1]] for a in atoms])
    g_ref, g_abs = oracle.force(*sub.geometry(), psi_h, wsub, with_abs=True)
    _parity(g[atoms], g_ref, g_abs, "batching force (sampled atoms)")
    plan.close()


def _pool8():
    """Eight systems of the request-stream pool: the largest band count, the
    largest cut-off and the largest grid are among them."""
    pool = wl.serving_pool(seed=4, nsystems=32)
    size = np.array([np.prod(s.n) * s.nbands for s in pool], dtype=np.float64)
    pick = {int(np.argmax([s.nbands for s in pool])), int(np.argmax([s.numax.max() for s in pool])),
            int(np.argmax([np.prod(s.n) for s in pool]))}
    for k in np.argsort(size):
        if len(pick) >= 8:
            break
        pick.add(int(k))
    return [pool[k] for k in sorted(pick)]


def test_serving_pool_subset_mixed():
    bd = _bd()
    from paper_1905_00480_amd import serve
    pool = _pool8()
    assert max(s.nbands for s in pool) == 128 and max(int(s.numax.max()) for s in pool) == 9
    srv = bd.Server(96 << 30, 4, 0)
    sids = serve.register(srv, pool, seed=4)
    inputs = [tuple(x.copy() for x in srv.inputs(sid)) for sid in sids]
    rng = np.random.default_rng(17)
    order = [(k, j) for k in range(len(pool)) for j in (0, 1, 2)]
    for i in rng.permutation(len(order)):
        k, j = order[i]
        srv.submit(sids[k], j)
    srv.drain()
    for k, s in enumerate(pool):
        psi, w = inputs[k]
        psi = psi.reshape(s.psi_shape)
        off = wl.coeff_offsets(s)
        # three atoms from the half with the smaller supports (oracle time)
        size = s.sigma * np.sqrt(2 * s.numax + 3)
        small = np.flatnonzero(size <= np.median(size))
        atoms = np.sort(rng.choice(small, min(3, small.size), replace=False))
        sub = s.subset(atoms)
        wsub = np.concatenate([w[off[a]:off[a + 1]] for a in atoms])
        c = srv.read(sids[k], 0)
        c_ref, c_abs = oracle.project(*sub.geometry(), psi, with_abs=True)
        _parity(np.concatenate([c[off[a]:off[a + 1]] for a in atoms]), c_ref, c_abs,
                "%s project" % s.name)
        g = srv.read(sids[k], 2).reshape(s.natoms, 3)
        g_ref, g_abs = oracle.force(*sub.geometry(), psi, wsub, with_abs=True)
        _parity(g[atoms], g_ref, g_abs, "%s force" % s.name)
        e = srv.read(sids[k], 1).reshape(-1, s.nbands)
        pts = rng.choice(e.shape[0], 12, replace=False)
        e_ref, e_abs = oracle.expand_at(*s.geometry(), w, pts, np.zeros((pts.size, s.nbands)),
                                        with_abs=True)
        _parity(e[pts], e_ref, e_abs, "%s expand (sampled points)" % s.name)
    srv.close()
