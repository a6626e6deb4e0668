"""Oracle for stored numerical projectors p_j(r) = P_k(|r|) Y_{l_k m}(r^).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's reference kernels (USU, sec. 6) project onto precomputed values
of numerical PAW projectors; its USU18 set holds two radial functions each
for l = 0, 1, 2 (s, s*, p, p*, d, d*: 18 projectors).  Here the projector
set is given as radial tables and sampled at every support point:

* radial table: P[k][m] = P_k(m dr), m = 0 .. nr-1 (uniform radial grid);
  between the nodes P_k is the cubic Lagrange interpolant through the four
  nodes s .. s+3, s = clamp(floor(r/dr) - 1, 0, nr - 4); for r >= (nr-1) dr
  the projector is zero (the table ends where the projector does);
* projectors j run over k, then m = -l_k .. l_k (the projector order of the
  set-up side); Y_lm are the real spherical harmonics of the set-up oracle
  (no Condon-Shortley sign, Y_11 ~ +x, Y_1-1 ~ +y), evaluated from their
  exact solid-harmonic polynomials r^l Y_lm; at r = 0 only l = 0 is nonzero;
* support S_a = the grid points within the cut-off radius rcut_a of the atom
  (the same sphere rule, images and clipping as the SHO projectors);
* projection c[a][j][b] = h^3 sum_{i in S_a} p_j(r_i - R_a) psi_b(i mod N),
  expansion psi_b(j) += sum_a sum_{i in S_a, i = j mod N} sum_j c p_j,
  coefficients in per-atom blocks [nproj][B]; sums in long double.
"""
import numpy as np

from . import setup as _setup
from . import support as _support


def nproj(ell):
    return int(sum(2 * int(l) + 1 for l in ell))


def interp(P, dr, r):
    """Cubic Lagrange interpolation of the table rows P[k][:] at radii r."""
    P = np.asarray(P, dtype=np.float64)
    P = P.reshape(-1, P.shape[-1])
    nr = P.shape[1]
    if nr < 4:
        raise ValueError("radial tables need at least 4 nodes")
    r = np.asarray(r, dtype=np.float64)
    t = r / dr
    m0 = np.floor(t).astype(np.int64)
    s = np.clip(m0 - 1, 0, nr - 4)
    u = t - s
    w = [-(u - 1) * (u - 2) * (u - 3) / 6, u * (u - 2) * (u - 3) / 2,
         -u * (u - 1) * (u - 3) / 2, u * (u - 1) * (u - 2) / 6]
    out = np.zeros((P.shape[0],) + r.shape)
    for q in range(4):
        out += w[q] * P[:, s + q]
    out[:, t >= nr - 1] = 0.0
    return out


def ylm(l, m, d):
    """Real Y_lm at directions d [K, 3] (rows need not be unit vectors);
    0 at d = 0 for l > 0, Y_00 there for l = 0."""
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    poly, k2 = _setup._solid(l, m)
    vals = np.zeros(d.shape[0])
    for (a, b, c), coef in poly.items():
        vals += float(coef) * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c
    r = np.sqrt(np.sum(d * d, axis=1))
    K = np.sqrt(float(k2) / np.pi)
    out = np.zeros_like(vals)
    nz = r > 0
    out[nz] = K * vals[nz] / r[nz] ** l
    if l == 0:
        out[~nz] = K * vals[~nz]
    return out


def projectors(ell, dr, P, d):
    """p_j at offsets d [K, 3] -> [K, nproj]."""
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt(np.sum(d * d, axis=1))
    rad = interp(P, dr, r)
    cols = []
    for k, l in enumerate(ell):
        for m in range(-int(l), int(l) + 1):
            cols.append(rad[k] * ylm(int(l), m, d))
    return np.stack(cols, axis=1)


def _points(n, h, periodic, centre, rcut):
    idx, mem = _support(n, h, periodic, centre, rcut)
    d = idx.astype(np.float64) * h - np.asarray(centre, dtype=np.float64)[None, :]
    return d, mem


def project(n, h, periodic, pos, rcut, ell, dr, P, psi, with_abs=False):
    """c (flat per-atom blocks [nproj][B]) and, with ``with_abs``, the abs-sum
    h^3 sum |p psi|."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    psi = np.asarray(psi, dtype=np.float64)
    B = psi.shape[-1]
    flat = psi.reshape(-1, B)
    npj = nproj(ell)
    h3 = np.longdouble(h) ** 3
    cs, ab = [], []
    for a in range(pos.shape[0]):
        d, mem = _points(n, h, periodic, pos[a], rcut[a])
        p = projectors(ell, dr, P, d).astype(np.longdouble)
        v = flat[mem].astype(np.longdouble)
        cs.append((h3 * (p.T @ v)).astype(np.float64).reshape(npj * B))
        ab.append((h3 * (np.abs(p).T @ np.abs(v))).astype(np.float64).reshape(npj * B))
    c = np.concatenate(cs) if cs else np.zeros(0)
    if with_abs:
        return c, (np.concatenate(ab) if ab else np.zeros(0))
    return c


def expand(n, h, periodic, pos, rcut, ell, dr, P, c, psi_in, with_abs=False):
    """psi_in + sum_a sum_j c p_j (and |psi_in| + sum |c p|)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    out = np.array(psi_in, dtype=np.float64, copy=True)
    B = out.shape[-1]
    acc = out.reshape(-1, B).astype(np.longdouble)
    absum = np.abs(acc)
    npj = nproj(ell)
    c = np.asarray(c, dtype=np.float64).reshape(pos.shape[0], npj, B)
    for a in range(pos.shape[0]):
        d, mem = _points(n, h, periodic, pos[a], rcut[a])
        p = projectors(ell, dr, P, d).astype(np.longdouble)
        ca = c[a].astype(np.longdouble)
        np.add.at(acc, mem, p @ ca)
        np.add.at(absum, mem, np.abs(p) @ np.abs(ca))
    res = acc.astype(np.float64).reshape(out.shape)
    if with_abs:
        return res, absum.astype(np.float64).reshape(out.shape)
    return res
