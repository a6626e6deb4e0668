"""CPU oracle for SHO projection / expansion / position derivatives.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package; it shares no code with the HIP library.

Thin ctypes marshalling over ``sho_oracle.c`` (plain triple sums written from
the paper's definitions, long-double accumulation).  Conventions:

* grid: ``n = (nx, ny, nz)`` points, spacing ``h`` (Bohr), point ``i`` at
  ``i*h``; ``periodic = (px, py, pz)`` flags.
* ``psi`` has shape ``(nz, ny, nx, B)`` (band index fastest), float64.
* coefficients are per-atom blocks ``[N_SHO(nu_a)][B]`` concatenated in atom
  order; index ``n`` runs nz outermost, then ny, nx fastest over
  ``nx+ny+nz <= nu_a``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsho_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # SHO_ORACLE_LIBRARY names another build of the oracle (the sanitized
    # libsho_oracle_asan.so of `build.py --sanitize`)
    path = os.environ.get("SHO_ORACLE_LIBRARY") or _LIB_PATH
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(path)
    lib.oracle_nsho.argtypes = [ctypes.c_int]
    lib.oracle_nsho.restype = ctypes.c_int
    lib.oracle_coeff_index.argtypes = [ctypes.c_int] * 4
    lib.oracle_coeff_index.restype = ctypes.c_int
    lib.oracle_box_radius.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.oracle_box_radius.restype = ctypes.c_double
    for f in (lib.oracle_phi, lib.oracle_dphi):
        f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp]
        f.restype = ctypes.c_int
    lib.oracle_support.argtypes = [_ip, ctypes.c_double, _ip, _dp, ctypes.c_double,
                                   ctypes.c_int64, _ip, _i64p]
    lib.oracle_support.restype = ctypes.c_int64
    geo = [_ip, ctypes.c_double, _ip, ctypes.c_int, _dp, _dp, _ip, _dp]
    lib.oracle_project.argtypes = geo + [_dp, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_project.restype = ctypes.c_int
    lib.oracle_expand.argtypes = geo + [_dp, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_expand.restype = ctypes.c_int
    lib.oracle_expand_at.argtypes = geo + [ctypes.c_int, _dp, ctypes.c_int64, _i64p,
                                           _dp, _dp, _dp]
    lib.oracle_expand_at.restype = ctypes.c_int
    lib.oracle_force.argtypes = geo + [_dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_force.restype = ctypes.c_int
    for f in (lib.oracle_project_k, lib.oracle_expand_k):
        f.argtypes = geo + [_dp, ctypes.c_int, _dp, _dp, _dp]
        f.restype = ctypes.c_int
    lib.fact_threads.argtypes = []
    lib.fact_threads.restype = ctypes.c_int
    for f in (lib.fact_project, lib.fact_expand):
        f.argtypes = geo + [ctypes.c_int, _dp, _dp]
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _grid(n, h, periodic):
    nn = (ctypes.c_int * 3)(*[int(v) for v in n])
    pp = (ctypes.c_int * 3)(*[1 if v else 0 for v in periodic])
    return nn, float(h), pp


def nsho(nu):
    """N_SHO(nu) = (nu+1)(nu+2)(nu+3)/6."""
    return _load().oracle_nsho(int(nu))


def coeff_index(nu, nx, ny, nz):
    return _load().oracle_coeff_index(int(nu), int(nx), int(ny), int(nz))


def box_radius(sigma, nu, h):
    """Default support radius sigma*sqrt(2 nu + 3) + 2h."""
    return _load().oracle_box_radius(float(sigma), int(nu), float(h))


def coeff_offsets(numax, nbands):
    """Start of each atom's coefficient block, in doubles ([natoms+1])."""
    off = [0]
    for nu in numax:
        off.append(off[-1] + nsho(nu) * int(nbands))
    return np.array(off, dtype=np.int64)


def phi(nu, sigma, u):
    """phi_n(u; sigma) for n = 0..nu -> array [nu+1, len(u)]."""
    u = _f64(np.atleast_1d(u))
    out = np.empty((nu + 1, u.size))
    if _load().oracle_phi(int(nu), float(sigma), u.size, _d(u), _d(out)):
        raise ValueError("oracle_phi: bad arguments")
    return out


def dphi(nu, sigma, u):
    """d/du phi_n(u; sigma) for n = 0..nu -> array [nu+1, len(u)]."""
    u = _f64(np.atleast_1d(u))
    out = np.empty((nu + 1, u.size))
    if _load().oracle_dphi(int(nu), float(sigma), u.size, _d(u), _d(out)):
        raise ValueError("oracle_dphi: bad arguments")
    return out


def support(n, h, periodic, centre, R):
    """Support points of one sphere: (unwrapped indices [K,3] as (x,y,z),
    memory indices [K])."""
    lib = _load()
    nn, hh, pp = _grid(n, h, periodic)
    c = _f64(centre, (3,))
    k = lib.oracle_support(nn, hh, pp, _d(c), float(R), 0, None, None)
    if k < 0:
        raise ValueError("oracle_support: bad grid")
    idx = np.empty((k, 3), dtype=np.int32)
    mem = np.empty(k, dtype=np.int64)
    lib.oracle_support(nn, hh, pp, _d(c), float(R), k,
                       idx.ctypes.data_as(_ip), mem.ctypes.data_as(_i64p))
    return idx, mem


def _atoms(pos, sigma, numax, rbox=None, spos=None):
    pos = _f64(pos, (-1, 3))
    na = pos.shape[0]
    return (na, pos, _f64(sigma, (na,)), _i32(numax).reshape(na),
            _f64(rbox, (na,)) if rbox is not None else None,
            _f64(spos, (na, 3)) if spos is not None else None)


def project(n, h, periodic, pos, sigma, numax, psi, rbox=None, spos=None,
            with_abs=False):
    """c = h^3 sum_{i in S_a} P_an(i) psi(i); returns c (flat per-atom blocks)
    and, with ``with_abs``, the abs-sum h^3 sum |P psi| of the same layout."""
    na, pos, sigma, numax, rbox, spos = _atoms(pos, sigma, numax, rbox, spos)
    psi = _f64(psi)
    B = psi.shape[-1]
    assert psi.size == int(n[0]) * int(n[1]) * int(n[2]) * B
    total = int(coeff_offsets(numax, B)[-1])
    c = np.zeros(total)
    ca = np.zeros(total) if with_abs else None
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_project(nn, hh, pp, na, _d(pos), _d(sigma),
                                numax.ctypes.data_as(_ip), _d(rbox), _d(spos), B,
                                _d(psi), _d(c), _d(ca))
    if rc:
        raise ValueError("oracle_project: bad arguments")
    return (c, ca) if with_abs else c


def threads():
    """OpenMP threads the CPU paths run with."""
    return int(_load().fact_threads())


def factorised_project(n, h, periodic, pos, sigma, numax, psi, rbox=None):
    """The factorised CPU path (sho_factorised.c): x, y and z passes per atom,
    double sums, OpenMP over atoms.  Same result as ``project`` up to
    rounding; the benchmark's CPU reference point, not the checker."""
    na, pos, sigma, numax, rbox, _ = _atoms(pos, sigma, numax, rbox, None)
    psi = _f64(psi)
    B = psi.shape[-1]
    assert psi.size == int(n[0]) * int(n[1]) * int(n[2]) * B
    c = np.zeros(int(coeff_offsets(numax, B)[-1]))
    nn, hh, pp = _grid(n, h, periodic)
    if _load().fact_project(nn, hh, pp, na, _d(pos), _d(sigma), numax.ctypes.data_as(_ip),
                            _d(rbox), B, _d(psi), _d(c)):
        raise ValueError("fact_project: bad arguments")
    return c


def factorised_expand(n, h, periodic, pos, sigma, numax, c, psi, rbox=None):
    """psi += expansion of c by the factorised CPU path, in place (psi must be
    a C-contiguous float64 array); returns psi."""
    na, pos, sigma, numax, rbox, _ = _atoms(pos, sigma, numax, rbox, None)
    assert psi.dtype == np.float64 and psi.flags.c_contiguous
    B = psi.shape[-1]
    c = _f64(c)
    assert c.size == int(coeff_offsets(numax, B)[-1])
    nn, hh, pp = _grid(n, h, periodic)
    if _load().fact_expand(nn, hh, pp, na, _d(pos), _d(sigma), numax.ctypes.data_as(_ip),
                           _d(rbox), B, _d(c), _d(psi)):
        raise ValueError("fact_expand: bad arguments")
    return psi


def expand(n, h, periodic, pos, sigma, numax, c, psi_in, rbox=None, spos=None,
           with_abs=False):
    """psi_out = psi_in + sum_a sum_n c P_an; returns psi_out (and abs-sum)."""
    na, pos, sigma, numax, rbox, spos = _atoms(pos, sigma, numax, rbox, spos)
    out = np.array(psi_in, dtype=np.float64, copy=True, order="C")
    B = out.shape[-1]
    c = _f64(c)
    assert c.size == int(coeff_offsets(numax, B)[-1])
    pab = np.abs(out) if with_abs else None
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_expand(nn, hh, pp, na, _d(pos), _d(sigma),
                               numax.ctypes.data_as(_ip), _d(rbox), _d(spos), B,
                               _d(c), _d(out), _d(pab))
    if rc:
        raise ValueError("oracle_expand: bad arguments")
    return (out, pab) if with_abs else out


def expand_at(n, h, periodic, pos, sigma, numax, c, points, psi_in_at=None,
              rbox=None, nbands=None, with_abs=False):
    """Expansion evaluated only at memory points ``points`` ([K] flat grid
    indices); returns [K, B] (and abs-sum)."""
    na, pos, sigma, numax, rbox, _ = _atoms(pos, sigma, numax, rbox)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    B = int(nbands) if nbands is not None else np.asarray(psi_in_at).shape[-1]
    c = _f64(c)
    pin = _f64(psi_in_at, (pts.size, B)) if psi_in_at is not None else None
    out = np.empty((pts.size, B))
    oab = np.empty((pts.size, B)) if with_abs else None
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_expand_at(nn, hh, pp, na, _d(pos), _d(sigma),
                                  numax.ctypes.data_as(_ip), _d(rbox), B, _d(c),
                                  pts.size, pts.ctypes.data_as(_i64p), _d(pin),
                                  _d(out), _d(oab))
    if rc:
        raise ValueError("oracle_expand_at failed (%d)" % rc)
    return (out, oab) if with_abs else out


def force(n, h, periodic, pos, sigma, numax, psi, w, rbox=None, spos=None,
          with_abs=False, with_dc=False):
    """g[a][d] = sum_{n,b} w * dc/dR_{a,d} (support frozen around ``spos``).
    Returns g [natoms,3], plus abs-sum and/or dc ([per-atom 3][N][B] blocks)."""
    na, pos, sigma, numax, rbox, spos = _atoms(pos, sigma, numax, rbox, spos)
    psi = _f64(psi)
    B = psi.shape[-1]
    w = _f64(w)
    total = int(coeff_offsets(numax, B)[-1])
    assert w.size == total
    g = np.zeros((na, 3))
    ga = np.zeros((na, 3)) if with_abs else None
    dc = np.zeros(3 * total) if with_dc else None
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_force(nn, hh, pp, na, _d(pos), _d(sigma),
                              numax.ctypes.data_as(_ip), _d(rbox), _d(spos), B,
                              _d(psi), _d(w), _d(g), _d(ga), _d(dc))
    if rc:
        raise ValueError("oracle_force: bad arguments")
    out = [g]
    if with_abs:
        out.append(ga)
    if with_dc:
        out.append(dc)
    return out[0] if len(out) == 1 else tuple(out)


def matrix_offsets(numax):
    """Offsets (doubles) of per-atom N_SHO x N_SHO blocks, atom order."""
    n = np.array([nsho(int(v)) for v in np.atleast_1d(numax)], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(n * n)])


def apply(n, h, periodic, pos, sigma, numax, psi, D, psi_in, rbox=None, with_abs=False):
    """Non-local application (sec. 3.2 steps 1-3): c = projection of psi,
    d_a = D_a c_a (a plain matrix product per atom), psi_out = psi_in +
    expansion of d.  With ``with_abs`` also the abs-sum of the whole chain,
    |psi_in| + sum |P| (|D| c_abs), which bounds the rounding of every step."""
    numax = np.atleast_1d(np.asarray(numax, dtype=np.int32))
    B = psi.shape[-1]
    c, c_abs = project(n, h, periodic, pos, sigma, numax, psi, rbox=rbox, with_abs=True)
    coff = coeff_offsets(numax, B)
    doff = matrix_offsets(numax)
    d = np.empty_like(c)
    d_abs = np.empty_like(c)
    for a in range(len(numax)):
        N = nsho(int(numax[a]))
        Da = np.asarray(D[doff[a]:doff[a + 1]]).reshape(N, N)
        ca = c[coff[a]:coff[a + 1]].reshape(N, B)
        d[coff[a]:coff[a + 1]] = (Da @ ca).ravel()
        d_abs[coff[a]:coff[a + 1]] = (np.abs(Da) @ c_abs[coff[a]:coff[a + 1]].reshape(N, B)).ravel()
    out = expand(n, h, periodic, pos, sigma, numax, d, psi_in, rbox=rbox)
    if not with_abs:
        return out
    _, out_abs = expand(n, h, periodic, pos, sigma, numax, d_abs, np.abs(psi_in), rbox=rbox,
                        with_abs=True)
    return out, out_abs


def _as_pairs(a):
    """Complex array -> float64 interleaved (re, im) pairs (a view if already
    float pairs)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1), dtype=np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def project_k(n, h, periodic, pos, sigma, numax, psi, kvec, rbox=None, with_abs=False):
    """Complex bands at wave vector ``kvec`` (Bohr^-1): c[a][n][b] =
    h^3 sum_{i in S_a} P_an(i) e^{i k.T_i} psi_b(i mod N).  ``psi`` complex
    (nz, ny, nx, B); returns complex c (flat per-atom blocks [N][B]) and, with
    ``with_abs``, the abs-sum h^3 sum |P| (|Re psi| + |Im psi|) (real)."""
    na, pos, sigma, numax, rbox, _ = _atoms(pos, sigma, numax, rbox)
    pp_ = _as_pairs(psi)
    B = pp_.shape[-2]
    total = int(coeff_offsets(numax, B)[-1])
    c = np.zeros(2 * total)
    ca = np.zeros(2 * total) if with_abs else None
    k = _f64(kvec, (3,))
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_project_k(nn, hh, pp, na, _d(pos), _d(sigma),
                                  numax.ctypes.data_as(_ip), _d(rbox), _d(k), B,
                                  _d(pp_), _d(c), _d(ca))
    if rc:
        raise ValueError("oracle_project_k: bad arguments")
    cz = c[0::2] + 1j * c[1::2]
    return (cz, ca[0::2]) if with_abs else cz


def expand_k(n, h, periodic, pos, sigma, numax, c, psi_in, kvec, rbox=None, with_abs=False):
    """psi_out = psi_in + sum_a sum_{images} e^{-i k.T} sum_n c P_an, complex
    arrays (psi (nz, ny, nx, B), c flat per-atom blocks); returns psi_out and,
    with ``with_abs``, |Re psi_in| + |Im psi_in| + sum |P| (|Re c| + |Im c|)."""
    na, pos, sigma, numax, rbox, _ = _atoms(pos, sigma, numax, rbox)
    out = _as_pairs(np.asarray(psi_in, dtype=np.complex128)).copy()
    B = out.shape[-2]
    cc = _as_pairs(np.asarray(c, dtype=np.complex128))
    assert cc.size == 2 * int(coeff_offsets(numax, B)[-1])
    pab = None
    if with_abs:
        pin = np.asarray(psi_in, dtype=np.complex128)
        s = np.abs(pin.real) + np.abs(pin.imag)
        pab = np.ascontiguousarray(np.stack([s, s], axis=-1))
    k = _f64(kvec, (3,))
    nn, hh, pp = _grid(n, h, periodic)
    rc = _load().oracle_expand_k(nn, hh, pp, na, _d(pos), _d(sigma),
                                 numax.ctypes.data_as(_ip), _d(rbox), _d(k), B,
                                 _d(cc), _d(out), _d(pab))
    if rc:
        raise ValueError("oracle_expand_k: bad arguments")
    z = out[..., 0] + 1j * out[..., 1]
    return (z, pab[..., 0]) if with_abs else z
