"""Seeded synthetic inputs for the SHO projection path.

This module only draws inputs: grids, atom positions, spreads sigma, basis
cut-offs nu_max, wave functions psi and coefficient / weight arrays.  It holds
none of the method's arithmetic, so both the HIP path and the CPU oracle can
consume the same arrays without sharing any computation.

The paper measures on a synthetic system (an fcc crystal in a 64^3 box,
sec. 6) and uses no public dataset; the workloads below follow its shape:
a uniform real-space grid, atoms with overlapping projection spheres, and
many real FP64 bands stored band-fastest (the band index is the vector lane,
sec. 6).

Random streams: ``numpy.random.default_rng`` (PCG64) children of one
``SeedSequence(seed)``: child 0 draws positions, child 1 sigma / nu_max,
child 2 psi, child 3 coefficients or weights.  Each array is reproducible on
its own, without drawing the others first.
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np


@dataclass
class System:
    """One projection problem: grid + atoms + band count."""
    name: str
    n: Tuple[int, int, int]          # points per axis (x, y, z)
    h: float                         # grid spacing, Bohr; point i at i*h
    periodic: Tuple[bool, bool, bool]
    pos: np.ndarray                  # [A, 3] Bohr
    sigma: np.ndarray                # [A] Bohr
    numax: np.ndarray                # [A] int32
    nbands: int
    seed: int = 0
    notes: str = ""
    rbox: Optional[np.ndarray] = field(default=None)  # optional support radii

    @property
    def natoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def psi_shape(self):
        return (self.n[2], self.n[1], self.n[0], self.nbands)

    @property
    def cell(self):
        return np.array(self.n, dtype=np.float64) * self.h

    def geometry(self):
        """Positional arguments shared by every entry point."""
        return (self.n, self.h, self.periodic, self.pos, self.sigma, self.numax)

    def subset(self, atoms: Sequence[int]) -> "System":
        """The same grid with only the listed atoms (for sampled checks)."""
        atoms = np.asarray(atoms, dtype=np.int64)
        return System(self.name + "[subset]", self.n, self.h, self.periodic,
                      self.pos[atoms].copy(), self.sigma[atoms].copy(),
                      self.numax[atoms].copy(), self.nbands, self.seed,
                      self.notes,
                      None if self.rbox is None else self.rbox[atoms].copy())


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


def nsho_count(nu) -> np.ndarray:
    """Number of (nx, ny, nz) with nx+ny+nz <= nu (sizes only, for buffers)."""
    nu = np.asarray(nu, dtype=np.int64)
    return (nu + 1) * (nu + 2) * (nu + 3) // 6


def uniform_positions(rng, natoms, cell):
    return rng.uniform(0.0, 1.0, size=(natoms, 3)) * np.asarray(cell)[None, :]


def rsa_positions(rng, natoms, cell, min_sep, periodic=(True, True, True),
                  max_tries=2_000_000):
    """Random sequential adsorption: uniform draws, rejected when closer than
    ``min_sep`` (minimum-image distance on periodic axes) to an accepted one."""
    cell = np.asarray(cell, dtype=np.float64)
    per = np.asarray(periodic, dtype=bool)
    out = np.empty((natoms, 3))
    k = 0
    tries = 0
    while k < natoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA placement did not converge")
        p = rng.uniform(0.0, 1.0, size=3) * cell
        if k:
            d = out[:k] - p[None, :]
            d = np.where(per[None, :], d - cell * np.round(d / cell), d)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_sep * min_sep:
                continue
        out[k] = p
        k += 1
    return out


def make_system(name, n, h, periodic, natoms, sigma, numax, nbands, seed,
                min_sep=None, sigma_range=None, numax_range=None, notes=""):
    """Generic generator: positions uniform (or RSA with ``min_sep``), sigma
    fixed or uniform in ``sigma_range``, nu_max fixed or uniform integer in
    ``numax_range`` (inclusive)."""
    n = tuple(int(v) for v in n)
    periodic = tuple(bool(v) for v in periodic)
    g_pos, g_par, _, _ = _streams(seed)
    cell = np.array(n, dtype=np.float64) * h
    if min_sep:
        pos = rsa_positions(g_pos, natoms, cell, min_sep, periodic)
    else:
        pos = uniform_positions(g_pos, natoms, cell)
    if sigma_range is not None:
        sig = g_par.uniform(sigma_range[0], sigma_range[1], size=natoms)
    else:
        sig = np.full(natoms, float(sigma))
    if numax_range is not None:
        nu = g_par.integers(numax_range[0], numax_range[1] + 1, size=natoms)
    else:
        nu = np.full(natoms, int(numax))
    return System(name, n, float(h), periodic, pos, sig.astype(np.float64),
                  nu.astype(np.int32), int(nbands), int(seed), notes)


# ------------------------------------------------------------- workloads ----

def tiny(seed=0) -> System:
    """1 atom at a random position in an isolated 16^3 grid, h = 0.25 Bohr,
    sigma = 0.5, nu_max = 3 (20 functions), 1 band."""
    return make_system("tiny", (16, 16, 16), 0.25, (False,) * 3, 1, 0.5, 3, 1,
                       seed)


def scale(seed=1, nbands=32) -> System:
    """Periodic 128^3 grid, h = 0.2 Bohr, 512 atoms (RSA, 2 Bohr minimum
    separation), sigma = 0.6, nu_max = 5 (56 functions), 32 bands."""
    return make_system("scale", (128, 128, 128), 0.2, (True,) * 3, 512, 0.6, 5,
                       nbands, seed, min_sep=2.0)


def batching(seed=2) -> System:
    """Periodic 160^3 grid, h = 0.18 Bohr, 2048 atoms uniform, nu_max uniform
    in 3..9, sigma uniform in [0.4, 1.2] Bohr, 64 bands."""
    return make_system("batching", (160, 160, 160), 0.18, (True,) * 3, 2048,
                       None, None, 64, seed, sigma_range=(0.4, 1.2),
                       numax_range=(3, 9))


def diff(seed=3) -> System:
    """Isolated 96^3 grid, h = 0.2 Bohr, 256 atoms uniform, sigma = 0.6,
    nu_max = 6 (84 functions), 16 bands."""
    return make_system("diff", (96, 96, 96), 0.2, (False,) * 3, 256, 0.6, 6, 16,
                       seed)


ANGSTROM = 1.0 / 0.529177210903  # Bohr per Angstrom


def paper_fcc(numax=5, nbands=1024, sigma=1.6) -> System:
    """The geometry of the paper's GPU benchmark (sec. 6), in Bohr: a cubic
    domain of 16 Angstrom with 64^3 points (h = 0.25 Angstrom), isolated; fcc
    lattice a = 4.08 Angstrom with a site at the origin; every atom whose
    projection sphere (radius 3.55 Angstrom) reaches a grid point; 1024 bands.
    sigma is not given by the paper: 1.6 Bohr puts the shell nu = 5 turning
    radius sigma sqrt(2 nu + 3) near the sphere radius and satisfies the
    sampling bound for nu <= 5.  All atoms share nu_max (one column of the
    paper's table per value)."""
    h = 0.25 * ANGSTROM
    n = 64
    a = 4.08 * ANGSTROM
    R = 3.55 * ANGSTROM
    top = (n - 1) * h
    lo = int(np.floor(-R / (a / 2))) - 1
    hi = int(np.ceil((top + R) / (a / 2))) + 1
    pts = []
    for i in range(lo, hi + 1):
        for j in range(lo, hi + 1):
            for k in range(lo, hi + 1):
                if (i + j + k) % 2:
                    continue
                p = np.array([i, j, k], dtype=np.float64) * (a / 2)
                q = np.clip(p, 0.0, top)
                if np.sqrt(np.sum((p - q) ** 2)) <= R:
                    pts.append(p)
    pos = np.array(pts)
    na = pos.shape[0]
    return System("paper_fcc", (n, n, n), h, (False,) * 3, pos,
                  np.full(na, float(sigma)), np.full(na, int(numax), dtype=np.int32),
                  int(nbands), 5, "fcc a = 4.08 A, 64^3, h = 0.25 A, R = 3.55 A",
                  np.full(na, R))


def small_periodic(seed=11, nbands=32, natoms=6, numax=5, sigma=0.6, n=32,
                   h=0.2) -> System:
    """Scale-shaped case small enough for the oracle in seconds: periodic
    32^3 (boxes wrap across the cell faces), several atoms, ragged band tail
    when ``nbands`` is not a multiple of the band tile."""
    return make_system("small_periodic", (n, n, n), h, (True,) * 3, natoms,
                       sigma, numax, nbands, seed)


def small_mixed(seed=12, nbands=20, natoms=8, n=(40, 36, 28), h=0.18,
                periodic=(True, False, True)) -> System:
    """Uneven atoms (nu_max 0..9, sigma 0.4..1.2) on a non-cubic grid with
    mixed periodic / isolated axes; a batching-shaped parity case."""
    return make_system("small_mixed", n, h, periodic, natoms, None, None,
                       nbands, seed, sigma_range=(0.4, 1.2),
                       numax_range=(0, 9))


def psi_for(system: System, seed: Optional[int] = None, dtype=np.float64):
    """psi ~ N(0, 1), shape (nz, ny, nx, B)."""
    g = _streams(system.seed if seed is None else seed)[2]
    return g.standard_normal(size=system.psi_shape, dtype=dtype)


def coeffs_for(system: System, seed: Optional[int] = None):
    """Coefficients (or weights) ~ N(0, 1), per-atom blocks [N_SHO][B]."""
    g = _streams(system.seed if seed is None else seed)[3]
    total = int(nsho_count(system.numax).sum()) * system.nbands
    return g.standard_normal(size=total)


def coeff_offsets(system: System):
    """Start of each atom's coefficient block in doubles, [natoms+1]."""
    cnt = nsho_count(system.numax) * system.nbands
    return np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)


# ------------------------------------------------- numerical projectors ----

def radial_set(rcut, ell=(0, 0, 1, 1, 2, 2), nr=512, seed=7):
    """Synthetic radial projector tables for a stored-projector (USU) plan:
    P_k(r) = r^l (1 + c1 r + c2 r^2) exp(-r^2 / (2 a^2)) (1 - (r/rcut)^2)^2 on
    the uniform grid r_i = i dr, i = 0..nr-1, dr = rcut / (nr - 1), with
    c1, c2 ~ U[-0.3, 0.3] and a ~ U[0.3, 0.5] rcut per function.  The default
    ell is the paper's USU18 set: two functions each for s, p and d (18
    projectors).  Returns (ell, dr, tables[nradial][nr])."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    ell = np.asarray(ell, dtype=np.int32)
    dr = float(rcut) / (nr - 1)
    r = np.arange(nr) * dr
    tab = np.empty((ell.size, nr))
    for k, l in enumerate(ell):
        c1, c2 = rng.uniform(-0.3, 0.3, size=2)
        a = rng.uniform(0.3, 0.5) * rcut
        tab[k] = (r ** int(l) * (1 + c1 * r + c2 * r * r) * np.exp(-r * r / (2 * a * a))
                  * (1 - (r / rcut) ** 2) ** 2)
    return ell, dr, tab


def radial_coeffs_for(system: System, nproj: int, seed: Optional[int] = None):
    """Coefficients ~ N(0, 1) for a stored-projector plan, blocks [nproj][B]."""
    g = _streams(system.seed if seed is None else seed)[3]
    return g.standard_normal(size=system.natoms * int(nproj) * system.nbands)


# --------------------------------------------------------------- serving ----

def serving_pool(seed=4, nsystems=32, hbm_cap_bytes=None):
    """Pool of systems for the request-stream workload: N uniform in
    {32, 48, ..., 160}, h = 0.2, natoms = clamp(round(rho L^3), 16, 4096) with
    rho uniform in [0.01, 0.125] Bohr^-3, nu_max in 3..9, sigma in
    [0.4, 1.2], B in {8, 16, 32, 64, 128}; periodic."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(5)[4])
    pool = []
    for k in range(nsystems):
        n = int(rng.choice(np.arange(32, 161, 16)))
        rho = rng.uniform(0.01, 0.125)
        L = n * 0.2
        natoms = int(np.clip(round(rho * L ** 3), 16, 4096))
        B = int(rng.choice([8, 16, 32, 64, 128]))
        s = make_system("serve%02d" % k, (n, n, n), 0.2, (True,) * 3, natoms,
                        None, None, B, seed * 1000 + k,
                        sigma_range=(0.4, 1.2), numax_range=(3, 9))
        pool.append(s)
    return pool


def poisson_arrivals(rate_hz, count, seed=4):
    """Arrival times (s) of a Poisson stream and a job kind per request
    (0 = project, 1 = expand, 2 = force)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    kinds = rng.integers(0, 3, size=count)
    return np.cumsum(gaps), kinds, rng
