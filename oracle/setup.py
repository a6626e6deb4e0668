"""Oracle for the set-up side of the SHO projectors (sec. 2.3-2.5, 3.5, 4).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain definitions,
written for checking, not speed.

* ``unitary(nu_max)``: the matrix U[c][s] = <Phi_c | Psi_s> between the
  Cartesian SHO states Phi_c = phi_nx(x) phi_ny(y) phi_nz(z) (the library's
  coefficient order) and the radial states Psi_s = R_{nr l}(r) Y_lm(r^)
  (radial order: nu ascending, l ascending with l = nu mod 2 .. nu, m = -l..l,
  nr = (nu - l)/2), sigma = 1 (U does not depend on sigma).  Both states are
  a polynomial times exp(-r^2/2); the overlap is evaluated exactly: the
  polynomials are expanded into monomials with rational coefficients and
  integrated against exp(-r^2) with the Gaussian moments
  int x^(2k) exp(-x^2) dx = (2k)!/(4^k k!) sqrt(pi).  All normalisation
  factors are square roots of rationals times powers of pi, and the powers
  of pi cancel, so every entry is (exact rational) x sqrt(exact rational).
* ``radial(nr, l, sigma, r)``: R_{nr l}(r) = N r~^l L_nr^(l+1/2)(r~^2)
  exp(-r~^2/2) sigma^(-3/2), r~ = r/sigma, N^2 = 2 nr!/Gamma(nr+l+3/2), so
  that int R^2 r^2 dr = 1 (scipy's generalised Laguerre polynomials).
* ``F`` / ``setup_matrix`` / ``quality``: F[j][s] = <p_j | Psi_s> for
  projectors p_j = P_k(r) Y_{l_k m}(r^) given on a radial quadrature
  (sum_i w_i g(r_i) ~ int g dr), M = F U^T (M[j][c] = <p_j | Phi_c>),
  script-D = M^T D M in the Cartesian basis (sec. 3.5), and
  Q_nu = sum_{nr <= (nu-l)/2} |<P | R_nr l>|^2 / <P | P> (sec. 4).

Real spherical harmonics: Y_l0 = K_l0 P_l(cos t); for m > 0
sqrt(2) K_lm P_l^m(cos t) cos(m f), for m < 0 sqrt(2) K_l|m| P_l^|m|(cos t)
sin(|m| f), K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m = (sin t)^m
d^m P_l / du^m without the Condon-Shortley sign (so Y_11 ~ +x, Y_1-1 ~ +y).
"""
from fractions import Fraction
from functools import lru_cache
from math import comb, factorial, sqrt

import numpy as np


def nsho(nu):
    return (nu + 1) * (nu + 2) * (nu + 3) // 6


def coeff_index(nu_max, nx, ny, nz):
    """Position of (nx, ny, nz) in the library's coefficient order (nz outer,
    then ny, nx fastest, nx + ny + nz <= nu_max), by enumeration."""
    k = 0
    for z in range(nu_max + 1):
        for y in range(nu_max + 1 - z):
            for x in range(nu_max + 1 - z - y):
                if (x, y, z) == (nx, ny, nz):
                    return k
                k += 1
    raise ValueError("not in the basis")


def radial_states(nu_max):
    """(nu, l, m, nr) in radial order."""
    out = []
    for nu in range(nu_max + 1):
        for l in range(nu % 2, nu + 1, 2):
            for m in range(-l, l + 1):
                out.append((nu, l, m, (nu - l) // 2))
    return out


def cartesian_states(nu_max):
    """(nx, ny, nz) in coefficient order."""
    return [(x, y, z) for z in range(nu_max + 1) for y in range(nu_max + 1 - z)
            for x in range(nu_max + 1 - z - y)]


# ------------------------------------------------------ exact polynomials --

def _hermite(n):
    """Physicists' H_n: {power: integer coefficient}."""
    return {n - 2 * k: (-1) ** k * factorial(n) * 2 ** (n - 2 * k)
            // (factorial(k) * factorial(n - 2 * k)) for k in range(n // 2 + 1)}


def _mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return {k: v for k, v in out.items() if v != 0}


def _add(p, q, s=1):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v != 0}


_R2 = {(2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1}


def _pow(p, k):
    out = {(0, 0, 0): 1}
    for _ in range(k):
        out = _mul(out, p)
    return out


def _xy_power(m):
    """(x + i y)^m = C + i S as two monomial dicts."""
    C, S = {}, {}
    for k in range(m + 1):
        c = comb(m, k)  # x^(m-k) (i y)^k
        if k % 4 == 0:
            C[(m - k, k, 0)] = c
        elif k % 4 == 1:
            S[(m - k, k, 0)] = c
        elif k % 4 == 2:
            C[(m - k, k, 0)] = -c
        else:
            S[(m - k, k, 0)] = -c
    return C, S


def _solid(l, m):
    """r^l Y_lm / K as (monomials with rational coefficients, K^2 rational
    part, where K^2 = (rational) / pi)."""
    am = abs(m)
    # r^(l-am) d^am P_l/du^am (z/r) = sum_k c_k z^(l-2k-am) r^(2k)
    poly = {}
    for k in range((l - am) // 2 + 1):
        c = Fraction((-1) ** k * comb(l, k) * comb(2 * l - 2 * k, l)
                     * factorial(l - 2 * k), 2 ** l * factorial(l - 2 * k - am))
        term = _mul({(0, 0, l - 2 * k - am): c}, _pow(_R2, k))
        poly = _add(poly, term)
    C, S = _xy_power(am)
    part = {(0, 0, 0): 1} if m == 0 else (C if m > 0 else S)
    poly = _mul(poly, part)
    k2 = Fraction(2 * l + 1, 4) * Fraction(factorial(l - am), factorial(l + am))
    if m != 0:
        k2 *= 2
    return poly, k2


def _laguerre(n, l):
    """L_n^(l+1/2)(t): {power of t: rational}."""
    a = Fraction(2 * l + 1, 2)
    out = {}
    for i in range(n + 1):
        # binom(n + a, n - i) = prod_{k=1}^{n-i} (a + i + k) / k
        b = Fraction(1)
        for k in range(1, n - i + 1):
            b *= (a + i + k) / k
        out[i] = (-1) ** i * b / factorial(i)
    return out


def _gamma_half_rational(k):
    """Gamma(k + 1/2) / sqrt(pi) as a rational."""
    return Fraction(factorial(2 * k), 4 ** k * factorial(k))


@lru_cache(maxsize=None)
def _radial_poly(nr, l, m):
    """Psi_s exp(r^2/2) = sqrt(q / pi^(3/2)) * poly, poly rational: (poly, q)."""
    S, k2 = _solid(l, m)
    L = _laguerre(nr, l)
    Lp = {}
    for i, c in L.items():
        Lp = _add(Lp, {kk: c * v for kk, v in _pow(_R2, i).items()})
    poly = _mul(S, Lp)
    # N^2 = 2 nr! / Gamma(nr + l + 3/2) = 2 nr! / (G * sqrt(pi)), K^2 = k2 / pi
    n2 = Fraction(2 * factorial(nr)) / _gamma_half_rational(nr + l + 1)
    return poly, n2 * k2


def _moment_rational(a):
    """int x^a exp(-x^2) dx / sqrt(pi)."""
    return 0 if a % 2 else _gamma_half_rational(a // 2)


@lru_cache(maxsize=None)
def _hermite_moment(n, a):
    """int H_n(x) x^a exp(-x^2) dx / sqrt(pi), rational."""
    return sum(Fraction(c) * _moment_rational(p + a) for p, c in _hermite(n).items())


def unitary(nu_max):
    """U[c][s] = <Phi_c | Psi_s>, [N_SHO][N_SHO], block diagonal in nu."""
    N = nsho(nu_max)
    cart = cartesian_states(nu_max)
    rad = radial_states(nu_max)
    U = np.zeros((N, N))
    for si, (nu, l, m, nr) in enumerate(rad):
        poly, q = _radial_poly(nr, l, m)
        for ci, (nx, ny, nz) in enumerate(cart):
            if nx + ny + nz != nu:
                continue
            acc = Fraction(0)
            for (a, b, c), v in poly.items():
                acc += v * _hermite_moment(nx, a) * _hermite_moment(ny, b) * _hermite_moment(nz, c)
            if acc == 0:
                continue
            # Phi_c exp(r^2/2) = H H H / sqrt(pi^(3/2) prod 2^n n!)
            qc = Fraction(1, 2 ** (nx + ny + nz) * factorial(nx) * factorial(ny) * factorial(nz))
            # pi powers: Phi pi^(-3/4), Psi pi^(-3/4), moments pi^(3/2)
            U[ci, si] = float(acc) * sqrt(float(qc * q))
    return U


# ------------------------------------------------------- radial functions --

def radial(nr, l, sigma, r):
    """R_{nr l}(r; sigma), normalised with weight r^2 dr."""
    from scipy.special import eval_genlaguerre, gammaln
    t = np.asarray(r, dtype=np.float64) / sigma
    logn = 0.5 * (np.log(2.0) + gammaln(nr + 1) - gammaln(nr + l + 1.5))
    return np.exp(logn) * t ** l * eval_genlaguerre(nr, l + 0.5, t * t) * np.exp(-0.5 * t * t) \
        * sigma ** -1.5


def projector_list(ell):
    """(k, l, m) of every projector j, m = -l..l per radial function k."""
    return [(k, l, m) for k, l in enumerate(ell) for m in range(-l, l + 1)]


def F_matrix(nu_max, sigma, ell, r, w, P):
    """F[j][s] = <p_j | Psi_s> = delta(l) delta(m) sum_i w_i r_i^2 P_k(r_i) R(r_i)."""
    r = np.asarray(r, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64).reshape(len(ell), r.size)
    projs = projector_list(ell)
    rad = radial_states(nu_max)
    F = np.zeros((len(projs), len(rad)))
    for j, (k, lk, mk) in enumerate(projs):
        for s, (nu, l, m, nr) in enumerate(rad):
            if l == lk and m == mk:
                F[j, s] = np.sum(w * r * r * P[k] * radial(nr, l, sigma, r))
    return F


def setup_matrix(nu_max, sigma, ell, r, w, P, D):
    """script-D = M^T D M, M = F U^T, in the coefficient order."""
    F = F_matrix(nu_max, sigma, ell, r, w, P)
    M = F @ unitary(nu_max).T
    D = np.asarray(D, dtype=np.float64).reshape(M.shape[0], M.shape[0])
    return M.T @ D @ M


def quality(nu_max, sigma, l, r, w, P):
    """Q_nu for nu = 0..nu_max (zero below l)."""
    r = np.asarray(r, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    norm = np.sum(w * r * r * P * P)
    Q = np.zeros(nu_max + 1)
    for nu in range(nu_max + 1):
        if nu < l:
            continue
        acc = 0.0
        for nr in range((nu - l) // 2 + 1):
            acc += np.sum(w * r * r * P * radial(nr, l, sigma, r)) ** 2
        Q[nu] = acc / norm
    return Q
