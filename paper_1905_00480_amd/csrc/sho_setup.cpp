// sho_setup.cpp -- host-side set-up of the SHO projector basis.
//
// What the paper does once per SCF cycle (sec. 3.5): the numerical radial
// projectors p_j = P_k(r) Y_lm are replaced by the Cartesian SHO basis, and
// the atomic matrix D becomes script-D = U^T F^T D F U in that basis, so that
// the grid kernels only ever project onto, and expand from, the separable
// functions phi_nx(x) phi_ny(y) phi_nz(z).  Here:
//
//  * U[c][s] = <Phi_c | Psi_s> between the Cartesian states (coefficient
//    order) and the radial states Psi_s = R_{nr l}(r) Y_lm (sec. 2.3-2.5).
//    Both are a polynomial of degree nu times exp(-r^2/2), so the product
//    Gauss-Hermite rule with nu + 1 nodes per axis integrates every entry
//    exactly (up to rounding).  The nodes are the roots of the orthonormal
//    Hermite polynomial h_{nu+1} (bracketed on a fine scan, then bisected);
//    the weights are the Christoffel numbers 1 / sum_{k<=nu} h_k(x)^2.
//  * Radial functions R_{nr l}(r) = N r~^l L_nr^(l+1/2)(r~^2) exp(-r~^2/2)
//    sigma^(-3/2), r~ = r/sigma, N^2 = 2 nr! / Gamma(nr+l+3/2), from the
//    three-term recurrence of the generalised Laguerre polynomials.
//  * Real solid harmonics r^l Y_lm from the associated Legendre recurrence
//    written in z and r^2, times the real / imaginary part of (x + i y)^|m|
//    (no Condon-Shortley sign: Y_11 ~ +x, Y_1-1 ~ +y).
//  * F[j][s] = <p_j | Psi_s> by the caller's radial quadrature, M = F U^T,
//    script-D = M^T D M; the representation quality Q_nu of sec. 4.
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "sho_internal.hpp"

namespace sho {
sho_status fail(sho_status code, const std::string &msg);
}

using sho::fail;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Orthonormal Hermite polynomials (weight exp(-x^2)) h_0..h_n at x.
void hermite_on(int n, double x, double *h) {
  h[0] = std::pow(kPi, -0.25);
  if (n >= 1) h[1] = std::sqrt(2.0) * x * h[0];
  for (int k = 1; k < n; ++k)
    h[k + 1] = std::sqrt(2.0 / (k + 1)) * x * h[k] - std::sqrt((double)k / (k + 1)) * h[k - 1];
}

// Gauss-Hermite rule with n nodes: sum_i w_i g(x_i) = int g(x) exp(-x^2) dx
// for polynomials g of degree <= 2n - 1.
void gauss_hermite(int n, std::vector<double> *x, std::vector<double> *w) {
  x->clear();
  w->clear();
  std::vector<double> h(n + 1);
  auto hn = [&](double t) {
    hermite_on(n, t, h.data());
    return h[n];
  };
  const double lim = std::sqrt(2.0 * n + 1.0) + 1.0;
  const int steps = 400 * n;
  double a = -lim, fa = hn(a);
  for (int i = 1; i <= steps; ++i) {
    const double b = -lim + 2.0 * lim * i / steps;
    const double fb = hn(b);
    if (fa == 0.0) {
      x->push_back(a);
    } else if (fa * fb < 0.0) {
      double lo = a, hi = b, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = hn(mid);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      x->push_back(0.5 * (lo + hi));
    }
    a = b;
    fa = fb;
  }
  for (double t : *x) {
    hermite_on(n - 1, t, h.data());
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += h[k] * h[k];
    w->push_back(1.0 / s);
  }
}

// Generalised Laguerre L_0..L_n^(alpha)(t).
void laguerre(int n, double alpha, double t, double *L) {
  L[0] = 1.0;
  if (n >= 1) L[1] = 1.0 + alpha - t;
  for (int k = 1; k < n; ++k)
    L[k + 1] = ((2.0 * k + 1.0 + alpha - t) * L[k] - (k + alpha) * L[k - 1]) / (k + 1.0);
}

double radial_norm(int nr, int l) {
  return std::exp(0.5 * (std::log(2.0) + std::lgamma(nr + 1.0) - std::lgamma(nr + l + 1.5)));
}

// R_{nr l}(r; sigma)
double radial_value(int nr, int l, double sigma, double r) {
  const double t = r / sigma;
  std::vector<double> L(nr + 1);
  laguerre(nr, l + 0.5, t * t, L.data());
  return radial_norm(nr, l) * std::pow(t, l) * L[nr] * std::exp(-0.5 * t * t) *
         std::pow(sigma, -1.5);
}

// Real solid harmonics r^l Y_lm for l <= lmax at (x, y, z): out[l*l + l + m].
void solid_harmonics(int lmax, double x, double y, double z, double *out) {
  const double r2 = x * x + y * y + z * z;
  std::vector<double> C(lmax + 1), S(lmax + 1), P(lmax + 1);
  C[0] = 1.0;
  S[0] = 0.0;
  for (int m = 1; m <= lmax; ++m) {
    C[m] = x * C[m - 1] - y * S[m - 1];
    S[m] = x * S[m - 1] + y * C[m - 1];
  }
  double dfact = 1.0;  // (2m - 1)!!
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) dfact *= (2.0 * m - 1.0);
    // P[l] = r^(l-m) d^m P_l / du^m (u = z/r), l = m..lmax
    P[m] = dfact;
    if (m + 1 <= lmax) P[m + 1] = (2.0 * m + 1.0) * z * P[m];
    for (int l = m + 2; l <= lmax; ++l)
      P[l] = ((2.0 * l - 1.0) * z * P[l - 1] - (l + m - 1.0) * r2 * P[l - 2]) / (l - m);
    for (int l = m; l <= lmax; ++l) {
      const double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) *
                                 std::exp(std::lgamma(l - m + 1.0) - std::lgamma(l + m + 1.0)));
      if (m == 0) {
        out[l * l + l] = K * P[l];
      } else {
        out[l * l + l + m] = std::sqrt(2.0) * K * P[l] * C[m];
        out[l * l + l - m] = std::sqrt(2.0) * K * P[l] * S[m];
      }
    }
  }
}

struct RadialState {
  int nu, l, m, nr;
};

std::vector<RadialState> radial_states(int nu_max) {
  std::vector<RadialState> v;
  for (int nu = 0; nu <= nu_max; ++nu)
    for (int l = nu % 2; l <= nu; l += 2)
      for (int m = -l; m <= l; ++m) v.push_back({nu, l, m, (nu - l) / 2});
  return v;
}

struct CartState {
  int nx, ny, nz;
};

std::vector<CartState> cart_states(int nu_max) {
  std::vector<CartState> v;
  for (int z = 0; z <= nu_max; ++z)
    for (int y = 0; y <= nu_max - z; ++y)
      for (int x = 0; x <= nu_max - z - y; ++x) v.push_back({x, y, z});
  return v;
}

// U [N][N] row-major (rows Cartesian, columns radial), shell by shell.
// False if a Gauss-Hermite rule did not come out with all its nodes.
bool build_unitary(int nu_max, double *U) {
  const auto cart = cart_states(nu_max);
  const auto rad = radial_states(nu_max);
  const size_t N = cart.size();
  for (size_t i = 0; i < N * N; ++i) U[i] = 0.0;
  std::vector<double> gx, gw, hx(nu_max + 1), hy(nu_max + 1), hz(nu_max + 1);
  std::vector<double> Y((nu_max + 1) * (nu_max + 1)), L(nu_max + 1);
  for (int nu = 0; nu <= nu_max; ++nu) {
    std::vector<int> cs, ss;
    for (size_t c = 0; c < N; ++c)
      if (cart[c].nx + cart[c].ny + cart[c].nz == nu) cs.push_back((int)c);
    for (size_t s = 0; s < N; ++s)
      if (rad[s].nu == nu) ss.push_back((int)s);
    gauss_hermite(nu + 1, &gx, &gw);
    const int nq = (int)gx.size();
    if (nq != nu + 1) return false;
    std::vector<double> cv(cs.size()), rv(ss.size());
    for (int i = 0; i < nq; ++i) {
      hermite_on(nu, gx[i], hx.data());
      for (int j = 0; j < nq; ++j) {
        hermite_on(nu, gx[j], hy.data());
        for (int k = 0; k < nq; ++k) {
          hermite_on(nu, gx[k], hz.data());
          const double x = gx[i], y = gx[j], z = gx[k];
          const double W = gw[i] * gw[j] * gw[k];
          for (size_t a = 0; a < cs.size(); ++a) {
            const CartState &q = cart[cs[a]];
            cv[a] = hx[q.nx] * hy[q.ny] * hz[q.nz];
          }
          solid_harmonics(nu, x, y, z, Y.data());
          const double r2 = x * x + y * y + z * z;
          for (size_t b = 0; b < ss.size(); ++b) {
            const RadialState &q = rad[ss[b]];
            laguerre(q.nr, q.l + 0.5, r2, L.data());
            rv[b] = W * radial_norm(q.nr, q.l) * L[q.nr] * Y[q.l * q.l + q.l + q.m];
          }
          for (size_t a = 0; a < cs.size(); ++a)
            for (size_t b = 0; b < ss.size(); ++b) U[cs[a] * N + ss[b]] += cv[a] * rv[b];
        }
      }
    }
  }
  return true;
}

bool sigma_ok(double s) { return std::isfinite(s) && s > 0.0; }

}  // namespace

extern "C" {

sho_status sho_setup_unitary(int32_t nu_max, double *U) {
  if (!U) return fail(SHO_E_INVALID, "U must not be NULL");
  if (nu_max < 0 || nu_max > SHO_NU_MAX) return fail(SHO_E_NU_RANGE, "nu_max out of range");
  if (!build_unitary(nu_max, U)) return fail(SHO_E_INVALID, "Gauss-Hermite nodes not found");
  return SHO_OK;
}

sho_status sho_setup_radial(int32_t nu_max, double sigma, int64_t npts, const double *r,
                            double *R) {
  if (nu_max < 0 || nu_max > SHO_SETUP_NU_MAX)
    return fail(SHO_E_NU_RANGE, "nu_max out of range");
  if (!sigma_ok(sigma)) return fail(SHO_E_INVALID, "sigma must be positive and finite");
  if (npts < 0 || (npts > 0 && (!r || !R))) return fail(SHO_E_INVALID, "NULL or negative size");
  int64_t k = 0;
  for (int nu = 0; nu <= nu_max; ++nu)
    for (int l = nu % 2; l <= nu; l += 2, ++k)
      for (int64_t i = 0; i < npts; ++i)
        R[k * npts + i] = radial_value((nu - l) / 2, l, sigma, r[i]);
  return SHO_OK;
}

sho_status sho_setup_matrix(int32_t nu_max, double sigma, int32_t nrad, const int32_t *ell,
                            int64_t ngrid, const double *r, const double *w, const double *P,
                            const double *D, double *out) {
  if (nu_max < 0 || nu_max > SHO_NU_MAX) return fail(SHO_E_NU_RANGE, "nu_max out of range");
  if (!sigma_ok(sigma)) return fail(SHO_E_INVALID, "sigma must be positive and finite");
  if (nrad < 0 || ngrid < 1 || !out || (nrad > 0 && (!ell || !r || !w || !P || !D)))
    return fail(SHO_E_INVALID, "NULL argument or bad size");
  int64_t nproj = 0;
  for (int32_t k = 0; k < nrad; ++k) {
    if (ell[k] < 0 || ell[k] > SHO_SETUP_NU_MAX)
      return fail(SHO_E_INVALID, "angular momentum out of range");
    nproj += 2 * ell[k] + 1;
  }
  const auto rad = radial_states(nu_max);
  const int64_t N = (int64_t)rad.size();
  std::vector<double> U(N * N);
  if (!build_unitary(nu_max, U.data()))
    return fail(SHO_E_INVALID, "Gauss-Hermite nodes not found");
  // F[j][s]: only s with the projector's (l, m) are non-zero
  std::vector<double> F(nproj * N, 0.0);
  int64_t j0 = 0;
  for (int32_t k = 0; k < nrad; ++k) {
    const int l = ell[k];
    for (int nr = 0; l + 2 * nr <= nu_max; ++nr) {
      double f = 0.0;
      for (int64_t i = 0; i < ngrid; ++i)
        f += w[i] * r[i] * r[i] * P[k * ngrid + i] * radial_value(nr, l, sigma, r[i]);
      for (int m = -l; m <= l; ++m)
        for (int64_t s = 0; s < N; ++s)
          if (rad[s].l == l && rad[s].nr == nr && rad[s].m == m) F[(j0 + m + l) * N + s] = f;
    }
    j0 += 2 * l + 1;
  }
  // M = F U^T, then out = M^T D M
  std::vector<double> M(nproj * N, 0.0), DM(nproj * N, 0.0);
  for (int64_t j = 0; j < nproj; ++j)
    for (int64_t c = 0; c < N; ++c) {
      double acc = 0.0;
      for (int64_t s = 0; s < N; ++s) acc += F[j * N + s] * U[c * N + s];
      M[j * N + c] = acc;
    }
  for (int64_t i = 0; i < nproj; ++i)
    for (int64_t c = 0; c < N; ++c) {
      double acc = 0.0;
      for (int64_t j = 0; j < nproj; ++j) acc += D[i * nproj + j] * M[j * N + c];
      DM[i * N + c] = acc;
    }
  for (int64_t a = 0; a < N; ++a)
    for (int64_t b = 0; b < N; ++b) {
      double acc = 0.0;
      for (int64_t i = 0; i < nproj; ++i) acc += M[i * N + a] * DM[i * N + b];
      out[a * N + b] = acc;
    }
  return SHO_OK;
}

sho_status sho_setup_quality(int32_t nu_max, double sigma, int32_t ell, int64_t ngrid,
                             const double *r, const double *w, const double *P, double *Q) {
  if (nu_max < 0 || nu_max > SHO_SETUP_NU_MAX)
    return fail(SHO_E_NU_RANGE, "nu_max out of range");
  if (!sigma_ok(sigma)) return fail(SHO_E_INVALID, "sigma must be positive and finite");
  if (ell < 0 || ngrid < 1 || !r || !w || !P || !Q)
    return fail(SHO_E_INVALID, "NULL argument or bad size");
  double norm = 0.0;
  for (int64_t i = 0; i < ngrid; ++i) norm += w[i] * r[i] * r[i] * P[i] * P[i];
  if (!(norm > 0.0)) return fail(SHO_E_INVALID, "projector has zero norm on the quadrature");
  double acc = 0.0;
  for (int nu = 0; nu <= nu_max; ++nu) {
    if (nu >= ell && (nu - ell) % 2 == 0) {
      const int nr = (nu - ell) / 2;
      double f = 0.0;
      for (int64_t i = 0; i < ngrid; ++i)
        f += w[i] * r[i] * r[i] * P[i] * radial_value(nr, ell, sigma, r[i]);
      acc += f * f;
    }
    Q[nu] = nu >= ell ? acc / norm : 0.0;
  }
  return SHO_OK;
}

}  // extern "C"
