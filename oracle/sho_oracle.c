/*
 * sho_oracle.c -- plain, slow CPU oracle for SHO projection, expansion and
 * position derivatives.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * What it computes, written directly from the paper's definitions
 * (Baumeister & Tsukamoto, "Analytical PAW Projector Functions for Reduced
 * Bandwidth Requirements", PASC'19):
 *
 *   phi_n(u; sigma)   1D harmonic-oscillator eigenfunction, Hermite polynomial
 *                     times Gaussian (sec. 2.2, eq. 1HO-eigenstate), with the
 *                     polynomial taken from the monic three-term recurrence of
 *                     sec. 3.7 and an L2(R) normalisation the paper leaves out
 *                     ("omitted ... for simplicity", sec. 2.2).
 *   P_an(i)           Cartesian product phi_nx phi_ny phi_nz (sec. 2.2,
 *                     eq. SHO-factorizable-basis), truncated to
 *                     nx+ny+nz <= nu_max (sec. 2.5, eq. SHO-basis).
 *   projection        c[a][n][b] = h^3 sum_{i in S_a} P_an(i) psi_b(i)
 *                     (sec. 3.2 step 1; the integral of sec. 3.5 sampled on
 *                     the grid) -- the plain triple sum, no factorisation.
 *   expansion         psi_b(j) += sum_a sum_{i in S_a, i = j mod N}
 *                     sum_n c[a][n][b] P_an(i)   (sec. 3.2 step 3, "add").
 *   derivative        g[a][d] = sum_{n,b} w[a][n][b] dc[a][n][b]/dR_{a,d},
 *                     support S_a frozen; d/du of the sampled functions taken
 *                     from the monic polynomial directly (H'_n = n H_{n-1}).
 *   complex bands     Bloch bands at a wave vector k (sec. 2.5: the basis
 *   at k              spans functions R^3 -> C): every periodic image of a
 *                     support point carries the phase e^{+-i k.T} of its
 *                     lattice translation T (oracle_project_k / _expand_k).
 *
 * Sums are accumulated in long double so that the oracle's own rounding error
 * stays far below the comparison tolerance.  Membership in the support is
 * decided in IEEE double in a fixed operation order (see in_support).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (oracle/build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NU_MAX 16

/* ---------------------------------------------------------------- basics -- */

/* N_SHO = (nu+1)(nu+2)(nu+3)/6, sec. 2.5 eq. SHO_basis_size */
int oracle_nsho(int nu) { return (nu + 1) * (nu + 2) * (nu + 3) / 6; }

/* Coefficient order: nz outermost, then ny, nx fastest, over nx+ny+nz <= nu.
 * Counted by brute force so that the index is obviously the position in
 * that enumeration. */
int oracle_coeff_index(int nu, int nx, int ny, int nz) {
  int idx = 0;
  for (int z = 0; z <= nu; ++z)
    for (int y = 0; y <= nu - z; ++y)
      for (int x = 0; x <= nu - z - y; ++x) {
        if (x == nx && y == ny && z == nz) return idx;
        ++idx;
      }
  return -1;
}

/* Paper's monic recurrence (sec. 3.7):
 *   H_0 = 1, H_1 = t, H_{n+1} = t H_n - (n/2) H_{n-1}. */
static void hermite_monic(int nmax, double t, double *H) {
  H[0] = 1.0;
  if (nmax >= 1) H[1] = t;
  for (int n = 1; n < nmax; ++n) H[n + 1] = t * H[n] - 0.5 * n * H[n - 1];
}

/* (2^n / (n! sqrt(pi) sigma))^(1/2): makes int phi_n^2 du = 1 for the monic
 * polynomial above (monic H_n = physicists' H_n / 2^n). */
static double phi_norm(int n, double sigma) {
  double f = 1.0;
  for (int k = 1; k <= n; ++k) f *= 2.0 / (double)k;
  return sqrt(f / (sqrt(M_PI) * sigma));
}

/* phi_n(u; sigma) for n = 0..nu into out[0..nu] */
static void phi_all(int nu, double sigma, double u, double *out) {
  double H[ORACLE_NU_MAX + 2];
  double t = u / sigma;
  hermite_monic(nu, t, H);
  double g = exp(-0.5 * t * t);
  for (int n = 0; n <= nu; ++n) out[n] = phi_norm(n, sigma) * H[n] * g;
}

/* d/du phi_n(u; sigma) = (1/sigma) N_n (n H_{n-1}(t) - t H_n(t)) e^{-t^2/2} */
static void dphi_all(int nu, double sigma, double u, double *out) {
  double H[ORACLE_NU_MAX + 2];
  double t = u / sigma;
  hermite_monic(nu, t, H);
  double g = exp(-0.5 * t * t);
  for (int n = 0; n <= nu; ++n) {
    double dH = (n > 0) ? (double)n * H[n - 1] : 0.0;
    out[n] = phi_norm(n, sigma) * (dH - t * H[n]) * g / sigma;
  }
}

/* Exported samplers: out[n*m + j] = phi_n(u[j]) */
int oracle_phi(int nu, double sigma, int m, const double *u, double *out) {
  if (nu < 0 || nu > ORACLE_NU_MAX || !(sigma > 0)) return -1;
  double v[ORACLE_NU_MAX + 1];
  for (int j = 0; j < m; ++j) {
    phi_all(nu, sigma, u[j], v);
    for (int n = 0; n <= nu; ++n) out[(int64_t)n * m + j] = v[n];
  }
  return 0;
}

int oracle_dphi(int nu, double sigma, int m, const double *u, double *out) {
  if (nu < 0 || nu > ORACLE_NU_MAX || !(sigma > 0)) return -1;
  double v[ORACLE_NU_MAX + 1];
  for (int j = 0; j < m; ++j) {
    dphi_all(nu, sigma, u[j], v);
    for (int n = 0; n <= nu; ++n) out[(int64_t)n * m + j] = v[n];
  }
  return 0;
}

/* ------------------------------------------------------------- geometry -- */

typedef struct {
  int n[3];        /* points per axis x, y, z */
  double h;        /* grid spacing; point i sits at i*h */
  int periodic[3]; /* 1: index taken modulo n; 0: points outside 0..n-1 dropped */
} ogrid;

/* Default box radius: classical turning radius of shell nu, sigma*sqrt(2nu+3)
 * (sec. 2.2 eq. SHO-energy-Cartesian with the potential r^2 sigma^-4 of
 * eq. SHO_Hamiltonian), plus two grid spacings. */
static double box_radius(double sigma, int nu, double h) {
  return sigma * sqrt(2.0 * nu + 3.0) + 2.0 * h;
}

/* Membership of unwrapped point i in the support sphere of radius R around
 * centre c.  Fixed IEEE-double operation order:
 *   d = i*h - c per axis;  r2 = (dx*dx + dy*dy) + dz*dz;  r2 <= R*R */
static int in_support(const int i[3], const double c[3], double h, double R) {
  double dx = (double)i[0] * h - c[0];
  double dy = (double)i[1] * h - c[1];
  double dz = (double)i[2] * h - c[2];
  double r2 = dx * dx + dy * dy;
  r2 = r2 + dz * dz;
  return r2 <= R * R;
}

static int wrap(int i, int n) {
  int m = i % n;
  return m < 0 ? m + n : m;
}

/* Scan range guaranteed to contain every member along one axis. */
static void scan_range(double c, double R, double h, int *lo, int *hi) {
  *lo = (int)floor((c - R) / h) - 1;
  *hi = (int)ceil((c + R) / h) + 1;
}

/* Visit every support point of one atom: calls fn(ctx, i_unwrapped, memidx) */
typedef void (*visit_fn)(void *ctx, const int i[3], int64_t mem);

static void visit_support(const ogrid *g, const double sc[3], double R,
                          visit_fn fn, void *ctx) {
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) scan_range(sc[d], R, g->h, &lo[d], &hi[d]);
  int i[3];
  for (i[2] = lo[2]; i[2] <= hi[2]; ++i[2]) {
    if (!g->periodic[2] && (i[2] < 0 || i[2] >= g->n[2])) continue;
    for (i[1] = lo[1]; i[1] <= hi[1]; ++i[1]) {
      if (!g->periodic[1] && (i[1] < 0 || i[1] >= g->n[1])) continue;
      for (i[0] = lo[0]; i[0] <= hi[0]; ++i[0]) {
        if (!g->periodic[0] && (i[0] < 0 || i[0] >= g->n[0])) continue;
        if (!in_support(i, sc, g->h, R)) continue;
        int64_t mem = ((int64_t)wrap(i[2], g->n[2]) * g->n[1] +
                       wrap(i[1], g->n[1])) * g->n[0] + wrap(i[0], g->n[0]);
        fn(ctx, i, mem);
      }
    }
  }
}

static int check_grid(const int n[3], double h, const int periodic[3],
                      ogrid *g) {
  if (!(h > 0)) return -1;
  for (int d = 0; d < 3; ++d) {
    if (n[d] <= 0) return -1;
    g->n[d] = n[d];
    g->periodic[d] = periodic[d] ? 1 : 0;
  }
  g->h = h;
  return 0;
}

/* Number of support points of one atom, and optionally their unwrapped
 * indices (out[3*k + d]) and memory indices (mem[k]). */
typedef struct {
  int64_t count, cap;
  int *out;
  int64_t *mem;
} collect_ctx;

static void collect_fn(void *p, const int i[3], int64_t m) {
  collect_ctx *c = (collect_ctx *)p;
  if (c->count < c->cap) {
    if (c->out)
      for (int d = 0; d < 3; ++d) c->out[3 * c->count + d] = i[d];
    if (c->mem) c->mem[c->count] = m;
  }
  c->count++;
}

int64_t oracle_support(const int n[3], double h, const int periodic[3],
                       const double centre[3], double R, int64_t cap,
                       int *out, int64_t *mem) {
  ogrid g;
  if (check_grid(n, h, periodic, &g)) return -1;
  collect_ctx c = {0, cap, out, mem};
  visit_support(&g, centre, R, collect_fn, &c);
  return c.count;
}

double oracle_box_radius(double sigma, int nu, double h) {
  return box_radius(sigma, nu, h);
}

/* Per-atom offsets of coefficient blocks [N_SHO(nu_a)][B], in doubles. */
static int64_t coeff_offset(const int *numax, int a, int B) {
  int64_t off = 0;
  for (int k = 0; k < a; ++k) off += (int64_t)oracle_nsho(numax[k]) * B;
  return off;
}

static int check_atoms(int natoms, const double *sigma, const int *numax,
                       int extra) {
  if (natoms < 0) return -1;
  for (int a = 0; a < natoms; ++a) {
    if (!(sigma[a] > 0)) return -1;
    if (numax[a] < 0 || numax[a] + extra > ORACLE_NU_MAX) return -1;
  }
  return 0;
}

/* ----------------------------------------------------------- projection -- */

typedef struct {
  const ogrid *g;
  const double *fc; /* function centre */
  double sigma;
  int nu, B;
  const double *psi;
  long double *acc; /* [N][B] */
  long double *abs; /* [N][B] */
} prj_ctx;

static void prj_fn(void *p, const int i[3], int64_t mem) {
  prj_ctx *c = (prj_ctx *)p;
  double fx[ORACLE_NU_MAX + 1], fy[ORACLE_NU_MAX + 1], fz[ORACLE_NU_MAX + 1];
  phi_all(c->nu, c->sigma, (double)i[0] * c->g->h - c->fc[0], fx);
  phi_all(c->nu, c->sigma, (double)i[1] * c->g->h - c->fc[1], fy);
  phi_all(c->nu, c->sigma, (double)i[2] * c->g->h - c->fc[2], fz);
  const double *ps = c->psi + mem * c->B;
  int idx = 0;
  for (int nz = 0; nz <= c->nu; ++nz)
    for (int ny = 0; ny <= c->nu - nz; ++ny)
      for (int nx = 0; nx <= c->nu - nz - ny; ++nx, ++idx) {
        double P = fx[nx] * fy[ny] * fz[nz];
        long double *acc = c->acc + (int64_t)idx * c->B;
        long double *ab = c->abs + (int64_t)idx * c->B;
        for (int b = 0; b < c->B; ++b) {
          acc[b] += (long double)P * ps[b];
          ab[b] += fabsl((long double)P * ps[b]);
        }
      }
}

/*
 * c[off_a + n*B + b] = h^3 sum_{i in S_a} P_an(i) psi[mem(i)*B + b]
 * psi layout [z][y][x][b]; c per-atom blocks in atom order.
 * rbox: per-atom support radius or NULL for the default rule.
 * spos: per-atom support centre [natoms][3] or NULL (= pos).  A separate
 *       support centre freezes the point set while the functions move.
 * cabs: optional, same layout as c: h^3 sum |P psi|.
 */
int oracle_project(const int n[3], double h, const int periodic[3],
                   int natoms, const double *pos, const double *sigma,
                   const int *numax, const double *rbox, const double *spos,
                   int B, const double *psi, double *c, double *cabs) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
  const double h3 = h * h * h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < natoms; ++a) {
    int nu = numax[a], N = oracle_nsho(nu);
    long double *acc = calloc((size_t)N * B, sizeof(long double));
    long double *ab = calloc((size_t)N * B, sizeof(long double));
    prj_ctx ctx = {&g, pos + 3 * a, sigma[a], nu, B, psi, acc, ab};
    double R = rbox ? rbox[a] : box_radius(sigma[a], nu, h);
    visit_support(&g, spos ? spos + 3 * a : pos + 3 * a, R, prj_fn, &ctx);
    int64_t off = coeff_offset(numax, a, B);
    for (int64_t k = 0; k < (int64_t)N * B; ++k) {
      c[off + k] = (double)(h3 * acc[k]);
      if (cabs) cabs[off + k] = (double)(h3 * ab[k]);
    }
    free(acc);
    free(ab);
  }
  return 0;
}

/* ------------------------------------------------------------ expansion -- */

typedef struct {
  const ogrid *g;
  const double *fc;
  double sigma;
  int nu, B, b0, b1;
  const double *cc; /* this atom's [N][B] */
  double *psi;
  double *pabs;
} add_ctx;

static void add_fn(void *p, const int i[3], int64_t mem) {
  add_ctx *c = (add_ctx *)p;
  double fx[ORACLE_NU_MAX + 1], fy[ORACLE_NU_MAX + 1], fz[ORACLE_NU_MAX + 1];
  phi_all(c->nu, c->sigma, (double)i[0] * c->g->h - c->fc[0], fx);
  phi_all(c->nu, c->sigma, (double)i[1] * c->g->h - c->fc[1], fy);
  phi_all(c->nu, c->sigma, (double)i[2] * c->g->h - c->fc[2], fz);
  for (int b = c->b0; b < c->b1; ++b) {
    long double s = 0, sa = 0;
    int idx = 0;
    for (int nz = 0; nz <= c->nu; ++nz)
      for (int ny = 0; ny <= c->nu - nz; ++ny)
        for (int nx = 0; nx <= c->nu - nz - ny; ++nx, ++idx) {
          double P = fx[nx] * fy[ny] * fz[nz];
          long double t = (long double)P * c->cc[(int64_t)idx * c->B + b];
          s += t;
          sa += fabsl(t);
        }
    c->psi[mem * c->B + b] += (double)s;
    if (c->pabs) c->pabs[mem * c->B + b] += (double)sa;
  }
}

/*
 * psi[mem*B+b] += sum_a sum_{i in S_a, mem(i)=mem} sum_n c[a][n][b] P_an(i)
 * psi is updated in place (accumulate semantics of sec. 3.2 step 3).
 * pabs (optional, grid layout): must hold |psi_in| on entry; receives
 * |psi_in| + sum |c P|.
 */
int oracle_expand(const int n[3], double h, const int periodic[3],
                  int natoms, const double *pos, const double *sigma,
                  const int *numax, const double *rbox, const double *spos,
                  int B, const double *c, double *psi, double *pabs) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
  /* Threads own disjoint band ranges, so no two threads touch one value. */
#pragma omp parallel
  {
    int nt = 1, t = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    t = omp_get_thread_num();
#endif
    int b0 = (int)((int64_t)B * t / nt), b1 = (int)((int64_t)B * (t + 1) / nt);
    if (b1 > b0)
      for (int a = 0; a < natoms; ++a) {
        add_ctx ctx = {&g,      pos + 3 * a, sigma[a], numax[a], B, b0, b1,
                       c + coeff_offset(numax, a, B), psi, pabs};
        double R = rbox ? rbox[a] : box_radius(sigma[a], numax[a], h);
        visit_support(&g, spos ? spos + 3 * a : pos + 3 * a, R, add_fn, &ctx);
      }
  }
  return 0;
}

/*
 * Expansion evaluated at selected memory points only:
 * out[k*B + b] = psi_in[k*B+b] + sum over atoms and over every unwrapped
 * support point i with mem(i) = pts[k] of sum_n c P.  psi_in (optional,
 * [npts][B]) holds the input values at those points.  oabs like out, with
 * |psi_in| + sum |c P|.
 */
typedef struct {
  int64_t target;
  int hit;
  int i[3];
  int nhits, cap;
  int *hits; /* unwrapped indices of the matches */
} find_ctx;

static void find_fn(void *p, const int i[3], int64_t mem) {
  find_ctx *f = (find_ctx *)p;
  if (mem != f->target) return;
  if (f->nhits < f->cap)
    for (int d = 0; d < 3; ++d) f->hits[3 * f->nhits + d] = i[d];
  f->nhits++;
}

int oracle_expand_at(const int n[3], double h, const int periodic[3],
                     int natoms, const double *pos, const double *sigma,
                     const int *numax, const double *rbox, int B,
                     const double *c, int64_t npts, const int64_t *pts,
                     const double *psi_in, double *out, double *oabs) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < npts; ++k) {
    long double *s = calloc((size_t)B, sizeof(long double));
    long double *sa = calloc((size_t)B, sizeof(long double));
    int hits[3 * 512];
    for (int b = 0; b < B; ++b) {
      double v = psi_in ? psi_in[k * B + b] : 0.0;
      s[b] = v;
      sa[b] = fabs(v);
    }
    for (int a = 0; a < natoms; ++a) {
      double R = rbox ? rbox[a] : box_radius(sigma[a], numax[a], h);
      find_ctx f = {pts[k], 0, {0, 0, 0}, 0, 512, hits};
      /* slow but plain: walk the whole support and keep the matches */
      visit_support(&g, pos + 3 * a, R, find_fn, &f);
      if (f.nhits > f.cap) {
#pragma omp atomic write
        fail = 1;
        continue;
      }
      const double *cc = c + coeff_offset(numax, a, B);
      int nu = numax[a];
      for (int q = 0; q < f.nhits; ++q) {
        double fx[ORACLE_NU_MAX + 1], fy[ORACLE_NU_MAX + 1],
            fz[ORACLE_NU_MAX + 1];
        phi_all(nu, sigma[a], (double)hits[3 * q] * h - pos[3 * a], fx);
        phi_all(nu, sigma[a], (double)hits[3 * q + 1] * h - pos[3 * a + 1], fy);
        phi_all(nu, sigma[a], (double)hits[3 * q + 2] * h - pos[3 * a + 2], fz);
        int idx = 0;
        for (int nz = 0; nz <= nu; ++nz)
          for (int ny = 0; ny <= nu - nz; ++ny)
            for (int nx = 0; nx <= nu - nz - ny; ++nx, ++idx) {
              double P = fx[nx] * fy[ny] * fz[nz];
              for (int b = 0; b < B; ++b) {
                long double t = (long double)P * cc[(int64_t)idx * B + b];
                s[b] += t;
                sa[b] += fabsl(t);
              }
            }
      }
    }
    for (int b = 0; b < B; ++b) {
      out[k * B + b] = (double)s[b];
      if (oabs) oabs[k * B + b] = (double)sa[b];
    }
    free(s);
    free(sa);
  }
  return fail ? -2 : 0;
}

/* ---------------------------------------------------------- derivative -- */

typedef struct {
  const ogrid *g;
  const double *fc;
  double sigma;
  int nu, B;
  const double *psi;
  long double *acc; /* [3][N][B] : sum dP/dR_d psi */
  long double *abs; /* [3][N][B] */
} frc_ctx;

static void frc_fn(void *p, const int i[3], int64_t mem) {
  frc_ctx *c = (frc_ctx *)p;
  double f[3][ORACLE_NU_MAX + 1], df[3][ORACLE_NU_MAX + 1];
  for (int d = 0; d < 3; ++d) {
    double u = (double)i[d] * c->g->h - c->fc[d];
    phi_all(c->nu, c->sigma, u, f[d]);
    dphi_all(c->nu, c->sigma, u, df[d]);
  }
  const double *ps = c->psi + mem * c->B;
  int N = oracle_nsho(c->nu);
  int idx = 0;
  for (int nz = 0; nz <= c->nu; ++nz)
    for (int ny = 0; ny <= c->nu - nz; ++ny)
      for (int nx = 0; nx <= c->nu - nz - ny; ++nx, ++idx) {
        /* dP/dR_d = -phi'_{n_d} * (other two factors): u = i*h - R */
        double dP[3] = {-df[0][nx] * f[1][ny] * f[2][nz],
                        -f[0][nx] * df[1][ny] * f[2][nz],
                        -f[0][nx] * f[1][ny] * df[2][nz]};
        for (int d = 0; d < 3; ++d) {
          long double *acc = c->acc + ((int64_t)d * N + idx) * c->B;
          long double *ab = c->abs + ((int64_t)d * N + idx) * c->B;
          for (int b = 0; b < c->B; ++b) {
            acc[b] += (long double)dP[d] * ps[b];
            ab[b] += fabsl((long double)dP[d] * ps[b]);
          }
        }
      }
}

/*
 * g[a][d] = sum_{n,b} w[off_a + n*B + b] * h^3 sum_{i in S_a} dP_an(i)/dR_d psi
 * with the support S_a frozen (built around spos, or pos when NULL).
 * gabs (optional): sum |w| h^3 sum |dP psi|.
 * dc (optional): [natoms-blocks][3][N][B] the coefficient derivatives.
 */
int oracle_force(const int n[3], double h, const int periodic[3], int natoms,
                 const double *pos, const double *sigma, const int *numax,
                 const double *rbox, const double *spos, int B,
                 const double *psi, const double *w, double *grad,
                 double *gabs, double *dc) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
  const double h3 = h * h * h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < natoms; ++a) {
    int nu = numax[a], N = oracle_nsho(nu);
    long double *acc = calloc((size_t)3 * N * B, sizeof(long double));
    long double *ab = calloc((size_t)3 * N * B, sizeof(long double));
    frc_ctx ctx = {&g, pos + 3 * a, sigma[a], nu, B, psi, acc, ab};
    double R = rbox ? rbox[a] : box_radius(sigma[a], nu, h);
    visit_support(&g, spos ? spos + 3 * a : pos + 3 * a, R, frc_fn, &ctx);
    int64_t off = coeff_offset(numax, a, B);
    for (int d = 0; d < 3; ++d) {
      long double s = 0, sa = 0;
      for (int64_t k = 0; k < (int64_t)N * B; ++k) {
        long double dck = h3 * acc[(int64_t)d * N * B + k];
        s += w[off + k] * dck;
        sa += fabsl((long double)w[off + k]) * h3 * ab[(int64_t)d * N * B + k];
        if (dc) dc[3 * off + (int64_t)d * N * B + k] = (double)dck;
      }
      grad[3 * a + d] = (double)s;
      if (gabs) gabs[3 * a + d] = (double)sa;
    }
    free(acc);
    free(ab);
  }
  return 0;
}

/* ------------------------------------------------- complex bands at k -- */

/*
 * Bloch bands (the SHO basis spans functions R^3 -> C, sec. 2.5): complex
 * psi with psi(r + T) = e^{i k.T} psi(r) for every lattice vector T of the
 * periodic axes.  Bands are interleaved (re, im) pairs: psi[mem][b][2],
 * c[off_a + n][b][2] with B complex bands.  An unwrapped support point i
 * lies at r_i = r_j + T_i, j = i mod N, T_i = (i - j) h, so that
 *   projection  c[a][n][b] = h^3 sum_{i in S_a} P_an(i) e^{+i k.T_i} psi_b(j)
 *   expansion   psi_b(j)  += sum_a sum_{i in S_a, i = j mod N}
 *                            e^{-i k.T_i} sum_n c[a][n][b] P_an(i)
 * The expansion builds the Bloch sum of the projectors with wave vector k,
 * and is the adjoint of the projection (up to h^3) in the complex inner
 * product.  Isolated axes have no images (T = 0 there).
 */
static double bloch_angle(const ogrid *g, const int i[3], const double k[3]) {
  double th = 0.0;
  for (int d = 0; d < 3; ++d) {
    const int j = wrap(i[d], g->n[d]);
    th += k[d] * ((double)(i[d] - j) * g->h);
  }
  return th;
}

typedef struct {
  const ogrid *g;
  const double *fc;
  double sigma;
  int nu, B;
  const double *k;
  const double *psi; /* [mem][B][2] */
  long double *acc;  /* [N][B][2] */
  long double *abs;  /* [N][B][2] */
} prjk_ctx;

static void prjk_fn(void *p, const int i[3], int64_t mem) {
  prjk_ctx *c = (prjk_ctx *)p;
  double fx[ORACLE_NU_MAX + 1], fy[ORACLE_NU_MAX + 1], fz[ORACLE_NU_MAX + 1];
  phi_all(c->nu, c->sigma, (double)i[0] * c->g->h - c->fc[0], fx);
  phi_all(c->nu, c->sigma, (double)i[1] * c->g->h - c->fc[1], fy);
  phi_all(c->nu, c->sigma, (double)i[2] * c->g->h - c->fc[2], fz);
  const double th = bloch_angle(c->g, i, c->k);
  const long double cs = cosl((long double)th), sn = sinl((long double)th);
  const double *ps = c->psi + mem * 2 * c->B;
  int idx = 0;
  for (int nz = 0; nz <= c->nu; ++nz)
    for (int ny = 0; ny <= c->nu - nz; ++ny)
      for (int nx = 0; nx <= c->nu - nz - ny; ++nx, ++idx) {
        const long double P = (long double)fx[nx] * fy[ny] * fz[nz];
        long double *acc = c->acc + (int64_t)idx * 2 * c->B;
        long double *ab = c->abs + (int64_t)idx * 2 * c->B;
        for (int b = 0; b < c->B; ++b) {
          const long double re = ps[2 * b], im = ps[2 * b + 1];
          acc[2 * b] += P * (cs * re - sn * im);
          acc[2 * b + 1] += P * (sn * re + cs * im);
          const long double m = fabsl(P) * (fabsl(re) + fabsl(im));
          ab[2 * b] += m;
          ab[2 * b + 1] += m;
        }
      }
}

int oracle_project_k(const int n[3], double h, const int periodic[3], int natoms,
                     const double *pos, const double *sigma, const int *numax,
                     const double *rbox, const double *kvec, int B, const double *psi,
                     double *c, double *cabs) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 || !kvec ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
  const double h3 = h * h * h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < natoms; ++a) {
    int nu = numax[a], N = oracle_nsho(nu);
    long double *acc = calloc((size_t)N * 2 * B, sizeof(long double));
    long double *ab = calloc((size_t)N * 2 * B, sizeof(long double));
    prjk_ctx ctx = {&g, pos + 3 * a, sigma[a], nu, B, kvec, psi, acc, ab};
    double R = rbox ? rbox[a] : box_radius(sigma[a], nu, h);
    visit_support(&g, pos + 3 * a, R, prjk_fn, &ctx);
    int64_t off = 2 * coeff_offset(numax, a, B);
    for (int64_t k = 0; k < (int64_t)N * 2 * B; ++k) {
      c[off + k] = (double)(h3 * acc[k]);
      if (cabs) cabs[off + k] = (double)(h3 * ab[k]);
    }
    free(acc);
    free(ab);
  }
  return 0;
}

typedef struct {
  const ogrid *g;
  const double *fc;
  double sigma;
  int nu, B, b0, b1;
  const double *k;
  const double *cc; /* this atom's [N][B][2] */
  double *psi;      /* [mem][B][2] */
  double *pabs;
} addk_ctx;

static void addk_fn(void *p, const int i[3], int64_t mem) {
  addk_ctx *c = (addk_ctx *)p;
  double fx[ORACLE_NU_MAX + 1], fy[ORACLE_NU_MAX + 1], fz[ORACLE_NU_MAX + 1];
  phi_all(c->nu, c->sigma, (double)i[0] * c->g->h - c->fc[0], fx);
  phi_all(c->nu, c->sigma, (double)i[1] * c->g->h - c->fc[1], fy);
  phi_all(c->nu, c->sigma, (double)i[2] * c->g->h - c->fc[2], fz);
  const double th = bloch_angle(c->g, i, c->k);
  const long double cs = cosl((long double)th), sn = sinl((long double)th);
  for (int b = c->b0; b < c->b1; ++b) {
    long double sr = 0, si = 0, sa = 0;
    int idx = 0;
    for (int nz = 0; nz <= c->nu; ++nz)
      for (int ny = 0; ny <= c->nu - nz; ++ny)
        for (int nx = 0; nx <= c->nu - nz - ny; ++nx, ++idx) {
          const long double P = (long double)fx[nx] * fy[ny] * fz[nz];
          const long double re = c->cc[((int64_t)idx * c->B + b) * 2];
          const long double im = c->cc[((int64_t)idx * c->B + b) * 2 + 1];
          sr += P * re;
          si += P * im;
          sa += fabsl(P) * (fabsl(re) + fabsl(im));
        }
    /* times e^{-i theta} */
    c->psi[(mem * c->B + b) * 2] += (double)(cs * sr + sn * si);
    c->psi[(mem * c->B + b) * 2 + 1] += (double)(cs * si - sn * sr);
    if (c->pabs) {
      c->pabs[(mem * c->B + b) * 2] += (double)sa;
      c->pabs[(mem * c->B + b) * 2 + 1] += (double)sa;
    }
  }
}

int oracle_expand_k(const int n[3], double h, const int periodic[3], int natoms,
                    const double *pos, const double *sigma, const int *numax,
                    const double *rbox, const double *kvec, int B, const double *c,
                    double *psi, double *pabs) {
  ogrid g;
  if (check_grid(n, h, periodic, &g) || B <= 0 || !kvec ||
      check_atoms(natoms, sigma, numax, 0))
    return -1;
#pragma omp parallel
  {
    int nt = 1, t = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    t = omp_get_thread_num();
#endif
    int b0 = (int)((int64_t)B * t / nt), b1 = (int)((int64_t)B * (t + 1) / nt);
    if (b1 > b0)
      for (int a = 0; a < natoms; ++a) {
        addk_ctx ctx = {&g,   pos + 3 * a, sigma[a], numax[a], B, b0, b1, kvec,
                        c + 2 * coeff_offset(numax, a, B), psi, pabs};
        double R = rbox ? rbox[a] : box_radius(sigma[a], numax[a], h);
        visit_support(&g, pos + 3 * a, R, addk_fn, &ctx);
      }
  }
  return 0;
}
