/*
 * sho_factorised.c -- factorised CPU implementation of the SHO projection and
 * expansion, the CPU reference point of the benchmark.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY, like the rest of oracle/: nothing in
 * the product path links, loads or calls it, and it shares no code, header or
 * table with the HIP library.  It is not the checker (sho_oracle.c is): the
 * tests pin it to the plain triple sum.
 *
 * It computes what sho_oracle.c computes, but the way the paper's method is
 * meant to run on a CPU (Baumeister & Tsukamoto, PASC'19): the projector of
 * the Cartesian SHO basis is a product of three 1D functions (sec. 2.2,
 * eq. SHO-factorizable-basis), so the sum over the support of one atom
 * separates into three successive 1D contractions (sec. 3.4):
 *
 *   T1[nx][b]      = sum_x phi_nx(x) psi(x,y,z)[b]          per (z, y) line
 *   T2[nx][ny][b] += phi_ny(y) T1[nx][b]                     per z plane
 *   c[n][b]       += h^3 phi_nz(z) T2[nx][ny][b]             nx+ny+nz <= nu
 *
 * and the expansion runs them backwards (z, then y, then x).  The 1D
 * functions are sampled once per atom and axis from the monic three-term
 * recurrence of sec. 3.7 with the L2 normalisation.  Double-precision sums,
 * OpenMP threads: over atoms for the projection; for the expansion first
 * over atoms (plane partials) and then over memory planes z, so that no two
 * threads add into the same values of psi.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FACT_NU_MAX 16

/* Threads a parallel region of this library runs with. */
int fact_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int fact_nsho(int nu) { return (nu + 1) * (nu + 2) * (nu + 3) / 6; }

static int fact_wrap(int i, int n) {
  int m = i % n;
  return m < 0 ? m + n : m;
}

/* phi_0..phi_nu at u: monic recurrence H_{n+1} = t H_n - (n/2) H_{n-1},
 * times (2^n / (n! sqrt(pi) sigma))^(1/2) e^{-t^2/2}, t = u / sigma. */
static void fact_phi(int nu, double sigma, double u, double *out) {
  const double t = u / sigma;
  const double g = exp(-0.5 * t * t);
  double hm = 0.0, h0 = 1.0, norm = 1.0 / sqrt(sqrt(M_PI) * sigma);
  for (int n = 0; n <= nu; ++n) {
    if (n > 0) norm *= sqrt(2.0 / (double)n);
    out[n] = norm * h0 * g;
    const double hn = t * h0 - 0.5 * n * hm;
    hm = h0;
    h0 = hn;
  }
}

/* Support geometry of one atom: the unwrapped index box that holds the
 * sphere, and per (z, y) line the x range inside it (membership decided in
 * IEEE double in the documented order: (dx*dx + dy*dy) + dz*dz <= R*R). */
typedef struct {
  int lo[3], m[3];  /* first unwrapped index and extent per axis */
  double *tab[3];   /* [m_d][nu+1] samples per axis */
  int *xa, *xb;     /* per line (jz * m[1] + jy): x table range [xa, xb) */
  int nu;
} fact_atom;

static int fact_atom_init(fact_atom *A, const int n[3], double h, const int periodic[3],
                          const double c[3], double sigma, int nu, double R) {
  A->nu = nu;
  for (int d = 0; d < 3; ++d) {
    int lo = (int)floor((c[d] - R) / h) - 1, hi = (int)ceil((c[d] + R) / h) + 1;
    if (!periodic[d]) {
      if (lo < 0) lo = 0;
      if (hi > n[d] - 1) hi = n[d] - 1;
    }
    A->lo[d] = lo;
    A->m[d] = hi >= lo ? hi - lo + 1 : 0;
    A->tab[d] = malloc(sizeof(double) * (size_t)(A->m[d] > 0 ? A->m[d] : 1) * (nu + 1));
    if (!A->tab[d]) return -1;
    for (int j = 0; j < A->m[d]; ++j)
      fact_phi(nu, sigma, (double)(lo + j) * h - c[d], A->tab[d] + (size_t)j * (nu + 1));
  }
  const size_t nl = (size_t)A->m[1] * A->m[2];
  A->xa = malloc(sizeof(int) * (nl ? nl : 1));
  A->xb = malloc(sizeof(int) * (nl ? nl : 1));
  if (!A->xa || !A->xb) return -1;
  for (int jz = 0; jz < A->m[2]; ++jz) {
    const double dz = (double)(A->lo[2] + jz) * h - c[2];
    for (int jy = 0; jy < A->m[1]; ++jy) {
      const double dy = (double)(A->lo[1] + jy) * h - c[1];
      int a = -1, b = -1;
      for (int jx = 0; jx < A->m[0]; ++jx) {
        const double dx = (double)(A->lo[0] + jx) * h - c[0];
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        if (r2 <= R * R) {
          if (a < 0) a = jx;
          b = jx + 1;
        }
      }
      /* a sphere meets a line in one interval */
      A->xa[(size_t)jz * A->m[1] + jy] = a < 0 ? 0 : a;
      A->xb[(size_t)jz * A->m[1] + jy] = a < 0 ? 0 : b;
    }
  }
  return 0;
}

static void fact_atom_free(fact_atom *A) {
  for (int d = 0; d < 3; ++d) free(A->tab[d]);
  free(A->xa);
  free(A->xb);
}

static double fact_radius(const double *rbox, int a, double sigma, int nu, double h) {
  return rbox ? rbox[a] : sigma * sqrt(2.0 * nu + 3.0) + 2.0 * h;
}

static int fact_check(const int n[3], double h, int natoms, const double *sigma,
                      const int *numax, int B) {
  if (!(h > 0) || B <= 0 || natoms < 0) return -1;
  for (int d = 0; d < 3; ++d)
    if (n[d] <= 0) return -1;
  for (int a = 0; a < natoms; ++a)
    if (!(sigma[a] > 0) || numax[a] < 0 || numax[a] > FACT_NU_MAX) return -1;
  return 0;
}

/* c (per-atom blocks [N_SHO(nu_a)][B], overwritten) <- projection of psi
 * ([z][y][x][B]).  Returns 0, or -1 on bad arguments or memory. */
int fact_project(const int n[3], double h, const int periodic[3], int natoms,
                 const double *pos, const double *sigma, const int *numax,
                 const double *rbox, int B, const double *psi, double *c) {
  if (fact_check(n, h, natoms, sigma, numax, B)) return -1;
  int64_t *off = malloc(sizeof(int64_t) * (size_t)(natoms + 1));
  if (!off) return -1;
  off[0] = 0;
  for (int a = 0; a < natoms; ++a) off[a + 1] = off[a] + (int64_t)fact_nsho(numax[a]) * B;
  const double h3 = h * h * h;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int a = 0; a < natoms; ++a) {
    const int nu = numax[a], NF = nu + 1;
    fact_atom A;
    memset(&A, 0, sizeof(A));
    double *T1 = malloc(sizeof(double) * (size_t)NF * B);
    double *T2 = malloc(sizeof(double) * (size_t)NF * NF * B);
    double *ca = c + off[a];
    memset(ca, 0, sizeof(double) * (size_t)fact_nsho(nu) * B);
    if (!T1 || !T2 || fact_atom_init(&A, n, h, periodic, pos + 3 * a, sigma[a], nu,
                                     fact_radius(rbox, a, sigma[a], nu, h))) {
      bad |= 1;
    } else {
      for (int jz = 0; jz < A.m[2]; ++jz) {
        const int zm = fact_wrap(A.lo[2] + jz, n[2]);
        memset(T2, 0, sizeof(double) * (size_t)NF * NF * B);
        int any = 0;
        for (int jy = 0; jy < A.m[1]; ++jy) {
          const size_t li = (size_t)jz * A.m[1] + jy;
          if (A.xa[li] >= A.xb[li]) continue;
          any = 1;
          const int ym = fact_wrap(A.lo[1] + jy, n[1]);
          memset(T1, 0, sizeof(double) * (size_t)NF * B);
          for (int jx = A.xa[li]; jx < A.xb[li]; ++jx) {
            const int xm = fact_wrap(A.lo[0] + jx, n[0]);
            const double *p = psi + (((int64_t)zm * n[1] + ym) * n[0] + xm) * B;
            const double *fx = A.tab[0] + (size_t)jx * NF;
            for (int k = 0; k < NF; ++k) {
              double *t = T1 + (size_t)k * B;
              for (int b = 0; b < B; ++b) t[b] += fx[k] * p[b];
            }
          }
          const double *fy = A.tab[1] + (size_t)jy * NF;
          for (int ny = 0; ny < NF; ++ny)
            for (int nx = 0; nx < NF - ny; ++nx) {
              double *t = T2 + ((size_t)ny * NF + nx) * B;
              const double *s = T1 + (size_t)nx * B;
              for (int b = 0; b < B; ++b) t[b] += fy[ny] * s[b];
            }
        }
        if (!any) continue;
        const double *fz = A.tab[2] + (size_t)jz * NF;
        int idx = 0;
        for (int nz = 0; nz <= nu; ++nz)
          for (int ny = 0; ny <= nu - nz; ++ny)
            for (int nx = 0; nx <= nu - nz - ny; ++nx, ++idx) {
              double *o = ca + (size_t)idx * B;
              const double *s = T2 + ((size_t)ny * NF + nx) * B;
              for (int b = 0; b < B; ++b) o[b] += fz[nz] * s[b];
            }
      }
      for (int64_t k = 0; k < (int64_t)fact_nsho(nu) * B; ++k) ca[k] *= h3;
    }
    fact_atom_free(&A);
    free(T1);
    free(T2);
  }
  free(off);
  return bad ? -1 : 0;
}

/* psi ([z][y][x][B]) += expansion of c (per-atom blocks). */
int fact_expand(const int n[3], double h, const int periodic[3], int natoms,
                const double *pos, const double *sigma, const int *numax,
                const double *rbox, int B, const double *c, double *psi) {
  if (fact_check(n, h, natoms, sigma, numax, B)) return -1;
  fact_atom *atoms = calloc((size_t)(natoms > 0 ? natoms : 1), sizeof(fact_atom));
  double **u2 = calloc((size_t)(natoms > 0 ? natoms : 1), sizeof(double *));
  int64_t *off = malloc(sizeof(int64_t) * (size_t)(natoms + 1));
  if (!atoms || !u2 || !off) {
    free(atoms);
    free(u2);
    free(off);
    return -1;
  }
  off[0] = 0;
  for (int a = 0; a < natoms; ++a) off[a + 1] = off[a] + (int64_t)fact_nsho(numax[a]) * B;
  int bad = 0;
  /* z pass per atom: U2[jz][ny][nx][b] = sum_nz phi_nz(z_jz) c[nx,ny,nz][b] */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int a = 0; a < natoms; ++a) {
    const int nu = numax[a], NF = nu + 1;
    fact_atom *A = &atoms[a];
    if (fact_atom_init(A, n, h, periodic, pos + 3 * a, sigma[a], nu,
                       fact_radius(rbox, a, sigma[a], nu, h))) {
      bad |= 1;
      continue;
    }
    u2[a] = calloc((size_t)(A->m[2] > 0 ? A->m[2] : 1) * NF * NF * B, sizeof(double));
    if (!u2[a]) {
      bad |= 1;
      continue;
    }
    const double *ca = c + off[a];
    for (int jz = 0; jz < A->m[2]; ++jz) {
      const double *fz = A->tab[2] + (size_t)jz * NF;
      double *U = u2[a] + (size_t)jz * NF * NF * B;
      int idx = 0;
      for (int nz = 0; nz <= nu; ++nz)
        for (int ny = 0; ny <= nu - nz; ++ny)
          for (int nx = 0; nx <= nu - nz - ny; ++nx, ++idx) {
            double *t = U + ((size_t)ny * NF + nx) * B;
            const double *s = ca + (size_t)idx * B;
            for (int b = 0; b < B; ++b) t[b] += fz[nz] * s[b];
          }
    }
  }
  if (!bad) {
    /* y and x passes, one memory plane per thread at a time */
#pragma omp parallel
    {
      double *U1 = malloc(sizeof(double) * (size_t)(FACT_NU_MAX + 1) * B);
#pragma omp for schedule(dynamic, 1)
      for (int zm = 0; zm < n[2]; ++zm) {
        if (!U1) continue;
        for (int a = 0; a < natoms; ++a) {
          const fact_atom *A = &atoms[a];
          const int NF = A->nu + 1;
          for (int jz = 0; jz < A->m[2]; ++jz) {
            if (fact_wrap(A->lo[2] + jz, n[2]) != zm) continue;
            const double *U = u2[a] + (size_t)jz * NF * NF * B;
            for (int jy = 0; jy < A->m[1]; ++jy) {
              const size_t li = (size_t)jz * A->m[1] + jy;
              if (A->xa[li] >= A->xb[li]) continue;
              const int ym = fact_wrap(A->lo[1] + jy, n[1]);
              const double *fy = A->tab[1] + (size_t)jy * NF;
              memset(U1, 0, sizeof(double) * (size_t)NF * B);
              for (int ny = 0; ny < NF; ++ny)
                for (int nx = 0; nx < NF - ny; ++nx) {
                  double *t = U1 + (size_t)nx * B;
                  const double *s = U + ((size_t)ny * NF + nx) * B;
                  for (int b = 0; b < B; ++b) t[b] += fy[ny] * s[b];
                }
              for (int jx = A->xa[li]; jx < A->xb[li]; ++jx) {
                const int xm = fact_wrap(A->lo[0] + jx, n[0]);
                double *p = psi + (((int64_t)zm * n[1] + ym) * n[0] + xm) * B;
                const double *fx = A->tab[0] + (size_t)jx * NF;
                for (int k = 0; k < NF; ++k) {
                  const double *s = U1 + (size_t)k * B;
                  for (int b = 0; b < B; ++b) p[b] += fx[k] * s[b];
                }
              }
            }
          }
        }
      }
      free(U1);
    }
  }
  for (int a = 0; a < natoms; ++a) {
    fact_atom_free(&atoms[a]);
    free(u2[a]);
  }
  free(atoms);
  free(u2);
  free(off);
  return bad ? -1 : 0;
}
