/*
 * sho.h -- C ABI of the MI355X (gfx950) SHO projection library, libsho.so.
 *
 * The library applies the two bandwidth-bound halves of the non-local PAW
 * operator with analytic projectors (Baumeister & Tsukamoto, PASC'19):
 *
 *   projection  (sec. 3.2 step 1, evaluated in the Cartesian SHO basis of
 *                sec. 3.5):
 *       c[a][n][b] = h^3 sum_{i in S_a} P_an(i) psi_b(i)
 *   expansion   (sec. 3.2 step 3, "add ... to"):
 *       psi_b(i) += sum_a sum_n c[a][n][b] P_an(i)
 *   derivative  (position derivative of the projection, support frozen):
 *       grad[a][d] = sum_{n,b} w[a][n][b] dc[a][n][b]/dR_{a,d}
 *
 * with P_an(x,y,z) = phi_nx(x-X_a) phi_ny(y-Y_a) phi_nz(z-Z_a), the product
 * of three L2-normalised 1D Hermite functions of spread sigma_a (sec. 2.2,
 * eqs. 1HO-eigenstate and SHO-factorizable-basis), truncated to
 * nx+ny+nz <= nu_a (sec. 2.5, eq. SHO-basis): N_SHO(nu) =
 * (nu+1)(nu+2)(nu+3)/6 functions per atom (eq. SHO_basis_size).  The 1D
 * functions are generated on the fly from their three-term recurrence
 * (sec. 3.7) unless the stored-projector variant is selected.
 *
 * Conventions
 *   grid      n[0..2] points along x, y, z; spacing h (Bohr); point i sits at
 *             i*h.  periodic[d] != 0: indices wrap modulo n[d]; otherwise
 *             support points outside 0..n[d]-1 are dropped.
 *   psi       device array of doubles, layout [n[2]][n[1]][n[0]][nbands]
 *             (band index fastest: the bands are the vector lanes, sec. 6).
 *   c, w      device array of doubles, per-atom blocks [N_SHO(nu_a)][nbands]
 *             concatenated in atom order (sho_plan_coeff_offsets).  Within a
 *             block n runs nz outermost, then ny, nx fastest.
 *   pos       host array [natoms][3] (Bohr), sigma host [natoms] (Bohr),
 *             numax host [natoms].
 *   support   S_a = unwrapped points i with (dx*dx + dy*dy) + dz*dz <= R_a^2,
 *             d = i*h - R_a evaluated in IEEE double in that order.
 *             R_a = rbox[a] if given, else sigma_a*sqrt(2 nu_a + 3) + 2h (the
 *             classical turning radius of shell nu_a, sec. 2.2, plus two
 *             spacings).  A point reached by several periodic images
 *             contributes once per image.
 *   streams   every compute call is asynchronous on the given hipStream_t
 *             (passed as void*, NULL = null stream).  Argument errors are
 *             reported synchronously and launch nothing.
 *   ownership the caller owns psi, c, w and grad; the library never frees
 *             them.  Host arrays are copied during the call.  A plan owns its
 *             device tables and frees them in sho_plan_destroy.
 *   buffers   before a launch every device pointer is checked against the
 *             HIP runtime's record of the allocation holding it: a host
 *             pointer, NULL, a range running past the end of that allocation,
 *             or psi overlapping c is refused with SHO_E_INVALID.  A buffer
 *             carved out of a larger pool allocation (a caching allocator's
 *             segment) is only checked against the pool's bounds, so callers
 *             must still pass buffers of the documented sizes.
 *   errors    every entry point returns a sho_status; on failure
 *             sho_last_error() gives a message (thread-local).  No C++
 *             exception crosses this interface.
 */
#ifndef SHO_H
#define SHO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sho_status;

#define SHO_OK 0
#define SHO_E_INVALID (-1)      /* bad argument (NULL, size, non-finite...) */
#define SHO_E_UNDERSAMPLED (-2) /* h > pi sigma / sqrt(2 nu + 1), sec. 3.6 */
#define SHO_E_NU_RANGE (-3)     /* nu outside 0..SHO_NU_MAX */
#define SHO_E_BOX (-4)          /* support box too wide for on-chip tables */
#define SHO_E_NOMEM (-5)        /* device or host allocation failed */
#define SHO_E_DEVICE (-6)       /* HIP runtime or launch error */
#define SHO_E_BUDGET (-7)       /* request exceeds the serving memory budget */

/* Largest nu_max accepted by project / expand.  The derivative uses
 * nu_max + 1 functions and accepts the same range. */
#define SHO_NU_MAX 10

/* Plan flags */
#define SHO_FLAG_STORED 0x1u              /* precompute P_an(i) for every
                                             support point into device memory
                                             (N_SHO doubles per point) and read
                                             it back in every projection and
                                             expansion: the stored-projector
                                             bandwidth baseline (sec. 6, the
                                             paper's USU kernels); nu <= 5.
                                             The derivative still generates
                                             its functions. */
#define SHO_FLAG_ALLOW_UNDERSAMPLED 0x2u  /* skip the sampling bound check */
#define SHO_FLAG_HOST_ONLY 0x4u           /* geometry and sizes only: no device
                                             call, no device memory; the
                                             compute calls refuse such a plan
                                             (for sizing and admission) */

typedef struct sho_grid {
  int32_t n[3];        /* points along x, y, z */
  double h;            /* grid spacing, Bohr */
  int32_t periodic[3]; /* nonzero: periodic axis */
} sho_grid;

typedef struct sho_plan_s *sho_plan_t;

typedef struct sho_plan_info {
  int32_t natoms;
  int32_t nbands;
  int32_t nu_max;          /* largest nu_a in the plan */
  int32_t flags;
  int64_t coeff_rows;      /* sum_a N_SHO(nu_a) */
  int64_t coeff_doubles;   /* coeff_rows * nbands: length of c and w */
  int64_t support_points;  /* sum_a |S_a| */
  int64_t lines;           /* (z, y) lines over all supports */
  int64_t planes;          /* z planes over all supports */
  int64_t device_bytes;    /* device memory owned by the plan */
  int64_t stored_bytes;    /* of which stored projector tables */
  int64_t union_points;    /* distinct grid points covered by any support */
  int64_t expand_points;   /* grid points the expansion reads and writes
                              (whole row chunks that some support touches) */
  int64_t expand_scratch_doubles; /* plane partials of the expansion */
} sho_plan_info;

/* N_SHO(nu) = (nu+1)(nu+2)(nu+3)/6 (sec. 2.5); -1 if nu < 0. */
int32_t sho_nsho(int32_t nu);

/* Message for the last failing call on this thread ("" if none). */
const char *sho_last_error(void);

/*
 * Build a reusable plan: per-atom supports (the projection spheres of sec. 6)
 * cut into (z, y) lines, uploaded to the current device.  Host-side work plus
 * synchronous uploads; the plan may then be used from any stream.
 *   rbox   optional host [natoms] support radii (NULL: default rule)
 *   flags  SHO_FLAG_* bits
 * Errors: SHO_E_INVALID, SHO_E_NU_RANGE, SHO_E_UNDERSAMPLED, SHO_E_BOX,
 * SHO_E_NOMEM, SHO_E_DEVICE.  *out is NULL on failure.
 */
sho_status sho_plan_create(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, sho_plan_t *out);

/* Free a plan's device tables.  Waits for the device first, so work already
 * queued with the plan finishes.  NULL is accepted. */
sho_status sho_plan_destroy(sho_plan_t plan);

sho_status sho_plan_get_info(sho_plan_t plan, sho_plan_info *info);

/* off[a] = first double of atom a's block in c / w, off[natoms] = total.
 * off: host array [natoms + 1]. */
sho_status sho_plan_coeff_offsets(sho_plan_t plan, int64_t *off);

/* |S_a| per atom into host array counts[natoms]. */
sho_status sho_plan_support_counts(sho_plan_t plan, int64_t *counts);

/*
 * Move the function centres to pos (host [natoms][3]) while keeping every
 * support S_a as built: the frozen-support setting in which the derivative
 * entry points are exact derivatives.  Synchronous (returns after the
 * upload on stream completed).  Not allowed on SHO_FLAG_STORED plans.
 */
sho_status sho_plan_set_centres(sho_plan_t plan, const double *pos,
                                void *stream);

/* c (device, coeff_doubles) <- projection of psi (device, grid x nbands).
 * c is overwritten; psi and c must not overlap. */
sho_status sho_plan_project(sho_plan_t plan, const double *psi, double *c,
                            void *stream);

/* psi (device) += expansion of c (device).  Accumulates; overlapping atoms
 * add in an unspecified order.  psi and c must not overlap. */
sho_status sho_plan_expand(sho_plan_t plan, const double *c, double *psi,
                           void *stream);

/* grad (device, [natoms][3]) <- sum_{n,b} w dc/dR, support frozen.
 * Overwritten.  w has the layout of c. */
sho_status sho_plan_force(sho_plan_t plan, const double *psi,
                          const double *w, double *grad, void *stream);

/*
 * Stateless forms: build (or reuse from a small internal cache keyed on the
 * exact argument bytes) a plan for the given geometry, then run the
 * operation on stream.  Same argument meaning as the plan calls above.
 */
sho_status sho_project(const sho_grid *grid, int32_t natoms,
                       const double *pos, const double *sigma,
                       const int32_t *numax, int32_t nbands, const double *psi,
                       double *c, uint32_t flags, void *stream);
sho_status sho_expand(const sho_grid *grid, int32_t natoms, const double *pos,
                      const double *sigma, const int32_t *numax,
                      int32_t nbands, const double *c, double *psi,
                      uint32_t flags, void *stream);
sho_status sho_force(const sho_grid *grid, int32_t natoms, const double *pos,
                     const double *sigma, const int32_t *numax, int32_t nbands,
                     const double *psi, const double *w, double *grad,
                     uint32_t flags, void *stream);

/*
 * Kernel timing for benchmarks: while enabled, every kernel launch made with
 * this plan is bracketed by HIP events recorded on the call's stream.
 * sho_plan_profile(plan, 1) clears and starts recording, (plan, 0) stops.
 * sho_plan_profile_read waits for the recorded events and returns, per
 * kernel kind, the number of launches and their mean duration in ms:
 *   SHO_KERNEL_PROJECT, SHO_KERNEL_EXPAND_PLANES (z pass of the expansion),
 *   SHO_KERNEL_EXPAND_ROWS (y and x passes), SHO_KERNEL_FORCE.
 * counts and mean_ms: host arrays [SHO_KERNEL_KINDS].  Not for use inside a
 * captured graph.
 */
#define SHO_KERNEL_PROJECT 0
#define SHO_KERNEL_EXPAND_PLANES 1
#define SHO_KERNEL_EXPAND_ROWS 2
#define SHO_KERNEL_FORCE 3
#define SHO_KERNEL_KINDS 4
sho_status sho_plan_profile(sho_plan_t plan, int32_t enable);
sho_status sho_plan_profile_read(sho_plan_t plan, int64_t *counts,
                                 double *mean_ms);

/* Drop every plan held by the stateless cache (waits for the device). */
sho_status sho_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* SHO_H */
