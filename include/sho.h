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
#define SHO_FLAG_PER_ATOM 0x8u            /* reference schedule: one launch per
                                             atom for the projection, the
                                             derivative and an atom-owner
                                             expansion (global atomics); the
                                             batched schedules are measured
                                             against it */
#define SHO_FLAG_FP32 0x10u               /* single-precision bands (the
                                             paper's float kernels, sec. 6):
                                             psi and c hold floats and go
                                             through sho_plan_project_f32 /
                                             sho_plan_expand_f32; nbands must
                                             be even (adjacent bands are
                                             processed in pairs); not with
                                             SHO_FLAG_STORED or
                                             SHO_FLAG_PER_ATOM.  The FP64
                                             entry points, the derivative, the
                                             atomic-matrix product and graphs
                                             refuse such a plan. */
#define SHO_FLAG_DETERMINISTIC 0x20u      /* bitwise reproducible results:
                                             every sum (over a support, over
                                             overlapping atoms, over band
                                             tiles) is taken in an order fixed
                                             by the plan, never through
                                             atomics.  The projection and the
                                             derivative keep one coefficient
                                             tile per wave, added in wave
                                             order, and one work item per
                                             atom; the expansion takes the
                                             owner form (SHO_EXPAND_OWNER).
                                             Repeated calls on the same inputs
                                             give identical bits.  FP64 only;
                                             not with SHO_FLAG_STORED,
                                             SHO_FLAG_PER_ATOM or
                                             SHO_FLAG_FP32 (SHO_E_INVALID). */
#define SHO_FLAG_BLOCH 0x40u              /* complex Bloch bands at a wave
                                             vector k (sec. 2.5: the basis
                                             spans functions R^3 -> C; set by
                                             sho_plan_set_kpoint, default 0).
                                             nbands counts complex bands;
                                             psi is [z][y][x][nbands][2] and c
                                             [N_SHO][nbands][2] (real,
                                             imaginary interleaved: complex128,
                                             or complex64 with SHO_FLAG_FP32).
                                             A support point reached through
                                             the periodic image translated by
                                             T contributes e^{+i k.T} psi to
                                             the projection and receives
                                             e^{-i k.T} sum_n c P_n from the
                                             expansion.  Single-launch
                                             schedules and the block form of
                                             the expansion only; not with
                                             SHO_FLAG_STORED, _PER_ATOM or
                                             _DETERMINISTIC; no derivative. */

/* Expansion forms (sho_plan_set_expand) */
#define SHO_EXPAND_ROWS 0
#define SHO_EXPAND_BLOCKS 1
#define SHO_EXPAND_OWNER 2

/* Projection launch schedules (sho_plan_set_schedule, sho_plan_tune) */
#define SHO_SCHED_BY_NU 0      /* one launch per cut-off nu */
#define SHO_SCHED_SINGLE 1     /* one launch over all work items, atoms in
                                  Morton order of their centres */
#define SHO_SCHED_SINGLE_LPT 2 /* one launch, work items by falling cost */
#define SHO_SCHED_SWEEP 3      /* one launch, work items (plane ranges of
                                  atoms) by the memory plane z they start at,
                                  then (x, y) Morton order: the workgroups
                                  resident at one time read a few consecutive
                                  planes, so overlapping supports are read
                                  close in time (cache reuse) */
#define SHO_SCHED_XCD 4        /* flag for any of the above: consecutive items
                                  of the order run on the same XCD (shared
                                  L2), each XCD taking one eighth */

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
  int64_t coeff_doubles;   /* coeff_rows * nbands: elements of c and w
                              (floats for SHO_FLAG_FP32 plans) */
  int64_t support_points;  /* sum_a |S_a| */
  int64_t lines;           /* (z, y) lines over all supports */
  int64_t planes;          /* z planes over all supports */
  int64_t device_bytes;    /* device memory owned by the plan; for a
                              SHO_FLAG_HOST_ONLY plan, what a device plan of
                              the same geometry and flags would own once it
                              has run every call (admission estimate) */
  int64_t stored_bytes;    /* of which stored projector tables */
  int64_t union_points;    /* distinct grid points covered by any support */
  int64_t expand_points;   /* grid points the expansion reads and writes:
                              the blocks (block form) or whole rows (row
                              form) that some support touches */
  int64_t expand_scratch_doubles; /* plane partials of the expansion */
  int64_t expand_blocks;   /* workgroup blocks of the block-form expansion */
  int64_t expand_entries;  /* (atom plane, block) pairs of that form */
} sho_plan_info;

/* N_SHO(nu) = (nu+1)(nu+2)(nu+3)/6 (sec. 2.5); -1 if nu < 0. */
int32_t sho_nsho(int32_t nu);

/* Message for the last failing call on this thread ("" if none). */
const char *sho_last_error(void);

/*
 * Build a reusable plan: per-atom supports (the projection spheres of sec. 6)
 * cut into (z, y) lines, uploaded to the current device.  Host-side work plus
 * synchronous uploads; the plan may then be used from any stream.  Calls of
 * one plan that use its device scratch (the expansion's plane partials) on
 * different streams are ordered by the library: each waits for the previous
 * one.  Work recorded into a captured graph is not ordered that way, so a
 * graph must not be replayed while another call of its plan runs.  A plan
 * must not be called from two host threads at once.
 *   rbox   optional host [natoms] support radii (NULL: default rule)
 *   flags  SHO_FLAG_* bits
 * Errors: SHO_E_INVALID (also when n[0] * nbands reaches 2^31 or nbands
 * 2^24, counting band pairs for SHO_FLAG_FP32: the kernels address a grid
 * line in 32-bit integers), SHO_E_NU_RANGE, SHO_E_UNDERSAMPLED, SHO_E_BOX,
 * SHO_E_NOMEM, SHO_E_DEVICE.  *out is NULL on failure.
 */
sho_status sho_plan_create(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, sho_plan_t *out);

/*
 * Stored numerical projectors (the paper's USU reference kernels, sec. 6:
 * precomputed projector values read from memory; its USU18 set holds two
 * radial functions each for l = 0, 1, 2):
 *   p_j(r) = P_k(|r - R_a|) Y_{l_k m}((r - R_a)^),  j over k, then m = -l_k..l_k
 * with P_k tabulated on a uniform radial grid, tables[k][i] = P_k(i dr),
 * i = 0..nr-1; between nodes P_k is the cubic Lagrange interpolant through
 * the nodes s..s+3, s = clamp(floor(r/dr) - 1, 0, nr - 4), and zero from
 * r = (nr-1) dr on.  Y_lm are the real spherical harmonics without the
 * Condon-Shortley sign (Y_11 ~ +x, Y_1,-1 ~ +y), unit-normalised on the
 * sphere; at r = 0 only l = 0 is nonzero.  The support of atom a is the
 * sphere of radius rcut[a] (same point rule, images and clipping as the SHO
 * supports).  The plan samples every p_j at every support point once, into
 * its device tables, and then projects and expands by reading them back on
 * the FP64 matrix cores (the stored kernels of SHO_FLAG_STORED plans):
 *   c[a][j][b] = h^3 sum_{i in S_a} p_j(i) psi_b(i),  psi_b += sum c p_j.
 * Coefficient blocks are [nproj][nbands] per atom, nproj = sum_k (2 l_k + 1).
 *   ell     host [nradial], 0..3;  nradial 1..16, nproj <= 56
 *   tables  host [nradial][nr], copied during the call;  nr >= 4, dr > 0
 *   rcut    host [natoms] support radii (Bohr)
 *   flags   0 or SHO_FLAG_HOST_ONLY
 * sho_plan_project / _expand / _destroy / _get_info / _coeff_offsets /
 * _support_counts / _set_expand and the graph calls accept the plan; the
 * derivative, moving centres, the atomic-matrix calls, FP32 and tuning are
 * refused (SHO_E_INVALID).  Errors: SHO_E_INVALID, SHO_E_BOX, SHO_E_NOMEM,
 * SHO_E_DEVICE.
 */
sho_status sho_plan_create_radial(const sho_grid *grid, int32_t natoms, const double *pos,
                                  const double *rcut, int32_t nradial, const int32_t *ell,
                                  int32_t nr, double dr, const double *tables,
                                  int32_t nbands, uint32_t flags, sho_plan_t *out);

/*
 * Bloch wave vector of a SHO_FLAG_BLOCH plan, k[3] in Bohr^-1 (host).  Waits
 * for the device (queued work reads the plan's phase tables), then stores
 * (cos, sin) of k.T for every run bundle and block entry of the plan on the
 * device; later calls use it.  The phase of an image is e^{i k.T},
 * T = (m_x n_x h, m_y n_y h, m_z n_z h) with the image counts m_d; a support
 * reaching more than 127 images along an axis is refused at plan creation
 * (SHO_E_BOX).  Graphs captured before are refused.  Errors: SHO_E_INVALID
 * (not a Bloch plan, non-finite k), SHO_E_DEVICE.
 */
sho_status sho_plan_set_kpoint(sho_plan_t plan, const double *k);

/* Free a plan's device tables.  Waits for the device first, so work already
 * queued with the plan finishes.  NULL is accepted. */
sho_status sho_plan_destroy(sho_plan_t plan);

/* Free the plan's own device scratch (the expansion's plane partials, also
 * the block projection's plane sums: sho_plan_info.expand_scratch_doubles
 * doubles), keeping its tables; the next call that needs the scratch
 * allocates it again.  For a plan kept while its system's buffers are
 * released (a server evicting a system it expects back).  Waits for the
 * device first (queued work finishes).  Graphs captured before are refused
 * afterwards (they hold the old address).  No-op for plans that hold no
 * scratch.  Errors: SHO_E_INVALID (NULL), SHO_E_DEVICE. */
sho_status sho_plan_release_scratch(sho_plan_t plan);

sho_status sho_plan_get_info(sho_plan_t plan, sho_plan_info *info);

/* off[a] = first element of atom a's block in c / w, off[natoms] = total.
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

/* psi (device) += alpha * expansion of c (device), i.e. the expansion of the
 * coefficients scaled by alpha (the scaling is applied to c inside the
 * kernels' z pass; c is not modified).  With alpha = h^3 this is the
 * gradient of a loss L(c) with respect to psi, dL/dpsi = h^3 expand(dL/dc),
 * since the projection carries the h^3 of the sampled integral (sec. 3.5).
 * FP64 plans only.  Errors as sho_plan_expand, and SHO_E_INVALID for a
 * non-finite alpha. */
sho_status sho_plan_expand_scaled(sho_plan_t plan, double alpha, const double *c,
                                  double *psi, void *stream);


/*
 * Allocation-free expansion, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): psi (device) += expansion of c (device), as sho_plan_expand,
 * but the plane partials live in a static device array of the library
 * (SHO_STATIC_SCRATCH_DOUBLES doubles, 32 MiB, one copy per device, held
 * until the process ends) instead of the plan's lazily allocated scratch.
 * The call allocates nothing and records no profiling events.  Every call on
 * one device shares that device's array and overwrites it: calls that
 * overlap in time on one device (other streams, other threads, other plans)
 * race and give wrong results; the caller must order them.  FP64 plans only.
 * Errors as sho_plan_expand, and SHO_E_INVALID when the plan's plane
 * partials (sho_plan_info.expand_scratch_doubles) exceed the array.
 */
#define SHO_STATIC_SCRATCH_DOUBLES 4194304
sho_status sho_plan_expand_noalloc(sho_plan_t plan, const double *c, double *psi,
                                   void *stream);

/*
 * Single precision (SHO_FLAG_FP32 plans), same layouts with float elements:
 * c[n][b] (device, coeff_doubles floats) <- projection of psi (device,
 * grid x nbands floats), and psi += expansion of c.  The 1D functions are
 * the double-precision samples rounded to float; all sums run in float.
 * Complex bands (Gamma point or isolated systems) are passed as interleaved
 * (real, imaginary) pairs, i.e. as 2 x nbands real bands, in either
 * precision: the SHO functions are real, so both parts transform alike.
 */
sho_status sho_plan_project_f32(sho_plan_t plan, const float *psi, float *c,
                                void *stream);
sho_status sho_plan_expand_f32(sho_plan_t plan, const float *c, float *psi,
                               void *stream);

/* grad (device, [natoms][3]) <- sum_{n,b} w dc/dR, support frozen.
 * Overwritten.  w has the layout of c. */
sho_status sho_plan_force(sho_plan_t plan, const double *psi,
                          const double *w, double *grad, void *stream);

/*
 * Non-local application (sec. 3.2, steps 1-3, with the atomic matrices in the
 * SHO basis of sec. 3.5: a real N_SHO x N_SHO matrix per atom):
 *   multiply:  d[a][n][b] = sum_m D_a[n][m] c[a][m][b]
 *   apply:     c <- project(psi); d <- multiply(D, c); out += expand(d)
 * D: device, per-atom row-major N_SHO(nu_a) x N_SHO(nu_a) blocks in atom
 * order, first double of atom a at matrix_offsets[a] (host [natoms + 1]).
 * c, d: device buffers of coeff_doubles (c and d must not overlap; both are
 * overwritten; out accumulates).  The products run on FP64 matrix cores.
 */
sho_status sho_plan_matrix_offsets(sho_plan_t plan, int64_t *off);
sho_status sho_plan_multiply(sho_plan_t plan, const double *D, const double *c,
                             double *d, void *stream);
sho_status sho_plan_apply(sho_plan_t plan, const double *psi, const double *D,
                          double *c, double *d, double *out, void *stream);

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
 *   SHO_KERNEL_PROJECT, SHO_KERNEL_EXPAND_Z (z pass of the expansion),
 *   SHO_KERNEL_EXPAND_XY (y and x passes, in either form; the whole
 *   expansion for stored and per-atom plans), SHO_KERNEL_FORCE.
 * counts and mean_ms: host arrays [SHO_KERNEL_KINDS].  Not for use inside a
 * captured graph.
 */
#define SHO_KERNEL_PROJECT 0
#define SHO_KERNEL_EXPAND_Z 1
#define SHO_KERNEL_EXPAND_XY 2
#define SHO_KERNEL_FORCE 3
#define SHO_KERNEL_KINDS 4
sho_status sho_plan_profile(sho_plan_t plan, int32_t enable);
sho_status sho_plan_profile_read(sho_plan_t plan, int64_t *counts,
                                 double *mean_ms);

/*
 * Work decomposition of the projection (sec. 6 measures prj and add over
 * many atoms of one system; these calls batch them).  schedule is one of
 * SHO_SCHED_BY_NU, _SINGLE, _SINGLE_LPT, _SWEEP, optionally | SHO_SCHED_XCD.  A work item is one
 * atom, or a share of an atom of more than target_points support points;
 * band_tile bands share a lane slot (power of two <= 64, 0 keeps the current
 * tile).  Plans with several cut-offs start with SHO_SCHED_SINGLE, others
 * with SHO_SCHED_BY_NU, target_points 16384 and the widest tile that fits.
 * set_schedule waits for the device (the work tables are replaced);
 * graphs made before it must be made again (sho_graph_launch refuses them).
 */
sho_status sho_plan_set_schedule(sho_plan_t plan, int32_t schedule,
                                 int32_t band_tile, int64_t target_points);
sho_status sho_plan_get_schedule(sho_plan_t plan, int32_t *schedule,
                                 int32_t *band_tile, int64_t *target_points);

/*
 * Form of the projection (sec. 3.2 step 1):
 *   SHO_PROJECT_ITEMS   work items of atoms (sho_plan_set_schedule): each
 *                       workgroup streams the psi box of one atom (or a share
 *                       of it), so a value held by k supports is read k times
 *                       (default);
 *   SHO_PROJECT_BLOCKS  one workgroup per block of block_rows x block_x points
 *                       of one plane and band_tile bands (8, 16, 32 or 64):
 *                       the block is read once and every atom plane touching
 *                       it adds its plane sums into the plan's plane-partial
 *                       scratch (atomics); a z pass writes c.  For heavily
 *                       overlapping supports (many atoms per grid value).
 * block_rows, block_x, band_tile = 0 pick 32 points, 16 bands and as many rows
 * as 8192 values allow; rows and points at most 255.  The block form is for
 * FP64 plans of real bands that are not stored, per-atom or deterministic
 * (SHO_E_INVALID otherwise); the derivative always uses work items.
 * set_project waits for the device; graphs made before it are refused.
 */
#define SHO_PROJECT_ITEMS 0
#define SHO_PROJECT_BLOCKS 1
sho_status sho_plan_set_project(sho_plan_t plan, int32_t form, int32_t block_rows,
                                int32_t block_x, int32_t band_tile);
sho_status sho_plan_get_project(sho_plan_t plan, int32_t *form, int32_t *block_rows,
                                int32_t *block_x, int32_t *band_tile);

/*
 * Form of the expansion's second half (sec. 3.2 step 3 after the z pass):
 *   0  rows:   one workgroup per chunk of one memory row; every run of the
 *              row loads its atom plane's partial sums;
 *   1  blocks: one workgroup per block of block_rows rows x block_x points of
 *              one plane; the partial sums of an atom plane are loaded once
 *              for all its runs in the block (default);
 *   2  owner:  one wavefront per strip of R rows x block_x points (16 or 32)
 *              of one plane and one tile of T bands (T = 16, or 8 for plans
 *              of at most 8 bands; R = 64 / T, block_rows must be 0 or R):
 *              each lane keeps its row's values in registers and adds the
 *              atoms touching the strip in the plan's order, without
 *              atomics, so the result is bitwise reproducible (the form of
 *              SHO_FLAG_DETERMINISTIC plans, which accept no other).
 * All read and write every touched value of psi once with plain loads and
 * stores.  For SHO_FLAG_STORED plans the forms are: 0 the atom-owner form
 * (global atomics, default for nu_max > 2), 1 the block form with the
 * products on matrix cores (default for nu_max <= 2).  block_rows = block_x = 0 picks the default shape; a shape whose
 * tile (rows x points x bands per tile: 8, 16, 32 or 64, the power of two
 * that covers nbands, at most 64) exceeds 4096 doubles, or whose rows or
 * points exceed 256 / (table row length: 8 doubles for nu_max <= 6, else
 * 16), is refused with SHO_E_INVALID.
 * set_expand waits for the device; graphs made before it are refused.
 */
sho_status sho_plan_set_expand(sho_plan_t plan, int32_t mode, int32_t block_rows,
                               int32_t block_x);
sho_status sho_plan_get_expand(sho_plan_t plan, int32_t *mode, int32_t *block_rows,
                               int32_t *block_x);

/*
 * Band tile of the expansion's block form (bands per lane slot: 8, 16, 32 or
 * 64; 0 restores the default rule: the power of two covering nbands, at most
 * 64).  Narrower tiles run more band tiles over larger blocks, so that the
 * plane partials of an atom plane are loaded for fewer blocks.  Rebuilds the
 * blocks in the default shape for the tile.  Not for SHO_FLAG_STORED plans.
 * Waits for the device; graphs made before it are refused.
 */
sho_status sho_plan_set_expand_tile(sho_plan_t plan, int32_t band_tile);
sho_status sho_plan_get_expand_tile(sho_plan_t plan, int32_t *band_tile);

typedef struct sho_tune_expand_result {
  int32_t mode;          /* chosen SHO_EXPAND_* */
  int32_t band_tile;     /* bands per lane slot of that form */
  int32_t block_rows;    /* block shape (block form) */
  int32_t block_x;
  double ms;             /* mean expansion time of the choice */
  double ms_before;      /* of the form the plan had before */
  int32_t candidates;    /* forms timed */
  int32_t pad;
} sho_tune_expand_result;

/*
 * Expansion tuner: times the expansion of c into psi (device buffers of the
 * plan's sizes; psi is used as scratch: it accumulates reps + 2 expansions
 * per candidate) under the block form with every band tile from 8 to the
 * one covering nbands and a few block shapes per tile (the default, half the
 * rows, half the width, twice the rows at half the width), and the row form
 * (FP64 plans of real bands), reps launches each after one warm-up, on
 * stream, and keeps the fastest.  Synchronous.  Refused (SHO_E_INVALID) on
 * stored, per-atom and deterministic plans.  result may be NULL.
 */
sho_status sho_plan_tune_expand(sho_plan_t plan, const void *c, void *psi, int32_t reps,
                                void *stream, sho_tune_expand_result *result);

typedef struct sho_tune_result {
  int32_t schedule;      /* chosen SHO_SCHED_* */
  int32_t band_tile;     /* chosen bands per lane slot */
  int64_t target_points; /* chosen work item size */
  double ms;             /* mean projection time of the choice */
  double ms_before;      /* of the schedule the plan had before */
  int32_t candidates;    /* schedules timed */
  int32_t project_form;  /* chosen SHO_PROJECT_* */
} sho_tune_result;

/*
 * Autotuner: times the projection of psi into c (both device buffers of the
 * plan's sizes; c is overwritten) under every schedule (with and without
 * SHO_SCHED_XCD) x work item size
 * {4096, 8192, 16384, 32768} x band tile {current, half}, and (FP64 plans of
 * real bands, not deterministic) the block form of the projection with band
 * tiles 8..32 and blocks 16..64 points wide, reps launches each after one
 * warm-up, on stream, and keeps the fastest (the item schedule is kept for
 * the derivative either way).  Synchronous.  result may be NULL.  psi and c hold the plan's element type (double, or float for
 * SHO_FLAG_FP32 plans).  Refused (SHO_E_INVALID) on stored and per-atom
 * plans.
 */
sho_status sho_plan_tune(sho_plan_t plan, const void *psi, void *c,
                         int32_t reps, void *stream, sho_tune_result *result);

/*
 * One captured HIP graph of project(psi -> c) followed by expand(c -> out)
 * (out accumulates, as in sho_plan_expand), replayable with one launch call.
 * The buffers are fixed at creation and must outlive the graph; psi and out
 * may be the same buffer.  The graph holds only kernel nodes (coefficients
 * are cleared by a fill kernel).  Destroy graphs before their plan; a graph
 * is refused after its plan's schedule changed.
 */
typedef struct sho_graph_s *sho_graph_t;
sho_status sho_graph_create(sho_plan_t plan, const double *psi, double *c,
                            double *out, sho_graph_t *graph);
/* The same for the whole application: project, multiply, expand. */
sho_status sho_graph_create_apply(sho_plan_t plan, const double *psi,
                                  const double *D, double *c, double *d,
                                  double *out, sho_graph_t *graph);
sho_status sho_graph_launch(sho_graph_t graph, void *stream);
sho_status sho_graph_destroy(sho_graph_t graph);

/*
 * Request server.  Systems (geometry, bands, host inputs psi and w) are
 * registered once; requests name a system and a job:
 *   SHO_JOB_PROJECT  c    <- project(psi)
 *   SHO_JOB_EXPAND   out  <- expand(w)        (out cleared first)
 *   SHO_JOB_FORCE    grad <- force(psi, w)
 * all on the system's resident buffers.  A system is made resident (plan
 * tables + psi, out, w, c, grad in device memory: its charge) on its first
 * request; when the charges would exceed budget_bytes, least recently used
 * other systems are evicted first.  An evicted system keeps its plan's
 * tables on the device (charged, without the plan's scratch, until they are
 * needed: then least recently used kept plans are freed too), so that its
 * next admission only uploads its inputs.  A system whose charge alone
 * exceeds the budget is refused with SHO_E_BUDGET.  Requests of one system run in
 * submission order on one of nstreams streams (1..16, default priority);
 * different systems overlap.  With two or more streams the first is kept
 * for short requests: those whose estimated cost (support points x bands x
 * a per-job factor) is at most both the median and half the mean of the
 * latest 256 requests' costs.  They never queue behind a long request; the
 * other requests go to the remaining stream with the least outstanding
 * estimated work.  plan_flags go to every plan (0, or
 * SHO_FLAG_PER_ATOM for the per-request reference); SHO_FLAG_HOST_ONLY makes
 * a server that only does the admission bookkeeping (no device use; every
 * request completes at once).
 *
 * submit is asynchronous (it waits only for evictions and admissions);
 * request_info returns the submit and completion times in seconds since the
 * server was made (t_done < 0 while running; completion is taken by a
 * polling thread when the request's event fires).  read copies a resident
 * system's latest output of a job into host memory (c: coeff_doubles, out:
 * grid * nbands, grad: natoms * 3) after that system's requests finished.
 * The host inputs are copied at registration into pinned host buffers that
 * the server owns; with psi or w NULL they start zeroed, and
 * sho_server_inputs returns the buffers so that the caller can fill them in
 * place (before the system's first request, or while it is not resident).
 * clock returns the server's time (seconds since creation, the clock of
 * request_info).  One server may be driven from one thread at a time.
 */
#define SHO_JOB_PROJECT 0
#define SHO_JOB_EXPAND 1
#define SHO_JOB_FORCE 2

typedef struct sho_server_s *sho_server_t;

typedef struct sho_server_stats {
  int64_t budget_bytes;
  int64_t resident_bytes;       /* sum of the resident systems' charges */
  int64_t peak_resident_bytes;
  int64_t requests, completed;
  int64_t admissions, evictions, rejected;
  int32_t systems, resident_systems;
  int64_t short_requests;       /* requests sent to the short-request stream */
  int64_t plan_reuses;          /* admissions that found the plan kept */
  int64_t plan_drops;           /* kept plans freed to make room */
} sho_server_stats;

sho_status sho_server_create(int64_t budget_bytes, int32_t nstreams,
                             uint32_t plan_flags, sho_server_t *server);
sho_status sho_server_add_system(sho_server_t server, const sho_grid *grid,
                                 int32_t natoms, const double *pos,
                                 const double *sigma, const int32_t *numax,
                                 int32_t nbands, const double *psi,
                                 const double *w, int32_t *system);
sho_status sho_server_submit(sho_server_t server, int32_t system, int32_t job,
                             int64_t *request);
/* Make a system resident now (admission as for a request, inputs uploaded,
 * waits for the upload); for loading systems before a request stream. */
sho_status sho_server_prefetch(sho_server_t server, int32_t system);
sho_status sho_server_drain(sho_server_t server);
sho_status sho_server_request_info(sho_server_t server, int64_t request,
                                   int32_t *system, int32_t *job,
                                   double *t_submit, double *t_done);
sho_status sho_server_read(sho_server_t server, int32_t system, int32_t job,
                           double *host);
sho_status sho_server_get_stats(sho_server_t server, sho_server_stats *stats);
sho_status sho_server_system_info(sho_server_t server, int32_t system,
                                  int64_t *charge_bytes, int32_t *resident);
sho_status sho_server_inputs(sho_server_t server, int32_t system, double **psi,
                             double **w);
sho_status sho_server_clock(sho_server_t server, double *now);
sho_status sho_server_destroy(sho_server_t server);

/* Drop every plan held by the stateless cache (waits for the device). */
sho_status sho_cache_clear(void);

/*
 * Set-up side (host only, no device call; once per SCF cycle, sec. 3.5).
 *
 * Radial SHO states Psi_s = R_{nr l}(r) Y_lm (sec. 2.3) are ordered by nu
 * ascending, then l = nu mod 2 .. nu in steps of 2, then m = -l..l, with
 * nr = (nu - l)/2 ("radial order").  R_{nr l}(r) = N r~^l L_nr^(l+1/2)(r~^2)
 * exp(-r~^2/2) sigma^(-3/2), r~ = r/sigma, normalised so that
 * int R^2 r^2 dr = 1.  Y_lm are real spherical harmonics without the
 * Condon-Shortley sign: m > 0 ~ cos(m phi), m < 0 ~ sin(|m| phi), so that
 * Y_11 ~ +x/r and Y_1-1 ~ +y/r.  Cartesian states Phi_c = phi_nx phi_ny phi_nz
 * are in the coefficient order of the projection (nz outer, ny, nx fastest).
 */
#define SHO_SETUP_NU_MAX 60   /* largest nu of the radial-only calls */

/* U[c][s] = <Phi_c | Psi_s> (sec. 2.5, the unitary map between the two
 * degenerate-shell bases; zero unless nx+ny+nz = l + 2 nr).  U: host
 * [N_SHO(nu_max)][N_SHO(nu_max)] row-major, rows Cartesian, columns radial
 * order; independent of sigma.  Errors: SHO_E_NU_RANGE (nu_max outside
 * 0..SHO_NU_MAX), SHO_E_INVALID (NULL). */
sho_status sho_setup_unitary(int32_t nu_max, double *U);

/* R[k][i] = R_{nr l}(r[i]; sigma) for every (nr, l) with l + 2 nr <= nu_max,
 * k in radial order without m (nu ascending, then l).  Host arrays:
 * r[npts], R[count][npts].  Errors: SHO_E_NU_RANGE (outside
 * 0..SHO_SETUP_NU_MAX), SHO_E_INVALID. */
sho_status sho_setup_radial(int32_t nu_max, double sigma, int64_t npts,
                            const double *r, double *R);

/*
 * The atomic matrix in the Cartesian SHO basis (sec. 3.5):
 *   out = M^T D M,  M[j][c] = <p_j | Phi_c> = sum_s F[j][s] U[c][s],
 *   F[j][s] = <p_j | Psi_s> = delta_{l l_j} delta_{m m_j} sum_i w_i r_i^2 P_k(r_i) R_s(r_i).
 * Projectors p_j = P_k(r) Y_{l_k m}: radial function k = 0..nrad-1 with
 * angular momentum ell[k], and m = -ell[k]..ell[k]; j runs over k, then m
 * (nproj = sum_k (2 ell[k] + 1)).  Host arrays: ell[nrad]; a radial
 * quadrature r[ngrid], w[ngrid] with sum_i w_i g(r_i) ~ int g(r) dr;
 * P[nrad][ngrid] projector values; D[nproj][nproj] row-major; out
 * [N_SHO(nu_max)][N_SHO(nu_max)] row-major in the coefficient order (the
 * per-atom block that sho_plan_multiply / sho_plan_apply take).  Functions
 * outside the basis (l_k > nu_max) contribute nothing.  Errors:
 * SHO_E_NU_RANGE, SHO_E_INVALID (NULL, ngrid < 1, negative l, sigma <= 0).
 */
sho_status sho_setup_matrix(int32_t nu_max, double sigma, int32_t nrad,
                            const int32_t *ell, int64_t ngrid, const double *r,
                            const double *w, const double *P, const double *D,
                            double *out);

/* Representation quality of one radial projector P(r) of angular momentum
 * ell in the radial SHO basis of spread sigma (sec. 4):
 *   Q[nu] = sum_{nr <= (nu - ell)/2} <P | R_{nr ell}>^2 / <P | P>, nu = 0..nu_max
 * (0 for nu < ell), inner products with weight r^2 on the caller's
 * quadrature.  Q[nu_max + 1] host output.  Errors: SHO_E_NU_RANGE (outside
 * 0..SHO_SETUP_NU_MAX), SHO_E_INVALID (NULL, zero norm, sigma <= 0). */
sho_status sho_setup_quality(int32_t nu_max, double sigma, int32_t ell,
                             int64_t ngrid, const double *r, const double *w,
                             const double *P, double *Q);

#ifdef __cplusplus
}
#endif

#endif /* SHO_H */
