// sho_launch.hpp -- kernel argument block and launchers of libsho.so.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

#include "sho_internal.hpp"

namespace sho {

// Sets the calling thread's message (sho_last_error) and returns code.
sho_status fail(sho_status code, const std::string &msg);
// SHO_E_DEVICE with the runtime's message for e (clears the sticky error).
sho_status hip_fail(hipError_t e, const char *what);

// Argument block of the projection / expansion / derivative kernels.
struct KArgs {
  const AtomRec *atoms;
  const LineRec *lines;
  const BundleRec *bundles;
  const WorkRec *work;       // work items of this launch (one nu)
  const double *tab;         // 1D tables of all atoms
  const double *stored;      // stored projectors (SHO_FLAG_STORED plans)
  const int64_t *run_poff;   // per run: first double of its stored block
  int32_t nwork;
  int32_t nlines;            // line records in the plan
  int32_t nx;                // grid points along x
  int32_t B;                 // bands: stride of one grid point
  int32_t tb_shift;          // log2(bands per lane slot)
  int32_t ntiles;            // band tiles per atom
  int32_t det;               // 1: deterministic sums (per-wave LDS tiles
                             // added in wave order; no atomics)
  int32_t bloch;             // 1: complex bands (re, im) at a wave vector k
  double h3;
  double alpha;              // expansion: psi += alpha * sum_n c P_n
  const double *bundle_phase;  // Bloch plans: (cos, sin) of k.T per bundle
};

// Argument block of the row-owner expansion.
struct EArgs {
  const AtomRec *atoms;
  const LineRec *lines;
  const int32_t *run_atom;
  const int32_t *row_runs;
  const RowRec *rows;
  const int64_t *u2_off;
  const int32_t *nu_atoms;
  const double *tab;
  int32_t nrows;        // entries of rows (a multiple of kRowsPerGroup)
  int32_t natoms_u2;    // entries of nu_atoms
  int32_t nx;
  int32_t B;
  int32_t tbe_shift;    // log2(bands per x phase): 5 or 6
  int32_t ntiles;       // band tiles of the row kernel
  int32_t ntiles_u2;    // band tiles (of 32) of the plane-partial kernel
  int32_t nu_max;       // largest nu among the atoms
  int32_t nu_begin[SHO_NU_MAX + 2];  // nu_atoms[nu_begin[nu] .. nu_begin[nu+1])
  // block form
  const BlockRec *blocks;
  const EntryRec *entries;
  const uint32_t *run_desc;
  const int64_t *desc_pbase;  // stored plans: per descriptor, P double of x = 0
  const double *P;            // stored plans: the projector tables
  int32_t nblocks;
  int32_t blk_rows;     // R
  int32_t blk_x;        // X
  int32_t ny;
  int32_t ncol;         // stored plans: 0, or the radial projectors per atom
  int32_t bloch;        // 1: complex bands (re, im) at a wave vector k
  double alpha;         // psi += alpha * sum_n c P_n (applied to c in the z pass)
  const double *entry_phase;  // Bloch plans: (cos, sin) of k.T per block entry
};

// Argument block of the stored-projector kernels.
struct SArgs {
  const AtomRec *atoms;
  const double *P;           // stored projector values
  const int64_t *atom_poff;  // [natoms] first double of each atom's block
  const int64_t *atom_pbeg;  // [natoms] first stored point of each atom
  const int32_t *pidx;       // grid memory index of every stored point
  const StoredItem *items;   // work items of this launch (one nu)
  int32_t nitems;
  int32_t B;
  int32_t ncol;              // stored values per point (= coefficient rows
                             // per atom) of the launch's atoms
  double h3;
  double alpha;              // expansion: psi += alpha * sum_n c P_n
};

// Radial projector sets (sho_plan_create_radial): p_j(r) = P_k(|r|) Y_lm(r^)
// with P_k tabulated on a uniform radial grid.
struct RArgs {
  const double *rad;         // [nrad][nr] table values P_k(m dr)
  int32_t nrad, nr, nproj;
  int32_t ell[kRadialMaxFuncs];
  double dr;
  double h;
};

// Samples the 1D tables of every atom (rows padded with zeros).
hipError_t launch_tables(const AtomRec *atoms, int32_t natoms, double h,
                         double *tab, int32_t mmax, hipStream_t s);
hipError_t launch_project(int nu, const KArgs &K, const double *psi, double *c,
                          hipStream_t s);
// Work items of any cut-off up to nu_max in one launch.
hipError_t launch_project_any(int nu_max, const KArgs &K, const double *psi,
                              double *c, hipStream_t s);
// Atom-owner expansion with global atomics (work items of one nu).
hipError_t launch_expand_atomic(int nu, const KArgs &K, const double *c,
                                double *psi, hipStream_t s);
// Expansion by rows: plane partials U2 from c, then every memory row adds the
// contributions of all runs that fall into it.  u2: E's u2 buffer.
hipError_t launch_expand_rows(const EArgs &E, const double *c, double *u2,
                              double *psi, hipStream_t s);
// The two halves of launch_expand_rows.
hipError_t launch_expand_planes(const EArgs &E, const double *c, double *u2,
                                hipStream_t s);
hipError_t launch_rows(const EArgs &E, const double *u2, double *psi,
                       hipStream_t s);
// Block form of the second half (blocks of R rows x X points).
hipError_t launch_blocks(const EArgs &E, const double *u2, double *psi,
                         hipStream_t s);
// Block form of the projection: every block of psi read once, the atom
// planes touching it add their plane sums into p2 (the plane-partial layout,
// zeroed first: launch_fill); launch_zpass then writes c = h3 * z pass of p2.
// E's block tables are the projection's (R x X blocks, band tile of
// 1 << E.tbe_shift bands, at most kProjTileDoubles values per block).
hipError_t launch_project_blocks(const EArgs &E, const double *psi, double *p2,
                                 hipStream_t s);
hipError_t launch_zpass(const EArgs &E, const double *p2, double *c, double h3,
                        hipStream_t s);
// Owner form of the second half: one wave per strip of 64/TB rows x X points
// (X = E.blk_x, 16 or 32), values in registers, entries in plan order.
hipError_t launch_owner(const EArgs &E, const double *u2, double *psi, hipStream_t s);
// Stored plans: the whole expansion in the block form, P_an read from the
// tables (per-block products on FP64 matrix cores); nu_max <= 5.
hipError_t launch_blocks_stored(const EArgs &E, const double *c, double *psi,
                                hipStream_t s);
// Stored-projector baseline: sample P_an at every support point, then
// project / expand by reading them back (nu <= 5).
hipError_t launch_store(const KArgs &K, const int32_t *run_atom, int32_t nruns,
                        double *stored, hipStream_t s);
// Radial plans: p_j at every support point into the stored tables.
hipError_t launch_store_radial(const KArgs &K, const RArgs &R, const int32_t *run_atom,
                               int32_t nruns, double *stored, hipStream_t s);
// c must be zeroed first (launch_fill): every item adds its chunk's share.
// S.ncol selects the table width (N_SHO(nu) or the radial projector count).
hipError_t launch_project_stored(const SArgs &S, const double *psi, double *c,
                                 hipStream_t s);
hipError_t launch_expand_stored(const SArgs &S, const double *c, double *psi,
                                hipStream_t s);
// d = D c per atom (D: per-atom N x N row-major blocks at doff[a]).
hipError_t launch_multiply(const AtomRec *atoms, int32_t natoms, const int64_t *doff,
                           const double *D, const double *c, double *d, int32_t B,
                           hipStream_t s);
// grad must be zeroed first (launch_fill).  With K.det, every (atom, band
// tile) writes its three sums to gpart[(atom * ntiles + tile) * 3 + d]
// instead, and launch_force_sum adds them in tile order into grad.
hipError_t launch_force(int nu, const KArgs &K, const double *psi,
                        const double *w, double *grad, hipStream_t s,
                        double *gpart = nullptr);
hipError_t launch_force_sum(const double *gpart, int32_t natoms, int32_t ntiles, double *grad,
                            hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

// Capacity of the static scratch of the allocation-free expansion (32 MiB).
constexpr int64_t kStaticScratchDoubles = (int64_t)1 << 22;
static_assert(kStaticScratchDoubles == SHO_STATIC_SCRATCH_DOUBLES, "static scratch size");
// Device address of the current device's static scratch (looked up once per
// device; no allocation).
hipError_t static_scratch(double **ptr);

// FP32 plans (an even number of bands, processed as pairs: K.B and E.B count
// pairs).  tab: the plan's tables rounded to FP32.
hipError_t launch_tables_f32(const double *tab, float *tab32, int64_t n, hipStream_t s);
hipError_t launch_project_f32(int nu, const KArgs &K, const float *tab, const float *psi,
                              float *c, hipStream_t s);
hipError_t launch_project_any_f32(int nu_max, const KArgs &K, const float *tab,
                                  const float *psi, float *c, hipStream_t s);
hipError_t launch_expand_planes_f32(const EArgs &E, const float *tab, const float *c,
                                    float *u2, hipStream_t s);
hipError_t launch_blocks_f32(const EArgs &E, const float *tab, const float *u2, float *psi,
                             hipStream_t s);

}  // namespace sho
