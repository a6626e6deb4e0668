// sho_internal.hpp -- data layout shared by the host plan builder, the C ABI
// layer and the gfx950 kernels of libsho.so.
//
// A plan cuts every atom's support sphere into z planes and each plane into
// (z, y) lines; a line is stored as one or two runs (cut where it crosses the
// periodic x boundary), each one contiguous block of psi.  Runs of one plane
// are grouped into bundles that one wavefront streams together, one run per
// lane slot.  Kernels contract x, y and z in turn (the factorised Cartesian
// basis of sec. 2.2) and never materialise a 3D projector; the 1D functions
// of every atom are sampled into small tables (the Tucker factors of
// sec. 3.4) that the kernels read through the scalar cache.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "sho.h"

namespace sho {

// Per-atom record, read by kernels.  Table entry j of axis d samples the 1D
// functions at unwrapped index (i0_d + j).
struct AtomRec {
  double cx, cy, cz;     // function centre (Bohr)
  double sigma;          // spread (Bohr)
  int32_t nu;            // basis cut-off nu_a
  int32_t ix0, iy0, iz0; // unwrapped index of table entry 0 per axis
  int32_t mx, my, mz;    // table extents per axis
  int32_t plane_begin;   // first plane record of this atom
  int32_t nplanes;
  int32_t line_begin;    // first run record of this atom
  int32_t nlines;        // runs of this atom
  int32_t tab_nfp;       // row stride of the 1D tables (doubles)
  int64_t coeff_row;     // sum of N_SHO(nu) over earlier atoms
  int64_t npoints;       // |S_a|
  int64_t tab_off;       // first double of this atom's 1D tables
};
static_assert(sizeof(AtomRec) == 104, "AtomRec layout");

// 1D tables of one atom: rows [x: mx][y: my][z: mz], row j of an axis holds
// phi_0..phi_{nf-1} at that grid index, padded with zeros to tab_nfp doubles.
// nf = nu + 2 (the derivative needs one function more than the basis).
inline int32_t table_nf(int32_t nu) { return nu + 2; }
inline int32_t table_nfp(int32_t nu) { return table_nf(nu) <= 8 ? 8 : 16; }

// One z plane of one atom's support.
struct PlaneRec {
  int32_t jz;          // table index along z
  int32_t line_begin;  // absolute index of the plane's first run
  int32_t nlines;
  int32_t npoints;
};

// One run of a (z, y) line: points x0 .. x0+len-1 (unwrapped) of memory row
// `row`.  Runs never cross the periodic x boundary, so a run is one
// contiguous block of len*nbands doubles of psi.
struct LineRec {
  int32_t row;   // (z mod nz) * ny + (y mod ny)
  int32_t x0m;   // memory x of the first point (x0 mod nx)
  int16_t jx0;   // table index of the first point along x
  int16_t jy;    // table index along y
  int16_t jz;    // table index along z (identifies the plane)
  int16_t len;   // number of points
};
static_assert(sizeof(LineRec) == 16, "LineRec layout");

// Up to `slots` runs of one atom plane, streamed together by one wavefront:
// the wave walks the table index jx over [jlo, jhi] (the union of the runs'
// x ranges) so that phi_x(jx) is the same for every lane.
struct BundleRec {
  int32_t run0;   // first run; slot s takes run0 + s
  int16_t nruns;  // runs in this bundle (<= slots)
  int16_t jz;     // plane (table index along z)
  int16_t jlo;    // union of the runs' table ranges along x
  int16_t jhi;
  int32_t pad;
};
static_assert(sizeof(BundleRec) == 16, "BundleRec layout");

// Waves per workgroup of the streaming kernels.
constexpr int kWaves = 8;
// Bytes of LDS the kernels may declare statically (the streaming kernels'
// staged line records and small reduction arrays); the coefficient tiles get
// the rest of a workgroup's LDS.
constexpr int kStaticLds = 1024 + kWaves * 64 * 16;

// One workgroup's share of an atom: a contiguous range of its bundles, cut
// into kWaves cost-balanced wave ranges.  `split` is set when the atom is
// shared by several work items (their partial results are added).
struct WorkRec {
  int32_t atom;
  int32_t split;
  int32_t wb[kWaves + 1];  // wave w takes bundles [wb[w], wb[w+1])
};
static_assert(sizeof(WorkRec) == 4 * (kWaves + 3), "WorkRec layout");

// Expansion work: one memory row (z, y) with the runs of every atom that fall
// into it.  One workgroup owns the row (per x chunk and band tile), so global
// memory sees one plain read and one plain write of it.
struct RowRec {
  int32_t row;        // (z mod nz) * ny + (y mod ny)
  int32_t run_begin;  // into the row-ordered run index list
  int32_t nruns;
  int32_t pad;
};
static_assert(sizeof(RowRec) == 16, "RowRec layout");

// Expansion work of the block form: R consecutive rows of one plane z times
// X consecutive x points.  One workgroup owns the block (per band tile); its
// entries are the (atom, plane, x shift) groups of runs that fall into it, so
// that the plane partials of an atom plane are loaded once for up to R rows.
struct BlockRec {
  int32_t z, y0, x0;
  int32_t entry_begin;
  int32_t nentries;  // -1: padding
  int32_t pad;
};
static_assert(sizeof(BlockRec) == 24, "BlockRec layout");

// Everything one wave needs for an entry, so that the entry costs one record
// load plus one round of data loads: where its plane partials start, where the
// table rows of the block's x range and rows start, which of them exist, and
// its runs as packed (row, x begin, x end) descriptors.
struct EntryRec {
  int64_t u2;          // first double of the atom plane's partials (band 0);
                       // stored plans: the atom's first coefficient row
  int32_t tab_x;       // table double of memory x = x0:  tab_off + (x0 + jshift) nfp
  int32_t tab_y;       // table double of block row 0:   tab_off + (mx + y0 + yshift) nfp
  int16_t nu, nfp;
  int16_t x_lo, x_hi;  // staged x rows that exist, relative to x0
  int16_t y_lo, y_hi;  // staged y rows that exist, relative to y0
  int32_t run_begin;   // into run_desc
  int32_t nruns;
  int8_t img[3];       // periodic image of the entry's runs: unwrapped minus
                       // memory position is img[d] * n[d] points per axis
  int8_t pad;
};
static_assert(sizeof(EntryRec) == 40, "EntryRec layout");

// Run descriptor of the block form: row r (relative to y0) | x begin << 8 |
// x end << 16 (both relative to x0, end exclusive).
inline uint32_t pack_run(int r, int xa, int xb) {
  return (uint32_t)r | ((uint32_t)xa << 8) | ((uint32_t)xb << 16);
}

// Expansion forms.
constexpr int32_t kExpandRows = 0;
constexpr int32_t kExpandBlocks = 1;
constexpr int32_t kExpandOwner = 2;  // one wave per strip, values in registers
constexpr int kBlockTileDoubles = 4096;  // LDS tile of a block workgroup
// Tile of the FP64 block expansion for plans up to cut-off numax: twice the
// size from 8 on, where the kernel's registers allow two waves per SIMD (two
// workgroups per CU) anyway, so that a block holds more of each atom plane
// and the plane partials are loaded fewer times.
constexpr int blk_tile_doubles(int numax) { return numax >= 8 ? 2 * kBlockTileDoubles : kBlockTileDoubles; }

// Rows handled by one expansion workgroup.
constexpr int kRowsPerGroup = 1;

// Blocks of R rows x X points of one plane with their entries (atom plane,
// image) and run descriptors: the work of the block forms.
struct BlockSet {
  int32_t rows = 0, x = 0;
  int64_t points = 0;                 // grid points inside the blocks
  std::vector<BlockRec> blocks;       // XCD-interleaved by plane
  std::vector<EntryRec> entries;
  std::vector<uint32_t> run_desc;
  std::vector<int32_t> run_desc_run;  // the run of every descriptor
};

// Host-side plan contents (built without any device call).
// A chunk of one atom's stored points [k0, k1) (stored-projector kernels).
struct StoredItem {
  int32_t atom;
  int32_t k0, k1;
  int32_t pad;
};
static_assert(sizeof(StoredItem) == 16, "StoredItem layout");

// One projection launch: items [begin, begin+count) of work_proj, all of
// cut-off nu (nu = -1: any cut-off up to nu_max, one launch).
struct ProjGroup {
  int32_t nu;
  int32_t begin;
  int32_t count;
};

struct HostPlan {
  sho_grid grid{};
  int32_t natoms = 0;
  int32_t nbands = 0;
  uint32_t flags = 0;
  int32_t nu_max = 0;
  int32_t m_max = 0;     // largest table extent over atoms and axes
  int32_t tb_shift = 0;  // log2(bands per lane slot)
  std::vector<AtomRec> atoms;
  std::vector<PlaneRec> planes;
  std::vector<LineRec> lines;
  std::vector<BundleRec> bundles;
  std::vector<WorkRec> work;           // by nu, then atoms in space order
  std::vector<int32_t> atom_work;      // [natoms+1] first item of each atom
                                       // in `work` (count: next - first)
  std::vector<WorkRec> work_proj;      // the projection's launch order
  std::vector<ProjGroup> proj_groups;  // its launches
  int32_t sched = 0;                   // kSched* of the projection
  int64_t target_points = 0;           // work item size of the schedule
  std::vector<int32_t> run_atom;       // atom of every run
  std::vector<int32_t> row_runs;       // run indices grouped by memory row
  std::vector<RowRec> rows;            // non-empty rows, XCD-aware order
  std::vector<int64_t> u2_off;         // [natoms] first double of the atom's
                                       // per-plane expansion partials
  std::vector<int32_t> nu_atoms;       // atoms with a support, sorted by nu
  int64_t u2_doubles = 0;
  int32_t expand_mode = kExpandBlocks;
  int32_t expand_tbe_shift = -1;        // block form: log2(bands per tile),
                                        // -1: the default rule
  int32_t blk_rows = 0, blk_x = 0;      // block shape of the block form
  int64_t block_points = 0;             // grid points inside the blocks
  std::vector<BlockRec> blocks;         // XCD-interleaved by plane
  std::vector<EntryRec> entries;
  std::vector<uint32_t> run_desc;
  std::vector<int32_t> run_desc_run;    // the run of every descriptor
  std::vector<int64_t> desc_pbase;      // stored plans: P double of block x 0
  int32_t proj_form = 0;                // kProjectItems or kProjectBlocks
  int32_t pblk_tb_shift = 0;            // log2(bands per lane slot), block form
  BlockSet pblk;                        // the projection's block form
  std::vector<int64_t> run_poff;      // stored projectors: first double of
                                      // each run's [len][N_SHO] block
  std::vector<int64_t> atom_poff;     // [natoms+1] first double of each atom
  std::vector<int64_t> atom_pbeg;     // [natoms+1] first stored point
  std::vector<int32_t> pidx;          // grid memory index of every point
  std::vector<StoredItem> sitems;     // point chunks, sorted by nu
  int64_t stored_doubles = 0;
  int32_t ncols = 0;          // radial plans: projectors per atom (stored
                              // columns and coefficient rows); 0: the SHO
                              // basis, N_SHO(nu_a) per atom
  int64_t union_points = 0;   // distinct grid points covered by any support
  int64_t rows_touched = 0;   // memory rows with at least one run
  std::vector<double> support_centre;  // [natoms][3], fixed at creation
  std::vector<int64_t> coeff_off;      // [natoms+1] in doubles
  std::vector<int64_t> dmat_off;       // [natoms+1] atomic matrices, doubles
  int64_t coeff_rows = 0;
  int64_t support_points = 0;
  int64_t table_doubles = 0;           // size of the 1D table buffer
  bool any_split = false;
};

inline int32_t nsho(int32_t nu) {
  return nu < 0 ? 0 : (nu + 1) * (nu + 2) * (nu + 3) / 6;
}

// Stored values per support point of atom A (columns of its projector table).
inline int32_t stored_cols(const HostPlan &P, const AtomRec &A) {
  return P.ncols > 0 ? P.ncols : nsho(A.nu);
}

// Largest number of radial projectors per atom (sho_plan_create_radial).
constexpr int32_t kRadialMaxProj = 56;
constexpr int32_t kRadialMaxFuncs = 16;
constexpr int32_t kRadialMaxL = 3;

// Compile-time column bound of the stored kernels for a table of ncol
// columns: the SHO sizes exactly, other counts the next larger of 20 or 56;
// 0 if more than 56.
inline int32_t stored_bound(int32_t ncol) {
  switch (ncol) {
    case 1: case 4: case 10: case 20: case 35: case 56:
      return ncol;
    default:
      return ncol <= 0 ? 0 : ncol <= 20 ? 20 : ncol <= 56 ? 56 : 0;
  }
}

// Builds the host plan geometry (supports, runs, tables layout); returns
// SHO_OK or an error code with *msg set.
sho_status build_host_plan(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, HostPlan *out,
                           std::string *msg);

// LDS bytes of a workgroup: a [N_SHO(nf-1)][tb] coefficient tile.
inline size_t lds_tile_bytes(int nf, int tb) {
  return (size_t)nf * (nf + 1) * (nf + 2) / 6 * tb * sizeof(double);
}

// Bands per lane slot (log2) for a workgroup LDS budget of `lds_limit`
// bytes: the derivative's tile at nu_max + 1 must fit.  -1 if even one band
// per slot does not.
int choose_tb_shift(int nbands, int nu_max, size_t lds_limit);

// Projection launch schedules.
constexpr int32_t kSchedByNu = 0;       // one launch per cut-off
constexpr int32_t kSchedSingle = 1;     // one launch, items in space order
constexpr int32_t kSchedSingleLpt = 2;  // one launch, items by falling cost
constexpr int32_t kSchedSweep = 3;      // one launch, items by first plane z,
                                        // then (x, y) Morton order
constexpr int32_t kSchedXcd = 4;        // flag: deal items to the 8 XCDs in
                                        // contiguous blocks of the order
constexpr int32_t kSchedCount = 4;      // base schedules
constexpr int32_t kXcds = 8;            // dispatch interleaves workgroups
                                        // over the XCDs by linear id

inline bool sched_valid(int32_t s) { return s >= 0 && (s & ~kSchedXcd) < kSchedCount; }

// Bundles (with 64 >> tb_shift slots) and work items: atoms of more than
// `target_points` support points are shared by several workgroups.  Atoms
// are visited in Morton order of their centres, so that workgroups running
// at the same time read neighbouring parts of psi (shared in L2 and the
// memory-side cache where supports overlap).  `sched` fixes the order of
// work_proj and its launches; with kSchedXcd, workgroup b of a launch of n
// items runs item (b mod 8) * ceil(n/8) + b / 8 (padding items have atom -1),
// so that each XCD works through one contiguous eighth of the order.
void build_work(HostPlan *P, int tb_shift, int64_t target_points, int32_t sched);

// Expansion tables: runs grouped by memory row, rows interleaved over the
// eight XCDs so that all rows of one plane share an L2, per-atom offsets of
// the plane partials U2[jz][pair][band].
void build_rows(HostPlan *P);

// Blocks of R rows x X points for the block form of the expansion (needs
// build_rows for run_atom).
void build_blocks(HostPlan *P, int32_t R, int32_t X);
void build_block_set(const HostPlan *P, int32_t R, int32_t X, BlockSet *out);

// Projection forms: work items of atoms (the run bundles of an atom streamed
// by one workgroup), or blocks of the grid (each block of psi read once,
// every atom plane touching it adds its share of the plane sums).
constexpr int32_t kProjectItems = 0;
constexpr int32_t kProjectBlocks = 1;
// LDS tile of a projection block (no write-back, so larger than the
// expansion's).
constexpr int kProjTileDoubles = 8192;

// log2 of the bands per lane slot of the expansion's y/x passes: the row form
// takes 32 or 64; the block form also 8 or 16, so that few bands still fill
// the wave with run slots.
inline int expand_tile_shift(int nbands, int mode, bool stored = false) {
  if (stored) return nbands > 16 ? 5 : 4;  // 16-band matrix-core blocks, <= 2
  if (mode == kExpandOwner) return nbands > 8 ? 4 : 3;
  if (nbands > 32) return 6;
  if (mode == kExpandRows || nbands > 16) return 5;
  return nbands > 8 ? 4 : 3;
}

// log2 of the band tile of the expansion's block form for plan P: the
// plan's setting (sho_plan_set_expand_tile) or the default rule.
inline int block_tile_shift(const HostPlan &P) {
  const bool stored = (P.flags & SHO_FLAG_STORED) != 0;
  if (!stored && P.expand_tbe_shift >= 0) return P.expand_tbe_shift;
  return expand_tile_shift(P.nbands, kExpandBlocks, stored);
}

// log2 of the band tile of the plan's current expansion form.
inline int plan_expand_shift(const HostPlan &P) {
  if (P.expand_mode == kExpandBlocks) return block_tile_shift(P);
  return expand_tile_shift(P.nbands, P.expand_mode, (P.flags & SHO_FLAG_STORED) != 0);
}

// Values (bands, or band pairs of SHO_FLAG_FP32 plans, which accumulate
// both bands of a pair in double) that one block's LDS tile holds.
inline int32_t block_tile_values(const HostPlan &P) {
  if (P.flags & SHO_FLAG_FP32) return kBlockTileDoubles / 2;
  if (P.flags & SHO_FLAG_STORED) return kBlockTileDoubles;
  return blk_tile_doubles(P.nu_max);
}

// Smallest power of two >= X.
inline int32_t pow2_ceil(int32_t X) {
  int32_t p = 1;
  while (p < X) p <<= 1;
  return p;
}

// Whether an R x X block fits: the LDS tile (R rows of pow2_ceil(X) points,
// the row stride of the block kernel's tile, per band tile) and the x-table
// staging of one wave (X rows of the widest table).
inline bool block_shape_ok(const HostPlan &P, int32_t R, int32_t X) {
  const int tbe = 1 << block_tile_shift(P);
  return R >= 1 && X >= 1 && X <= 256 &&
         (int64_t)R * pow2_ceil(X) * tbe <= block_tile_values(P) &&
         X * table_nfp(P.nu_max) <= 256 && R * table_nfp(P.nu_max) <= 256;
}

// Owner form: a strip is 64 / (bands per tile) rows (one per lane group of a
// wave) by X points, X one of the widths the kernel is built for.
inline int32_t owner_rows(const HostPlan &P) {
  return 64 >> expand_tile_shift(P.nbands, kExpandOwner);
}
inline bool owner_width_ok(int32_t X) { return X == 16 || X == 32; }

// Default block shape: as wide in x as the staging allows (at most 32 points,
// 16 for 64-band tiles), then as many rows as the tile holds and the y
// staging allows.
inline void default_block_shape(const HostPlan &P, int32_t *R, int32_t *X) {
  const int tbe = 1 << block_tile_shift(P);
  const int nfp = table_nfp(P.nu_max);
  *X = std::min(256 / nfp, tbe == 64 ? 16 : 32);
  *R = std::min(block_tile_values(P) / (*X * tbe), 256 / nfp);
}

// Layout of the stored projector tables (SHO_FLAG_STORED plans): the points
// of every atom in run order, each with its N_SHO values; chunks of at most
// `chunk` points per work item.
void build_stored(HostPlan *P, int32_t chunk);

// Stored plans: for every block run descriptor, the stored-table double of
// its row at block-local x = 0 (needs build_blocks and build_stored).
void build_desc_pbase(HostPlan *P);

// Points per stored-projector work item.
constexpr int32_t kStoredChunk = 1024;

// Largest nu the stored-projector variant supports (56 functions).
constexpr int32_t kStoredNuMax = 5;

// Largest table extent the kernels accept per axis.
constexpr int32_t kMaxTable = 512;

// Support points per work item before an atom is shared by workgroups.
constexpr int64_t kTargetPoints = 16384;

}  // namespace sho
