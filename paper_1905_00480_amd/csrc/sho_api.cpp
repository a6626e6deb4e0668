// sho_api.cpp -- C ABI of libsho.so: plans, uploads, launch orchestration,
// error reporting and the small plan cache behind the stateless calls.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "sho_launch.hpp"

namespace {
thread_local std::string g_err;
}  // namespace

namespace sho {

sho_status fail(sho_status code, const std::string &msg) {
  g_err = msg;
  return code;
}

sho_status hip_fail(hipError_t e, const char *what) {
  (void)hipGetLastError();
  return fail(SHO_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace sho

namespace {

using sho::fail;
using sho::hip_fail;

struct ProfEvent {
  int kind;
  hipEvent_t a, b;
};

struct Group {
  int32_t nu;
  int32_t work_begin;  // into the device work-item array
  int32_t count;       // work items
};

}  // namespace

struct sho_plan_s {
  sho::HostPlan hp;
  int device = 0;
  size_t lds_limit = 0;
  std::vector<Group> groups;
  sho::AtomRec *d_atoms = nullptr;
  sho::LineRec *d_lines = nullptr;
  sho::BundleRec *d_bundles = nullptr;
  sho::WorkRec *d_work = nullptr;
  double *d_tab = nullptr;
  bool fp32 = false;          // SHO_FLAG_FP32: hp.nbands counts band pairs
  bool bloch = false;         // SHO_FLAG_BLOCH: complex bands, hp.nbands counts
                              // real lanes (FP64: 2 per band; FP32: 1 pair)
  double kvec[3] = {0.0, 0.0, 0.0};  // Bloch wave vector (Bohr^-1)
  double *d_bundle_phase = nullptr;  // Bloch plans: (cos, sin) of k.T per bundle
  double *d_entry_phase = nullptr;   //   and per expansion block entry
  float *d_tab32 = nullptr;   // FP32 plans: the tables rounded to float
  int32_t *d_run_atom = nullptr;
  int32_t *d_row_runs = nullptr;
  sho::RowRec *d_rows = nullptr;
  int64_t *d_u2_off = nullptr;
  int32_t *d_nu_atoms = nullptr;
  double *d_u2 = nullptr;  // expansion plane partials, allocated on first use
  double *d_stored = nullptr;     // stored projectors (SHO_FLAG_STORED)
  int64_t *d_run_poff = nullptr;
  int64_t *d_atom_poff = nullptr;
  int64_t *d_atom_pbeg = nullptr;
  int32_t *d_pidx = nullptr;
  sho::StoredItem *d_sitems = nullptr;
  std::vector<Group> sgroups;     // stored work items by nu
  sho::WorkRec *d_work_proj = nullptr;  // the projection's launch order
  int64_t sched_version = 0;      // bumped whenever the work items change
  int64_t sched_bytes = 0;        // device bytes of the schedule tables
  double *d_gpart = nullptr;           // deterministic derivative: per-tile sums
  int64_t *d_doff = nullptr;           // per-atom offsets of the atomic matrices
  int64_t *d_desc_pbase = nullptr;     // stored plans: block descriptors -> P
  sho::BlockRec *d_blocks = nullptr;   // block form of the expansion
  sho::BlockRec *d_pblocks = nullptr;  // block form of the projection
  sho::EntryRec *d_pentries = nullptr;
  uint32_t *d_prun_desc = nullptr;
  int64_t pblk_bytes = 0;
  sho::EntryRec *d_entries = nullptr;
  uint32_t *d_run_desc = nullptr;
  int64_t blk_bytes = 0;
  bool prof_on = false;
  std::vector<ProfEvent> prof;
  // Ordering of the plan's own scratch (plane partials) across streams: the
  // event marks the end of the last call that used it, on scratch_stream.
  hipEvent_t scratch_ev = nullptr;
  hipStream_t scratch_stream = nullptr;
  bool scratch_used = false;
  int64_t scratch_gen = 0;  // bumped when the scratch is released
  int64_t device_bytes = 0;
  int64_t stored_bytes = 0;
};

namespace {

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src, int64_t *bytes) {
  const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc((void **)dst, n);
  if (e != hipSuccess) return e;
  *bytes += (int64_t)n;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T),
                                  hipMemcpyHostToDevice);
  return e;
}

void free_plan_device(sho_plan_s *p) {
  for (double **q : {&p->d_bundle_phase, &p->d_entry_phase}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  if (p->scratch_ev) (void)hipEventDestroy(p->scratch_ev);
  p->scratch_ev = nullptr;
  if (p->d_atoms) (void)hipFree(p->d_atoms);
  if (p->d_lines) (void)hipFree(p->d_lines);
  if (p->d_bundles) (void)hipFree(p->d_bundles);
  if (p->d_work) (void)hipFree(p->d_work);
  if (p->d_work_proj) (void)hipFree(p->d_work_proj);
  p->d_work_proj = nullptr;
  for (void **q : {(void **)&p->d_blocks, (void **)&p->d_entries, (void **)&p->d_run_desc,
                   (void **)&p->d_pblocks, (void **)&p->d_pentries, (void **)&p->d_prun_desc}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  if (p->d_tab) (void)hipFree(p->d_tab);
  if (p->d_tab32) (void)hipFree(p->d_tab32);
  p->d_tab32 = nullptr;
  for (void *q : {(void *)p->d_run_atom, (void *)p->d_row_runs, (void *)p->d_rows,
                  (void *)p->d_u2_off, (void *)p->d_nu_atoms, (void *)p->d_u2})
    if (q) (void)hipFree(q);
  p->d_run_atom = nullptr;
  p->d_row_runs = nullptr;
  p->d_rows = nullptr;
  p->d_u2_off = nullptr;
  p->d_nu_atoms = nullptr;
  p->d_u2 = nullptr;
  if (p->d_doff) (void)hipFree(p->d_doff);
  p->d_doff = nullptr;
  if (p->d_gpart) (void)hipFree(p->d_gpart);
  p->d_gpart = nullptr;
  if (p->d_desc_pbase) (void)hipFree(p->d_desc_pbase);
  p->d_desc_pbase = nullptr;
  for (void *q : {(void *)p->d_stored, (void *)p->d_run_poff, (void *)p->d_atom_poff,
                  (void *)p->d_atom_pbeg, (void *)p->d_pidx, (void *)p->d_sitems})
    if (q) (void)hipFree(q);
  p->d_stored = nullptr;
  p->d_run_poff = nullptr;
  p->d_atom_poff = nullptr;
  p->d_atom_pbeg = nullptr;
  p->d_pidx = nullptr;
  p->d_sitems = nullptr;
  p->d_atoms = nullptr;
  p->d_lines = nullptr;
  p->d_bundles = nullptr;
  p->d_work = nullptr;
  p->d_tab = nullptr;
}

// (Re)uploads the schedule-dependent tables: bundles and both work-item
// orders; regroups the items by nu.
// Bloch plans: (cos, sin) of the phase angle k.T, T = (m_x n_x, m_y n_y,
// m_z n_z) h for image counts m, per bundle of the projection (the image of
// its runs) and per block entry of the expansion.
void phase_of(const sho_plan_s *p, int64_t mx, int64_t my, int64_t mz, double *cs) {
  const sho_grid &g = p->hp.grid;
  double th = p->kvec[0] * ((double)(mx * g.n[0]) * g.h);
  th += p->kvec[1] * ((double)(my * g.n[1]) * g.h);
  th += p->kvec[2] * ((double)(mz * g.n[2]) * g.h);
  cs[0] = std::cos(th);
  cs[1] = std::sin(th);
}

hipError_t upload_phases(sho_plan_s *p) {
  if (!p->bloch || (p->hp.flags & SHO_FLAG_HOST_ONLY)) return hipSuccess;
  const sho::HostPlan &hp = p->hp;
  std::vector<double> bph(2 * std::max<size_t>(hp.bundles.size(), 1), 0.0);
  std::vector<int32_t> run_atom(hp.lines.size(), 0);
  for (int32_t a = 0; a < hp.natoms; ++a)
    for (int32_t r = hp.atoms[a].line_begin; r < hp.atoms[a].line_begin + hp.atoms[a].nlines; ++r)
      run_atom[r] = a;
  for (size_t b = 0; b < hp.bundles.size(); ++b) {
    const sho::LineRec &L = hp.lines[hp.bundles[b].run0];
    const sho::AtomRec &A = hp.atoms[run_atom[hp.bundles[b].run0]];
    const int32_t ny = hp.grid.n[1];
    phase_of(p, (A.ix0 + L.jx0 - L.x0m) / hp.grid.n[0], (A.iy0 + L.jy - L.row % ny) / ny,
             (A.iz0 + L.jz - L.row / ny) / hp.grid.n[2], &bph[2 * b]);
  }
  std::vector<double> eph(2 * std::max<size_t>(hp.entries.size(), 1), 0.0);
  for (size_t i = 0; i < hp.entries.size(); ++i)
    phase_of(p, hp.entries[i].img[0], hp.entries[i].img[1], hp.entries[i].img[2], &eph[2 * i]);
  int64_t bytes = 0;
  for (double **q : {&p->d_bundle_phase, &p->d_entry_phase}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  hipError_t e = upload(&p->d_bundle_phase, bph, &bytes);
  if (e == hipSuccess) e = upload(&p->d_entry_phase, eph, &bytes);
  return e;
}

hipError_t upload_schedule(sho_plan_s *p) {
  for (void **q : {(void **)&p->d_bundles, (void **)&p->d_work, (void **)&p->d_work_proj}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  hipError_t e;
  int64_t &bytes = p->sched_bytes;
  bytes = 0;
  if ((e = upload(&p->d_bundles, p->hp.bundles, &bytes)) != hipSuccess ||
      (e = upload(&p->d_work, p->hp.work, &bytes)) != hipSuccess ||
      (e = upload(&p->d_work_proj, p->hp.work_proj, &bytes)) != hipSuccess)
    return e;
  p->groups.clear();
  const auto &work = p->hp.work;
  for (size_t i = 0; i < work.size();) {
    const int32_t nu = p->hp.atoms[work[i].atom].nu;
    Group g{nu, (int32_t)i, 0};
    while (i < work.size() && p->hp.atoms[work[i].atom].nu == nu) {
      g.count++;
      ++i;
    }
    p->groups.push_back(g);
  }
  p->sched_version++;
  return upload_phases(p);
}

// (Re)uploads the block tables of the expansion.
hipError_t upload_blocks(sho_plan_s *p) {
  const bool stored = (p->hp.flags & SHO_FLAG_STORED) && !p->hp.run_poff.empty();
  if (stored) sho::build_desc_pbase(&p->hp);
  if (p->d_desc_pbase) (void)hipFree(p->d_desc_pbase);
  p->d_desc_pbase = nullptr;
  for (void **q : {(void **)&p->d_blocks, (void **)&p->d_entries, (void **)&p->d_run_desc}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  int64_t &bytes = p->blk_bytes;
  bytes = 0;
  hipError_t e;
  if ((e = upload(&p->d_blocks, p->hp.blocks, &bytes)) != hipSuccess ||
      (e = upload(&p->d_entries, p->hp.entries, &bytes)) != hipSuccess ||
      (e = upload(&p->d_run_desc, p->hp.run_desc, &bytes)) != hipSuccess)
    return e;
  if (stored && (e = upload(&p->d_desc_pbase, p->hp.desc_pbase, &bytes)) != hipSuccess)
    return e;
  return upload_phases(p);
}

// (Re)uploads the block tables of the projection's block form.
hipError_t upload_pblocks(sho_plan_s *p) {
  for (void **q : {(void **)&p->d_pblocks, (void **)&p->d_pentries, (void **)&p->d_prun_desc}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  int64_t &bytes = p->pblk_bytes;
  bytes = 0;
  hipError_t e;
  if ((e = upload(&p->d_pblocks, p->hp.pblk.blocks, &bytes)) != hipSuccess ||
      (e = upload(&p->d_pentries, p->hp.pblk.entries, &bytes)) != hipSuccess ||
      (e = upload(&p->d_prun_desc, p->hp.pblk.run_desc, &bytes)) != hipSuccess)
    return e;
  return hipSuccess;
}

// Radial projector set of a plan made by sho_plan_create_radial.
struct RadialInput {
  int32_t nrad, nr, nproj;
  double dr;
  const int32_t *ell;     // [nrad]
  const double *tables;   // host [nrad][nr]
};

sho::SArgs make_sargs(const sho_plan_s *p, const Group &g) {
  sho::SArgs S;
  S.atoms = p->d_atoms;
  S.P = p->d_stored;
  S.atom_poff = p->d_atom_poff;
  S.atom_pbeg = p->d_atom_pbeg;
  S.pidx = p->d_pidx;
  S.items = p->d_sitems + g.work_begin;
  S.nitems = g.count;
  S.B = p->hp.nbands;
  S.ncol = p->hp.ncols > 0 ? p->hp.ncols : sho::nsho(g.nu);
  const double h = p->hp.grid.h;
  S.h3 = h * h * h;
  S.alpha = 1.0;
  return S;
}

sho::KArgs make_args(const sho_plan_s *p, const Group &g) {
  sho::KArgs K;
  K.atoms = p->d_atoms;
  K.lines = p->d_lines;
  K.bundles = p->d_bundles;
  K.work = p->d_work + g.work_begin;
  K.tab = p->d_tab;
  K.stored = p->d_stored;
  K.run_poff = p->d_run_poff;
  K.nwork = g.count;
  K.nlines = (int32_t)std::max<size_t>(p->hp.lines.size(), 1);
  K.nx = p->hp.grid.n[0];
  K.B = p->hp.nbands;
  K.tb_shift = p->hp.tb_shift;
  K.ntiles = (p->hp.nbands + (1 << K.tb_shift) - 1) >> K.tb_shift;
  K.det = (p->hp.flags & SHO_FLAG_DETERMINISTIC) ? 1 : 0;
  K.bloch = p->bloch ? 1 : 0;
  const double h = p->hp.grid.h;
  K.h3 = h * h * h;
  K.alpha = 1.0;
  K.bundle_phase = p->d_bundle_phase;
  return K;
}

void prof_clear(sho_plan_s *p) {
  for (ProfEvent &ev : p->prof) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  p->prof.clear();
}

// Runs f (a sequence of launches on s), bracketed by events when profiling.
template <typename F>
hipError_t timed(sho_plan_s *p, bool prof, int kind, hipStream_t s, F &&f) {
  if (!prof) return f();
  ProfEvent ev{kind, nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev.a);
  if (e == hipSuccess) e = hipEventCreate(&ev.b);
  if (e == hipSuccess) e = hipEventRecord(ev.a, s);
  if (e != hipSuccess) return e;
  e = f();
  hipError_t e2 = hipEventRecord(ev.b, s);
  p->prof.push_back(ev);
  return e != hipSuccess ? e : e2;
}

sho::EArgs make_eargs(const sho_plan_s *p) {
  sho::EArgs E;
  E.atoms = p->d_atoms;
  E.lines = p->d_lines;
  E.run_atom = p->d_run_atom;
  E.row_runs = p->d_row_runs;
  E.rows = p->d_rows;
  E.u2_off = p->d_u2_off;
  E.nu_atoms = p->d_nu_atoms;
  E.tab = p->d_tab;
  E.nrows = (int32_t)p->hp.rows.size();
  E.natoms_u2 = (int32_t)p->hp.nu_atoms.size();
  E.nx = p->hp.grid.n[0];
  E.B = p->hp.nbands;
  E.tbe_shift = sho::plan_expand_shift(p->hp);
  E.desc_pbase = p->d_desc_pbase;
  E.P = p->d_stored;
  E.ntiles = (p->hp.nbands + (1 << E.tbe_shift) - 1) >> E.tbe_shift;
  E.ntiles_u2 = (p->hp.nbands + 31) / 32;
  E.nu_max = p->hp.nu_max;
  E.blocks = p->d_blocks;
  E.entries = p->d_entries;
  E.run_desc = p->d_run_desc;
  E.nblocks = (int32_t)p->hp.blocks.size();
  E.blk_rows = p->hp.blk_rows;
  E.blk_x = p->hp.blk_x;
  E.ny = p->hp.grid.n[1];
  E.ncol = p->hp.ncols;
  E.bloch = p->bloch ? 1 : 0;
  E.alpha = 1.0;
  E.entry_phase = p->d_entry_phase;
  for (int nu = 0; nu <= SHO_NU_MAX + 1; ++nu) E.nu_begin[nu] = 0;
  {
    int nu = 0;
    for (size_t i = 0; i <= p->hp.nu_atoms.size(); ++i) {
      const int cur = i < p->hp.nu_atoms.size() ? p->hp.atoms[p->hp.nu_atoms[i]].nu
                                                : SHO_NU_MAX + 1;
      while (nu <= cur && nu <= SHO_NU_MAX + 1) E.nu_begin[nu++] = (int32_t)i;
    }
  }
  return E;
}

// Arguments of the projection's block form: the expansion's, with the
// projection's block tables and band tile.
sho::EArgs make_peargs(const sho_plan_s *p) {
  sho::EArgs E = make_eargs(p);
  E.blocks = p->d_pblocks;
  E.entries = p->d_pentries;
  E.run_desc = p->d_prun_desc;
  E.nblocks = (int32_t)p->hp.pblk.blocks.size();
  E.blk_rows = p->hp.pblk.rows;
  E.blk_x = p->hp.pblk.x;
  E.tbe_shift = p->hp.pblk_tb_shift;
  E.ntiles = (p->hp.nbands + (1 << E.tbe_shift) - 1) >> E.tbe_shift;
  return E;
}

// A device buffer of at least `bytes` bytes must start at ptr: checked
// against the runtime's allocation record so that a wrong size or a host
// pointer is refused before any kernel touches it.
bool device_range_ok(const void *ptr, int64_t bytes) {
  if (!ptr) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (attr.type != hipMemoryTypeDevice && !attr.isManaged) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const char *b = static_cast<const char *>(base);
  const char *q = static_cast<const char *>(ptr);
  return q >= b && (int64_t)(q - b) + bytes <= (int64_t)size;
}

int64_t psi_bytes(const sho_plan_s *p) {
  return (int64_t)p->hp.grid.n[0] * p->hp.grid.n[1] * p->hp.grid.n[2] *
         p->hp.nbands * (int64_t)sizeof(double);
}

// Device bytes a plan of this geometry allocates (tables, work items, 1D
// tables, expansion scratch, stored tables), each rounded up as the
// allocations are.
int64_t estimate_device_bytes(const sho::HostPlan &hp) {
  auto b = [](int64_t n, int64_t size) { return std::max<int64_t>(n, 1) * size; };
  const int64_t nl = (int64_t)hp.lines.size();
  int64_t t = b(hp.natoms, sizeof(sho::AtomRec)) + b(nl, sizeof(sho::LineRec)) +
              b((int64_t)hp.bundles.size(), sizeof(sho::BundleRec)) +
              2 * b((int64_t)hp.work.size(), sizeof(sho::WorkRec)) +
              b(hp.table_doubles, 8) + 2 * b(nl, 4) +
              b((int64_t)hp.rows.size(), sizeof(sho::RowRec)) + b(hp.natoms, 8) +
              b(hp.natoms, 4) + b(hp.u2_doubles, 8) +
              b((int64_t)hp.blocks.size(), sizeof(sho::BlockRec)) +
              b((int64_t)hp.entries.size(), sizeof(sho::EntryRec)) +
              b((int64_t)hp.run_desc.size(), 4);
  if (hp.flags & SHO_FLAG_STORED) {
    int64_t stored = 0;
    for (const auto &A : hp.atoms) stored += (int64_t)A.npoints * sho::stored_cols(hp, A);
    const int64_t items = (hp.support_points + sho::kStoredChunk - 1) / sho::kStoredChunk +
                          hp.natoms;
    t += b(stored, 8) + b(nl + 1, 8) + 2 * b(hp.natoms + 1, 8) + b(hp.support_points, 4) +
         b(items, sizeof(sho::StoredItem));
  }
  return t;
}

void build_default_blocks(sho::HostPlan *hp) {
  if (hp->flags & SHO_FLAG_DETERMINISTIC) {
    hp->expand_mode = sho::kExpandOwner;
    sho::build_blocks(hp, sho::owner_rows(*hp), 32);
    return;
  }
  int32_t R = 0, X = 0;
  sho::default_block_shape(*hp, &R, &X);
  sho::build_blocks(hp, R, X);
  // stored plans: the block form wins while the products are short (measured
  // up to nu_max = 2, 10 columns), the atom-owner form with atomics beyond
  const bool long_rows = hp->ncols > 0 ? hp->ncols > 10 : hp->nu_max > 2;
  if ((hp->flags & SHO_FLAG_STORED) && long_rows) hp->expand_mode = sho::kExpandRows;
}

// Plans with several cut-offs run the projection as one launch.
int32_t default_schedule(const sho::HostPlan &hp) {
  if (hp.flags & SHO_FLAG_BLOCH) return sho::kSchedSingle;  // one kernel family
  for (const auto &A : hp.atoms)
    if (A.npoints > 0 && A.nu != hp.atoms[0].nu) return sho::kSchedSingle;
  return sho::kSchedByNu;
}

int64_t coeff_bytes(const sho_plan_s *p) {
  return p->hp.coeff_rows * p->hp.nbands * (int64_t)sizeof(double);
}

// Item range of atom a in `work` (per-atom launches).
Group atom_group(const sho_plan_s *p, int32_t a) {
  const int32_t b = p->hp.atom_work[a];
  int32_t n = 0;  // the items of one atom are contiguous
  while (b + n < (int32_t)p->hp.work.size() && p->hp.work[b + n].atom == a) ++n;
  return Group{p->hp.atoms[a].nu, b, n};
}

// Precision of an entry point: 0 double, 1 float, -1 either (the plan's).
sho_status check_project(const sho_plan_s *p, const void *psi, const void *c,
                         int want_f32 = 0) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (p->hp.flags & SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "host-only plan cannot run kernels");
  if (want_f32 >= 0 && (want_f32 != 0) != p->fp32)
    return fail(SHO_E_INVALID, p->fp32 ? "plan holds FP32 bands: use the _f32 entry points"
                                       : "plan holds FP64 bands: use the FP64 entry points");
  if (p->hp.coeff_rows == 0) return SHO_OK;
  if (!device_range_ok(psi, psi_bytes(p)) || !device_range_ok(c, coeff_bytes(p)))
    return fail(SHO_E_INVALID, "psi and c must be device buffers of the plan's sizes");
  if ((const char *)c < (const char *)psi + psi_bytes(p) &&
      (const char *)psi < (const char *)c + coeff_bytes(p))
    return fail(SHO_E_INVALID, "psi and c overlap");
  return SHO_OK;
}

// Expansion scratch (plane partials), allocated on first use.
sho_status ensure_u2(sho_plan_s *p) {
  if (p->d_u2 || (p->hp.flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM))) return SHO_OK;
  const int64_t n = std::max<int64_t>(p->hp.u2_doubles, 1) * sizeof(double);
  hipError_t e = hipMalloc((void **)&p->d_u2, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->d_u2 = nullptr;
    return e == hipErrorOutOfMemory ? fail(SHO_E_NOMEM, "device allocation failed")
                                    : hip_fail(e, "expansion scratch");
  }
  p->device_bytes += n;
  return SHO_OK;
}

// The projection's launches on s (arguments already checked).
hipError_t run_project(sho_plan_s *p, const void *psi_v, void *c_v, hipStream_t s,
                       bool prof) {
  const double *psi = static_cast<const double *>(psi_v);
  double *c = static_cast<double *>(c_v);
  // atoms whose support missed the grid entirely keep zero coefficients;
  // atoms shared by several work items (and every stored point chunk) are
  // summed into zeroed coefficients
  const bool blocks = p->hp.proj_form == sho::kProjectBlocks;
  bool zero = (p->hp.any_split && !blocks) || (p->hp.flags & SHO_FLAG_STORED);
  for (const auto &A : p->hp.atoms) zero |= (A.npoints == 0);
  if (zero) {
    hipError_t e = sho::launch_fill(c, p->hp.coeff_rows * p->hp.nbands, 0.0, s);
    if (e != hipSuccess) return e;
  }
  if (blocks) {
    // the plane sums go through the plan's plane-partial scratch
    return timed(p, prof, SHO_KERNEL_PROJECT, s, [&]() {
      const sho::EArgs E = make_peargs(p);
      hipError_t e1 = sho::launch_fill(p->d_u2, p->hp.u2_doubles, 0.0, s);
      if (e1 == hipSuccess) e1 = sho::launch_project_blocks(E, psi, p->d_u2, s);
      const double h = p->hp.grid.h;
      if (e1 == hipSuccess) e1 = sho::launch_zpass(E, p->d_u2, c, h * h * h, s);
      return e1;
    });
  }
  return timed(p, prof, SHO_KERNEL_PROJECT, s, [&]() {
    if (p->hp.flags & SHO_FLAG_STORED) {
      for (const Group &g : p->sgroups) {
        hipError_t e1 = sho::launch_project_stored(make_sargs(p, g), psi, c, s);
        if (e1 != hipSuccess) return e1;
      }
      return hipSuccess;
    }
    if (p->hp.flags & SHO_FLAG_PER_ATOM) {
      for (int32_t a = 0; a < p->hp.natoms; ++a) {
        const Group g = atom_group(p, a);
        if (!g.count) continue;
        hipError_t e1 = sho::launch_project(g.nu, make_args(p, g), psi, c, s);
        if (e1 != hipSuccess) return e1;
      }
      return hipSuccess;
    }
    for (const sho::ProjGroup &pg : p->hp.proj_groups) {
      sho::KArgs K = make_args(p, Group{pg.nu, 0, pg.count});
      K.work = p->d_work_proj + pg.begin;
      hipError_t e1;
      if (p->fp32) {
        const float *pf = static_cast<const float *>(psi_v);
        float *cf = static_cast<float *>(c_v);
        e1 = pg.nu < 0 ? sho::launch_project_any_f32(p->hp.nu_max, K, p->d_tab32, pf, cf, s)
                       : sho::launch_project_f32(pg.nu, K, p->d_tab32, pf, cf, s);
      } else {
        e1 = pg.nu < 0 ? sho::launch_project_any(p->hp.nu_max, K, psi, c, s)
                       : sho::launch_project(pg.nu, K, psi, c, s);
      }
      if (e1 != hipSuccess) return e1;
    }
    return hipSuccess;
  });
}

// True if s is capturing a graph (no cross-stream ordering is recorded then).
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

// Calls that use the plan's scratch on different streams are ordered: the
// call on s waits for the end of the previous one (outside graph capture).
hipError_t scratch_acquire(sho_plan_s *p, hipStream_t s) {
  if (!p->scratch_used || p->scratch_stream == s || capturing(s)) return hipSuccess;
  return hipStreamWaitEvent(s, p->scratch_ev, 0);
}

hipError_t scratch_release(sho_plan_s *p, hipStream_t s) {
  if (capturing(s)) return hipSuccess;
  hipError_t e = hipEventRecord(p->scratch_ev, s);
  if (e == hipSuccess) {
    p->scratch_stream = s;
    p->scratch_used = true;
  }
  return e;
}

// The expansion's launches on s (arguments checked, scratch allocated):
// psi += alpha * expansion of c, with the plane partials in u2 (the plan's
// own scratch or the static one; unused by stored and per-atom plans).
hipError_t run_expand(sho_plan_s *p, const void *c_v, void *psi_v, hipStream_t s,
                      bool prof, double *u2_buf, double alpha = 1.0) {
  const double *c = static_cast<const double *>(c_v);
  double *psi = static_cast<double *>(psi_v);
  if (p->fp32) {
    // FP32 plans: plane partials and the block form only
    sho::EArgs E = make_eargs(p);
    float *u2 = reinterpret_cast<float *>(u2_buf);
    hipError_t e = timed(p, prof, SHO_KERNEL_EXPAND_Z, s, [&]() {
      return sho::launch_expand_planes_f32(E, p->d_tab32, static_cast<const float *>(c_v),
                                           u2, s);
    });
    if (e == hipSuccess)
      e = timed(p, prof, SHO_KERNEL_EXPAND_XY, s, [&]() {
        return sho::launch_blocks_f32(E, p->d_tab32, u2, static_cast<float *>(psi_v), s);
      });
    return e;
  }
  if (p->hp.flags & SHO_FLAG_STORED) {
    if (p->hp.expand_mode == sho::kExpandBlocks) {
      sho::EArgs E = make_eargs(p);
      E.alpha = alpha;
      return timed(p, prof, SHO_KERNEL_EXPAND_XY, s,
                   [&]() { return sho::launch_blocks_stored(E, c, psi, s); });
    }
    return timed(p, prof, SHO_KERNEL_EXPAND_XY, s, [&]() {
      for (const Group &g : p->sgroups) {
        sho::SArgs S = make_sargs(p, g);
        S.alpha = alpha;
        hipError_t e1 = sho::launch_expand_stored(S, c, psi, s);
        if (e1 != hipSuccess) return e1;
      }
      return hipSuccess;
    });
  }
  if (p->hp.flags & SHO_FLAG_PER_ATOM) {
    return timed(p, prof, SHO_KERNEL_EXPAND_XY, s, [&]() {
      for (int32_t a = 0; a < p->hp.natoms; ++a) {
        const Group g = atom_group(p, a);
        if (!g.count) continue;
        sho::KArgs K = make_args(p, g);
        K.alpha = alpha;
        hipError_t e1 = sho::launch_expand_atomic(g.nu, K, c, psi, s);
        if (e1 != hipSuccess) return e1;
      }
      return hipSuccess;
    });
  }
  sho::EArgs E = make_eargs(p);
  E.alpha = alpha;
  hipError_t e = timed(p, prof, SHO_KERNEL_EXPAND_Z, s,
                       [&]() { return sho::launch_expand_planes(E, c, u2_buf, s); });
  if (e == hipSuccess)
    e = timed(p, prof, SHO_KERNEL_EXPAND_XY, s, [&]() {
      switch (p->hp.expand_mode) {
        case sho::kExpandBlocks:
          return sho::launch_blocks(E, u2_buf, psi, s);
        case sho::kExpandOwner:
          return sho::launch_owner(E, u2_buf, psi, s);
        default:
          return sho::launch_rows(E, u2_buf, psi, s);
      }
    });
  return e;
}

// run_project with the block form's plane sums in the plan's own scratch,
// ordered against the scratch's other users (the item form uses none).
hipError_t run_project_own(sho_plan_s *p, const void *psi, void *c, hipStream_t s, bool prof) {
  if (p->hp.proj_form != sho::kProjectBlocks) return run_project(p, psi, c, s, prof);
  hipError_t e = scratch_acquire(p, s);
  if (e == hipSuccess) e = run_project(p, psi, c, s, prof);
  if (e == hipSuccess) e = scratch_release(p, s);
  return e;
}

// run_expand on the plan's own scratch, ordered against its other users.
hipError_t run_expand_own(sho_plan_s *p, const void *c, void *psi, hipStream_t s, bool prof,
                          double alpha = 1.0) {
  hipError_t e = scratch_acquire(p, s);
  if (e == hipSuccess) e = run_expand(p, c, psi, s, prof, p->d_u2, alpha);
  if (e == hipSuccess) e = scratch_release(p, s);
  return e;
}

// Device side of a new plan whose host geometry p->hp is built: work split,
// tables, uploads, stored projector tables (sampled SHO functions, or the
// radial set rad), scratch.  Takes ownership of p (deleted on failure).
sho_status finish_plan(sho_plan_s *p, uint32_t flags, int32_t nbands, bool f32,
                       const RadialInput *rad, sho_plan_t *out) {
  // FP32 plans keep the projection's coefficient tile in double for both
  // bands of a pair: half the LDS budget per lane value; deterministic plans
  // keep one tile per wave
  const size_t lds_div = f32 ? 2 : (flags & SHO_FLAG_DETERMINISTIC) ? sho::kWaves : 1;
  if (flags & SHO_FLAG_HOST_ONLY) {
    // geometry and sizes only; work split as for a 64 KiB workgroup LDS
    const int tbs = sho::choose_tb_shift(nbands, p->hp.nu_max, (65536 - sho::kStaticLds) / lds_div);
    if (tbs < 0 || (p->bloch && !f32 && tbs < 1)) {
      delete p;
      return fail(SHO_E_BOX, "coefficient tile too large for the workgroup LDS");
    }
    sho::build_work(&p->hp, tbs, sho::kTargetPoints, default_schedule(p->hp));
    sho::build_rows(&p->hp);
    build_default_blocks(&p->hp);
    *out = p;
    return SHO_OK;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  int shm = 0;
  e = hipDeviceGetAttribute(&shm, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  p->lds_limit = (size_t)std::max(shm - sho::kStaticLds, 0) / lds_div;  // static LDS of the kernels
  const int tbs = sho::choose_tb_shift(nbands, p->hp.nu_max, p->lds_limit);
  if (tbs < 0 || (p->bloch && !f32 && tbs < 1)) {
    delete p;
    return fail(SHO_E_BOX, "coefficient tile too large for the workgroup LDS");
  }
  sho::build_work(&p->hp, tbs, sho::kTargetPoints, default_schedule(p->hp));
  sho::build_rows(&p->hp);
  build_default_blocks(&p->hp);
  std::vector<double> no_tab;
  if ((e = upload(&p->d_atoms, p->hp.atoms, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_lines, p->hp.lines, &p->device_bytes)) != hipSuccess ||
      (e = upload_schedule(p)) != hipSuccess || (e = upload_blocks(p)) != hipSuccess ||
      (e = upload(&p->d_doff, p->hp.dmat_off, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_run_atom, p->hp.run_atom, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_row_runs, p->hp.row_runs, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_rows, p->hp.rows, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_u2_off, p->hp.u2_off, &p->device_bytes)) != hipSuccess ||
      (e = upload(&p->d_nu_atoms, p->hp.nu_atoms, &p->device_bytes)) != hipSuccess ||
      (e = hipMalloc((void **)&p->d_tab,
                     std::max<int64_t>(p->hp.table_doubles, 1) * sizeof(double))) !=
          hipSuccess) {
    free_plan_device(p);
    delete p;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? fail(SHO_E_NOMEM, "device allocation failed")
                                    : hip_fail(e, "plan upload");
  }
  p->device_bytes += std::max<int64_t>(p->hp.table_doubles, 1) * sizeof(double);
  e = sho::launch_tables(p->d_atoms, p->hp.natoms, p->hp.grid.h, p->d_tab, p->hp.m_max,
                         nullptr);
  if (e == hipSuccess && f32) {
    const int64_t tb = std::max<int64_t>(p->hp.table_doubles, 1) * sizeof(float);
    e = hipMalloc((void **)&p->d_tab32, tb);
    if (e == hipSuccess) {
      p->device_bytes += tb;
      e = sho::launch_tables_f32(p->d_tab, p->d_tab32, p->hp.table_doubles, nullptr);
    }
  }
  if (e == hipSuccess && (flags & SHO_FLAG_STORED)) {
    sho::HostPlan &hp = p->hp;
    sho::build_stored(&hp, sho::kStoredChunk);
    e = upload_blocks(p);
    for (size_t i = 0; i < hp.sitems.size();) {
      const int32_t nu = hp.atoms[hp.sitems[i].atom].nu;
      Group g{nu, (int32_t)i, 0};
      while (i < hp.sitems.size() && hp.atoms[hp.sitems[i].atom].nu == nu) {
        g.count++;
        ++i;
      }
      p->sgroups.push_back(g);
    }
    const int64_t sb = std::max<int64_t>(hp.stored_doubles, 1) * sizeof(double);
    if (e == hipSuccess &&
        (e = upload(&p->d_run_poff, hp.run_poff, &p->device_bytes)) == hipSuccess &&
        (e = upload(&p->d_atom_poff, hp.atom_poff, &p->device_bytes)) == hipSuccess &&
        (e = upload(&p->d_atom_pbeg, hp.atom_pbeg, &p->device_bytes)) == hipSuccess &&
        (e = upload(&p->d_pidx, hp.pidx, &p->device_bytes)) == hipSuccess &&
        (e = upload(&p->d_sitems, hp.sitems, &p->device_bytes)) == hipSuccess &&
        (e = hipMalloc((void **)&p->d_stored, sb)) == hipSuccess) {
      p->stored_bytes = sb;
      p->device_bytes += sb;
      Group all{0, 0, 0};
      sho::KArgs K = make_args(p, all);
      if (rad) {
        // the radial tables are needed only while the stored values are sampled
        double *d_rad = nullptr;
        const size_t rb = (size_t)rad->nrad * rad->nr * sizeof(double);
        e = hipMalloc((void **)&d_rad, rb);
        if (e == hipSuccess)
          e = hipMemcpy(d_rad, rad->tables, rb, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
          sho::RArgs R{};
          R.rad = d_rad;
          R.nrad = rad->nrad;
          R.nr = rad->nr;
          R.nproj = rad->nproj;
          for (int32_t k = 0; k < rad->nrad; ++k) R.ell[k] = rad->ell[k];
          R.dr = rad->dr;
          R.h = hp.grid.h;
          e = sho::launch_store_radial(K, R, p->d_run_atom, (int32_t)hp.lines.size(),
                                       p->d_stored, nullptr);
          if (e == hipSuccess) e = hipDeviceSynchronize();
        }
        if (d_rad) (void)hipFree(d_rad);
      } else {
        e = sho::launch_store(K, p->d_run_atom, (int32_t)hp.lines.size(), p->d_stored,
                              nullptr);
      }
    }
  }
  if (e == hipSuccess && (flags & SHO_FLAG_DETERMINISTIC)) {
    // per-(atom, band tile) derivative sums, for any band tile down to one
    const int64_t gb = std::max<int64_t>((int64_t)p->hp.natoms * nbands * 3, 1) * sizeof(double);
    e = hipMalloc((void **)&p->d_gpart, gb);
    if (e == hipSuccess) p->device_bytes += gb;
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->scratch_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_plan_device(p);
    delete p;
    return hip_fail(e, "table sampling");
  }
  *out = p;
  return SHO_OK;
}


}  // namespace

// ----------------------------------------------------------------- C ABI --

extern "C" {

int32_t sho_nsho(int32_t nu) { return nu < 0 ? -1 : sho::nsho(nu); }

const char *sho_last_error(void) { return g_err.c_str(); }

sho_status sho_plan_create(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, sho_plan_t *out) {
  if (!out) return fail(SHO_E_INVALID, "out must not be NULL");
  *out = nullptr;
  const bool f32 = (flags & SHO_FLAG_FP32) != 0;
  const bool bloch = (flags & SHO_FLAG_BLOCH) != 0;
  if (bloch) {
    if (nbands <= 0 || nbands > (1 << 29))
      return fail(SHO_E_INVALID, "Bloch plans need a positive number of complex bands");
    if (flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM | SHO_FLAG_DETERMINISTIC))
      return fail(SHO_E_INVALID, "SHO_FLAG_BLOCH does not combine with SHO_FLAG_STORED, "
                                 "SHO_FLAG_PER_ATOM or SHO_FLAG_DETERMINISTIC");
    nbands *= 2;  // real and imaginary parts
  }
  if (f32) {
    if (nbands <= 0 || nbands % 2)
      return fail(SHO_E_INVALID, "FP32 plans need a positive, even number of bands");
    if (flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM))
      return fail(SHO_E_INVALID,
                  "SHO_FLAG_FP32 does not combine with SHO_FLAG_STORED or SHO_FLAG_PER_ATOM");
    nbands /= 2;  // the kernels work on band pairs
  }
  if ((flags & SHO_FLAG_DETERMINISTIC) &&
      (flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM | SHO_FLAG_FP32)))
    return fail(SHO_E_INVALID,
                "SHO_FLAG_DETERMINISTIC does not combine with SHO_FLAG_STORED, "
                "SHO_FLAG_PER_ATOM or SHO_FLAG_FP32");
  sho_plan_s *p = new (std::nothrow) sho_plan_s();
  if (!p) return fail(SHO_E_NOMEM, "host allocation failed");
  p->fp32 = f32;
  p->bloch = bloch;
  std::string msg;
  sho_status st = sho::build_host_plan(grid, natoms, pos, sigma, numax, rbox,
                                       nbands, flags, &p->hp, &msg);
  if (st != SHO_OK) {
    delete p;
    return fail(st, msg);
  }
  if (bloch) {
    // image counts along each axis must fit the entry records (|m| <= 127)
    for (const auto &A : p->hp.atoms) {
      if (A.npoints == 0) continue;
      const int32_t i0[3] = {A.ix0, A.iy0, A.iz0}, m[3] = {A.mx, A.my, A.mz};
      for (int d = 0; d < 3; ++d) {
        const int64_t n = p->hp.grid.n[d];
        auto img = [&](int64_t i) { return i >= 0 ? i / n : -((-i + n - 1) / n); };
        if (std::llabs(img(i0[d])) > 127 || std::llabs(img((int64_t)i0[d] + m[d] - 1)) > 127) {
          delete p;
          return fail(SHO_E_BOX, "a support reaches more than 127 periodic images");
        }
      }
    }
  }
  return finish_plan(p, flags, nbands, f32, nullptr, out);
}

sho_status sho_plan_create_radial(const sho_grid *grid, int32_t natoms, const double *pos,
                                  const double *rcut, int32_t nradial, const int32_t *ell,
                                  int32_t nr, double dr, const double *tables,
                                  int32_t nbands, uint32_t flags, sho_plan_t *out) {
  if (!out) return fail(SHO_E_INVALID, "out must not be NULL");
  *out = nullptr;
  if (flags & ~(uint32_t)SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "radial plans take no flags but SHO_FLAG_HOST_ONLY");
  if (nradial < 1 || nradial > sho::kRadialMaxFuncs || !ell || !tables)
    return fail(SHO_E_INVALID, "need 1..16 radial functions with their l and tables");
  if (nr < 4 || !(dr > 0.0) || !std::isfinite(dr))
    return fail(SHO_E_INVALID, "radial tables need nr >= 4 nodes and a finite dr > 0");
  int32_t nproj = 0;
  for (int32_t k = 0; k < nradial; ++k) {
    if (ell[k] < 0 || ell[k] > sho::kRadialMaxL)
      return fail(SHO_E_INVALID, "angular momenta must lie in 0..3");
    nproj += 2 * ell[k] + 1;
  }
  if (nproj > sho::kRadialMaxProj)
    return fail(SHO_E_INVALID, "at most 56 projectors per atom");
  for (int64_t i = 0; i < (int64_t)nradial * nr; ++i)
    if (!std::isfinite(tables[i])) return fail(SHO_E_INVALID, "non-finite radial table value");
  if (natoms < 0 || (natoms > 0 && (!pos || !rcut)))
    return fail(SHO_E_INVALID, "positions and cut-off radii are required");
  for (int32_t a = 0; a < natoms; ++a)
    if (!(rcut[a] > 0.0) || !std::isfinite(rcut[a]))
      return fail(SHO_E_INVALID, "cut-off radii must be finite and positive");
  // the support geometry is that of an SHO plan with nu = 0 and the cut-off
  // as support radius (sigma = rcut only satisfies the sampling bound; the
  // SHO tables of such a plan are not used)
  if (!grid || !(grid->h > 0.0)) return fail(SHO_E_INVALID, "grid with a positive spacing required");
  std::vector<int32_t> nu0(std::max(natoms, 1), 0);
  std::vector<double> sig(std::max(natoms, 1), grid->h);
  for (int32_t a = 0; a < natoms; ++a) sig[a] = std::max(rcut[a], grid->h);
  sho_plan_s *p = new (std::nothrow) sho_plan_s();
  if (!p) return fail(SHO_E_NOMEM, "host allocation failed");
  const uint32_t pflags = flags | SHO_FLAG_STORED;
  std::string msg;
  sho_status st = sho::build_host_plan(grid, natoms, pos, sig.data(), nu0.data(), rcut,
                                       nbands, pflags, &p->hp, &msg);
  if (st != SHO_OK) {
    delete p;
    return fail(st, msg);
  }
  // coefficient blocks [nproj][B] per atom
  sho::HostPlan &hp = p->hp;
  hp.ncols = nproj;
  hp.coeff_rows = 0;
  for (int32_t a = 0; a < natoms; ++a) {
    hp.atoms[a].coeff_row = hp.coeff_rows;
    hp.coeff_rows += nproj;
    hp.coeff_off[a + 1] = hp.coeff_rows * nbands;
  }
  const RadialInput rad{nradial, nr, nproj, dr, ell, tables};
  return finish_plan(p, pflags, nbands, false, &rad, out);
}

sho_status sho_plan_destroy(sho_plan_t p) {
  if (!p) return SHO_OK;
  if (p->hp.flags & SHO_FLAG_HOST_ONLY) {
    delete p;
    return SHO_OK;
  }
  prof_clear(p);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  hipError_t e = hipDeviceSynchronize();
  free_plan_device(p);
  if (cur != p->device) (void)hipSetDevice(cur);
  delete p;
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  return SHO_OK;
}

sho_status sho_plan_release_scratch(sho_plan_t p) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (!p->d_u2) return SHO_OK;
  // queued calls and graph launches may still read the scratch
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipFree(p->d_u2);
  if (cur != p->device) (void)hipSetDevice(cur);
  p->d_u2 = nullptr;
  p->device_bytes -= std::max<int64_t>(p->hp.u2_doubles, 1) * sizeof(double);
  p->scratch_used = false;
  p->scratch_gen++;
  if (e != hipSuccess) return hip_fail(e, "hipFree");
  return SHO_OK;
}

sho_status sho_plan_profile(sho_plan_t p, int32_t enable) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (p->hp.flags & SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "host-only plan cannot run kernels");
  if (enable) prof_clear(p);
  p->prof_on = enable != 0;
  return SHO_OK;
}

sho_status sho_plan_profile_read(sho_plan_t p, int64_t *counts, double *mean_ms) {
  if (!p || !counts || !mean_ms) return fail(SHO_E_INVALID, "NULL argument");
  double sum[SHO_KERNEL_KINDS] = {0, 0, 0, 0};
  for (int k = 0; k < SHO_KERNEL_KINDS; ++k) counts[k] = 0;
  for (ProfEvent &ev : p->prof) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(ev.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
    if (e != hipSuccess) return hip_fail(e, "profile events");
    sum[ev.kind] += ms;
    counts[ev.kind]++;
  }
  for (int k = 0; k < SHO_KERNEL_KINDS; ++k)
    mean_ms[k] = counts[k] ? sum[k] / (double)counts[k] : 0.0;
  return SHO_OK;
}

sho_status sho_plan_get_info(sho_plan_t p, sho_plan_info *info) {
  if (!p || !info) return fail(SHO_E_INVALID, "NULL plan or info");
  info->natoms = p->hp.natoms;
  const int64_t per_lane = p->fp32 ? 2 : 1;  // bands per kernel lane
  // Bloch plans: complex bands (two reals each)
  info->nbands = (int32_t)(p->hp.nbands * per_lane / (p->bloch ? 2 : 1));
  info->nu_max = p->hp.nu_max;
  info->flags = (int32_t)p->hp.flags;
  info->coeff_rows = p->hp.coeff_rows;
  info->coeff_doubles = p->hp.coeff_rows * p->hp.nbands * per_lane;
  info->support_points = p->hp.support_points;
  info->lines = (int64_t)p->hp.lines.size();
  info->planes = (int64_t)p->hp.planes.size();
  info->device_bytes = (p->hp.flags & SHO_FLAG_HOST_ONLY)
                           ? estimate_device_bytes(p->hp)
                           : p->device_bytes + p->sched_bytes + p->blk_bytes;
  info->expand_blocks = (int64_t)p->hp.blocks.size();
  info->expand_entries = (int64_t)p->hp.entries.size();
  info->stored_bytes = p->stored_bytes;
  info->union_points = p->hp.union_points;
  // the row kernel moves whole chunks of touched rows: with 32 or 64 bands
  // per tile a chunk spans 64 or 32 points (2048 doubles)
  info->expand_points = p->hp.expand_mode != sho::kExpandRows
                            ? p->hp.block_points
                            : p->hp.rows_touched * (int64_t)p->hp.grid.n[0];
  info->expand_scratch_doubles = p->hp.u2_doubles;
  return SHO_OK;
}

sho_status sho_plan_coeff_offsets(sho_plan_t p, int64_t *off) {
  if (!p || !off) return fail(SHO_E_INVALID, "NULL plan or output");
  std::memcpy(off, p->hp.coeff_off.data(),
              p->hp.coeff_off.size() * sizeof(int64_t));
  if (p->fp32)  // element offsets: two floats per band pair
    for (size_t a = 0; a < p->hp.coeff_off.size(); ++a) off[a] *= 2;
  return SHO_OK;
}

sho_status sho_plan_support_counts(sho_plan_t p, int64_t *counts) {
  if (!p || !counts) return fail(SHO_E_INVALID, "NULL plan or output");
  for (int32_t a = 0; a < p->hp.natoms; ++a) counts[a] = p->hp.atoms[a].npoints;
  return SHO_OK;
}

sho_status sho_plan_set_kpoint(sho_plan_t p, const double *k) {
  if (!p || !k) return fail(SHO_E_INVALID, "NULL plan or k");
  if (!p->bloch) return fail(SHO_E_INVALID, "not a Bloch plan (SHO_FLAG_BLOCH)");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(k[d])) return fail(SHO_E_INVALID, "k must be finite");
  if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
    hipError_t e = hipDeviceSynchronize();  // queued work reads the phase tables
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }
  for (int d = 0; d < 3; ++d) p->kvec[d] = k[d];
  hipError_t e = upload_phases(p);
  if (e != hipSuccess) return hip_fail(e, "phase upload");
  p->sched_version++;  // graphs captured with the previous k are refused
  return SHO_OK;
}

sho_status sho_plan_set_centres(sho_plan_t p, const double *pos, void *stream) {
  if (!p || (!pos && p->hp.natoms)) return fail(SHO_E_INVALID, "NULL plan or pos");
  if (p->hp.flags & SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "host-only plan has no device tables");
  if (p->hp.flags & SHO_FLAG_STORED)
    return fail(SHO_E_INVALID, "stored-projector plans cannot move their centres");
  for (int32_t a = 0; a < p->hp.natoms; ++a)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(pos[3 * a + d]))
        return fail(SHO_E_INVALID, "non-finite position");
  for (int32_t a = 0; a < p->hp.natoms; ++a) {
    p->hp.atoms[a].cx = pos[3 * a];
    p->hp.atoms[a].cy = pos[3 * a + 1];
    p->hp.atoms[a].cz = pos[3 * a + 2];
  }
  if (!p->hp.natoms) return SHO_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(p->d_atoms, p->hp.atoms.data(),
                                p->hp.atoms.size() * sizeof(sho::AtomRec),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = sho::launch_tables(p->d_atoms, p->hp.natoms, p->hp.grid.h, p->d_tab,
                           p->hp.m_max, s);
  if (e == hipSuccess && p->fp32)
    e = sho::launch_tables_f32(p->d_tab, p->d_tab32, p->hp.table_doubles, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "centre upload");
  return SHO_OK;
}

sho_status sho_plan_project(sho_plan_t p, const double *psi, double *c,
                            void *stream) {
  sho_status st = check_project(p, psi, c);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  // the block form's plane sums live in the plan's scratch, which
  // sho_plan_release_scratch may have freed
  if (p->hp.proj_form == sho::kProjectBlocks && (st = ensure_u2(p)) != SHO_OK) return st;
  hipError_t e = run_project_own(p, psi, c, (hipStream_t)stream, p->prof_on);
  if (e != hipSuccess) return hip_fail(e, "project launch");
  return SHO_OK;
}

sho_status sho_plan_expand(sho_plan_t p, const double *c, double *psi,
                           void *stream) {
  sho_status st = check_project(p, psi, c);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  hipError_t e = run_expand_own(p, c, psi, (hipStream_t)stream, p->prof_on);
  if (e != hipSuccess) return hip_fail(e, "expand launch");
  return SHO_OK;
}

sho_status sho_plan_expand_scaled(sho_plan_t p, double alpha, const double *c, double *psi,
                                  void *stream) {
  if (!std::isfinite(alpha)) return fail(SHO_E_INVALID, "alpha must be finite");
  sho_status st = check_project(p, psi, c);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  hipError_t e = run_expand_own(p, c, psi, (hipStream_t)stream, p->prof_on, alpha);
  if (e != hipSuccess) return hip_fail(e, "expand launch");
  return SHO_OK;
}

sho_status sho_plan_expand_noalloc(sho_plan_t p, const double *c, double *psi, void *stream) {
  sho_status st = check_project(p, psi, c);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  const bool uses_u2 = !(p->hp.flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM));
  if (uses_u2 && p->hp.u2_doubles > sho::kStaticScratchDoubles)
    return fail(SHO_E_INVALID,
                "plane partials need " + std::to_string(p->hp.u2_doubles) +
                    " doubles, the static scratch holds " +
                    std::to_string(sho::kStaticScratchDoubles));
  double *u2 = nullptr;
  hipError_t e = hipSuccess;
  if (uses_u2 && (e = sho::static_scratch(&u2)) != hipSuccess)
    return hip_fail(e, "static scratch address");
  // no profiling events: nothing is created or allocated on this path
  e = run_expand(p, c, psi, (hipStream_t)stream, false, u2);
  if (e != hipSuccess) return hip_fail(e, "expand launch");
  return SHO_OK;
}

sho_status sho_plan_project_f32(sho_plan_t p, const float *psi, float *c, void *stream) {
  sho_status st = check_project(p, psi, c, 1);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  hipError_t e = run_project(p, psi, c, (hipStream_t)stream, p->prof_on);
  if (e != hipSuccess) return hip_fail(e, "project launch");
  return SHO_OK;
}

sho_status sho_plan_expand_f32(sho_plan_t p, const float *c, float *psi, void *stream) {
  sho_status st = check_project(p, psi, c, 1);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  hipError_t e = run_expand_own(p, c, psi, (hipStream_t)stream, p->prof_on);
  if (e != hipSuccess) return hip_fail(e, "expand launch");
  return SHO_OK;
}

sho_status sho_plan_force(sho_plan_t p, const double *psi, const double *w,
                          double *grad, void *stream) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (p->fp32) return fail(SHO_E_INVALID, "the derivative is FP64 only");
  if (p->hp.ncols > 0) return fail(SHO_E_INVALID, "radial plans have no derivative");
  if (p->bloch) return fail(SHO_E_INVALID, "Bloch plans have no derivative");
  if (p->hp.flags & SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "host-only plan cannot run kernels");
  if (p->hp.natoms == 0) return SHO_OK;
  if (!device_range_ok(psi, psi_bytes(p)) || !device_range_ok(w, coeff_bytes(p)) ||
      !device_range_ok(grad, 3 * (int64_t)p->hp.natoms * (int64_t)sizeof(double)))
    return fail(SHO_E_INVALID, "psi, w and grad must be device buffers of the plan's sizes");
  hipStream_t s = (hipStream_t)stream;
  const bool det = (p->hp.flags & SHO_FLAG_DETERMINISTIC) != 0;
  // deterministic plans write every (atom, band tile) sum, then add them in
  // tile order; the others add into a zeroed grad with atomics
  hipError_t e = det ? hipSuccess : sho::launch_fill(grad, 3 * (int64_t)p->hp.natoms, 0.0, s);
  if (e == hipSuccess && det) e = sho::launch_fill(p->d_gpart, 3 * (int64_t)p->hp.natoms *
                                                                   p->hp.nbands, 0.0, s);
  if (e != hipSuccess) return hip_fail(e, "fill");
  e = timed(p, p->prof_on, SHO_KERNEL_FORCE, s, [&]() {
    if (p->hp.flags & SHO_FLAG_PER_ATOM) {
      for (int32_t a = 0; a < p->hp.natoms; ++a) {
        const Group g = atom_group(p, a);
        if (!g.count) continue;
        hipError_t e1 = sho::launch_force(g.nu, make_args(p, g), psi, w, grad, s);
        if (e1 != hipSuccess) return e1;
      }
      return hipSuccess;
    }
    sho::KArgs K0 = make_args(p, Group{0, 0, 0});
    for (const Group &g : p->groups) {
      hipError_t e1 = sho::launch_force(g.nu, make_args(p, g), psi, w, grad, s,
                                        det ? p->d_gpart : nullptr);
      if (e1 != hipSuccess) return e1;
    }
    return det ? sho::launch_force_sum(p->d_gpart, p->hp.natoms, K0.ntiles, grad, s)
               : hipSuccess;
  });
  if (e != hipSuccess) return hip_fail(e, "force launch");
  return SHO_OK;
}

sho_status sho_plan_set_schedule(sho_plan_t p, int32_t schedule, int32_t band_tile,
                                 int64_t target_points) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (!sho::sched_valid(schedule)) return fail(SHO_E_INVALID, "unknown schedule");
  if (target_points < 256 || target_points > (int64_t)1 << 30)
    return fail(SHO_E_INVALID, "target_points outside [256, 2^30]");
  int tbs = -1;
  for (int k = 0; k <= 6; ++k)
    if ((1 << k) == band_tile) tbs = k;
  if (band_tile == 0) tbs = p->hp.tb_shift;
  if (tbs < 0) return fail(SHO_E_INVALID, "band_tile must be 0 or a power of two <= 64");
  if (p->bloch && (schedule & ~sho::kSchedXcd) == sho::kSchedByNu)
    return fail(SHO_E_INVALID, "Bloch plans run single-launch schedules");
  if (p->bloch && !p->fp32 && tbs < 1)
    return fail(SHO_E_INVALID, "Bloch plans keep the real and imaginary lanes in one tile");
  const size_t limit = (p->hp.flags & SHO_FLAG_HOST_ONLY)
                           ? (65536 - sho::kStaticLds) / (p->fp32 ? 2
                                               : (p->hp.flags & SHO_FLAG_DETERMINISTIC) ? sho::kWaves
                                                                                        : 1)
                           : p->lds_limit;
  if (sho::lds_tile_bytes(p->hp.nu_max + 2, 1 << tbs) > limit)
    return fail(SHO_E_BOX, "band tile too wide for the workgroup LDS");
  if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
    hipError_t e = hipDeviceSynchronize();  // tables may be in use
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }
  sho::build_work(&p->hp, tbs, target_points, schedule);
  if (p->hp.flags & SHO_FLAG_HOST_ONLY) return SHO_OK;
  hipError_t e = upload_schedule(p);
  if (e != hipSuccess) return hip_fail(e, "schedule upload");
  return SHO_OK;
}

sho_status sho_plan_get_schedule(sho_plan_t p, int32_t *schedule, int32_t *band_tile,
                                 int64_t *target_points) {
  if (!p || !schedule || !band_tile || !target_points)
    return fail(SHO_E_INVALID, "NULL argument");
  *schedule = p->hp.sched;
  *band_tile = 1 << p->hp.tb_shift;
  *target_points = p->hp.target_points;
  return SHO_OK;
}

sho_status sho_plan_set_project(sho_plan_t p, int32_t form, int32_t block_rows,
                                int32_t block_x, int32_t band_tile) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (form != sho::kProjectItems && form != sho::kProjectBlocks)
    return fail(SHO_E_INVALID, "unknown projection form");
  if (form == sho::kProjectBlocks &&
      ((p->hp.flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM | SHO_FLAG_DETERMINISTIC)) ||
       p->fp32 || p->bloch))
    return fail(SHO_E_INVALID, "the block form of the projection is for FP64 plans of real "
                               "bands without SHO_FLAG_STORED, _PER_ATOM, _DETERMINISTIC");
  const bool dev = !(p->hp.flags & SHO_FLAG_HOST_ONLY);
  if (form == sho::kProjectItems) {
    p->hp.proj_form = form;
    p->sched_version++;
    return SHO_OK;
  }
  int tbs = -1;
  const int tb = band_tile ? band_tile : 16;
  for (int k = 3; k <= 6; ++k)
    if ((1 << k) == tb) tbs = k;
  if (tbs < 0) return fail(SHO_E_INVALID, "band_tile must be 0, 8, 16, 32 or 64");
  const int32_t X = block_x ? block_x : 32;
  if (X < 1 || X > 255) return fail(SHO_E_INVALID, "block_x outside 1..255");
  const int64_t per_row = (int64_t)sho::pow2_ceil(X) << tbs;
  const int32_t R = block_rows ? block_rows
                               : (int32_t)std::min<int64_t>(255, sho::kProjTileDoubles / per_row);
  if (R < 1 || R > 255 || R * per_row > sho::kProjTileDoubles)
    return fail(SHO_E_INVALID, "block of rows x points x band tile exceeds 8192 values");
  if (dev) {
    hipError_t e = hipDeviceSynchronize();  // the old tables may be in use
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }
  sho::build_block_set(&p->hp, R, X, &p->hp.pblk);
  p->hp.pblk_tb_shift = tbs;
  if (dev) {
    hipError_t e = upload_pblocks(p);
    if (e != hipSuccess) return hip_fail(e, "block upload");
    sho_status st = ensure_u2(p);
    if (st != SHO_OK) return st;
  }
  p->hp.proj_form = form;
  p->sched_version++;
  return SHO_OK;
}

sho_status sho_plan_get_project(sho_plan_t p, int32_t *form, int32_t *block_rows,
                                int32_t *block_x, int32_t *band_tile) {
  if (!p || !form || !block_rows || !block_x || !band_tile)
    return fail(SHO_E_INVALID, "NULL argument");
  *form = p->hp.proj_form;
  *block_rows = p->hp.pblk.rows;
  *block_x = p->hp.pblk.x;
  *band_tile = p->hp.pblk.rows ? 1 << p->hp.pblk_tb_shift : 0;
  return SHO_OK;
}

sho_status sho_plan_set_expand(sho_plan_t p, int32_t mode, int32_t block_rows,
                               int32_t block_x) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (mode != sho::kExpandRows && mode != sho::kExpandBlocks && mode != sho::kExpandOwner)
    return fail(SHO_E_INVALID, "unknown expansion form");
  if (p->fp32 && mode != sho::kExpandBlocks)
    return fail(SHO_E_INVALID, "FP32 plans expand in the block form only");
  if (p->bloch && mode != sho::kExpandBlocks)
    return fail(SHO_E_INVALID, "Bloch plans expand in the block form only");
  if ((p->hp.flags & SHO_FLAG_STORED) && mode == sho::kExpandOwner)
    return fail(SHO_E_INVALID, "stored plans expand in the row or block form");
  if ((p->hp.flags & SHO_FLAG_DETERMINISTIC) && mode != sho::kExpandOwner)
    return fail(SHO_E_INVALID, "deterministic plans expand in the owner form only");
  if (mode == sho::kExpandOwner) {
    const int32_t R = sho::owner_rows(p->hp);
    const int32_t X = block_x ? block_x : 32;
    if ((block_rows && block_rows != R) || !sho::owner_width_ok(X))
      return fail(SHO_E_INVALID, "owner form: block_rows must be 0 or 64 / band tile, "
                                 "block_x 0, 16 or 32");
    if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    }
    sho::build_blocks(&p->hp, R, X);
    if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
      hipError_t e = upload_blocks(p);
      if (e != hipSuccess) return hip_fail(e, "block upload");
    }
  }
  if (mode == sho::kExpandBlocks) {
    int32_t R = block_rows, X = block_x;
    if (R == 0 && X == 0) sho::default_block_shape(p->hp, &R, &X);
    if (!sho::block_shape_ok(p->hp, R, X))
      return fail(SHO_E_INVALID, "block shape does not fit the LDS tile or the table staging");
    if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    }
    sho::build_blocks(&p->hp, R, X);
    if (!(p->hp.flags & SHO_FLAG_HOST_ONLY)) {
      hipError_t e = upload_blocks(p);
      if (e != hipSuccess) return hip_fail(e, "block upload");
    }
  }
  p->hp.expand_mode = mode;
  p->sched_version++;
  return SHO_OK;
}

sho_status sho_plan_get_expand(sho_plan_t p, int32_t *mode, int32_t *block_rows,
                               int32_t *block_x) {
  if (!p || !mode || !block_rows || !block_x) return fail(SHO_E_INVALID, "NULL argument");
  *mode = p->hp.expand_mode;
  *block_rows = p->hp.blk_rows;
  *block_x = p->hp.blk_x;
  return SHO_OK;
}

sho_status sho_plan_set_expand_tile(sho_plan_t p, int32_t band_tile) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (p->hp.flags & SHO_FLAG_STORED)
    return fail(SHO_E_INVALID, "stored plans keep their matrix-core band tile");
  int tbs = -1;
  for (int k = 3; k <= 6; ++k)
    if ((1 << k) == band_tile) tbs = k;
  if (band_tile != 0 && tbs < 0)
    return fail(SHO_E_INVALID, "band_tile must be 0, 8, 16, 32 or 64");
  const bool dev = !(p->hp.flags & SHO_FLAG_HOST_ONLY);
  if (dev) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }
  p->hp.expand_tbe_shift = tbs;
  if (p->hp.expand_mode == sho::kExpandBlocks) {
    int32_t R = 0, X = 0;
    sho::default_block_shape(p->hp, &R, &X);
    sho::build_blocks(&p->hp, R, X);
    if (dev) {
      hipError_t e = upload_blocks(p);
      if (e != hipSuccess) return hip_fail(e, "block upload");
    }
  }
  p->sched_version++;
  return SHO_OK;
}

sho_status sho_plan_get_expand_tile(sho_plan_t p, int32_t *band_tile) {
  if (!p || !band_tile) return fail(SHO_E_INVALID, "NULL argument");
  *band_tile = 1 << sho::block_tile_shift(p->hp);
  return SHO_OK;
}

sho_status sho_plan_tune_expand(sho_plan_t p, const void *c, void *psi, int32_t reps,
                                void *stream, sho_tune_expand_result *result) {
  sho_status st = check_project(p, psi, c, -1);
  if (st != SHO_OK) return st;
  if (reps < 1 || reps > 1000) return fail(SHO_E_INVALID, "reps outside 1..1000");
  if (p->hp.flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM | SHO_FLAG_DETERMINISTIC))
    return fail(SHO_E_INVALID, "stored, per-atom and deterministic plans have fixed forms");
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  struct Cand {
    int32_t mode, tbs, R, X;
  };
  std::vector<Cand> cands;
  int nb_shift = 3;
  while ((1 << nb_shift) < p->hp.nbands && nb_shift < 6) ++nb_shift;
  const int32_t nfp = sho::table_nfp(p->hp.nu_max);
  for (int32_t tbs = 3; tbs <= nb_shift; ++tbs) {
    const int32_t keep = p->hp.expand_tbe_shift;
    p->hp.expand_tbe_shift = tbs;
    int32_t R = 0, X = 0;
    sho::default_block_shape(p->hp, &R, &X);
    for (const auto &rx : {std::make_pair(R, X), std::make_pair(std::max(1, R / 2), X),
                           std::make_pair(R, std::max(1, X / 2)),
                           std::make_pair(std::min(256 / nfp, 2 * R), std::max(1, X / 2))})
      if (sho::block_shape_ok(p->hp, rx.first, rx.second))
        cands.push_back({sho::kExpandBlocks, tbs, rx.first, rx.second});
    p->hp.expand_tbe_shift = keep;
  }
  if (!p->fp32 && !p->bloch) cands.push_back({sho::kExpandRows, -1, 0, 0});
  hipEvent_t ea = nullptr, eb = nullptr;
  hipError_t e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  auto time_current = [&](double *ms) -> hipError_t {
    hipError_t e1 = run_expand_own(p, c, psi, s, false);  // warm-up
    if (e1 == hipSuccess) e1 = hipEventRecord(ea, s);
    for (int r = 0; r < reps && e1 == hipSuccess; ++r) e1 = run_expand_own(p, c, psi, s, false);
    if (e1 == hipSuccess) e1 = hipEventRecord(eb, s);
    if (e1 == hipSuccess) e1 = hipEventSynchronize(eb);
    float t = 0.f;
    if (e1 == hipSuccess) e1 = hipEventElapsedTime(&t, ea, eb);
    *ms = (double)t / reps;
    return e1;
  };
  const Cand before{p->hp.expand_mode, p->hp.expand_tbe_shift, p->hp.blk_rows, p->hp.blk_x};
  double ms_before = 0.0;
  if (e == hipSuccess) e = time_current(&ms_before);
  double best = ms_before;
  Cand pick = before;
  int32_t tried = 1;
  auto apply = [&](const Cand &cd) -> hipError_t {
    hipError_t e1 = hipStreamSynchronize(s);
    if (e1 != hipSuccess) return e1;
    p->hp.expand_mode = cd.mode;
    p->hp.expand_tbe_shift = cd.tbs;
    if (cd.mode == sho::kExpandBlocks) {
      sho::build_blocks(&p->hp, cd.R, cd.X);
      e1 = upload_blocks(p);
    }
    return e1;
  };
  for (const Cand &cd : cands) {
    if (e != hipSuccess) break;
    if ((e = apply(cd)) != hipSuccess) break;
    double ms = 0.0;
    if ((e = time_current(&ms)) != hipSuccess) break;
    ++tried;
    if (ms < best) {
      best = ms;
      pick = cd;
    }
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  if (e != hipSuccess) return hip_fail(e, "tuning");
  if ((e = apply(pick)) != hipSuccess) return hip_fail(e, "expansion form upload");
  p->sched_version++;
  if (result) {
    result->mode = pick.mode;
    result->band_tile = 1 << sho::plan_expand_shift(p->hp);
    result->block_rows = p->hp.blk_rows;
    result->block_x = p->hp.blk_x;
    result->ms = best;
    result->ms_before = ms_before;
    result->candidates = tried;
    result->pad = 0;
  }
  return SHO_OK;
}

sho_status sho_plan_tune(sho_plan_t p, const void *psi, void *c, int32_t reps,
                         void *stream, sho_tune_result *result) {
  sho_status st = check_project(p, psi, c, -1);
  if (st != SHO_OK) return st;
  if (reps < 1 || reps > 1000) return fail(SHO_E_INVALID, "reps outside 1..1000");
  if (p->hp.flags & (SHO_FLAG_STORED | SHO_FLAG_PER_ATOM))
    return fail(SHO_E_INVALID, "stored and per-atom plans have a fixed schedule");
  const bool blocks_ok =
      !(p->hp.flags & SHO_FLAG_DETERMINISTIC) && !p->fp32 && !p->bloch;
  if (blocks_ok && (st = ensure_u2(p)) != SHO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  struct Cand {
    int32_t sched, tbs;
    int64_t target;
  };
  std::vector<Cand> cands;
  const int32_t tb0 = p->hp.tb_shift;
  const int32_t tb_min = (p->bloch && !p->fp32) ? 1 : 0;  // Bloch: re, im in one tile
  for (int32_t sc : {0, 1, 2, 3, 4, 5, 6, 7}) {
    if (p->bloch && (sc & ~sho::kSchedXcd) == sho::kSchedByNu) continue;
    for (int64_t tp : {(int64_t)4096, (int64_t)8192, (int64_t)16384, (int64_t)32768})
      for (int32_t tb = tb0; tb >= std::max(tb_min, tb0 - 1); --tb) cands.push_back({sc, tb, tp});
  }
  const Cand before{p->hp.sched, tb0, p->hp.target_points};
  const int32_t form0 = p->hp.proj_form;
  hipEvent_t ea = nullptr, eb = nullptr;
  hipError_t e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  auto time_current = [&](double *ms) -> hipError_t {
    hipError_t e1 = run_project(p, psi, c, s, false);  // warm-up
    if (e1 == hipSuccess) e1 = hipEventRecord(ea, s);
    for (int r = 0; r < reps && e1 == hipSuccess; ++r) e1 = run_project(p, psi, c, s, false);
    if (e1 == hipSuccess) e1 = hipEventRecord(eb, s);
    if (e1 == hipSuccess) e1 = hipEventSynchronize(eb);
    float t = 0.f;
    if (e1 == hipSuccess) e1 = hipEventElapsedTime(&t, ea, eb);
    *ms = (double)t / reps;
    return e1;
  };
  double ms_before = 0.0;
  if (e == hipSuccess) e = time_current(&ms_before);
  // item form: schedules x item sizes x band tiles
  p->hp.proj_form = sho::kProjectItems;
  double best = form0 == sho::kProjectItems ? ms_before : 1e300;
  Cand pick = before;
  int32_t tried = 1;
  for (const Cand &cd : cands) {
    if (e != hipSuccess) break;
    if (form0 == sho::kProjectItems && cd.sched == before.sched && cd.tbs == before.tbs &&
        cd.target == before.target)
      continue;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    sho::build_work(&p->hp, cd.tbs, cd.target, cd.sched);
    if ((e = upload_schedule(p)) != hipSuccess) break;
    double ms = 0.0;
    if ((e = time_current(&ms)) != hipSuccess) break;
    ++tried;
    if (ms < best) {
      best = ms;
      pick = cd;
    }
  }
  // block form: band tile x block width (rows: as many as the tile holds)
  struct BCand {
    int32_t tbs, x;
  };
  BCand bpick{0, 0};
  double bbest = 1e300;
  if (blocks_ok) {
    for (const BCand &bc : {BCand{4, 32}, BCand{3, 32}, BCand{5, 16}, BCand{4, 16}, BCand{3, 64}}) {
      if (e != hipSuccess) break;
      if ((1 << bc.tbs) > 2 * std::max<int32_t>(p->hp.nbands, 8)) continue;
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) break;
      const int64_t per_row = (int64_t)sho::pow2_ceil(bc.x) << bc.tbs;
      sho::build_block_set(&p->hp, (int32_t)std::min<int64_t>(255, sho::kProjTileDoubles / per_row),
                           bc.x, &p->hp.pblk);
      p->hp.pblk_tb_shift = bc.tbs;
      if ((e = upload_pblocks(p)) != hipSuccess) break;
      p->hp.proj_form = sho::kProjectBlocks;
      double ms = 0.0;
      e = time_current(&ms);
      p->hp.proj_form = sho::kProjectItems;
      if (e != hipSuccess) break;
      ++tried;
      if (ms < bbest) {
        bbest = ms;
        bpick = bc;
      }
    }
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  if (e != hipSuccess) return hip_fail(e, "tuning");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "tuning");
  sho::build_work(&p->hp, pick.tbs, pick.target, pick.sched);
  if ((e = upload_schedule(p)) != hipSuccess) return hip_fail(e, "schedule upload");
  const bool use_blocks = bbest < best;
  if (use_blocks) {
    const int64_t per_row = (int64_t)sho::pow2_ceil(bpick.x) << bpick.tbs;
    sho::build_block_set(&p->hp, (int32_t)std::min<int64_t>(255, sho::kProjTileDoubles / per_row),
                         bpick.x, &p->hp.pblk);
    p->hp.pblk_tb_shift = bpick.tbs;
    if ((e = upload_pblocks(p)) != hipSuccess) return hip_fail(e, "block upload");
    p->hp.proj_form = sho::kProjectBlocks;
  }
  p->sched_version++;
  if (result) {
    result->schedule = pick.sched;
    result->band_tile = 1 << pick.tbs;
    result->target_points = pick.target;
    result->ms = use_blocks ? bbest : best;
    result->ms_before = ms_before;
    result->candidates = tried;
    result->project_form = use_blocks ? sho::kProjectBlocks : sho::kProjectItems;
  }
  return SHO_OK;
}

sho_status sho_plan_matrix_offsets(sho_plan_t p, int64_t *off) {
  if (!p || !off) return fail(SHO_E_INVALID, "NULL plan or output");
  std::memcpy(off, p->hp.dmat_off.data(), p->hp.dmat_off.size() * sizeof(int64_t));
  return SHO_OK;
}

namespace {

sho_status check_multiply(const sho_plan_s *p, const double *D, const double *c,
                          const double *d) {
  if (!p) return fail(SHO_E_INVALID, "NULL plan");
  if (p->hp.flags & SHO_FLAG_HOST_ONLY)
    return fail(SHO_E_INVALID, "host-only plan cannot run kernels");
  if (p->fp32) return fail(SHO_E_INVALID, "the atomic-matrix product is FP64 only");
  if (p->hp.ncols > 0)
    return fail(SHO_E_INVALID, "radial plans carry no atomic matrices in the SHO basis");
  if (p->hp.coeff_rows == 0) return SHO_OK;
  const int64_t db = p->hp.dmat_off.back() * (int64_t)sizeof(double);
  if (!device_range_ok(D, db) || !device_range_ok(c, coeff_bytes(p)) ||
      !device_range_ok(d, coeff_bytes(p)))
    return fail(SHO_E_INVALID, "D, c and d must be device buffers of the plan's sizes");
  if ((const char *)c < (const char *)d + coeff_bytes(p) &&
      (const char *)d < (const char *)c + coeff_bytes(p))
    return fail(SHO_E_INVALID, "c and d overlap");
  return SHO_OK;
}

hipError_t run_multiply(sho_plan_s *p, const double *D, const double *c, double *d,
                        hipStream_t s) {
  return sho::launch_multiply(p->d_atoms, p->hp.natoms, p->d_doff, D, c, d, p->hp.nbands, s);
}

}  // namespace

sho_status sho_plan_multiply(sho_plan_t p, const double *D, const double *c, double *d,
                             void *stream) {
  sho_status st = check_multiply(p, D, c, d);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  hipError_t e = run_multiply(p, D, c, d, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "multiply launch");
  return SHO_OK;
}

sho_status sho_plan_apply(sho_plan_t p, const double *psi, const double *D, double *c,
                          double *d, double *out, void *stream) {
  sho_status st = check_project(p, psi, c);
  if (st == SHO_OK) st = check_multiply(p, D, c, d);
  if (st == SHO_OK) st = check_project(p, out, d);
  if (st != SHO_OK || p->hp.coeff_rows == 0) return st;
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = run_project_own(p, psi, c, s, p->prof_on);
  if (e == hipSuccess) e = run_multiply(p, D, c, d, s);
  if (e == hipSuccess) e = run_expand_own(p, d, out, s, p->prof_on);
  if (e != hipSuccess) return hip_fail(e, "apply launch");
  return SHO_OK;
}

// ------------------------------------------------------------- graphs --

struct sho_graph_s {
  sho_plan_t plan = nullptr;
  int64_t sched_version = 0;
  int64_t scratch_gen = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // extern "C"

namespace {

// Captures f(stream) into an instantiated graph owned by a new sho_graph_s.
template <typename F>
sho_status capture(sho_plan_t p, F &&f, sho_graph_t *g) {
  sho_graph_s *G = new (std::nothrow) sho_graph_s();
  if (!G) return fail(SHO_E_NOMEM, "host allocation failed");
  G->plan = p;
  G->sched_version = p->sched_version;
  G->scratch_gen = p->scratch_gen;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = p->hp.coeff_rows ? f(cs) : hipSuccess;
    e = hipStreamEndCapture(cs, &G->graph);
    if (e1 != hipSuccess) e = e1;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return hip_fail(e, "graph capture");
  }
  *g = G;
  return SHO_OK;
}

}  // namespace

extern "C" {

sho_status sho_graph_create(sho_plan_t p, const double *psi, double *c, double *out,
                            sho_graph_t *g) {
  if (!g) return fail(SHO_E_INVALID, "NULL graph output");
  *g = nullptr;
  sho_status st = check_project(p, psi, c);
  if (st != SHO_OK) return st;
  if (!device_range_ok(out, psi_bytes(p)))
    return fail(SHO_E_INVALID, "out must be a device buffer of the grid's size");
  if ((const char *)c < (const char *)out + psi_bytes(p) &&
      (const char *)out < (const char *)c + coeff_bytes(p))
    return fail(SHO_E_INVALID, "out and c overlap");
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  return capture(p, [&](hipStream_t cs) {
    hipError_t e1 = run_project(p, psi, c, cs, false);
    if (e1 == hipSuccess) e1 = run_expand(p, c, out, cs, false, p->d_u2);
    return e1;
  }, g);
}

sho_status sho_graph_create_apply(sho_plan_t p, const double *psi, const double *D,
                                  double *c, double *d, double *out, sho_graph_t *g) {
  if (!g) return fail(SHO_E_INVALID, "NULL graph output");
  *g = nullptr;
  sho_status st = check_project(p, psi, c);
  if (st == SHO_OK) st = check_multiply(p, D, c, d);
  if (st == SHO_OK) st = check_project(p, out, d);
  if (st != SHO_OK) return st;
  if ((st = ensure_u2(p)) != SHO_OK) return st;
  return capture(p, [&](hipStream_t cs) {
    hipError_t e1 = run_project(p, psi, c, cs, false);
    if (e1 == hipSuccess) e1 = run_multiply(p, D, c, d, cs);
    if (e1 == hipSuccess) e1 = run_expand(p, d, out, cs, false, p->d_u2);
    return e1;
  }, g);
}

sho_status sho_graph_launch(sho_graph_t g, void *stream) {
  if (!g) return fail(SHO_E_INVALID, "NULL graph");
  if (g->plan->sched_version != g->sched_version)
    return fail(SHO_E_INVALID, "the plan's schedule changed after the graph was made");
  if (g->plan->scratch_gen != g->scratch_gen)
    return fail(SHO_E_INVALID, "the plan's scratch was released after the graph was made");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return SHO_OK;
}

sho_status sho_graph_destroy(sho_graph_t g) {
  if (!g) return SHO_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return SHO_OK;
}

}  // extern "C"

// ----------------------------------------------------- stateless + cache --

namespace {

std::mutex g_cache_mu;
std::list<std::pair<std::string, sho_plan_t>> g_cache;  // most recent first
constexpr size_t kCacheSize = 8;

std::string cache_key(const sho_grid *grid, int32_t natoms, const double *pos,
                      const double *sigma, const int32_t *numax,
                      int32_t nbands, uint32_t flags, int device) {
  std::string k;
  auto put = [&k](const void *p, size_t n) {
    k.append(reinterpret_cast<const char *>(p), n);
  };
  put(grid, sizeof(sho_grid));
  put(&natoms, sizeof natoms);
  put(&nbands, sizeof nbands);
  put(&flags, sizeof flags);
  put(&device, sizeof device);
  if (natoms > 0) {
    put(pos, 3 * sizeof(double) * (size_t)natoms);
    put(sigma, sizeof(double) * (size_t)natoms);
    put(numax, sizeof(int32_t) * (size_t)natoms);
  }
  return k;
}

// Runs f(plan) with the plan for this geometry, built or reused from the
// cache.  The cache lock is held until f returns (f only queues work), so
// that no other thread can evict and destroy the plan while it is in use.
template <typename F>
sho_status with_cached_plan(const sho_grid *grid, int32_t natoms, const double *pos,
                            const double *sigma, const int32_t *numax, int32_t nbands,
                            uint32_t flags, F &&f) {
  if (!grid || natoms < 0 || (natoms > 0 && (!pos || !sigma || !numax)))
    return fail(SHO_E_INVALID, "NULL geometry arguments");
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string key = cache_key(grid, natoms, pos, sigma, numax, nbands, flags, dev);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
    if (it->first == key) {
      g_cache.splice(g_cache.begin(), g_cache, it);
      return f(g_cache.front().second);
    }
  }
  sho_plan_t p = nullptr;
  sho_status st = sho_plan_create(grid, natoms, pos, sigma, numax, nullptr,
                                  nbands, flags, &p);
  if (st != SHO_OK) return st;
  g_cache.emplace_front(std::move(key), p);
  while (g_cache.size() > kCacheSize) {
    sho_plan_destroy(g_cache.back().second);
    g_cache.pop_back();
  }
  return f(p);
}

}  // namespace

extern "C" {

sho_status sho_project(const sho_grid *grid, int32_t natoms, const double *pos,
                       const double *sigma, const int32_t *numax,
                       int32_t nbands, const double *psi, double *c,
                       uint32_t flags, void *stream) {
  return with_cached_plan(grid, natoms, pos, sigma, numax, nbands, flags,
                          [&](sho_plan_t p) { return sho_plan_project(p, psi, c, stream); });
}

sho_status sho_expand(const sho_grid *grid, int32_t natoms, const double *pos,
                      const double *sigma, const int32_t *numax,
                      int32_t nbands, const double *c, double *psi,
                      uint32_t flags, void *stream) {
  return with_cached_plan(grid, natoms, pos, sigma, numax, nbands, flags,
                          [&](sho_plan_t p) { return sho_plan_expand(p, c, psi, stream); });
}

sho_status sho_force(const sho_grid *grid, int32_t natoms, const double *pos,
                     const double *sigma, const int32_t *numax, int32_t nbands,
                     const double *psi, const double *w, double *grad,
                     uint32_t flags, void *stream) {
  return with_cached_plan(grid, natoms, pos, sigma, numax, nbands, flags, [&](sho_plan_t p) {
    return sho_plan_force(p, psi, w, grad, stream);
  });
}

sho_status sho_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  sho_status st = SHO_OK;
  for (auto &kv : g_cache) {
    sho_status s2 = sho_plan_destroy(kv.second);
    if (s2 != SHO_OK) st = s2;
  }
  g_cache.clear();
  return st;
}

}  // extern "C"
