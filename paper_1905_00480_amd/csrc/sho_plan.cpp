// sho_plan.cpp -- host-side geometry: validation and support tables.
//
// Compiled without floating-point contraction (-ffp-contract=off) so that the
// support membership test below is evaluated in exactly the IEEE double
// operation order the interface documents:
//     d = i*h - centre  (per axis),  r2 = (dx*dx + dy*dy) + dz*dz,
//     member  <=>  r2 <= R*R.
// The support is the projection sphere of sec. 6 of the paper; its default
// radius sigma*sqrt(2 nu + 3) + 2h is the classical turning radius of the
// highest shell nu (E sigma^2 = 2 nu + 3, sec. 2.2) plus two spacings.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>

#include "sho_internal.hpp"

namespace sho {
namespace {

int32_t wrap_index(int64_t i, int32_t n) {
  int64_t m = i % n;
  return (int32_t)(m < 0 ? m + n : m);
}

bool finite3(const double *p) {
  return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

}  // namespace

sho_status build_host_plan(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, HostPlan *out,
                           std::string *msg) {
  char buf[256];
  if (!grid || !out) {
    *msg = "grid and output pointers must not be NULL";
    return SHO_E_INVALID;
  }
  if (natoms < 0 || (natoms > 0 && (!pos || !sigma || !numax))) {
    *msg = "natoms < 0 or NULL atom arrays";
    return SHO_E_INVALID;
  }
  if (nbands <= 0) {
    *msg = "nbands must be positive";
    return SHO_E_INVALID;
  }
  const double h = grid->h;
  if (!(h > 0) || !std::isfinite(h)) {
    *msg = "grid spacing h must be positive and finite";
    return SHO_E_INVALID;
  }
  int64_t npts = 1;
  for (int d = 0; d < 3; ++d) {
    if (grid->n[d] <= 0) {
      *msg = "grid point counts must be positive";
      return SHO_E_INVALID;
    }
    npts *= grid->n[d];
  }
  if ((int64_t)grid->n[2] * grid->n[1] > std::numeric_limits<int32_t>::max() ||
      npts > std::numeric_limits<int64_t>::max() / 8 / nbands) {
    *msg = "grid too large";
    return SHO_E_INVALID;
  }
  // the kernels address a point within a grid line as x * nbands in 32-bit
  // integer (24-bit multiplies)
  if (nbands >= (1 << 24) || (int64_t)grid->n[0] * nbands > std::numeric_limits<int32_t>::max()) {
    *msg = "grid line too long for the band count (n[0] * nbands must stay below 2^31, "
           "nbands below 2^24)";
    return SHO_E_INVALID;
  }
  const uint32_t known =
      SHO_FLAG_STORED | SHO_FLAG_ALLOW_UNDERSAMPLED | SHO_FLAG_HOST_ONLY | SHO_FLAG_PER_ATOM |
      SHO_FLAG_FP32 | SHO_FLAG_DETERMINISTIC | SHO_FLAG_BLOCH;
  if (flags & ~known) {
    *msg = "unknown flag bits";
    return SHO_E_INVALID;
  }

  HostPlan &P = *out;
  P = HostPlan();
  P.grid = *grid;
  P.natoms = natoms;
  P.nbands = nbands;
  P.flags = flags;
  P.atoms.resize(natoms);
  P.support_centre.assign(pos, pos + 3 * (size_t)natoms);
  P.coeff_off.resize(natoms + 1);
  P.coeff_off[0] = 0;
  P.dmat_off.assign(natoms + 1, 0);

  for (int32_t a = 0; a < natoms; ++a) {
    const double *c = pos + 3 * a;
    const double s = sigma[a];
    const int32_t nu = numax[a];
    if (!finite3(c) || !(s > 0) || !std::isfinite(s)) {
      snprintf(buf, sizeof buf, "atom %d: non-finite position or sigma <= 0", a);
      *msg = buf;
      return SHO_E_INVALID;
    }
    if ((flags & SHO_FLAG_STORED) && nu > kStoredNuMax) {
      snprintf(buf, sizeof buf,
               "atom %d: nu_max %d above %d, the stored-projector limit", a, nu,
               kStoredNuMax);
      *msg = buf;
      return SHO_E_NU_RANGE;
    }
    if (nu < 0 || nu > SHO_NU_MAX) {
      snprintf(buf, sizeof buf, "atom %d: nu_max %d outside 0..%d", a, nu,
               SHO_NU_MAX);
      *msg = buf;
      return SHO_E_NU_RANGE;
    }
    // sampling bound, sec. 3.6 eq. max_grid_spacing
    const double hmax = M_PI * s / std::sqrt(2.0 * nu + 1.0);
    if (!(flags & SHO_FLAG_ALLOW_UNDERSAMPLED) && h > hmax) {
      snprintf(buf, sizeof buf,
               "atom %d: h = %g exceeds pi*sigma/sqrt(2nu+1) = %g", a, h, hmax);
      *msg = buf;
      return SHO_E_UNDERSAMPLED;
    }
    double R = s * std::sqrt(2.0 * nu + 3.0) + 2.0 * h;
    if (rbox) {
      R = rbox[a];
      if (!(R > 0) || !std::isfinite(R)) {
        snprintf(buf, sizeof buf, "atom %d: rbox must be positive", a);
        *msg = buf;
        return SHO_E_INVALID;
      }
    }
    const double R2 = R * R;
    // scan ranges that surely contain every member
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = (int64_t)std::floor((c[d] - R) / h) - 1;
      hi[d] = (int64_t)std::ceil((c[d] + R) / h) + 1;
      if (!grid->periodic[d]) {
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > grid->n[d] - 1) hi[d] = grid->n[d] - 1;
      }
      if (hi[d] - lo[d] + 1 > 4 * kMaxTable) {
        snprintf(buf, sizeof buf, "atom %d: support box too wide", a);
        *msg = buf;
        return SHO_E_BOX;
      }
    }
    AtomRec &A = P.atoms[a];
    A = AtomRec();
    A.cx = c[0];
    A.cy = c[1];
    A.cz = c[2];
    A.sigma = s;
    A.nu = nu;
    A.plane_begin = (int32_t)P.planes.size();
    A.line_begin = (int32_t)P.lines.size();
    int64_t xmin = INT64_MAX, xmax = INT64_MIN, ymin = INT64_MAX,
            ymax = INT64_MIN, zmin = INT64_MAX, zmax = INT64_MIN;
    struct RawLine { int64_t z, y, x0, len; };
    std::vector<RawLine> raw;
    for (int64_t iz = lo[2]; iz <= hi[2]; ++iz) {
      const double dz = (double)iz * h - c[2];
      for (int64_t iy = lo[1]; iy <= hi[1]; ++iy) {
        const double dy = (double)iy * h - c[1];
        int64_t x0 = 0, len = 0;
        for (int64_t ix = lo[0]; ix <= hi[0]; ++ix) {
          const double dx = (double)ix * h - c[0];
          double r2 = dx * dx + dy * dy;
          r2 = r2 + dz * dz;
          if (r2 <= R2) {
            if (len == 0) x0 = ix;
            ++len;
          } else if (len) {
            break;  // the members of a line are contiguous (sphere)
          }
        }
        if (!len) continue;
        raw.push_back({iz, iy, x0, len});
        xmin = std::min(xmin, x0);
        xmax = std::max(xmax, x0 + len - 1);
        ymin = std::min(ymin, iy);
        ymax = std::max(ymax, iy);
        zmin = std::min(zmin, iz);
        zmax = std::max(zmax, iz);
      }
    }
    if (!raw.empty()) {
      A.ix0 = (int32_t)xmin;
      A.iy0 = (int32_t)ymin;
      A.iz0 = (int32_t)zmin;
      A.mx = (int32_t)(xmax - xmin + 1);
      A.my = (int32_t)(ymax - ymin + 1);
      A.mz = (int32_t)(zmax - zmin + 1);
      if (A.mx > kMaxTable || A.my > kMaxTable || A.mz > kMaxTable) {
        snprintf(buf, sizeof buf,
                 "atom %d: support box spans more than %d points per axis", a,
                 kMaxTable);
        *msg = buf;
        return SHO_E_BOX;
      }
      P.m_max = std::max(P.m_max, std::max(A.mx, std::max(A.my, A.mz)));
    }
    int64_t cur_z = INT64_MIN;
    for (const RawLine &r : raw) {
      if (r.z != cur_z) {
        PlaneRec pl;
        pl.jz = (int32_t)(r.z - zmin);
        pl.line_begin = (int32_t)P.lines.size();
        pl.nlines = 0;
        pl.npoints = 0;
        P.planes.push_back(pl);
        cur_z = r.z;
      }
      // cut the line where it crosses the periodic x boundary
      int64_t k0 = 0;
      while (k0 < r.len) {
        const int32_t xm = wrap_index(r.x0 + k0, grid->n[0]);
        int64_t run = std::min<int64_t>(r.len - k0, (int64_t)grid->n[0] - xm);
        LineRec L;
        L.row = wrap_index(r.z, grid->n[2]) * grid->n[1] + wrap_index(r.y, grid->n[1]);
        L.x0m = xm;
        L.jx0 = (int16_t)(r.x0 + k0 - xmin);
        L.jy = (int16_t)(r.y - ymin);
        L.jz = (int16_t)(r.z - zmin);
        L.len = (int16_t)run;
        P.lines.push_back(L);
        k0 += run;
      }
      P.planes.back().nlines++;
      P.planes.back().npoints += (int32_t)r.len;
      A.npoints += r.len;
    }
    if (P.lines.size() > (size_t)std::numeric_limits<int32_t>::max()) {
      *msg = "too many support lines";
      return SHO_E_INVALID;
    }
    A.nplanes = (int32_t)P.planes.size() - A.plane_begin;
    A.nlines = (int32_t)P.lines.size() - A.line_begin;
    A.coeff_row = P.coeff_rows;
    A.tab_nfp = table_nfp(nu);
    A.tab_off = P.table_doubles;
    P.table_doubles += (int64_t)(A.mx + A.my + A.mz) * A.tab_nfp;
    P.coeff_rows += nsho(nu);
    P.coeff_off[a + 1] = P.coeff_rows * nbands;
    P.dmat_off[a + 1] = P.dmat_off[a] + (int64_t)nsho(nu) * nsho(nu);
    P.support_points += A.npoints;
    P.nu_max = std::max(P.nu_max, nu);
  }
  return SHO_OK;
}

int choose_tb_shift(int nbands, int nu_max, size_t lds_limit) {
  int shift = 0;
  while ((1 << shift) < nbands && shift < 6) ++shift;
  // the derivative contracts nu_max + 2 functions (tile of N_SHO(nu_max+1))
  while (shift > 0 && lds_tile_bytes(nu_max + 2, 1 << shift) > lds_limit) --shift;
  if (lds_tile_bytes(nu_max + 2, 1 << shift) > lds_limit) return -1;
  return shift;
}

namespace {

// 3D Morton key of a point given in cells of four grid points per axis.
uint64_t morton_key(const HostPlan *P, int32_t a) {
  uint64_t key = 0;
  uint32_t q[3];
  for (int d = 0; d < 3; ++d) {
    const int32_t n = P->grid.n[d];
    int64_t i = (int64_t)std::floor(P->support_centre[3 * a + d] / P->grid.h);
    if (P->grid.periodic[d]) i = ((i % n) + n) % n;
    i = std::min<int64_t>(std::max<int64_t>(i, 0), n - 1);
    q[d] = (uint32_t)(i >> 2);
  }
  for (int bit = 0; bit < 16; ++bit)
    for (int d = 0; d < 3; ++d)
      key |= (uint64_t)((q[d] >> bit) & 1u) << (3 * bit + (2 - d));
  return key;
}

// 2D Morton key of the (x, y) position of a centre, cells of four points.
uint64_t morton_xy(const HostPlan *P, int32_t a) {
  uint64_t key = 0;
  uint32_t q[2];
  for (int d = 0; d < 2; ++d) {
    const int32_t n = P->grid.n[d];
    int64_t i = (int64_t)std::floor(P->support_centre[3 * a + d] / P->grid.h);
    if (P->grid.periodic[d]) i = ((i % n) + n) % n;
    i = std::min<int64_t>(std::max<int64_t>(i, 0), n - 1);
    q[d] = (uint32_t)(i >> 2);
  }
  for (int bit = 0; bit < 16; ++bit)
    for (int d = 0; d < 2; ++d) key |= (uint64_t)((q[d] >> bit) & 1u) << (2 * bit + (1 - d));
  return key;
}

}  // namespace

void build_work(HostPlan *P, int tb_shift, int64_t target_points, int32_t sched) {
  const int slots = 64 >> tb_shift;
  P->tb_shift = tb_shift;
  P->sched = sched;
  P->target_points = target_points;
  P->bundles.clear();
  P->work.clear();
  P->work_proj.clear();
  P->proj_groups.clear();
  P->any_split = false;
  // bundles: the runs of each atom plane, ordered by their first x index so
  // that runs of similar extent share a bundle, in groups of `slots`
  std::vector<int32_t> atom_bundle_begin(P->natoms + 1, 0);
  std::vector<int64_t> cost;  // per bundle: x steps of the wave
  for (int32_t a = 0; a < P->natoms; ++a) {
    atom_bundle_begin[a] = (int32_t)P->bundles.size();
    const AtomRec &A = P->atoms[a];
    for (int32_t pi = A.plane_begin; pi < A.plane_begin + A.nplanes; ++pi) {
      const PlaneRec &pl = P->planes[pi];
      // runs of this plane: [pl.line_begin, next plane's line_begin)
      const int32_t rb = pl.line_begin;
      const int32_t re = (pi + 1 < A.plane_begin + A.nplanes)
                             ? P->planes[pi + 1].line_begin
                             : A.line_begin + A.nlines;
      // Bloch plans: runs of one periodic image together (a bundle carries
      // one phase), then by first x index
      const bool bloch = (P->flags & SHO_FLAG_BLOCH) != 0;
      auto image = [&](const LineRec &L) {  // image counts along x and y
        const int64_t mx = (int64_t)(A.ix0 + L.jx0 - L.x0m) / P->grid.n[0];
        const int64_t my = (int64_t)(A.iy0 + L.jy - L.row % P->grid.n[1]) / P->grid.n[1];
        return mx * 1024 + my;
      };
      if (bloch)
        std::stable_sort(P->lines.begin() + rb, P->lines.begin() + re,
                         [&](const LineRec &x, const LineRec &y) {
                           const int64_t ix = image(x), iy = image(y);
                           return ix != iy ? ix < iy : x.jx0 < y.jx0;
                         });
      else
        std::stable_sort(P->lines.begin() + rb, P->lines.begin() + re,
                         [](const LineRec &x, const LineRec &y) { return x.jx0 < y.jx0; });
      for (int32_t r = rb, rn = rb; r < re; r = rn) {
        rn = std::min(re, r + slots);
        if (bloch)
          for (int32_t k = r + 1; k < rn; ++k)
            if (image(P->lines[k]) != image(P->lines[r])) {
              rn = k;
              break;
            }
        BundleRec b;
        b.run0 = r;
        b.nruns = (int16_t)(rn - r);
        b.jz = P->lines[r].jz;
        int lo = INT32_MAX, hi = INT32_MIN;
        for (int32_t k = r; k < r + b.nruns; ++k) {
          lo = std::min(lo, (int)P->lines[k].jx0);
          hi = std::max(hi, (int)P->lines[k].jx0 + P->lines[k].len - 1);
        }
        b.jlo = (int16_t)lo;
        b.jhi = (int16_t)hi;
        b.pad = 0;
        P->bundles.push_back(b);
        // x steps, in whole batches of 8 loads, plus per-bundle overhead
        cost.push_back((hi - lo + 8) / 8 * 8 + 2);
      }
    }
  }
  atom_bundle_begin[P->natoms] = (int32_t)P->bundles.size();
  // atoms in Morton order of their centres
  std::vector<int32_t> order(P->natoms);
  std::vector<uint64_t> key(P->natoms);
  for (int32_t a = 0; a < P->natoms; ++a) {
    order[a] = a;
    key[a] = morton_key(P, a);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  // work items, grouped by nu
  std::vector<int32_t> first(P->natoms, 0), count(P->natoms, 0);
  std::vector<int64_t> item_cost;
  for (int32_t nu = 0; nu <= SHO_NU_MAX; ++nu) {
    for (int32_t a : order) {
      const AtomRec &A = P->atoms[a];
      if (A.nu != nu || A.npoints == 0) continue;
      const int32_t bb = atom_bundle_begin[a], be = atom_bundle_begin[a + 1];
      const int64_t parts =
          (P->flags & SHO_FLAG_DETERMINISTIC)  // one item per atom: no atomics into c
              ? 1
              : std::max<int64_t>(1, (A.npoints + target_points - 1) / target_points);
      std::vector<int64_t> cum(be - bb + 1, 0);
      for (int32_t i = bb; i < be; ++i) cum[i - bb + 1] = cum[i - bb] + cost[i];
      const int64_t total = cum.back();
      auto cut = [&](int64_t target) {
        return bb + (int32_t)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
      };
      first[a] = (int32_t)P->work.size();
      count[a] = (int32_t)parts;
      for (int64_t q = 0; q < parts; ++q) {
        WorkRec W;
        W.atom = a;
        W.split = parts > 1 ? 1 : 0;
        const int64_t c0 = total * q / parts, c1 = total * (q + 1) / parts;
        for (int w = 0; w <= kWaves; ++w)
          W.wb[w] = std::min(std::max(cut(c0 + (c1 - c0) * w / kWaves), bb), be);
        if (q == 0) W.wb[0] = bb;
        if (q == parts - 1) W.wb[kWaves] = be;
        P->work.push_back(W);
        // cost of the item: x steps of its waves times the functions per step
        item_cost.push_back((cum[W.wb[kWaves] - bb] - cum[W.wb[0] - bb]) * (nu + 2));
      }
      P->any_split |= parts > 1;
    }
  }
  P->atom_work.assign(P->natoms + 1, (int32_t)P->work.size());
  for (int32_t a = 0; a < P->natoms; ++a)
    P->atom_work[a] = count[a] ? first[a] : (int32_t)P->work.size();
  // the projection's launches
  const int32_t base = sched & ~kSchedXcd;
  std::vector<WorkRec> order_items;
  std::vector<ProjGroup> groups;
  if (base == kSchedByNu) {
    order_items = P->work;
    for (size_t i = 0; i < order_items.size();) {
      const int32_t nu = P->atoms[order_items[i].atom].nu;
      ProjGroup g{nu, (int32_t)i, 0};
      while (i < order_items.size() && P->atoms[order_items[i].atom].nu == nu) {
        ++g.count;
        ++i;
      }
      groups.push_back(g);
    }
  } else {
    for (int32_t a : order)
      for (int32_t i = 0; i < count[a]; ++i) order_items.push_back(P->work[first[a] + i]);
    if (base == kSchedSingleLpt) {
      std::vector<int32_t> idx(P->work.size());
      for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int32_t)i;
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int32_t x, int32_t y) { return item_cost[x] > item_cost[y]; });
      order_items.clear();
      for (int32_t i : idx) order_items.push_back(P->work[i]);
    }
    if (base == kSchedSweep) {
      // plane sweep: items by the memory plane of their first bundle, then
      // by the (x, y) Morton key of their atom, so that the workgroups
      // resident at one time cover a few consecutive planes of psi and the
      // overlapping supports of neighbouring atoms are read close in time
      const int32_t nz = P->grid.n[2];
      std::vector<std::pair<uint64_t, int32_t>> keyed(order_items.size());
      for (size_t i = 0; i < order_items.size(); ++i) {
        const WorkRec &W = order_items[i];
        const AtomRec &A = P->atoms[W.atom];
        int64_t z = (int64_t)A.iz0 + P->bundles[W.wb[0]].jz;
        if (P->grid.periodic[2]) z = ((z % nz) + nz) % nz;
        z = std::min<int64_t>(std::max<int64_t>(z, 0), nz - 1);
        keyed[i] = {((uint64_t)z << 40) | morton_xy(P, W.atom), (int32_t)i};
      }
      std::stable_sort(keyed.begin(), keyed.end(),
                       [](const std::pair<uint64_t, int32_t> &x,
                          const std::pair<uint64_t, int32_t> &y) { return x.first < y.first; });
      std::vector<WorkRec> sorted;
      sorted.reserve(order_items.size());
      for (const auto &k : keyed) sorted.push_back(order_items[k.second]);
      order_items.swap(sorted);
    }
    if (!order_items.empty()) groups.push_back(ProjGroup{-1, 0, (int32_t)order_items.size()});
  }
  if (!(sched & kSchedXcd)) {
    P->work_proj = order_items;
    P->proj_groups = groups;
    return;
  }
  WorkRec pad{};
  pad.atom = -1;
  for (const ProjGroup &g : groups) {
    const int32_t per = (g.count + kXcds - 1) / kXcds;
    ProjGroup ng{g.nu, (int32_t)P->work_proj.size(), per * kXcds};
    for (int32_t b = 0; b < per * kXcds; ++b) {
      const int32_t src = (b % kXcds) * per + b / kXcds;
      P->work_proj.push_back(src < g.count ? order_items[g.begin + src] : pad);
    }
    P->proj_groups.push_back(ng);
  }
}

void build_stored(HostPlan *P, int32_t chunk) {
  const int32_t nx = P->grid.n[0];
  P->run_poff.assign(P->lines.size() + 1, 0);
  P->atom_poff.assign(P->natoms + 1, 0);
  P->atom_pbeg.assign(P->natoms + 1, 0);
  P->pidx.clear();
  P->pidx.reserve(P->support_points);
  int64_t off = 0;
  for (int32_t a = 0; a < P->natoms; ++a) {
    const AtomRec &A = P->atoms[a];
    const int64_t ns = stored_cols(*P, A);
    P->atom_poff[a] = off;
    P->atom_pbeg[a] = (int64_t)P->pidx.size();
    for (int32_t r = A.line_begin; r < A.line_begin + A.nlines; ++r) {
      const LineRec &L = P->lines[r];
      P->run_poff[r] = off;
      off += (int64_t)L.len * ns;
      for (int32_t k = 0; k < L.len; ++k)
        P->pidx.push_back(L.row * nx + L.x0m + k);
    }
  }
  P->atom_poff[P->natoms] = off;
  P->atom_pbeg[P->natoms] = (int64_t)P->pidx.size();
  P->run_poff[P->lines.size()] = off;
  P->stored_doubles = off;
  // work items: chunks of each atom's points, atoms ordered by nu
  std::vector<int32_t> order(P->natoms);
  for (int32_t a = 0; a < P->natoms; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return P->atoms[x].nu < P->atoms[y].nu;
  });
  P->sitems.clear();
  for (int32_t a : order) {
    const int32_t np = (int32_t)(P->atom_pbeg[a + 1] - P->atom_pbeg[a]);
    for (int32_t k = 0; k < np; k += chunk)
      P->sitems.push_back(StoredItem{a, k, std::min(np, k + chunk), 0});
  }
}

void build_rows(HostPlan *P) {
  const int64_t nrows_grid = (int64_t)P->grid.n[2] * P->grid.n[1];
  P->run_atom.assign(P->lines.size(), -1);
  for (int32_t a = 0; a < P->natoms; ++a) {
    const AtomRec &A = P->atoms[a];
    for (int32_t r = A.line_begin; r < A.line_begin + A.nlines; ++r) P->run_atom[r] = a;
  }
  // counting sort of runs by memory row (stable: atom order, then run order)
  std::vector<int32_t> count(nrows_grid + 1, 0);
  for (const LineRec &L : P->lines) count[L.row + 1]++;
  for (int64_t r = 0; r < nrows_grid; ++r) count[r + 1] += count[r];
  P->row_runs.assign(P->lines.size(), 0);
  std::vector<int32_t> fill(count.begin(), count.end() - 1);
  for (int32_t i = 0; i < (int32_t)P->lines.size(); ++i)
    P->row_runs[fill[P->lines[i].row]++] = i;
  // distinct covered points: union of the runs' x ranges per row
  P->union_points = 0;
  P->rows_touched = 0;
  std::vector<uint8_t> mark(P->grid.n[0]);
  for (int64_t r = 0; r < nrows_grid; ++r) {
    if (count[r + 1] == count[r]) continue;
    P->rows_touched++;
    std::fill(mark.begin(), mark.end(), 0);
    for (int32_t k = count[r]; k < count[r + 1]; ++k) {
      const LineRec &L = P->lines[P->row_runs[k]];
      for (int x = L.x0m; x < L.x0m + L.len; ++x) mark[x] = 1;
    }
    for (uint8_t m : mark) P->union_points += m;
  }
  // non-empty rows, one list per plane class z mod 8, interleaved in groups
  // of kRowsPerGroup so that workgroup g (dispatched to XCD g mod 8) works on
  // planes of one class
  std::vector<std::vector<RowRec>> cls(8);
  for (int64_t r = 0; r < nrows_grid; ++r) {
    const int32_t n = count[r + 1] - count[r];
    if (!n) continue;
    const int32_t z = (int32_t)(r / P->grid.n[1]);
    cls[z % 8].push_back(RowRec{(int32_t)r, count[r], n, 0});
  }
  P->rows.clear();
  std::vector<size_t> at(8, 0);
  for (bool any = true; any;) {
    any = false;
    for (int k = 0; k < 8; ++k) {
      for (int j = 0; j < kRowsPerGroup; ++j) {
        if (at[k] < cls[k].size()) {
          P->rows.push_back(cls[k][at[k]++]);
          any = true;
        } else {
          // pad the group so the next group starts on the next XCD
          P->rows.push_back(RowRec{-1, 0, 0, 0});
        }
      }
    }
  }
  // drop trailing groups made only of padding
  while (!P->rows.empty() && P->rows.size() >= (size_t)kRowsPerGroup) {
    bool empty = true;
    for (size_t j = P->rows.size() - kRowsPerGroup; j < P->rows.size(); ++j)
      empty &= P->rows[j].row < 0;
    if (!empty) break;
    P->rows.resize(P->rows.size() - kRowsPerGroup);
  }
  // plane partials: per atom mz planes x pairs x bands
  P->u2_off.assign(P->natoms, 0);
  P->u2_doubles = 0;
  for (int32_t a = 0; a < P->natoms; ++a) {
    const AtomRec &A = P->atoms[a];
    const int64_t np = (int64_t)(A.nu + 1) * (A.nu + 2) / 2;
    P->u2_off[a] = P->u2_doubles;
    P->u2_doubles += (int64_t)A.mz * np * P->nbands;
  }
  P->nu_atoms.clear();
  for (int32_t nu = 0; nu <= SHO_NU_MAX; ++nu)
    for (int32_t a = 0; a < P->natoms; ++a)
      if (P->atoms[a].nu == nu && P->atoms[a].npoints > 0) P->nu_atoms.push_back(a);
}

void build_block_set(const HostPlan *P, int32_t R, int32_t X, BlockSet *out) {
  const int32_t nx = P->grid.n[0], ny = P->grid.n[1];
  const int64_t nyb = (ny + R - 1) / R, nxb = (nx + X - 1) / X;
  out->rows = R;
  out->x = X;
  struct Item {
    int64_t block;
    int32_t atom, jz, jshift, yshift, row, run;
  };
  std::vector<Item> items;
  items.reserve(P->lines.size() * 3 / 2);
  for (int32_t r = 0; r < (int32_t)P->lines.size(); ++r) {
    const LineRec &L = P->lines[r];
    const int32_t z = L.row / ny, y = L.row % ny;
    for (int32_t cx = L.x0m / X; cx <= (L.x0m + L.len - 1) / X; ++cx)
      items.push_back(Item{((int64_t)z * nyb + y / R) * nxb + cx, P->run_atom[r], L.jz,
                           L.jx0 - L.x0m, L.jy - y, L.row, r});
  }
  std::sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
    if (a.block != b.block) return a.block < b.block;
    if (a.atom != b.atom) return a.atom < b.atom;
    if (a.jz != b.jz) return a.jz < b.jz;
    if (a.jshift != b.jshift) return a.jshift < b.jshift;
    if (a.yshift != b.yshift) return a.yshift < b.yshift;
    if (a.row != b.row) return a.row < b.row;
    return a.run < b.run;
  });
  out->entries.clear();
  out->run_desc.clear();
  out->run_desc_run.clear();
  std::vector<std::vector<BlockRec>> cls(8);
  for (size_t i = 0; i < items.size();) {
    const int64_t blk = items[i].block;
    BlockRec B;
    const int64_t cx = blk % nxb, yz = blk / nxb;
    B.z = (int32_t)(yz / nyb);
    B.y0 = (int32_t)(yz % nyb) * R;
    B.x0 = (int32_t)cx * X;
    B.entry_begin = (int32_t)out->entries.size();
    B.nentries = 0;
    B.pad = 0;
    while (i < items.size() && items[i].block == blk) {
      const Item &it = items[i];
      const AtomRec &A = P->atoms[it.atom];
      const int64_t np = (int64_t)(A.nu + 1) * (A.nu + 2) / 2;
      EntryRec E;
      E.u2 = P->u2_off[it.atom] + (int64_t)it.jz * np * P->nbands;
      const int32_t jx0 = B.x0 + it.jshift;   // table x index of memory x0
      const int32_t jy0 = B.y0 + it.yshift;   // table y index of block row 0
      E.tab_x = (int32_t)(A.tab_off + (int64_t)jx0 * A.tab_nfp);
      E.tab_y = (int32_t)(A.tab_off + (int64_t)(A.mx + jy0) * A.tab_nfp);
      E.nu = (int16_t)A.nu;
      E.nfp = (int16_t)A.tab_nfp;
      E.x_lo = (int16_t)std::max(0, -jx0);
      E.x_hi = (int16_t)std::min(X, A.mx - jx0);
      E.y_lo = (int16_t)std::max(0, -jy0);
      E.y_hi = (int16_t)std::min(R, A.my - jy0);
      E.run_begin = (int32_t)out->run_desc.size();
      E.nruns = 0;
      // image counts (clamped; Bloch plans refuse supports beyond 127 images)
      {
        const int32_t nz = P->grid.n[2];
        const int64_t dxyz[3] = {(int64_t)A.ix0 + it.jshift, (int64_t)A.iy0 + it.yshift,
                                 (int64_t)A.iz0 + it.jz - B.z};
        const int32_t nd[3] = {nx, ny, nz};
        for (int d = 0; d < 3; ++d) {
          const int64_t m = dxyz[d] / nd[d];
          E.img[d] = (int8_t)std::min<int64_t>(std::max<int64_t>(m, -127), 127);
        }
        E.pad = 0;
      }
      // at most 64 runs per entry (one descriptor per lane)
      while (i < items.size() && E.nruns < 64 && items[i].block == blk &&
             items[i].atom == it.atom && items[i].jz == it.jz &&
             items[i].jshift == it.jshift && items[i].yshift == it.yshift) {
        const LineRec &L = P->lines[items[i].run];
        const int32_t xa = std::max((int32_t)L.x0m, B.x0) - B.x0;
        const int32_t xb = std::min((int32_t)L.x0m + L.len, B.x0 + X) - B.x0;
        out->run_desc.push_back(pack_run(L.row % ny - B.y0, xa, xb));
        out->run_desc_run.push_back(items[i].run);
        E.nruns++;
        ++i;
      }
      out->entries.push_back(E);
      B.nentries++;
    }
    // the block's waves take its entries round robin: costliest first, so
    // that the waves finish closer together (cost: plane partial loads, y
    // passes per run, x steps per point)
    {
      auto cost = [&](const EntryRec &E) {
        const int64_t nf = E.nu + 1, np = nf * (nf + 1) / 2;
        int64_t pts = 0;
        for (int32_t k = E.run_begin; k < E.run_begin + E.nruns; ++k) {
          const uint32_t d = out->run_desc[k];
          pts += (int64_t)((d >> 16) & 0xff) - (int64_t)((d >> 8) & 0xff);
        }
        return np * (1 + E.nruns) + nf * pts;
      };
      std::stable_sort(out->entries.begin() + B.entry_begin, out->entries.end(),
                       [&](const EntryRec &a, const EntryRec &b) { return cost(a) > cost(b); });
      // then dealt to the 4 waves in snake order (round k goes 0..3 when k
      // is even, 3..0 when odd), so that wave w's k-th entry sits at list
      // position 4k + w
      constexpr int32_t kWavesB = 4;  // waves of a block workgroup
      const int32_t n = B.nentries;
      std::vector<EntryRec> dealt(n);
      for (int32_t i = 0; i < n; ++i) {
        const int32_t k = i / kWavesB, r = i % kWavesB;
        const int32_t w = (k % 2 == 0) ? r : kWavesB - 1 - r;
        const int32_t pos = k * kWavesB + w;
        dealt[pos < n ? pos : i] = out->entries[B.entry_begin + i];
      }
      std::copy(dealt.begin(), dealt.end(), out->entries.begin() + B.entry_begin);
    }
    cls[B.z % 8].push_back(B);
  }
  // blocks of planes z = k mod 8 go to workgroups g = k mod 8 (XCD k)
  out->blocks.clear();
  std::vector<size_t> at(8, 0);
  const BlockRec pad{0, 0, 0, 0, -1, 0};
  for (bool any = true; any;) {
    any = false;
    for (int k = 0; k < 8; ++k) {
      if (at[k] < cls[k].size()) {
        out->blocks.push_back(cls[k][at[k]++]);
        any = true;
      } else {
        out->blocks.push_back(pad);
      }
    }
  }
  while (!out->blocks.empty() && out->blocks.back().nentries < 0) out->blocks.pop_back();
  out->points = 0;
  for (const BlockRec &B : out->blocks)
    if (B.nentries >= 0)
      out->points += (int64_t)(std::min(B.y0 + R, ny) - B.y0) * (std::min(B.x0 + X, nx) - B.x0);
}

void build_blocks(HostPlan *P, int32_t R, int32_t X) {
  BlockSet bs;
  build_block_set(P, R, X, &bs);
  P->blk_rows = bs.rows;
  P->blk_x = bs.x;
  P->block_points = bs.points;
  P->blocks.swap(bs.blocks);
  P->entries.swap(bs.entries);
  P->run_desc.swap(bs.run_desc);
  P->run_desc_run.swap(bs.run_desc_run);
}

void build_desc_pbase(HostPlan *P) {
  P->desc_pbase.assign(P->run_desc.size(), 0);
  for (const BlockRec &B : P->blocks) {
    if (B.nentries < 0) continue;
    for (int32_t e = B.entry_begin; e < B.entry_begin + B.nentries; ++e) {
      EntryRec &E = P->entries[e];
      const AtomRec &A = P->atoms[P->run_atom[P->run_desc_run[E.run_begin]]];
      const int64_t ns = stored_cols(*P, A);
      E.u2 = A.coeff_row;
      for (int32_t k = E.run_begin; k < E.run_begin + E.nruns; ++k) {
        const LineRec &L = P->lines[P->run_desc_run[k]];
        P->desc_pbase[k] = P->run_poff[P->run_desc_run[k]] + (int64_t)(B.x0 - L.x0m) * ns;
      }
    }
  }
}

}  // namespace sho
