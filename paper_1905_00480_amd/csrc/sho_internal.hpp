// sho_internal.hpp -- data layout shared by the host plan builder, the C ABI
// layer and the gfx950 kernels of libsho.so.
//
// A plan cuts every atom's support sphere into z planes and each plane into
// (z, y) lines; each line is one contiguous run of x points, i.e. one
// contiguous run of x*nbands doubles of psi in memory.  Kernels stream the
// lines from HBM, contract x, y and z in turn (the factorised Cartesian basis
// of sec. 2.2) and never materialise a 3D projector.
#pragma once

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
  int32_t line_begin;    // first line record of this atom
  int32_t nlines;
  int32_t pad0;
  int64_t coeff_row;     // sum of N_SHO(nu) over earlier atoms
  int64_t npoints;       // |S_a|
  int64_t point_begin;   // first support point (line order) of this atom
};
static_assert(sizeof(AtomRec) == 104, "AtomRec layout");

// One z plane of one atom's support.
struct PlaneRec {
  int32_t jz;          // table index along z
  int32_t line_begin;  // absolute index of the plane's first line
  int32_t nlines;
  int32_t npoints;
};

// One (z, y) line: points x0 .. x0+len-1 (unwrapped) of memory row `row`.
struct LineRec {
  int32_t row;   // (z mod nz) * ny + (y mod ny)
  int32_t x0m;   // x0 mod nx: memory x of the first point
  int16_t jx0;   // table index of the first point along x
  int16_t jy;    // table index along y
  int32_t len;   // number of points
};
static_assert(sizeof(LineRec) == 16, "LineRec layout");

// Host-side plan contents (built without any device call).
struct HostPlan {
  sho_grid grid{};
  int32_t natoms = 0;
  int32_t nbands = 0;
  uint32_t flags = 0;
  int32_t nu_max = 0;
  int32_t m_max = 0;  // largest table extent over atoms and axes
  std::vector<AtomRec> atoms;
  std::vector<PlaneRec> planes;
  std::vector<LineRec> lines;
  std::vector<double> support_centre;  // [natoms][3], fixed at creation
  std::vector<int64_t> coeff_off;      // [natoms+1] in doubles
  int64_t coeff_rows = 0;
  int64_t support_points = 0;
};

inline int32_t nsho(int32_t nu) {
  return nu < 0 ? 0 : (nu + 1) * (nu + 2) * (nu + 3) / 6;
}

// Builds the host plan; returns SHO_OK or an error code with *msg set.
sho_status build_host_plan(const sho_grid *grid, int32_t natoms,
                           const double *pos, const double *sigma,
                           const int32_t *numax, const double *rbox,
                           int32_t nbands, uint32_t flags, HostPlan *out,
                           std::string *msg);

// Largest table extent the kernels accept per axis.
constexpr int32_t kMaxTable = 512;

}  // namespace sho
