// sho_launch.hpp -- kernel argument block and launchers of libsho.so.
#pragma once

#include <hip/hip_runtime_api.h>

#include "sho_internal.hpp"

namespace sho {

// Argument block of the projection / expansion / derivative kernels.
struct KArgs {
  const AtomRec *atoms;
  const PlaneRec *planes;
  const LineRec *lines;
  const int32_t *atom_list;  // atoms handled by this launch (one nu)
  int32_t nlist;
  int32_t nx;                // grid points along x (wrap of a line)
  int32_t B;                 // bands: stride of one grid point
  int32_t tb_shift;          // log2(bands per line slot)
  int32_t ntiles;            // band tiles per atom
  int32_t mstride;           // table rows per axis in LDS
  double h, h3;
};

// LDS bytes of a workgroup: three tables [mstride][nf] and a [N_SHO(nf-1)][tb]
// coefficient tile.
size_t lds_bytes(int nf, int mstride, int tb);

hipError_t launch_project(int nu, const KArgs &K, const double *psi, double *c,
                          hipStream_t s);
hipError_t launch_expand(int nu, const KArgs &K, const double *c, double *psi,
                         hipStream_t s);
// grad must be zeroed first (launch_fill)
hipError_t launch_force(int nu, const KArgs &K, const double *psi,
                        const double *w, double *grad, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace sho
