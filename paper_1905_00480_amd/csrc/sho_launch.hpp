// sho_launch.hpp -- kernel argument block and launchers of libsho.so.
#pragma once

#include <hip/hip_runtime_api.h>

#include "sho_internal.hpp"

namespace sho {

// Argument block of the projection / expansion / derivative kernels.
struct KArgs {
  const AtomRec *atoms;
  const LineRec *lines;
  const BundleRec *bundles;
  const WorkRec *work;       // work items of this launch (one nu)
  const double *tab;         // 1D tables of all atoms
  int32_t nwork;
  int32_t nx;                // grid points along x
  int32_t B;                 // bands: stride of one grid point
  int32_t tb_shift;          // log2(bands per lane slot)
  int32_t ntiles;            // band tiles per atom
  int32_t pad;
  double h3;
};

// Samples the 1D tables of every atom (rows padded with zeros).
hipError_t launch_tables(const AtomRec *atoms, int32_t natoms, double h,
                         double *tab, int32_t mmax, hipStream_t s);
hipError_t launch_project(int nu, const KArgs &K, const double *psi, double *c,
                          hipStream_t s);
hipError_t launch_expand(int nu, const KArgs &K, const double *c, double *psi,
                         hipStream_t s);
// grad must be zeroed first (launch_fill)
hipError_t launch_force(int nu, const KArgs &K, const double *psi,
                        const double *w, double *grad, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace sho
