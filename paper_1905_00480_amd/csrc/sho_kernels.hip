// sho_kernels.hip -- gfx950 kernels for SHO projection, expansion and the
// position derivative (Baumeister & Tsukamoto, PASC'19).
//
// Work decomposition (one launch per distinct nu in a plan):
//   * one workgroup (8 wave64) per (atom, band tile);
//   * the tile's bands are the lanes: lane = (line slot, band), TB bands per
//     slot, 64/TB line slots per wave (band index is fastest in memory, so a
//     slot's loads of one grid point are one coalesced TB*8-byte run);
//   * waves take the atom's z planes round robin; inside a plane the slots take
//     lines round robin.
//
// Projection (sec. 3.2 step 1 in the factorised basis of sec. 2.2):
//   x pass  T1[nx]     = sum_x phi_nx(x) psi(x,y,z)       registers, streams HBM
//   y pass  T2[nx][ny] = sum_y phi_ny(y) T1[nx]           registers
//   z pass  C[nx,ny,nz]+= phi_nz(z) T2[nx][ny]            LDS tile, ds_add_f64
// Expansion (step 3) runs the same passes backwards and adds into psi with
// global_atomic_add_f64 (supports of different atoms overlap).
// The 1D functions are sampled per workgroup into LDS by the normalised
// three-term recurrence (the monic recurrence of sec. 3.7 rescaled so that
// every phi_n has unit L2 norm), once per atom and axis.
#include <hip/hip_runtime.h>

#include "sho_launch.hpp"

namespace sho {



constexpr int kBlock = 512;

// ---------------------------------------------------------------- tables --

// tab[(axis*mstride + j)*NF + n] = phi_n(u) at u = (i0_axis + j)*h - centre.
// phi_0 = pi^{-1/4} sigma^{-1/2} e^{-t^2/2}, phi_1 = sqrt(2) t phi_0,
// phi_{n+1} = sqrt(2/(n+1)) t phi_n - sqrt(n/(n+1)) phi_{n-1},  t = u/sigma.
template <int NF>
__device__ inline void fill_tables(const AtomRec &A, const KArgs &K,
                                   double *tab) {
  const double inv_s = 1.0 / A.sigma;
  const double p0 = 0.7511255444649425 * sqrt(inv_s);
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int i0 = axis == 0 ? A.ix0 : (axis == 1 ? A.iy0 : A.iz0);
    const double c = axis == 0 ? A.cx : (axis == 1 ? A.cy : A.cz);
    for (int j = threadIdx.x; j < K.mstride; j += blockDim.x) {
      const double u = (double)(i0 + j) * K.h - c;
      const double x = u * inv_s;
      double *row = tab + ((size_t)axis * K.mstride + j) * NF;
      double fm = 0.0;
      double f = p0 * exp(-0.5 * x * x);
      row[0] = f;
#pragma unroll
      for (int n = 0; n + 1 < NF; ++n) {
        const double fn = sqrt(2.0 / (n + 1)) * x * f - sqrt((double)n / (n + 1)) * fm;
        fm = f;
        f = fn;
        row[n + 1] = f;
      }
    }
  }
}

// ------------------------------------------------------- projection core --

// Accumulates sum_{i in S_a} P_an(i) psi(i) (no h^3) for the workgroup's
// band tile into cacc[n*TB + bl] (LDS, zeroed by the caller).
template <int NU>
__device__ inline void project_core(const KArgs &K, const AtomRec &A,
                                    int tile, const double *__restrict__ psi,
                                    const double *tab, double *cacc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  const int TB = 1 << K.tb_shift;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int slot = lane >> K.tb_shift;
  const int lpw = 64 >> K.tb_shift;
  const int bl = lane & (TB - 1);
  const int b = tile * TB + bl;
  const bool bok = b < K.B;
  const double *phx = tab;
  const double *phy = tab + (size_t)K.mstride * NF;
  const double *phz = tab + (size_t)2 * K.mstride * NF;
  const int64_t rowlen = (int64_t)K.nx * K.B;

  for (int p = wave; p < A.nplanes; p += nwaves) {
    const PlaneRec pl = K.planes[A.plane_begin + p];
    double T2[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) T2[q] = 0.0;
    for (int l = slot; l < pl.nlines; l += lpw) {
      const LineRec ln = K.lines[pl.line_begin + l];
      double T1[NF];
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = 0.0;
      const double *src = psi + (int64_t)ln.row * rowlen + b;
      const double *fx = phx + (int)ln.jx0 * NF;
      int xm = ln.x0m;
#pragma unroll 4
      for (int k = 0; k < ln.len; ++k) {
        const double v = bok ? src[(int64_t)xm * K.B] : 0.0;
#pragma unroll
        for (int n = 0; n < NF; ++n) T1[n] = fma(fx[k * NF + n], v, T1[n]);
        xm = (xm + 1 == K.nx) ? 0 : xm + 1;
      }
      const double *fy = phy + (int)ln.jy * NF;
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const double f = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) T2[q] = fma(f, T1[nx], T2[q]);
      }
    }
    // fold the line slots of this wave (same band, different lines)
    for (int s = 32; s >= TB; s >>= 1) {
#pragma unroll
      for (int q = 0; q < NP; ++q) T2[q] += __shfl_xor(T2[q], s);
    }
    if (slot == 0 && bok) {
      const double *fz = phz + pl.jz * NF;
      int idx = 0;
#pragma unroll
      for (int nz = 0; nz < NF; ++nz) {
        const double f = fz[nz];
        int q = 0;
#pragma unroll
        for (int ny = 0; ny < NF; ++ny) {
#pragma unroll
          for (int nx = 0; nx < NF - ny; ++nx, ++q) {
            if (nx + ny + nz <= NU) {
              atomicAdd(&cacc[idx * TB + bl], f * T2[q]);
              ++idx;
            }
          }
        }
      }
    }
  }
}

template <int NU>
__global__ __launch_bounds__(kBlock) void k_project(
    KArgs K, const double *__restrict__ psi, double *__restrict__ c) {
  constexpr int NF = NU + 1;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  extern __shared__ double lds[];
  const int ia = blockIdx.x / K.ntiles;
  const int tile = blockIdx.x - ia * K.ntiles;
  const AtomRec A = K.atoms[K.atom_list[ia]];
  const int TB = 1 << K.tb_shift;
  double *tab = lds;
  double *cacc = lds + (size_t)3 * K.mstride * NF;
  fill_tables<NF>(A, K, tab);
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) cacc[t] = 0.0;
  __syncthreads();
  project_core<NU>(K, A, tile, psi, tab, cacc);
  __syncthreads();
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bb = tile * TB + (t & (TB - 1));
    if (bb < K.B) c[(A.coeff_row + n) * K.B + bb] = K.h3 * cacc[t];
  }
}

// -------------------------------------------------------------- expansion --

template <int NU>
__global__ __launch_bounds__(kBlock) void k_expand(
    KArgs K, const double *__restrict__ c, double *psi) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  extern __shared__ double lds[];
  const int ia = blockIdx.x / K.ntiles;
  const int tile = blockIdx.x - ia * K.ntiles;
  const AtomRec A = K.atoms[K.atom_list[ia]];
  const int TB = 1 << K.tb_shift;
  double *tab = lds;
  double *cin = lds + (size_t)3 * K.mstride * NF;
  fill_tables<NF>(A, K, tab);
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bb = tile * TB + (t & (TB - 1));
    cin[t] = bb < K.B ? c[(A.coeff_row + n) * K.B + bb] : 0.0;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int slot = lane >> K.tb_shift;
  const int lpw = 64 >> K.tb_shift;
  const int bl = lane & (TB - 1);
  const int b = tile * TB + bl;
  const bool bok = b < K.B;
  const double *phx = tab;
  const double *phy = tab + (size_t)K.mstride * NF;
  const double *phz = tab + (size_t)2 * K.mstride * NF;
  const int64_t rowlen = (int64_t)K.nx * K.B;

  for (int p = wave; p < A.nplanes; p += nwaves) {
    const PlaneRec pl = K.planes[A.plane_begin + p];
    // z pass: U2[nx][ny] = sum_nz phi_nz(z) C[nx,ny,nz]
    double U2[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) U2[q] = 0.0;
    {
      const double *fz = phz + pl.jz * NF;
      int idx = 0;
#pragma unroll
      for (int nz = 0; nz < NF; ++nz) {
        const double f = fz[nz];
        int q = 0;
#pragma unroll
        for (int ny = 0; ny < NF; ++ny) {
#pragma unroll
          for (int nx = 0; nx < NF - ny; ++nx, ++q) {
            if (nx + ny + nz <= NU) {
              U2[q] = fma(f, cin[idx * TB + bl], U2[q]);
              ++idx;
            }
          }
        }
      }
    }
    for (int l = slot; l < pl.nlines; l += lpw) {
      const LineRec ln = K.lines[pl.line_begin + l];
      // y pass: U1[nx] = sum_ny phi_ny(y) U2[nx][ny]
      double U1[NF];
#pragma unroll
      for (int n = 0; n < NF; ++n) U1[n] = 0.0;
      const double *fy = phy + (int)ln.jy * NF;
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const double f = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[nx] = fma(f, U2[q], U1[nx]);
      }
      // x pass: psi(x) += sum_nx phi_nx(x) U1[nx]
      double *dst = psi + (int64_t)ln.row * rowlen + b;
      const double *fx = phx + (int)ln.jx0 * NF;
      int xm = ln.x0m;
#pragma unroll 4
      for (int k = 0; k < ln.len; ++k) {
        double v = 0.0;
#pragma unroll
        for (int n = 0; n < NF; ++n) v = fma(fx[k * NF + n], U1[n], v);
        if (bok) unsafeAtomicAdd(dst + (int64_t)xm * K.B, v);
        xm = (xm + 1 == K.nx) ? 0 : xm + 1;
      }
    }
  }
}

// ------------------------------------------------------------- derivative --

// Index of (nx, ny, nz) in the nz-major / ny / nx-fastest order at cut-off nu.
__device__ inline int coeff_index(int nx, int ny, int nz, int nu) {
  auto N3 = [](int m) { return m < 0 ? 0 : (m + 1) * (m + 2) * (m + 3) / 6; };
  auto N2 = [](int m) { return m < 0 ? 0 : (m + 1) * (m + 2) / 2; };
  return N3(nu) - N3(nu - nz) + N2(nu - nz) - N2(nu - nz - ny) + nx;
}

__device__ inline void coeff_decode(int n, int nu, int &nx, int &ny, int &nz) {
  nz = 0;
  for (;;) {
    const int cnt = (nu - nz + 1) * (nu - nz + 2) / 2;
    if (n < cnt) break;
    n -= cnt;
    ++nz;
  }
  ny = 0;
  for (;;) {
    const int cnt = nu - nz - ny + 1;
    if (n < cnt) break;
    n -= cnt;
    ++ny;
  }
  nx = n;
}

// Projection at nu+1 = NU1 on the atom's (nu) support, then the ladder
//   dC[n]/dX = -(1/sigma) [ sqrt(nx/2) C~(nx-1) - sqrt((nx+1)/2) C~(nx+1) ]
// (phi_n' = (1/sigma)[sqrt(n/2) phi_{n-1} - sqrt((n+1)/2) phi_{n+1}]) and the
// contraction grad[a][d] += sum_{n,b} w[n][b] dC[n][b]/dR_d.
// grad must be zero before the launch (band tiles add into it).
template <int NU1>
__global__ __launch_bounds__(kBlock) void k_force(
    KArgs K, const double *__restrict__ psi, const double *__restrict__ w,
    double *grad) {
  constexpr int NF = NU1 + 1;
  constexpr int NS1 = NF * (NF + 1) * (NF + 2) / 6;
  constexpr int NU = NU1 - 1;
  constexpr int NS = (NU + 1) * (NU + 2) * (NU + 3) / 6;
  extern __shared__ double lds[];
  __shared__ double red[3][kBlock / 64];
  const int ia = blockIdx.x / K.ntiles;
  const int tile = blockIdx.x - ia * K.ntiles;
  const int a = K.atom_list[ia];
  const AtomRec A = K.atoms[a];
  const int TB = 1 << K.tb_shift;
  double *tab = lds;
  double *cacc = lds + (size_t)3 * K.mstride * NF;
  fill_tables<NF>(A, K, tab);
  for (int t = threadIdx.x; t < NS1 * TB; t += blockDim.x) cacc[t] = 0.0;
  __syncthreads();
  project_core<NU1>(K, A, tile, psi, tab, cacc);
  __syncthreads();

  double g[3] = {0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bl = t & (TB - 1);
    const int bb = tile * TB + bl;
    if (bb >= K.B) continue;
    int m[3];
    coeff_decode(n, NU, m[0], m[1], m[2]);
    const double wv = w[(A.coeff_row + n) * K.B + bb];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int up[3] = {m[0], m[1], m[2]};
      up[d] += 1;
      double v = -sqrt(0.5 * (m[d] + 1)) *
                 cacc[coeff_index(up[0], up[1], up[2], NU1) * TB + bl];
      if (m[d] > 0) {
        int dn[3] = {m[0], m[1], m[2]};
        dn[d] -= 1;
        v += sqrt(0.5 * m[d]) * cacc[coeff_index(dn[0], dn[1], dn[2], NU1) * TB + bl];
      }
      g[d] = fma(wv, v, g[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v = g[d];
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
    if ((threadIdx.x & 63) == 0) red[d][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[threadIdx.x][k];
    atomicAdd(&grad[3 * a + threadIdx.x], -K.h3 / A.sigma * s);
  }
}

__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- launch --

size_t lds_bytes(int nf, int mstride, int tb) {
  const size_t ns = (size_t)nf * (nf + 1) * (nf + 2) / 6;
  return ((size_t)3 * mstride * nf + ns * tb) * sizeof(double);
}

template <int NU>
static hipError_t launch_project_nu(const KArgs &K, const double *psi,
                                    double *c, hipStream_t s) {
  const size_t shm = lds_bytes(NU + 1, K.mstride, 1 << K.tb_shift);
  hipLaunchKernelGGL(k_project<NU>, dim3(K.nlist * K.ntiles), dim3(kBlock), shm,
                     s, K, psi, c);
  return hipGetLastError();
}

template <int NU>
static hipError_t launch_expand_nu(const KArgs &K, const double *c,
                                   double *psi, hipStream_t s) {
  const size_t shm = lds_bytes(NU + 1, K.mstride, 1 << K.tb_shift);
  hipLaunchKernelGGL(k_expand<NU>, dim3(K.nlist * K.ntiles), dim3(kBlock), shm,
                     s, K, c, psi);
  return hipGetLastError();
}

template <int NU1>
static hipError_t launch_force_nu(const KArgs &K, const double *psi,
                                  const double *w, double *grad,
                                  hipStream_t s) {
  const size_t shm = lds_bytes(NU1 + 1, K.mstride, 1 << K.tb_shift);
  hipLaunchKernelGGL(k_force<NU1>, dim3(K.nlist * K.ntiles), dim3(kBlock), shm,
                     s, K, psi, w, grad);
  return hipGetLastError();
}

#define SHO_NU_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

hipError_t launch_project(int nu, const KArgs &K, const double *psi, double *c,
                          hipStream_t s) {
  switch (nu) {
#define X(N) case N: return launch_project_nu<N>(K, psi, c, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand(int nu, const KArgs &K, const double *c, double *psi,
                         hipStream_t s) {
  switch (nu) {
#define X(N) case N: return launch_expand_nu<N>(K, c, psi, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_force(int nu, const KArgs &K, const double *psi,
                        const double *w, double *grad, hipStream_t s) {
  switch (nu) {
#define X(N) case N: return launch_force_nu<N + 1>(K, psi, w, grad, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace sho
