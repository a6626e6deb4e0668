// sho_kernels.hip -- gfx950 kernels for SHO projection, expansion and the
// position derivative (Baumeister & Tsukamoto, PASC'19).
//
// Work decomposition
//   * grid = (work items, band tiles); a work item is one atom, or a share of
//     a large atom, cut into kWaves cost-balanced ranges of run bundles;
//   * one workgroup = kWaves wave64; wave w streams its own bundles;
//   * lane = (slot, band): TB bands per slot, 64/TB slots per wave, slot s
//     takes run s of the bundle.  All runs of a bundle lie in one atom plane
//     and the wave steps the table index jx over the union of their x ranges,
//     so phi_x(jx) is wave-uniform and is read through the scalar cache.  A
//     run is one contiguous block of psi (band index fastest): each load
//     instruction reads TB*8 contiguous bytes per slot.
//
// Projection (sec. 3.2 step 1, in the factorised basis of sec. 2.2):
//   x pass  T1[nx]      = sum_x phi_nx(x) psi(x,y,z)   registers, streams HBM
//   y pass  T2[nx][ny] += phi_ny(y) T1[nx]            registers
//   z pass  C[nx,ny,nz] += phi_nz(z) T2[nx][ny]       at each plane change:
//                                                     slots folded, LDS tile
// Expansion (step 3) runs the passes backwards: the z pass per atom plane
// (plane partials U2), then one workgroup per memory row adds the y and x
// passes of every run that falls into the row, so that each value of psi is
// read and written once with plain loads and stores, in a fixed order.
// The 1D functions are sampled once per plan into small per-atom tables by
// the normalised three-term recurrence (the monic recurrence of sec. 3.7
// rescaled so that every phi_n has unit L2 norm).
#include <hip/hip_runtime.h>

#include <mutex>

#include "sho_device.hpp"
#include "sho_launch.hpp"

namespace sho {

constexpr int kBlock = 64 * kWaves;

#define SHO_NU_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
constexpr int kBatch = 8;  // loads in flight per lane and batch
constexpr int kLineStage = 64;  // line records per wave held in LDS
static_assert(kWaves * kLineStage * sizeof(LineRec) + 1024 <= kStaticLds,
              "static LDS of the streaming kernels");

// waves per SIMD the register allocator must allow (4 keeps <= 128 VGPRs).
// Deterministic plans keep eight coefficient tiles in LDS (one per wave), so
// few of their workgroups fit on a CU (one at nu = 5 and 32-band tiles); they
// may use the registers of two waves per SIMD instead of spilling to fit four.
constexpr int waves_per_eu(int nf, bool det = false) { return nf <= 6 && !det ? 4 : 2; }

// dst[t] = value(t) for t < count, with U global loads in flight per thread
// (all loads of a round are issued before the first LDS write waits).
template <int U, typename F>
__device__ inline void fill_lds(double *dst, int count, F &&value) {
  for (int t0 = 0; t0 < count; t0 += U * (int)blockDim.x) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x + (int)threadIdx.x;
      v[u] = t < count ? value(t) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x + (int)threadIdx.x;
      if (t < count) dst[t] = v[u];
    }
  }
}

// ---------------------------------------------------------------- tables --

// Row j of axis d of atom a: phi_n(u), u = (i0_d + j)*h - centre_d, for
// n < nu+2, then zeros up to the row stride.
// phi_0 = pi^{-1/4} sigma^{-1/2} e^{-t^2/2}, phi_1 = sqrt(2) t phi_0,
// phi_{n+1} = sqrt(2/(n+1)) t phi_n - sqrt(n/(n+1)) phi_{n-1},  t = u/sigma.
__global__ __launch_bounds__(256) void k_tables(const AtomRec *__restrict__ atoms,
                                                double h, double *__restrict__ tab) {
  const AtomRec A = atoms[blockIdx.x];
  const int nf = A.nu + 2;
  const int nfp = A.tab_nfp;
  const int rows = A.mx + A.my + A.mz;
  const double inv_s = 1.0 / A.sigma;
  const double p0 = 0.7511255444649425 * sqrt(inv_s);
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    int i;
    double c;
    if (r < A.mx) {
      i = A.ix0 + r;
      c = A.cx;
    } else if (r < A.mx + A.my) {
      i = A.iy0 + (r - A.mx);
      c = A.cy;
    } else {
      i = A.iz0 + (r - A.mx - A.my);
      c = A.cz;
    }
    const double x = ((double)i * h - c) * inv_s;
    double *row = tab + A.tab_off + (int64_t)r * nfp;
    double fm = 0.0;
    double f = p0 * exp(-0.5 * x * x);
    row[0] = f;
    for (int n = 0; n + 1 < nf; ++n) {
      const double fn = sqrt(2.0 / (n + 1)) * x * f - sqrt((double)n / (n + 1)) * fm;
      fm = f;
      f = fn;
      row[n + 1] = f;
    }
    for (int n = nf; n < nfp; ++n) row[n] = 0.0;
  }
}

// ------------------------------------------------------------- lane state --

struct Lanes {
  int slot;  // run slot of this lane
  int TB;    // bands per slot
  int bl;    // band within the tile
  bool bok;  // band exists
  int bc;    // band used for addressing (clamped into range)
};

__device__ inline Lanes lane_geometry(const KArgs &K, int tile) {
  Lanes L;
  const int lane = threadIdx.x & 63;
  L.TB = 1 << K.tb_shift;
  L.slot = lane >> K.tb_shift;
  L.bl = lane & (L.TB - 1);
  const int b = tile * L.TB + L.bl;
  L.bok = b < K.B;
  L.bc = L.bok ? b : K.B - 1;
  return L;
}


// The run a lane streams in the current bundle.  Slots beyond the bundle's
// run count mirror its last run (valid addresses) and contribute nothing.
struct RunState {
  const double *base;  // psi at the run's first point, this lane's band
  int jx0;             // table index of the first point
  int len;
  int jy;
  int active;  // int, not bool: a struct without padding bytes stays in
               // registers when the loop carries it
};

__device__ inline RunState run_state(const KArgs &K, const Lanes &L,
                                     const double *psi, const BundleRec &bd) {
  const int s = min(L.slot, bd.nruns - 1);
  const LineRec ln = K.lines[bd.run0 + s];
  RunState r;
  r.base = psi + ((int64_t)ln.row * K.nx + ln.x0m) * K.B + L.bc;
  r.jx0 = ln.jx0;
  r.len = ln.len;
  r.jy = ln.jy;
  r.active = L.slot < bd.nruns;
  return r;
}

// The runs of a wave's bundles are consecutive line records.  The wave
// copies kLineStage of them at a time into its LDS stage (one 16-byte load
// per lane), so that moving to the next bundle reads its runs from LDS: a
// global load there would make the wave wait for every load in flight
// before it, the streamed psi of the current bundle included.
__device__ inline void stage_lines(const KArgs &K, int base, LineRec *st) {
  const int lane = threadIdx.x & 63;
  const int i = min(base + lane, K.nlines - 1);
  reinterpret_cast<int4 *>(st)[lane] = reinterpret_cast<const int4 *>(K.lines)[i];
  __builtin_amdgcn_wave_barrier();
}

// The stage, one per wave of a workgroup (a single variable, so that a kernel
// whose branches instantiate several cut-offs still allocates it once).
__shared__ LineRec g_line_stage[kWaves][kLineStage];

// run_state with the line records of [base, base + kLineStage) staged in st;
// restages first if bd's runs reach past them.
__device__ inline RunState run_state_staged(const KArgs &K, const Lanes &L, const double *psi,
                                            const BundleRec &bd, LineRec *st, int &base) {
  if (bd.run0 + bd.nruns > base + kLineStage) {
    base = bd.run0;
    stage_lines(K, base, st);
  }
  const int s = min(L.slot, bd.nruns - 1);
  const LineRec ln = st[bd.run0 + s - base];
  RunState r;
  r.base = psi + ((int64_t)ln.row * K.nx + ln.x0m) * K.B + L.bc;
  r.jx0 = ln.jx0;
  r.len = ln.len;
  r.jy = ln.jy;
  r.active = L.slot < bd.nruns;
  return r;
}

// Complex bands: lanes hold the real (even band) and imaginary (odd band)
// part of one band, in neighbouring lanes.  v <- e^{+-i th} v for the pair:
// sgn_s = -s on real lanes and +s on imaginary lanes multiplies by e^{+i th};
// the opposite signs by e^{-i th}.
__device__ inline double rotate_pair(double v, double c, double sgn_s) {
  const double p = __shfl_xor(v, 1);
  return fma(sgn_s, p, c * v);
}

// Issues kBatch loads: table indices jb .. jb+kBatch-1 of the lane's run,
// clamped into the run (the clamped copies get zero weight).
__device__ inline void load_batch(const KArgs &K, const RunState &r, int jb,
                                  double *v) {
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const int k = min(max(jb + u - r.jx0, 0), r.len - 1);
    v[u] = r.base[k * K.B];
  }
}

// z pass of the projection for one plane: fold the slots (same band,
// different runs of the plane), then C[n] += phi_nz(z) T2[nx][ny].
template <int NU, bool DET>
__device__ inline void flush_plane(cptr<double> fz, double *T2, double *cacc,
                                   const Lanes &L) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  for (int s = 32; s >= L.TB; s >>= 1) {
#pragma unroll
    for (int q = 0; q < NP; ++q) T2[q] += __shfl_xor(T2[q], s);
  }
  if (L.slot == 0 && L.bok) {
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
            // deterministic plans: the wave's own tile, one lane per value
            if constexpr (DET)
              cacc[idx * L.TB + L.bl] += f * T2[q];
            else
              atomicAdd(&cacc[idx * L.TB + L.bl], f * T2[q]);
            ++idx;
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) T2[q] = 0.0;
}

// ------------------------------------------------------- projection core --

// Adds sum over the runs of bundles [b0,b1) of P_n(i) psi(i) (no h^3), for
// the workgroup's band tile, into cacc[n*TB + bl] (LDS).  One batch of loads
// is always in flight while the previous one is contracted.
template <int NU, bool DET, bool CPLX = false>
__device__ inline void project_bundles(const KArgs &K, const AtomRec &A,
                                       const Lanes &L, int b0, int b1,
                                       const double *__restrict__ psi,
                                       double *cacc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  if (b0 >= b1) return;
  const int nfp = A.tab_nfp;
  const cptr<double> tx = as_const(K.tab) + A.tab_off;
  const double *ty = K.tab + A.tab_off + (int64_t)A.mx * nfp;
  const cptr<double> tz = tx + (int64_t)(A.mx + A.my) * nfp;

  double T1[NF], T2[NP];
#pragma unroll
  for (int n = 0; n < NF; ++n) T1[n] = 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) T2[q] = 0.0;
  LineRec *st = g_line_stage[wave_id()];
  int bi = b0;
  BundleRec bd = load_uniform(K.bundles + bi);
  int sbase = bd.run0;
  stage_lines(K, sbase, st);
  RunState rs = run_state_staged(K, L, psi, bd, st, sbase);
  int jb = bd.jlo;
  // One batch: request the next batch (of this bundle or the next one) into
  // nxt, contract cur, and at the bundle's end take the y pass and, at the
  // plane's end, the z pass.  Returns false after the last batch.  The loop
  // below alternates the two buffers instead of copying nxt into cur (a copy
  // would wait for the loads just issued), and runs both steps of a round
  // unconditionally, the second idle (live false: loads of valid addresses,
  // zero weights) once the first was the last: an exit between the two
  // would let the compiler's waits count the first step's loads as in
  // flight at the top of the loop.
  auto step = [&](double (&cur)[kBatch], double (&nxt)[kBatch], bool live) -> bool {
    BundleRec nbd = bd;
    RunState nrs = rs;
    int njb = jb + kBatch;
    const bool end = live && njb > bd.jhi;  // last batch of the bundle
    const bool more = live && (njb <= bd.jhi || bi + 1 < b1);
    // the y table row of this lane's run, requested before the next batch so
    // that waiting for it leaves that batch in flight
    double fy[NF];
    if (end) {
      const double *ry = ty + rs.jy * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) fy[n] = ry[n];
    }
    if (end && more) {
      nbd = load_uniform(K.bundles + bi + 1);
      nrs = run_state_staged(K, L, psi, nbd, st, sbase);
      njb = nbd.jlo;
    }
    // issued also after the last batch (valid addresses of the last run,
    // unused): a load on one path only makes the waits of the other path
    // count it as still in flight
    load_batch(K, nrs, njb, nxt);
    // every loaded value is consumed (zero weight past the bundle's end), so
    // that no load is left pending into registers that are loaded again
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int jx = jb + u;
      const int k = jx - rs.jx0;
      const bool ok = live && jx <= bd.jhi && rs.active && k >= 0 && k < rs.len;
      const double xv = ok ? cur[u] : 0.0;
      const cptr<double> f = tx + min(jx, (int)bd.jhi) * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = fma(f[n], xv, T1[n]);
    }
    if (end) {
      if constexpr (CPLX) {
        // the bundle's runs share one periodic image T, which carries
        // e^{+i k.T} (cos, sin from the plan's table: scalar loads)
        const cptr<double> ph = as_const(K.bundle_phase) + 2 * bi;
        const double pc = ph[0], ps = ph[1];
        const double sg = (L.bl & 1) ? ps : -ps;
#pragma unroll
        for (int n = 0; n < NF; ++n) T1[n] = rotate_pair(T1[n], pc, sg);
      }
      // y pass with this lane's run
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const double fv = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) T2[q] = fma(fv, T1[nx], T2[q]);
      }
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = 0.0;
      if (!more || nbd.jz != bd.jz) flush_plane<NU, DET>(tz + bd.jz * nfp, T2, cacc, L);
      ++bi;
    }
    bd = nbd;
    rs = nrs;
    jb = njb;
    return more;
  };
  double v[kBatch], w[kBatch];
  load_batch(K, rs, jb, v);
  bool more = true;
  do {
    more = step(v, w, true);
    more = step(w, v, more);
  } while (more);
}

// One work item of the projection: zero the LDS tile, stream the item's
// bundles, write (or, for a shared atom, add) h^3 C into c.
template <int NU, bool DET, bool CPLX = false>
__device__ inline void project_item(const KArgs &K, cptr<WorkRec> W, const AtomRec &A,
                                    const double *__restrict__ psi,
                                    double *__restrict__ c, double *cacc) {
  constexpr int NF = NU + 1;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  const int tile = blockIdx.y;
  const int TB = 1 << K.tb_shift;
  const int nt = NS * TB;  // one coefficient tile
  constexpr int tiles = DET ? kWaves : 1;
  for (int t = threadIdx.x; t < nt * tiles; t += blockDim.x) cacc[t] = 0.0;
  __syncthreads();
  const int w = wave_id();
  const Lanes L = lane_geometry(K, tile);
  project_bundles<NU, DET, CPLX>(K, A, L, W->wb[w], W->wb[w + 1], psi,
                                 DET ? cacc + w * nt : cacc);
  __syncthreads();
  const bool split = W->split != 0;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bb = tile * TB + (t & (TB - 1));
    if (bb >= K.B) continue;
    double v = cacc[t];
    for (int k = 1; k < tiles; ++k) v += cacc[k * nt + t];  // waves in order
    double *dst = c + (A.coeff_row + n) * K.B + bb;
    if (split)
      unsafeAtomicAdd(dst, K.h3 * v);
    else
      *dst = K.h3 * v;
  }
}

template <int NU, bool DET>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NU + 1, DET)))) void k_project(
    KArgs K, const double *__restrict__ psi, double *__restrict__ c) {
  extern __shared__ double cacc[];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  if (W->atom < 0) return;  // padding of an XCD-dealt launch
  const AtomRec A = load_uniform(K.atoms + W->atom);
  project_item<NU, DET>(K, W, A, psi, c, cacc);
}

// All cut-offs in one launch: the item's atom selects the instantiation
// (a wave-uniform branch).  Registers are those of the largest case, so the
// single launch serves plans whose cut-offs differ.
template <int NUMAX, bool DET, bool CPLX = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NUMAX + 1, DET)))) void k_project_any(
    KArgs K, const double *__restrict__ psi, double *__restrict__ c) {
  extern __shared__ double cacc[];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  if (W->atom < 0) return;  // padding of an XCD-dealt launch
  const AtomRec A = load_uniform(K.atoms + W->atom);
  switch (A.nu) {
#define X(N)                                                  \
  case N:                                                     \
    if constexpr (N <= NUMAX) project_item<N, DET, CPLX>(K, W, A, psi, c, cacc); \
    break;
    SHO_NU_CASES(X)
#undef X
  }
}

// Expansion of one atom's box with global FP64 atomics (atom-owner form):
// the z pass into registers per plane, the y pass per run, the x pass adds
// into psi.  Used by the per-atom launch schedule.
template <int NU>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NU + 1)))) void k_expand_atomic(
    KArgs K, const double *__restrict__ c, double *psi) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  extern __shared__ double cin[];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  const int tile = blockIdx.y;
  const AtomRec A = load_uniform(K.atoms + W->atom);
  const int TB = 1 << K.tb_shift;
  fill_lds<4>(cin, NS * TB, [&](int t) {
    const int n = t >> K.tb_shift;
    const int bb = tile * TB + (t & (TB - 1));
    return bb < K.B ? K.alpha * c[(A.coeff_row + n) * K.B + bb] : 0.0;
  });
  __syncthreads();
  const int w = wave_id();
  const Lanes L = lane_geometry(K, tile);
  const int nfp = A.tab_nfp;
  const cptr<double> tx = as_const(K.tab) + A.tab_off;
  const double *ty = K.tab + A.tab_off + (int64_t)A.mx * nfp;
  const cptr<double> tz = tx + (int64_t)(A.mx + A.my) * nfp;
  const int b1 = W->wb[w + 1];
  double U2[NP];
  int cur_jz = -1;
  for (int bi = W->wb[w]; bi < b1; ++bi) {
    const BundleRec bd = load_uniform(K.bundles + bi);
    if (bd.jz != cur_jz) {
      // z pass: U2[nx][ny] = sum_nz phi_nz(z) C[nx,ny,nz]
      cur_jz = bd.jz;
      const cptr<double> fz = tz + cur_jz * nfp;
#pragma unroll
      for (int q = 0; q < NP; ++q) U2[q] = 0.0;
      // one layer nz per iteration (not unrolled: with every layer's LDS
      // reads in flight at once the large cut-offs ran out of registers);
      // layer nz holds the pairs nx + ny <= NU - nz, ny outer, nx fastest
      int base = 0;
#pragma unroll 1
      for (int nz = 0; nz < NF; ++nz) {
        const double fv = fz[nz];
        const int lim = NU - nz;
        int q = 0;
#pragma unroll
        for (int ny = 0; ny < NF; ++ny) {
          const int row = base + ny * (lim + 1) - ny * (ny - 1) / 2;
#pragma unroll
          for (int nx = 0; nx < NF - ny; ++nx, ++q)
            if (nx + ny <= lim) U2[q] = fma(fv, cin[(row + nx) * TB + L.bl], U2[q]);
        }
        base += (lim + 1) * (lim + 2) / 2;
      }
    }
    const RunState rs = run_state(K, L, psi, bd);
    // y pass: U1[nx] = sum_ny phi_ny(y) U2[nx][ny] for this lane's run
    double U1[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) U1[n] = 0.0;
    const double *fy = ty + rs.jy * nfp;
    int q = 0;
#pragma unroll
    for (int ny = 0; ny < NF; ++ny) {
      const double fv = fy[ny];
#pragma unroll
      for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[nx] = fma(fv, U2[q], U1[nx]);
    }
    // x pass: psi(x) += sum_nx phi_nx(x) U1[nx]
    double *dst = const_cast<double *>(rs.base);
    const bool live = rs.active && L.bok;
    for (int jb = bd.jlo; jb <= bd.jhi; jb += kBatch) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int jx = jb + u;
        if (jx <= bd.jhi) {
          const cptr<double> f = tx + jx * nfp;
          double v = 0.0;
#pragma unroll
          for (int n = 0; n < NF; ++n) v = fma(f[n], U1[n], v);
          const int k = jx - rs.jx0;
          if (live && k >= 0 && k < rs.len) unsafeAtomicAdd(dst + k * K.B, v);
        }
      }
    }
  }
}

// --------------------------------------------------- expansion by rows --

// Plane partials of the expansion, U2[jz][q][b] = sum_nz phi_nz(z_jz) C[nx,ny,nz][b]
// for every plane jz of every atom (pairs q: ny outer, nx inner).  One
// workgroup per (atom, tile of 32 bands).
constexpr int kU2Tile = 32;

template <int NU>
__global__ __launch_bounds__(256) void k_u2(EArgs E, const double *__restrict__ c,
                                            double *__restrict__ u2) {
  constexpr int NF = NU + 1;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  constexpr int NP = NF * (NF + 1) / 2;
  __shared__ double cs[NS * kU2Tile];
  const int a = E.nu_atoms[E.nu_begin[NU] + blockIdx.x];
  const AtomRec A = load_uniform(E.atoms + a);
  const int b0 = blockIdx.y * kU2Tile;
  fill_lds<8>(cs, NS * kU2Tile, [&](int t) {
    const int n = t / kU2Tile, bl = t % kU2Tile;
    return (b0 + bl < E.B) ? E.alpha * c[(A.coeff_row + n) * E.B + b0 + bl] : 0.0;
  });
  __syncthreads();
  const double *tz = E.tab + A.tab_off + (int64_t)(A.mx + A.my) * A.tab_nfp;
  double *dst = u2 + E.u2_off[a];
  // thread = (plane jz, band bl); it writes all pairs of that plane and band
  for (int t = threadIdx.x; t < A.mz * kU2Tile; t += blockDim.x) {
    const int bl = t % kU2Tile;
    const int jz = t / kU2Tile;
    if (b0 + bl >= E.B) continue;
    double fz[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) fz[n] = tz[(int64_t)jz * A.tab_nfp + n];
    double *out = dst + (int64_t)jz * NP * E.B + b0 + bl;
    int q = 0;
#pragma unroll
    for (int ny = 0; ny < NF; ++ny) {
#pragma unroll
      for (int nx = 0; nx < NF - ny; ++nx, ++q) {
        double acc = 0.0;
        // C index of (nx, ny, nz): nz-major, then ny, nx fastest
#pragma unroll
        for (int nz = 0; nz < NF; ++nz) {
          if (nx + ny + nz <= NU) {
            // offset of (0, ny, nz) within the nz-major order
            int base = 0;
#pragma unroll
            for (int k = 0; k < nz; ++k) base += (NU - k + 1) * (NU - k + 2) / 2;
#pragma unroll
            for (int j = 0; j < ny; ++j) base += NU - nz - j + 1;
            acc = fma(fz[nz], cs[(base + nx) * kU2Tile + bl], acc);
          }
        }
        out[(int64_t)q * E.B] = acc;
      }
    }
  }
}

// Doubles of one row chunk held in LDS by the row kernel, and of each wave's
// staging area for 1D table rows.
constexpr int kRowChunkDoubles = 2048;
constexpr int kStageDoubles = 256;  // 256/nfp table rows (32 or 16 points)
constexpr int kRowWaves = 4;
constexpr int kRowBlock = 64 * kRowWaves;

// Adds the contribution of one run, clipped to x in [xa, xb), into the LDS
// copy of the row chunk that starts at memory x = xc0:
//   U1[nx] = sum_ny phi_ny(y) U2[jz][nx,ny],  psi(x) += sum_nx phi_nx(x) U1[nx].
// Lanes are (x phase, band); phase xp takes the points xa+xp, xa+xp+XP, ...
// The x-table rows of up to 256/nfp points are first copied into the wave's
// LDS staging area with one vector load per lane, issued together with the
// U2 loads, so a run costs one memory latency.
template <int NU, int XP>
__device__ inline void add_run(const EArgs &E, const AtomRec &A,
                               const LineRec &ln, const double *u2a, int xa,
                               int xb, int xc0, double *rowbuf, double *stage,
                               int TB, int xp, int bl, int bc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  const int nfp = A.tab_nfp;
  const int lane = threadIdx.x & 63;
  const double *tx = E.tab + A.tab_off;
  const cptr<double> fy = as_const(E.tab) + A.tab_off + (int64_t)(A.mx + ln.jy) * nfp;
  const double *ub = u2a + (int64_t)ln.jz * NP * E.B + bc;
  const int jshift = ln.jx0 - ln.x0m;  // table index of memory x
  double u2v[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) u2v[q] = ub[(int64_t)q * E.B];
  double U1[NF];
  bool first = true;
  const int stage_pts = kStageDoubles / nfp;
  for (int xs = xa; xs < xb; xs += stage_pts) {
    const int npt = min(stage_pts, xb - xs);
    // stage rows jshift+xs .. +npt-1 (npt*nfp doubles, <= 4 per lane)
    const int nd = npt * nfp;
    const double *src = tx + (int64_t)(xs + jshift) * nfp;
    double tmp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = lane * 4 + k;
      tmp[k] = i < nd ? src[i] : 0.0;
    }
    if (first) {
#pragma unroll
      for (int n = 0; n < NF; ++n) U1[n] = 0.0;
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const double fv = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[nx] = fma(fv, u2v[q], U1[nx]);
      }
      first = false;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) stage[lane * 4 + k] = tmp[k];
    for (int x = xs; x < xs + npt; x += XP) {
      const int xl = x + xp;
      const double *f = stage + (min(xl, xs + npt - 1) - xs) * nfp;
      double val = 0.0;
#pragma unroll
      for (int n = 0; n < NF; ++n) val = fma(f[n], U1[n], val);
      if (xl < xs + npt) atomicAdd(&rowbuf[(xl - xc0) * TB + bl], val);
    }
  }
}

// One workgroup per (memory row, x chunk, band tile): the chunk of psi is read
// into LDS once, every run of any atom that falls into it adds its part
// (waves take runs round robin), and the chunk is written back once.  No two
// workgroups touch the same values, so global memory sees plain loads and
// stores only.  Small workgroups let several of them, in different phases
// (load, add, store), share a CU.
template <int XP, int NUMAX>
__global__ __launch_bounds__(kRowBlock) void k_expand_rows(EArgs E,
                                                          const double *__restrict__ u2,
                                                          double *psi) {
  extern __shared__ double lds[];
  double *rowbuf = lds;
  const RowRec rr = load_uniform(E.rows + blockIdx.x);
  if (rr.row < 0) return;
  const int w = wave_id();
  double *stage = lds + kRowChunkDoubles + w * kStageDoubles;
  const int TB = 1 << E.tbe_shift;
  const int xchunk = kRowChunkDoubles >> E.tbe_shift;
  const int xc0 = (int)blockIdx.y * xchunk;
  const int xc1 = min(xc0 + xchunk, E.nx);
  const int tile = blockIdx.z;
  const int64_t rowoff = (int64_t)rr.row * E.nx;
  const int nval = (xc1 - xc0) << E.tbe_shift;
  fill_lds<kRowChunkDoubles / kRowBlock>(rowbuf, nval, [&](int t) {
    const int x = t >> E.tbe_shift;
    const int b = tile * TB + (t & (TB - 1));
    return b < E.B ? psi[(rowoff + xc0 + x) * E.B + b] : 0.0;
  });
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int xp = lane >> E.tbe_shift;
  const int bl = lane & (TB - 1);
  const int b = tile * TB + bl;
  const int bc = b < E.B ? b : E.B - 1;
  const cptr<int32_t> runs = as_const(E.row_runs) + rr.run_begin;
  for (int i = w; i < rr.nruns; i += kRowWaves) {
    const int run = runs[i];
    const LineRec ln = load_uniform(E.lines + run);
    const int xa = max((int)ln.x0m, xc0);
    const int xb = min((int)ln.x0m + ln.len, xc1);
    if (xa >= xb) continue;
    const int a = as_const(E.run_atom)[run];
    const AtomRec A = load_uniform(E.atoms + a);
    const double *u2a = u2 + as_const(E.u2_off)[a];
    switch (A.nu) {
#define X(N)                                                                  \
  case N:                                                                     \
    if constexpr (N <= NUMAX)                                                 \
      add_run<N, XP>(E, A, ln, u2a, xa, xb, xc0, rowbuf, stage, TB, xp, bl, bc); \
    break;
      X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
#undef X
    }
  }
  __syncthreads();
  constexpr int kPer = kRowChunkDoubles / kRowBlock;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int t = u * kRowBlock + (int)threadIdx.x;
    v[u] = t < nval ? rowbuf[t] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int t = u * kRowBlock + (int)threadIdx.x;
    const int x = t >> E.tbe_shift;
    const int b = tile * TB + (t & (TB - 1));
    if (t < nval && b < E.B) psi[(rowoff + xc0 + x) * E.B + b] = v[u];
  }
}

// ---------------------------------------------- expansion by blocks --

constexpr int kBlkWaves = 4;
constexpr int kBlkBlock = 64 * kBlkWaves;
constexpr int kBlkXStage = 256;  // doubles per wave: the x-table rows of a block

// Adds every run of one entry (one atom plane, one image) into the LDS tile
// of the block.  Lanes are (run slot, band): with 32 bands per tile two runs
// of the entry (two rows of the block) are added at once.  All runs of an
// entry share the atom's x table, so phi_x(x) is wave-uniform and comes from
// the scalar cache; the plane partials are loaded once per entry.
// Runs of one slot handled together: phi_x(x) is read once per x and applied
// to all of them.  Four where the kernel's register budget is set by a larger
// cut-off anyway, else two.
constexpr int blk_group(int nu, int numax) {
  return ((numax > 5 && nu <= 5) || (numax >= 8 && nu <= 7) || (numax >= 9 && nu <= 8)) ? 4 : 2;
}

// The lane's run descriptor of an entry (lane < nruns), requested one entry
// ahead of its use.
__device__ inline uint32_t entry_desc(const EArgs &E, const EntryRec &en) {
  const int lane = threadIdx.x & 63;
  return lane < en.nruns ? as_const(E.run_desc)[en.run_begin + lane] : 0u;
}

// The y-table row of run i of an entry (i clamped into the runs).
__device__ inline const double *entry_fy(const EArgs &E, const EntryRec &en, uint32_t mydesc,
                                         int i, int gend) {
  const uint32_t d = __shfl(mydesc, min(i, gend - 1));
  return E.tab + en.tab_y + (int)(d & 0xff) * en.nfp;
}

template <int NU, int NUMAX, bool CPLX>
__device__ inline void add_entry(const EArgs &E, const EntryRec &en, uint32_t mydesc,
                                 const EntryRec &nen, bool has_next, uint32_t &ndesc, int ei,
                                 const double *u2, int nxl, double *tile, double *xstage,
                                 int TB, int slot, int bl, int bc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  constexpr int G = blk_group(NU, NUMAX);
  const int nfp = en.nfp;
  const int lane = threadIdx.x & 63;
  const int slots = 64 / TB;
  // one round of loads: plane partials, the x-table rows of the block's x
  // range (staged in LDS; rows that do not exist stay unset), the y-table
  // rows of the first group's runs, then the next entry's run descriptors
  const double *ub = u2 + en.u2 + bc;
  double u2v[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) u2v[q] = ub[(int64_t)q * E.B];
  // (up to cut-off 5: above, the registers would cost occupancy)
  constexpr bool kPreY = NUMAX <= 5;
  double fy0[kPreY ? G : 1][NF];
  if constexpr (kPreY) {
    const int gend = min(G * slots, (int)en.nruns);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const double *fy = entry_fy(E, en, mydesc, j * slots + slot, gend);
#pragma unroll
      for (int n = 0; n < NF; ++n) fy0[j][n] = fy[n];
    }
  }
  if constexpr (CPLX) {
    // the entry's image T receives e^{-i k.T} times the plane partials
    // (cos, sin from the plan's table: scalar loads)
    const cptr<double> ph = as_const(E.entry_phase) + 2 * ei;
    const double cs = ph[0], sn = ph[1];
    const double sg = (bl & 1) ? -sn : sn;
#pragma unroll
    for (int q = 0; q < NP; ++q) u2v[q] = rotate_pair(u2v[q], cs, sg);
  }
  double tx[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = lane * 4 + k;
    const int pt = i / nfp;
    tx[k] = (pt >= en.x_lo && pt < en.x_hi) ? E.tab[en.tab_x + i] : 0.0;
  }
  if (has_next) ndesc = entry_desc(E, nen);
#pragma unroll
  for (int k = 0; k < 4; ++k) xstage[lane * 4 + k] = tx[k];
  for (int g0 = 0; g0 < en.nruns; g0 += G * slots) {
    const int gend = min(g0 + G * slots, en.nruns);
    // wave-uniform x range of the group
    int lo = 255, hi = 0;
    for (int k = g0; k < gend; ++k) {
      const uint32_t d = __builtin_amdgcn_readlane(mydesc, k);
      lo = min(lo, (int)((d >> 8) & 0xff));
      hi = max(hi, (int)((d >> 16) & 0xff));
    }
    // this lane's runs g0 + j slots + slot, j < G: rows, ranges, y passes
    int rr[G], xa[G], xb[G];
    double U1[G][NF];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int i = g0 + j * slots + slot;
      const uint32_t d = __shfl(mydesc, min(i, gend - 1));
      rr[j] = d & 0xff;
      xa[j] = i < gend ? (int)((d >> 8) & 0xff) : 0;
      xb[j] = i < gend ? (int)((d >> 16) & 0xff) : 0;
      // the first group's rows were requested with the plane partials
      double fy[NF];
      if (kPreY && g0 == 0) {
#pragma unroll
        for (int n = 0; n < NF; ++n) fy[n] = fy0[kPreY ? j : 0][n];
      } else {
        const double *ry = E.tab + en.tab_y + rr[j] * nfp;
#pragma unroll
        for (int n = 0; n < NF; ++n) fy[n] = ry[n];
      }
#pragma unroll
      for (int n = 0; n < NF; ++n) U1[j][n] = 0.0;
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const double fv = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[j][nx] = fma(fv, u2v[q], U1[j][nx]);
      }
    }
    for (int x = lo; x < hi; ++x) {
      const double *f = xstage + x * nfp;
      double fx[NF];
#pragma unroll
      for (int n = 0; n < NF; ++n) fx[n] = f[n];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        double val = 0.0;
#pragma unroll
        for (int n = 0; n < NF; ++n) val = fma(fx[n], U1[j][n], val);
        if (x >= xa[j] && x < xb[j])
          atomicAdd(&tile[(rr[j] * nxl + x) * TB + bl], val);
      }
    }
  }
}

// One workgroup per (block, band tile): the block's values of psi are read
// into LDS once, every entry adds its runs (waves take entries round robin),
// and the block is written back once with plain stores.  The tile is laid
// out as [row][X2][band] with X2 the block width rounded up to a power of
// two, so that a tile slot splits into (row, x, band) with shifts and masks
// instead of divisions (the index arithmetic of the fill and write-back is a
// large share of the kernel's instructions); slots past the grid's last
// column hold zeros and are not written back.
template <int NUMAX, bool CPLX>
__global__ __launch_bounds__(kBlkBlock) void k_expand_blocks(EArgs E,
                                                            const double *__restrict__ u2,
                                                            double *psi) {
  extern __shared__ double lds[];
  constexpr int kTile = blk_tile_doubles(NUMAX);
  const BlockRec bk = load_uniform(E.blocks + blockIdx.x);
  if (bk.nentries < 0) return;
  const int w = wave_id();
  double *tile = lds;
  const int TB = 1 << E.tbe_shift;
  const int btile = blockIdx.y;
  const int xe = min(bk.x0 + E.blk_x, E.nx);
  const int nxl = xe - bk.x0;
  const int nrow = min(bk.y0 + E.blk_rows, E.ny) - bk.y0;
  const int x2s = E.blk_x <= 1 ? 0 : 32 - __clz(E.blk_x - 1);
  const int rs = x2s + E.tbe_shift;
  const int nval = nrow << rs;  // tile slots, padding columns included
  const int64_t gbase = ((int64_t)(bk.z * E.ny + bk.y0) * E.nx + bk.x0) * E.B + btile * TB;
  const int64_t grow = (int64_t)E.nx * E.B;
  // slot t <-> psi index g; false past the grid's last column or for a
  // padding band
  auto slot = [&](int64_t base, int t, int64_t &g) -> bool {
    const int r = t >> rs;
    const int x = (t >> E.tbe_shift) & ((1 << x2s) - 1);
    const int l = t & (TB - 1);
    g = base + r * grow + (int64_t)__umul24(x, E.B) + l;
    return x < nxl && btile * TB + l < E.B;
  };
  // 16-byte chunks (two bands) when every band pair is whole: the tile is
  // filled by direct loads into LDS (no registers, no LDS writes).  (A
  // write-back in 16-byte chunks, ds_read_b128 + 16-byte stores, measured
  // slower than the 8-byte one below.)
  const bool wide = TB >= 2 && (E.B & 1) == 0;
  if (wide) {
    // chunk c of the tile is slot 2c; each wave moves 64 chunks (1 KiB) per
    // load, lane i into the wave's LDS address + 16 i.  Slots that hold no
    // value of the block (padding columns and bands, chunks past nval) are
    // loaded from the block's first point: never added to by an entry that
    // is written back.
    const int nchunk = nval >> 1;
    const int lane = threadIdx.x & 63;
    for (int c0 = w * 64; c0 < nchunk; c0 += kBlkBlock) {
      const int c = c0 + lane;
      int64_t g = gbase;
      int64_t gc = 0;
      if (c < nchunk && slot(gbase, 2 * c, gc)) g = gc;
      // non-temporal (cache policy nt), like the write-back below: the
      // block is read and written once, and should not evict from the
      // memory-side cache the psi that the projection reads again
      __builtin_amdgcn_global_load_lds(psi + g, (__attribute__((address_space(3))) void *)(tile + 2 * c0),
                                       16, 0, 2);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  } else {
    fill_lds<kTile / kBlkBlock>(tile, nval, [&](int t) {
      int64_t g = 0;
      return slot(gbase, t, g) ? psi[g] : 0.0;
    });
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lslot = lane >> E.tbe_shift;
  const int bl = lane & (TB - 1);
  const int b = btile * TB + bl;
  const int bc = b < E.B ? b : E.B - 1;
  double *xstage = lds + kTile + w * kBlkXStage;
  // entries round robin over the waves; the next entry's record is requested
  // before the current one is processed
  EntryRec en;
  uint32_t desc = 0u;
  if (w < bk.nentries) {
    en = load_uniform(E.entries + bk.entry_begin + w);
    desc = entry_desc(E, en);
  }
  for (int i = w; i < bk.nentries; i += kBlkWaves) {
    EntryRec nxt = en;
    const bool has_next = i + kBlkWaves < bk.nentries;
    if (has_next) nxt = load_uniform(E.entries + bk.entry_begin + i + kBlkWaves);
    uint32_t ndesc = 0u;
    switch (en.nu) {
#define X(N)                                                                          \
  case N:                                                                             \
    if constexpr (N <= NUMAX)                                                         \
      add_entry<N, NUMAX, CPLX>(E, en, desc, nxt, has_next, ndesc, bk.entry_begin + i, u2, \
                                1 << x2s, tile, xstage, TB, lslot, bl, bc);          \
    break;
      X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
#undef X
    }
    en = nxt;
    desc = ndesc;
  }
  __syncthreads();
  // the write-back forms its addresses again (the base is made opaque)
  // instead of holding them in registers across the entries
  int64_t gb = gbase;
  asm volatile("" : "+s"(gb));
  constexpr int kPer = kTile / kBlkBlock;
  for (int t0 = 0; t0 < nval; t0 += kPer * kBlkBlock) {
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      v[u] = t < nval ? tile[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      int64_t g = 0;
      if (t < nval && slot(gb, t, g)) __builtin_nontemporal_store(v[u], psi + g);
    }
  }
}

// ------------------------------------------------ projection by blocks --

// Block form of the projection, for plans whose supports overlap much: one
// workgroup per (block of R rows x X points of one plane, band tile) reads
// the block's values of psi into LDS once, and every entry (atom plane,
// image) touching the block adds its share of the atom plane's sums,
//   T2[nx][ny] = sum_{rows y} phi_ny(y) sum_x phi_nx(x) psi(x, y, z),
// to the plane partials P2[jz][pair][band] (global atomics; the layout of
// the expansion's plane partials).  k_zpass then takes the z pass,
// c[n] = h^3 sum_jz phi_nz(z_jz) P2[jz][nx,ny].  Each value of psi is read
// from memory once per band tile however many supports hold it; the price is
// one atomic add per pair and band for every entry.
// Lanes are (run slot, band) as in the expansion's block form; phi_x is
// wave-uniform (scalar loads), phi_y per lane.
template <int NU>
__device__ inline void proj_entry(const EArgs &E, const EntryRec &en, double *p2,
                                  const double *tile, int x2, int TB, int slot, int bl,
                                  int bc, bool bok) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  const int nfp = en.nfp;
  const int lane = threadIdx.x & 63;
  const int slots = 64 / TB;
  const uint32_t mydesc = lane < en.nruns ? as_const(E.run_desc)[en.run_begin + lane] : 0u;
  const cptr<double> tx = as_const(E.tab) + en.tab_x;
  double T2[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) T2[q] = 0.0;
  for (int g0 = 0; g0 < en.nruns; g0 += slots) {
    const int gend = min(g0 + slots, (int)en.nruns);
    int lo = 255, hi = 0;  // wave-uniform x range of the group
    for (int k = g0; k < gend; ++k) {
      const uint32_t d = __builtin_amdgcn_readlane(mydesc, k);
      lo = min(lo, (int)((d >> 8) & 0xff));
      hi = max(hi, (int)((d >> 16) & 0xff));
    }
    const int i = g0 + slot;
    const uint32_t d = __shfl(mydesc, min(i, gend - 1));
    const int r = d & 0xff;
    const int xa = i < gend ? (int)((d >> 8) & 0xff) : 0;
    const int xb = i < gend ? (int)((d >> 16) & 0xff) : 0;
    const double *trow = tile + ((r * x2) << __builtin_ctz(TB)) + bl;
    double T1[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) T1[n] = 0.0;
    for (int x = lo; x < hi; ++x) {
      const double v = (x >= xa && x < xb) ? trow[x * TB] : 0.0;
      const cptr<double> f = tx + x * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = fma(f[n], v, T1[n]);
    }
    const double *fy = E.tab + en.tab_y + r * nfp;
    int q = 0;
#pragma unroll
    for (int ny = 0; ny < NF; ++ny) {
      const double fv = fy[ny];
#pragma unroll
      for (int nx = 0; nx < NF - ny; ++nx, ++q) T2[q] = fma(fv, T1[nx], T2[q]);
    }
  }
  for (int sft = 32; sft >= TB; sft >>= 1) {
#pragma unroll
    for (int q = 0; q < NP; ++q) T2[q] += __shfl_xor(T2[q], sft);
  }
  if (slot == 0 && bok) {
    double *dst = p2 + en.u2 + bc;
#pragma unroll
    for (int q = 0; q < NP; ++q) unsafeAtomicAdd(dst + (int64_t)q * E.B, T2[q]);
  }
}

template <int NUMAX>
__global__ __launch_bounds__(kBlkBlock) void k_project_blocks(EArgs E,
                                                             const double *__restrict__ psi,
                                                             double *p2) {
  extern __shared__ double lds[];
  const BlockRec bk = load_uniform(E.blocks + blockIdx.x);
  if (bk.nentries < 0) return;
  const int w = wave_id();
  double *tile = lds;
  const int TB = 1 << E.tbe_shift;
  const int btile = blockIdx.y;
  const int xe = min(bk.x0 + E.blk_x, E.nx);
  const int nxl = xe - bk.x0;
  const int nrow = min(bk.y0 + E.blk_rows, E.ny) - bk.y0;
  const int x2s = E.blk_x <= 1 ? 0 : 32 - __clz(E.blk_x - 1);
  const int rs = x2s + E.tbe_shift;
  const int nval = nrow << rs;
  const int64_t gbase = ((int64_t)(bk.z * E.ny + bk.y0) * E.nx + bk.x0) * E.B + btile * TB;
  const int64_t grow = (int64_t)E.nx * E.B;
  fill_lds<16>(tile, nval, [&](int t) {
    const int r = t >> rs;
    const int x = (t >> E.tbe_shift) & ((1 << x2s) - 1);
    const int l = t & (TB - 1);
    return (x < nxl && btile * TB + l < E.B)
               ? psi[gbase + r * grow + (int64_t)__umul24(x, E.B) + l]
               : 0.0;
  });
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lslot = lane >> E.tbe_shift;
  const int bl = lane & (TB - 1);
  const int b = btile * TB + bl;
  const bool bok = b < E.B;
  const int bc = bok ? b : E.B - 1;
  for (int i = w; i < bk.nentries; i += kBlkWaves) {
    const EntryRec en = load_uniform(E.entries + bk.entry_begin + i);
    switch (en.nu) {
#define X(N)                                                                      \
  case N:                                                                         \
    if constexpr (N <= NUMAX) proj_entry<N>(E, en, p2, tile, 1 << x2s, TB, lslot, bl, bc, bok); \
    break;
      SHO_NU_CASES(X)
#undef X
    }
  }
}

// z pass of the block projection: c[n][b] = h^3 sum_jz phi_nz(z_jz) P2[jz][nx,ny][b]
// for every atom of cut-off NU; thread = (pair, band), each plane partial
// read once.
template <int NU>
__global__ __launch_bounds__(256) void k_zpass(EArgs E, const double *__restrict__ p2,
                                               double *__restrict__ c, double h3) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  const int a = E.nu_atoms[E.nu_begin[NU] + blockIdx.x];
  const AtomRec A = load_uniform(E.atoms + a);
  const int b0 = blockIdx.y * kU2Tile;
  const cptr<double> tz = as_const(E.tab) + A.tab_off + (int64_t)(A.mx + A.my) * A.tab_nfp;
  const double *src = p2 + E.u2_off[a];
  for (int t = threadIdx.x; t < NP * kU2Tile; t += blockDim.x) {
    const int q = t / kU2Tile, bl = t % kU2Tile;
    const int b = b0 + bl;
    if (b >= E.B) continue;
    // pair q -> (nx, ny), ny outer
    int ny = 0, qq = q;
    while (qq >= NF - ny) {
      qq -= NF - ny;
      ++ny;
    }
    const int nx = qq;
    double acc[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) acc[n] = 0.0;
    for (int jz = 0; jz < A.mz; ++jz) {
      const double v = src[((int64_t)jz * NP + q) * E.B + b];
      const cptr<double> fz = tz + jz * A.tab_nfp;
#pragma unroll
      for (int nz = 0; nz < NF; ++nz) acc[nz] = fma(fz[nz], v, acc[nz]);
    }
    // C index of (nx, ny, nz): nz-major, then ny, nx fastest
#pragma unroll
    for (int nz = 0; nz < NF; ++nz) {
      if (nx + ny + nz <= NU) {
        int base = 0;
        for (int k = 0; k < nz; ++k) base += (NU - k + 1) * (NU - k + 2) / 2;
        for (int j = 0; j < ny; ++j) base += NU - nz - j + 1;
        c[(A.coeff_row + base + nx) * E.B + b] = h3 * acc[nz];
      }
    }
  }
}

// ------------------------------------------------ expansion by owners --

// Owner form of the expansion's y and x passes.  One wave owns a strip of R
// rows x X points of one plane for one tile of TB bands (R = 64 / TB): lane
// (r, b) keeps the X values psi(z, y0 + r, x0 .. x0 + X - 1)[b] in
// registers, reads them once, adds the contribution of every entry (atom
// plane and image) that touches the strip, in the plan's fixed entry order,
// and writes them once.  No value is shared between lanes, so there are no
// atomics and the sum over atoms is taken in the same order on every run.
// Per entry a lane forms U1[nx] = sum_ny phi_ny(y) U2[nx][ny] for its row
// from the plane partials, then the x pass adds sum_nx phi_nx(x) U1[nx] to
// the points of its row's run; phi_x is wave-uniform (scalar loads).
template <int NU, int X>
__device__ inline void owner_entry(const EArgs &E, const EntryRec &en, const double *u2,
                                   double (&acc)[X], int r, int bc) {
  constexpr int NF = NU + 1;
  const int nfp = en.nfp;
  // this lane's run (at most one per row) and the union of the entry's runs
  const cptr<uint32_t> desc = as_const(E.run_desc) + en.run_begin;
  int xa = 0, xb = 0, lo = X, hi = 0, rr = -1;
  for (int k = 0; k < en.nruns; ++k) {
    const uint32_t d = desc[k];
    const int dr = d & 0xff, da = (d >> 8) & 0xff, db = (d >> 16) & 0xff;
    lo = min(lo, da);
    hi = max(hi, db);
    if (rr < 0) rr = dr;  // a row of the entry, for the lanes without a run
    if (dr == r) {
      xa = da;
      xb = db;
    }
  }
  const int ry = xa < xb ? r : rr;
  // y pass of this lane's row
  const double *fy = E.tab + en.tab_y + ry * nfp;
  const double *ub = u2 + en.u2 + bc;
  double U1[NF];
#pragma unroll
  for (int n = 0; n < NF; ++n) U1[n] = 0.0;
  int q = 0;
#pragma unroll
  for (int ny = 0; ny < NF; ++ny) {
    const double fv = fy[ny];
#pragma unroll
    for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[nx] = fma(fv, ub[(int64_t)q * E.B], U1[nx]);
  }
  // x pass over the union of the runs (a wave-uniform range)
  const cptr<double> tx = as_const(E.tab) + en.tab_x;
#pragma unroll
  for (int x = 0; x < X; ++x) {
    if (x >= lo && x < hi) {
      const cptr<double> f = tx + x * nfp;
      double v = 0.0;
#pragma unroll
      for (int n = 0; n < NF; ++n) v = fma(f[n], U1[n], v);
      if (x >= xa && x < xb) acc[x] += v;
    }
  }
}

template <int NUMAX, int X>
__global__ __launch_bounds__(64) void k_expand_owner(EArgs E, const double *__restrict__ u2,
                                                      double *psi) {
  if ((int)blockIdx.x >= E.nblocks) return;  // launch rounded up to 8 XCDs
  const BlockRec bk = load_uniform(E.blocks + blockIdx.x);
  if (bk.nentries < 0) return;
  const int lane = threadIdx.x;
  const int TB = 1 << E.tbe_shift;
  const int r = lane >> E.tbe_shift;
  const int b = (int)blockIdx.y * TB + (lane & (TB - 1));
  const bool live = b < E.B && bk.y0 + r < E.ny;
  const int bc = b < E.B ? b : E.B - 1;
  const int nxl = min(X, E.nx - bk.x0);
  double *base = psi + ((int64_t)(bk.z * E.ny + (live ? bk.y0 + r : bk.y0)) * E.nx + bk.x0) *
                           E.B + bc;
  double acc[X];
#pragma unroll
  for (int x = 0; x < X; ++x) acc[x] = (live && x < nxl) ? base[(int64_t)x * E.B] : 0.0;
  for (int i = 0; i < bk.nentries; ++i) {
    const EntryRec en = load_uniform(E.entries + bk.entry_begin + i);
    switch (en.nu) {
#define X_(N)                                                      \
  case N:                                                          \
    if constexpr (N <= NUMAX) owner_entry<N, X>(E, en, u2, acc, r, bc); \
    break;
      X_(0) X_(1) X_(2) X_(3) X_(4) X_(5) X_(6) X_(7) X_(8) X_(9) X_(10)
#undef X_
    }
  }
#pragma unroll
  for (int x = 0; x < X; ++x)
    if (live && x < nxl) base[(int64_t)x * E.B] = acc[x];
}

// ------------------------------------------------- stored projectors --

// P[run][k][n] = phi_nx(x) phi_ny(y) phi_nz(z) at point k of the run, for all
// n of the atom's basis (nz-major order).  One workgroup per run.
__global__ __launch_bounds__(256) void k_store(KArgs K, const int32_t *__restrict__ run_atom,
                                               double *__restrict__ stored) {
  const int run = blockIdx.x;
  const LineRec ln = K.lines[run];
  const AtomRec A = K.atoms[run_atom[run]];
  const int nu = A.nu;
  const int ns = (nu + 1) * (nu + 2) * (nu + 3) / 6;
  const int nfp = A.tab_nfp;
  const double *tx = K.tab + A.tab_off;
  const double *fy = tx + (int64_t)(A.mx + ln.jy) * nfp;
  const double *fz = tx + (int64_t)(A.mx + A.my + ln.jz) * nfp;
  double *out = stored + K.run_poff[run];
  for (int t = threadIdx.x; t < ln.len * ns; t += blockDim.x) {
    const int k = t / ns;
    int n = t - k * ns;
    int nz = 0;
    while (n >= (nu - nz + 1) * (nu - nz + 2) / 2) {
      n -= (nu - nz + 1) * (nu - nz + 2) / 2;
      ++nz;
    }
    int ny = 0;
    while (n >= nu - nz - ny + 1) {
      n -= nu - nz - ny + 1;
      ++ny;
    }
    const int nx = n;
    const double *fx = tx + (int64_t)(ln.jx0 + k) * nfp;
    out[t] = fx[nx] * fy[ny] * fz[nz];
  }
}

// Real solid harmonic r^l Y_lm(r^) at offset (x, y, z) for l <= 3, m = -l..l:
// the real spherical harmonics without the Condon-Shortley sign (Y_11 ~ +x,
// Y_1,-1 ~ +y), normalised on the unit sphere.
__device__ inline double solid_harmonic(int l, int m, double x, double y, double z) {
  const double pi = 3.14159265358979323846;
  const double r2 = x * x + y * y + z * z;
  switch (l * 8 + m + 3) {
    case 0 * 8 + 3: return 0.5 / sqrt(pi);
    case 1 * 8 + 2: return sqrt(0.75 / pi) * y;
    case 1 * 8 + 3: return sqrt(0.75 / pi) * z;
    case 1 * 8 + 4: return sqrt(0.75 / pi) * x;
    case 2 * 8 + 1: return 0.5 * sqrt(15.0 / pi) * x * y;
    case 2 * 8 + 2: return 0.5 * sqrt(15.0 / pi) * y * z;
    case 2 * 8 + 3: return 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - r2);
    case 2 * 8 + 4: return 0.5 * sqrt(15.0 / pi) * x * z;
    case 2 * 8 + 5: return 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    case 3 * 8 + 0: return 0.25 * sqrt(17.5 / pi) * y * (3.0 * x * x - y * y);
    case 3 * 8 + 1: return 0.5 * sqrt(105.0 / pi) * x * y * z;
    case 3 * 8 + 2: return 0.25 * sqrt(10.5 / pi) * y * (5.0 * z * z - r2);
    case 3 * 8 + 3: return 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0 * r2);
    case 3 * 8 + 4: return 0.25 * sqrt(10.5 / pi) * x * (5.0 * z * z - r2);
    case 3 * 8 + 5: return 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    case 3 * 8 + 6: return 0.25 * sqrt(17.5 / pi) * x * (x * x - 3.0 * y * y);
    default: return 0.0;
  }
}

// Radial plans: P[run][k][j] = P_kr(r) Y_lm(r^) at point k of the run, r the
// offset from the atom, for every projector j (radial function kr, then m).
// P_kr between the table nodes is the cubic Lagrange interpolant through the
// nodes s .. s+3, s = clamp(floor(r/dr) - 1, 0, nr - 4); zero from the last
// node on.  One workgroup per run, thread = (point, projector).
__global__ __launch_bounds__(256) void k_store_radial(KArgs K, RArgs R,
                                                      const int32_t *__restrict__ run_atom,
                                                      double *__restrict__ stored) {
  const int run = blockIdx.x;
  const LineRec ln = K.lines[run];
  const AtomRec A = K.atoms[run_atom[run]];
  const int np = R.nproj;
  double *out = stored + K.run_poff[run];
  const double y = (double)(A.iy0 + ln.jy) * R.h - A.cy;
  const double z = (double)(A.iz0 + ln.jz) * R.h - A.cz;
  for (int t = threadIdx.x; t < ln.len * np; t += blockDim.x) {
    const int k = t / np;
    int j = t - k * np;
    int kr = 0;
    while (j >= 2 * R.ell[kr] + 1) {  // projector j -> (radial function, m)
      j -= 2 * R.ell[kr] + 1;
      ++kr;
    }
    const int l = R.ell[kr], m = j - l;
    const double x = (double)(A.ix0 + ln.jx0 + k) * R.h - A.cx;
    const double r = sqrt(x * x + y * y + z * z);
    const double tt = r / R.dr;
    double rad = 0.0;
    if (tt < (double)(R.nr - 1)) {
      const int s0 = min(max((int)floor(tt) - 1, 0), R.nr - 4);
      const double u = tt - (double)s0;
      const double *row = R.rad + (int64_t)kr * R.nr + s0;
      rad = -(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0 * row[0] +
            u * (u - 2.0) * (u - 3.0) / 2.0 * row[1] -
            u * (u - 1.0) * (u - 3.0) / 2.0 * row[2] + u * (u - 1.0) * (u - 2.0) / 6.0 * row[3];
    }
    double ang;
    if (l == 0)
      ang = solid_harmonic(0, 0, x, y, z);
    else if (r > 0.0)
      ang = solid_harmonic(l, m, x, y, z) / (l == 1 ? r : l == 2 ? r * r : r * r * r);
    else
      ang = 0.0;
    out[t] = rad * ang;
  }
}

// The stored forms are dense contractions per atom, run on FP64 MFMA
// (v_mfma_f64_16x16x4f64, D[16][16] += A[16][4] B[4][16]).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it receives D[4 r + l / 16][l % 16]
// in accumulator register r.
typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ inline dx4 mfma_f64(double a, double b, dx4 d) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
}

constexpr int kStoredBlock = 256;  // 4 waves
constexpr int kStoredTile = 32;    // bands per workgroup (two 16-band MFMA columns)

// c[n][b] += h^3 sum_k P[k][n] psi(k)[b] over the item's points k: MFMA with
// i = n (16 per block), j = b, and four points per step along the sum.  Each
// wave takes every fourth step; the waves meet in LDS, then one atomic add
// per coefficient and band goes to c.  The table has S.ncol <= NS columns.
template <int NS>
__global__ __launch_bounds__(kStoredBlock) void k_project_stored(
    SArgs S, const double *__restrict__ psi, double *__restrict__ c) {
  constexpr int NBN = (NS + 15) / 16;
  const int ncol = S.ncol;
  constexpr int U = 2;  // steps in flight per wave
  __shared__ double red[NBN * 16 * kStoredTile];
  const StoredItem it = load_uniform(S.items + blockIdx.x);
  const int a = it.atom;
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int q = lane >> 4, col = lane & 15;
  const int b0 = blockIdx.y * kStoredTile;
  const int bA = b0 + col, bB = b0 + 16 + col;
  const bool okA = bA < S.B, okB = bB < S.B;
  const double *P = S.P + S.atom_poff[a];
  const int32_t *pidx = S.pidx + S.atom_pbeg[a];
  for (int t = threadIdx.x; t < NBN * 16 * kStoredTile; t += kStoredBlock) red[t] = 0.0;
  dx4 acc[NBN][2];
#pragma unroll
  for (int nb = 0; nb < NBN; ++nb) acc[nb][0] = acc[nb][1] = dx4{0.0, 0.0, 0.0, 0.0};
  for (int k = it.k0 + 4 * w; k < it.k1; k += 4 * 4 * U) {
    double av[U][NBN], vA[U], vB[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kp = k + 16 * u + q;
      const bool ok = kp < it.k1;
      const int kc = ok ? kp : it.k1 - 1;
      const double *prow = P + (int64_t)kc * ncol;
      const double *vrow = psi + (int64_t)pidx[kc] * S.B;
#pragma unroll
      for (int nb = 0; nb < NBN; ++nb) {
        const int n = nb * 16 + col;
        av[u][nb] = (ok && n < ncol) ? prow[n] : 0.0;
      }
      vA[u] = (ok && okA) ? vrow[bA] : 0.0;
      vB[u] = (ok && okB) ? vrow[bB] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int nb = 0; nb < NBN; ++nb) {
        acc[nb][0] = mfma_f64(av[u][nb], vA[u], acc[nb][0]);
        acc[nb][1] = mfma_f64(av[u][nb], vB[u], acc[nb][1]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < NBN; ++nb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = nb * 16 + 4 * r + q;
      atomicAdd(&red[n * kStoredTile + col], acc[nb][0][r]);
      atomicAdd(&red[n * kStoredTile + 16 + col], acc[nb][1][r]);
    }
  }
  __syncthreads();
  const int64_t row0 = S.atoms[a].coeff_row;
  for (int t = threadIdx.x; t < ncol * kStoredTile; t += kStoredBlock) {
    const int n = t / kStoredTile;
    const int b = b0 + (t % kStoredTile);
    if (b < S.B) unsafeAtomicAdd(c + (row0 + n) * S.B + b, S.h3 * red[t]);
  }
}

// psi(k)[b] += sum_n P[k][n] c[n][b]: MFMA with i = point (16 per tile),
// j = band and four coefficients per step along the sum; the atom's
// coefficients stay in registers.  Overlapping atoms meet in global FP64
// atomics.  The table has S.ncol <= NS columns.
template <int NS>
__global__ __launch_bounds__(kStoredBlock) void k_expand_stored(
    SArgs S, const double *__restrict__ c, double *psi) {
  constexpr int NK = (NS + 3) / 4;
  const int ncol = S.ncol;
  const StoredItem it = load_uniform(S.items + blockIdx.x);
  const int a = it.atom;
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int q = lane >> 4, col = lane & 15;
  const int b0 = blockIdx.y * kStoredTile;
  const int bA = b0 + col, bB = b0 + 16 + col;
  const bool okA = bA < S.B, okB = bB < S.B;
  const double *P = S.P + S.atom_poff[a];
  const int32_t *pidx = S.pidx + S.atom_pbeg[a];
  const int64_t row0 = S.atoms[a].coeff_row;
  // sum over n in the order n = q NK + m: contiguous P reads per lane
  double cA[NK], cB[NK];
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    const int n = q * NK + m;
    cA[m] = (n < ncol && okA) ? S.alpha * c[(row0 + n) * S.B + bA] : 0.0;
    cB[m] = (n < ncol && okB) ? S.alpha * c[(row0 + n) * S.B + bB] : 0.0;
  }
  for (int k = it.k0 + 16 * w; k < it.k1; k += 16 * 4) {
    const int kp = k + col;
    const bool ok = kp < it.k1;
    const double *prow = P + (int64_t)(ok ? kp : it.k1 - 1) * ncol;
    double av[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      const int n = q * NK + m;
      av[m] = (ok && n < ncol) ? prow[n] : 0.0;
    }
    int32_t mi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kr = k + 4 * r + q;
      mi[r] = kr < it.k1 ? pidx[kr] : -1;
    }
    dx4 dA = {0.0, 0.0, 0.0, 0.0}, dB = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      dA = mfma_f64(av[m], cA[m], dA);
      dB = mfma_f64(av[m], cB[m], dB);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (mi[r] < 0) continue;
      double *dst = psi + (int64_t)mi[r] * S.B;
      if (okA) unsafeAtomicAdd(dst + bA, dA[r]);
      if (okB) unsafeAtomicAdd(dst + bB, dB[r]);
    }
  }
}

// ------------------------------------------ stored, block form expansion --

// Adds the runs of one entry from the stored tables: for 16 points of a run
// at a time, D[point][band] = sum_n P[point][n] c[n][band] on FP64 MFMA
// (i = point, j = band, four n per step; the atom's coefficients of this
// lane's bands stay in registers), then LDS atomic adds into the block tile.
// The atom's table has ncol <= NS columns.
template <int NS>
__device__ inline void add_entry_stored(const EArgs &E, const EntryRec &en,
                                        const double *__restrict__ c, int nxl, double *tile,
                                        int TB, int btile, int ncol) {
  constexpr int NK = (NS + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, col = lane & 15;
  const int64_t row0 = en.u2;
  const int bA = btile * TB + col, bB = bA + 16;
  const bool okA = bA < E.B, okB = TB > 16 && bB < E.B;
  // the sum over n runs in the order n = q NK + m (lane quarter q, step m),
  // so that each lane reads one contiguous stretch of its point's P row
  double cA[NK], cB[NK];
#pragma unroll
  for (int m = 0; m < NK; ++m) {
    const int n = q * NK + m;
    cA[m] = (n < ncol && okA) ? E.alpha * c[(row0 + n) * E.B + bA] : 0.0;
    cB[m] = (n < ncol && okB) ? E.alpha * c[(row0 + n) * E.B + bB] : 0.0;
  }
  const uint32_t mydesc = lane < en.nruns ? as_const(E.run_desc)[en.run_begin + lane] : 0u;
  const int64_t mybase = lane < en.nruns ? E.desc_pbase[en.run_begin + lane] : 0;
  for (int i = 0; i < en.nruns; ++i) {
    const uint32_t d = __builtin_amdgcn_readlane(mydesc, i);
    const int r = d & 0xff, xa = (d >> 8) & 0xff, xb = (d >> 16) & 0xff;
    const int64_t pb = ((int64_t)__builtin_amdgcn_readlane((int)(mybase >> 32), i) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)(mybase & 0xffffffff), i);
    double *trow = tile + (int64_t)r * nxl * TB;
    for (int p0 = xa; p0 < xb; p0 += 16) {
      const int pt = p0 + col;  // A row of this lane
      const bool ok = pt < xb;
      const double *prow = E.P + pb + (int64_t)(ok ? pt : xb - 1) * ncol;
      dx4 dA = {0.0, 0.0, 0.0, 0.0}, dB = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < NK; ++m) {
        const int n = q * NK + m;
        const double av = (ok && n < ncol) ? prow[n] : 0.0;
        dA = mfma_f64(av, cA[m], dA);
        dB = mfma_f64(av, cB[m], dB);
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int x = p0 + 4 * rr + q;
        if (x < xb) {
          atomicAdd(&trow[x * TB + col], dA[rr]);
          if (TB > 16) atomicAdd(&trow[x * TB + 16 + col], dB[rr]);
        }
      }
    }
  }
}

// NUMAX: the largest cut-off of an SHO plan; RNS > 0: radial plan, the
// column bound of its E.ncol projectors.
template <int NUMAX, int RNS>
__global__ __launch_bounds__(kBlkBlock) void k_expand_blocks_stored(
    EArgs E, const double *__restrict__ c, double *psi) {
  extern __shared__ double lds[];
  const BlockRec bk = load_uniform(E.blocks + blockIdx.x);
  if (bk.nentries < 0) return;
  const int w = wave_id();
  double *tile = lds;
  const int TB = 1 << E.tbe_shift;
  const int btile = blockIdx.y;
  const int xe = min(bk.x0 + E.blk_x, E.nx);
  const int nxl = xe - bk.x0;
  const int nrow = min(bk.y0 + E.blk_rows, E.ny) - bk.y0;
  const int rowbase = bk.z * E.ny + bk.y0;
  const int per_row = nxl << E.tbe_shift;
  const int nval = nrow * per_row;
  auto gidx = [&](int t, int &b) -> int64_t {
    const int r = t / per_row;
    const int rem = t - r * per_row;
    const int x = rem >> E.tbe_shift;
    b = btile * TB + (rem & (TB - 1));
    return ((int64_t)(rowbase + r) * E.nx + bk.x0 + x) * E.B + b;
  };
  fill_lds<kBlockTileDoubles / kBlkBlock>(tile, nval, [&](int t) {
    int bb;
    const int64_t g = gidx(t, bb);
    return bb < E.B ? psi[g] : 0.0;
  });
  __syncthreads();
  for (int i = w; i < bk.nentries; i += kBlkWaves) {
    const EntryRec en = load_uniform(E.entries + bk.entry_begin + i);
    if constexpr (RNS > 0) {
      add_entry_stored<RNS>(E, en, c, nxl, tile, TB, btile, E.ncol);
    } else {
      switch (en.nu) {
#define X(N)                                                                         \
  case N:                                                                            \
    if constexpr (N <= NUMAX)                                                        \
      add_entry_stored<(N + 1) * (N + 2) * (N + 3) / 6>(E, en, c, nxl, tile, TB, btile, \
                                                        (N + 1) * (N + 2) * (N + 3) / 6); \
    break;
        X(0) X(1) X(2) X(3) X(4) X(5)
#undef X
      }
    }
  }
  __syncthreads();
  constexpr int kPer = kBlockTileDoubles / kBlkBlock;
  for (int t0 = 0; t0 < nval; t0 += kPer * kBlkBlock) {
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      v[u] = t < nval ? tile[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      if (t < nval) {
        int bb;
        const int64_t g = gidx(t, bb);
        if (bb < E.B) psi[g] = v[u];
      }
    }
  }
}

// ------------------------------------------------------- multiplication --

// d[a][n][b] = sum_m D_a[n][m] c[a][m][b] (sec. 3.2 step 2 with the atomic
// matrix carried into the SHO basis, sec. 3.5): per atom a dense N x N times
// N x B product, on FP64 MFMA with i = n, j = b and four m per step.  One
// workgroup per (atom, 32-band tile); wave w takes the 16-row blocks
// w, w+4, ...
__global__ __launch_bounds__(kStoredBlock) void k_multiply(const AtomRec *__restrict__ atoms,
                                                           const int64_t *__restrict__ doff,
                                                           const double *__restrict__ D,
                                                           const double *__restrict__ c,
                                                           double *__restrict__ d, int32_t B) {
  const int a = blockIdx.x;
  const int nu = load_uniform(&atoms[a].nu);
  const int64_t row0 = load_uniform(&atoms[a].coeff_row);
  const int N = (nu + 1) * (nu + 2) * (nu + 3) / 6;
  const double *Da = D + doff[a];
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int q = lane >> 4, col = lane & 15;
  const int b0 = blockIdx.y * kStoredTile;
  const int bA = b0 + col, bB = b0 + 16 + col;
  const bool okA = bA < B, okB = bB < B;
  const int nblk = (N + 15) / 16;
  for (int nb = w; nb < nblk; nb += 4) {
    dx4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int n = nb * 16 + col;
#pragma unroll 4
    for (int m0 = 0; m0 < N; m0 += 4) {
      const int m = m0 + q;
      const double av = (n < N && m < N) ? Da[(int64_t)n * N + m] : 0.0;
      const double cA = (m < N && okA) ? c[(row0 + m) * B + bA] : 0.0;
      const double cB = (m < N && okB) ? c[(row0 + m) * B + bB] : 0.0;
      acc0 = mfma_f64(av, cA, acc0);
      acc1 = mfma_f64(av, cB, acc1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nn = nb * 16 + 4 * r + q;
      if (nn < N) {
        if (okA) d[(row0 + nn) * B + bA] = acc0[r];
        if (okB) d[(row0 + nn) * B + bB] = acc1[r];
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
// grad must be zero before the launch (work items and band tiles add).
template <int NU1, bool DET>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NU1 + 1, DET)))) void k_force(
    KArgs K, const double *__restrict__ psi, const double *__restrict__ w,
    double *grad, double *gpart) {
  constexpr int NF = NU1 + 1;
  constexpr int NS1 = NF * (NF + 1) * (NF + 2) / 6;
  constexpr int NU = NU1 - 1;
  constexpr int NS = (NU + 1) * (NU + 2) * (NU + 3) / 6;
  extern __shared__ double cacc[];
  __shared__ double red[3][kWaves];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  const int tile = blockIdx.y;
  const int a = W->atom;
  const AtomRec A = load_uniform(K.atoms + a);
  const int TB = 1 << K.tb_shift;
  const int nt = NS1 * TB;
  constexpr int tiles = DET ? kWaves : 1;
  for (int t = threadIdx.x; t < nt * tiles; t += blockDim.x) cacc[t] = 0.0;
  __syncthreads();
  const int wv = wave_id();
  const Lanes L = lane_geometry(K, tile);
  project_bundles<NU1, DET>(K, A, L, W->wb[wv], W->wb[wv + 1], psi, DET ? cacc + wv * nt : cacc);
  __syncthreads();
  if constexpr (DET) {  // the waves' tiles, added in wave order into the first
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      double v = cacc[t];
      for (int k = 1; k < tiles; ++k) v += cacc[k * nt + t];
      cacc[t] = v;
    }
    __syncthreads();
  }

  double g[3] = {0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bl = t & (TB - 1);
    const int bb = tile * TB + bl;
    if (bb >= K.B) continue;
    int m[3];
    coeff_decode(n, NU, m[0], m[1], m[2]);
    const double wn = w[(A.coeff_row + n) * K.B + bb];
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
      g[d] = fma(wn, v, g[d]);
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
    for (int k = 0; k < kWaves; ++k) s += red[threadIdx.x][k];
    if constexpr (DET)
      gpart[((int64_t)a * K.ntiles + tile) * 3 + threadIdx.x] = -K.h3 / A.sigma * s;
    else
      unsafeAtomicAdd(&grad[3 * a + threadIdx.x], -K.h3 / A.sigma * s);
  }
}

// grad[a][d] = sum over band tiles, in tile order, of the deterministic
// derivative's per-tile sums.
__global__ void k_force_sum(const double *__restrict__ gpart, int32_t natoms, int32_t ntiles,
                            double *__restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (atom, direction)
  if (i >= 3 * natoms) return;
  const int a = i / 3, d = i % 3;
  double v = 0.0;
  for (int t = 0; t < ntiles; ++t) v += gpart[((int64_t)a * ntiles + t) * 3 + d];
  grad[i] = v;
}

__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- launch --

static dim3 grid_of(const KArgs &K) {
  return dim3((unsigned)K.nwork, (unsigned)K.ntiles);
}

// LDS of a projection workgroup: one coefficient tile, or one per wave for
// deterministic sums.
static size_t proj_lds(const KArgs &K, int nf) {
  return lds_tile_bytes(nf, 1 << K.tb_shift) * (K.det ? kWaves : 1);
}

template <int NU>
static hipError_t launch_project_nu(const KArgs &K, const double *psi,
                                    double *c, hipStream_t s) {
  const size_t shm = proj_lds(K, NU + 1);
  if (K.det)
    hipLaunchKernelGGL((k_project<NU, true>), grid_of(K), dim3(kBlock), shm, s, K, psi, c);
  else
    hipLaunchKernelGGL((k_project<NU, false>), grid_of(K), dim3(kBlock), shm, s, K, psi, c);
  return hipGetLastError();
}

template <int NU1>
static hipError_t launch_force_nu(const KArgs &K, const double *psi,
                                  const double *w, double *grad,
                                  hipStream_t s, double *gpart) {
  const size_t shm = proj_lds(K, NU1 + 1);
  if (K.det) {
    if (!gpart) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_force<NU1, true>), grid_of(K), dim3(kBlock), shm, s, K, psi, w, grad,
                       gpart);
  } else {
    hipLaunchKernelGGL((k_force<NU1, false>), grid_of(K), dim3(kBlock), shm, s, K, psi, w, grad,
                       gpart);
  }
  return hipGetLastError();
}


template <int NUMAX>
static hipError_t launch_project_any_nu(const KArgs &K, const double *psi,
                                        double *c, hipStream_t s) {
  const size_t shm = proj_lds(K, NUMAX + 1);
  if (K.det)
    hipLaunchKernelGGL((k_project_any<NUMAX, true>), grid_of(K), dim3(kBlock), shm, s, K, psi,
                       c);
  else if (K.bloch)
    hipLaunchKernelGGL((k_project_any<NUMAX, false, true>), grid_of(K), dim3(kBlock), shm, s, K,
                       psi, c);
  else
    hipLaunchKernelGGL((k_project_any<NUMAX, false>), grid_of(K), dim3(kBlock), shm, s, K, psi,
                       c);
  return hipGetLastError();
}

hipError_t launch_project_any(int nu_max, const KArgs &K, const double *psi,
                              double *c, hipStream_t s) {
  if (K.nwork <= 0) return hipSuccess;
  switch (nu_max) {
#define X(N) case N: return launch_project_any_nu<N>(K, psi, c, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <int NU>
static hipError_t launch_expand_atomic_nu(const KArgs &K, const double *c,
                                          double *psi, hipStream_t s) {
  const size_t shm = lds_tile_bytes(NU + 1, 1 << K.tb_shift);
  hipLaunchKernelGGL(k_expand_atomic<NU>, grid_of(K), dim3(kBlock), shm, s, K, c, psi);
  return hipGetLastError();
}

hipError_t launch_expand_atomic(int nu, const KArgs &K, const double *c,
                                double *psi, hipStream_t s) {
  if (K.nwork <= 0) return hipSuccess;
  switch (nu) {
#define X(N) case N: return launch_expand_atomic_nu<N>(K, c, psi, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_project(int nu, const KArgs &K, const double *psi, double *c,
                          hipStream_t s) {
  if (K.bloch) return hipErrorInvalidValue;  // Bloch plans run k_project_any
  switch (nu) {
#define X(N) case N: return launch_project_nu<N>(K, psi, c, s);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_force(int nu, const KArgs &K, const double *psi,
                        const double *w, double *grad, hipStream_t s, double *gpart) {
  if (K.nwork <= 0) return hipSuccess;
  switch (nu) {
#define X(N) case N: return launch_force_nu<N + 1>(K, psi, w, grad, s, gpart);
    SHO_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand_planes(const EArgs &E, const double *c, double *u2,
                                hipStream_t s) {
  for (int nu = 0; nu <= SHO_NU_MAX; ++nu) {
    const int cnt = E.nu_begin[nu + 1] - E.nu_begin[nu];
    if (cnt <= 0) continue;
    const dim3 g((unsigned)cnt, (unsigned)E.ntiles_u2);
    switch (nu) {
#define X(N)                                                            \
  case N:                                                               \
    hipLaunchKernelGGL(k_u2<N>, g, dim3(256), 0, s, E, c, u2);          \
    break;
      SHO_NU_CASES(X)
#undef X
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rows(const EArgs &E, const double *u2, double *psi,
                       hipStream_t s) {
  if (E.bloch) return hipErrorInvalidValue;  // Bloch plans expand in the block form
  if (E.nrows > 0) {
    const int xchunk = kRowChunkDoubles >> E.tbe_shift;
    const dim3 g((unsigned)E.nrows, (unsigned)((E.nx + xchunk - 1) / xchunk),
                 (unsigned)E.ntiles);
    const size_t shm = (kRowChunkDoubles + kRowWaves * kStageDoubles) * sizeof(double);
    switch (E.nu_max) {
#define X(N)                                                                      \
  case N:                                                                         \
    if (E.tbe_shift == 6)                                                         \
      hipLaunchKernelGGL((k_expand_rows<1, N>), g, dim3(kRowBlock), shm, s, E, u2, psi); \
    else                                                                          \
      hipLaunchKernelGGL((k_expand_rows<2, N>), g, dim3(kRowBlock), shm, s, E, u2, psi); \
    break;
      SHO_NU_CASES(X)
#undef X
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_blocks(const EArgs &E, const double *u2, double *psi,
                         hipStream_t s) {
  if (E.nblocks > 0) {
    const dim3 g((unsigned)E.nblocks, (unsigned)E.ntiles);
    size_t shm = 0;
    switch (E.nu_max) {
#define X(N)                                                                          \
  case N:                                                                             \
    shm = (blk_tile_doubles(N) + kBlkWaves * kBlkXStage) * sizeof(double);           \
    if (E.bloch)                                                                      \
      hipLaunchKernelGGL((k_expand_blocks<N, true>), g, dim3(kBlkBlock), shm, s, E, u2, \
                         psi);                                                        \
    else                                                                              \
      hipLaunchKernelGGL((k_expand_blocks<N, false>), g, dim3(kBlkBlock), shm, s, E, u2, \
                         psi);                                                        \
    break;
      SHO_NU_CASES(X)
#undef X
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_owner(const EArgs &E, const double *u2, double *psi, hipStream_t s) {
  if (E.bloch) return hipErrorInvalidValue;  // Bloch plans expand in the block form
  if (E.nblocks <= 0) return hipSuccess;
  // whole groups of 8 workgroups, so that block g runs on XCD g mod 8 for
  // every band tile (the plan deals the planes' strips to the XCDs that way)
  const unsigned gx = (unsigned)((E.nblocks + 7) / 8 * 8);
  const dim3 g(gx, (unsigned)E.ntiles);
  switch (E.nu_max * 64 + E.blk_x) {
#define X_(N)                                                                         \
  case N * 64 + 16:                                                                   \
    hipLaunchKernelGGL((k_expand_owner<N, 16>), g, dim3(64), 0, s, E, u2, psi);      \
    break;                                                                            \
  case N * 64 + 32:                                                                   \
    hipLaunchKernelGGL((k_expand_owner<N, 32>), g, dim3(64), 0, s, E, u2, psi);      \
    break;
    SHO_NU_CASES(X_)
#undef X_
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_blocks_stored(const EArgs &E, const double *c, double *psi,
                                hipStream_t s) {
  if (E.nblocks > 0) {
    const dim3 g((unsigned)E.nblocks, (unsigned)E.ntiles);
    const size_t shm = kBlockTileDoubles * sizeof(double);
    if (E.ncol > 0) {
      switch (stored_bound(E.ncol)) {
#define X(N)                                                                         \
  case N:                                                                            \
    hipLaunchKernelGGL((k_expand_blocks_stored<0, N>), g, dim3(kBlkBlock), shm, s, E, c, \
                       psi);                                                         \
    break;
        X(1) X(4) X(10) X(20) X(35) X(56)
#undef X
        default:
          return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
    switch (E.nu_max) {
#define X(N)                                                                        \
  case N:                                                                           \
    hipLaunchKernelGGL((k_expand_blocks_stored<N, 0>), g, dim3(kBlkBlock), shm, s, E, c, \
                       psi);                                                        \
    break;
      X(0) X(1) X(2) X(3) X(4) X(5)
#undef X
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_expand_rows(const EArgs &E, const double *c, double *u2,
                              double *psi, hipStream_t s) {
  hipError_t e = launch_expand_planes(E, c, u2, s);
  if (e != hipSuccess) return e;
  return launch_rows(E, u2, psi, s);
}


hipError_t launch_store(const KArgs &K, const int32_t *run_atom, int32_t nruns,
                        double *stored, hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_store, dim3((unsigned)nruns), dim3(256), 0, s, K, run_atom, stored);
  return hipGetLastError();
}

hipError_t launch_store_radial(const KArgs &K, const RArgs &R, const int32_t *run_atom,
                               int32_t nruns, double *stored, hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_store_radial, dim3((unsigned)nruns), dim3(256), 0, s, K, R, run_atom,
                     stored);
  return hipGetLastError();
}

static dim3 stored_grid(const SArgs &S) {
  return dim3((unsigned)S.nitems, (unsigned)((S.B + kStoredTile - 1) / kStoredTile));
}

#define SHO_STORED_BOUNDS(X) X(1) X(4) X(10) X(20) X(35) X(56)

hipError_t launch_project_stored(const SArgs &S, const double *psi, double *c,
                                 hipStream_t s) {
  if (S.nitems <= 0) return hipSuccess;
  switch (stored_bound(S.ncol)) {
#define X(N)                                                                   \
  case N:                                                                      \
    hipLaunchKernelGGL(k_project_stored<N>, stored_grid(S), dim3(kStoredBlock), 0, s, S, \
                       psi, c);                                                \
    return hipGetLastError();
    SHO_STORED_BOUNDS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand_stored(const SArgs &S, const double *c, double *psi,
                                hipStream_t s) {
  if (S.nitems <= 0) return hipSuccess;
  switch (stored_bound(S.ncol)) {
#define X(N)                                                                  \
  case N:                                                                     \
    hipLaunchKernelGGL(k_expand_stored<N>, stored_grid(S), dim3(kStoredBlock), 0, s, S, \
                       c, psi);                                               \
    return hipGetLastError();
    SHO_STORED_BOUNDS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_multiply(const AtomRec *atoms, int32_t natoms, const int64_t *doff,
                           const double *D, const double *c, double *d, int32_t B,
                           hipStream_t s) {
  if (natoms <= 0) return hipSuccess;
  const dim3 g((unsigned)natoms, (unsigned)((B + kStoredTile - 1) / kStoredTile));
  hipLaunchKernelGGL(k_multiply, g, dim3(kStoredBlock), 0, s, atoms, doff, D, c, d, B);
  return hipGetLastError();
}

hipError_t launch_tables(const AtomRec *atoms, int32_t natoms, double h,
                         double *tab, int32_t mmax, hipStream_t s) {
  (void)mmax;
  if (natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tables, dim3((unsigned)natoms), dim3(256), 0, s, atoms, h, tab);
  return hipGetLastError();
}

hipError_t launch_force_sum(const double *gpart, int32_t natoms, int32_t ntiles, double *grad,
                            hipStream_t s) {
  if (natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_sum, dim3((unsigned)((3 * natoms + 255) / 256)), dim3(256), 0, s,
                     gpart, natoms, ntiles, grad);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_project_blocks(const EArgs &E, const double *psi, double *p2,
                                 hipStream_t s) {
  if (E.nblocks <= 0) return hipSuccess;
  if (E.bloch) return hipErrorInvalidValue;
  const dim3 g((unsigned)E.nblocks, (unsigned)E.ntiles);
  const size_t shm = kProjTileDoubles * sizeof(double);
  switch (E.nu_max) {
#define X(N)                                                                          \
  case N:                                                                             \
    hipLaunchKernelGGL((k_project_blocks<N>), g, dim3(kBlkBlock), shm, s, E, psi, p2); \
    break;
    SHO_NU_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zpass(const EArgs &E, const double *p2, double *c, double h3,
                        hipStream_t s) {
  for (int nu = 0; nu <= SHO_NU_MAX; ++nu) {
    const int cnt = E.nu_begin[nu + 1] - E.nu_begin[nu];
    if (cnt <= 0) continue;
    const dim3 g((unsigned)cnt, (unsigned)E.ntiles_u2);
    switch (nu) {
#define X(N)                                                                 \
  case N:                                                                    \
    hipLaunchKernelGGL(k_zpass<N>, g, dim3(256), 0, s, E, p2, c, h3);        \
    break;
      SHO_NU_CASES(X)
#undef X
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------- static expansion scratch --

// Plane partials of the allocation-free expansion: one copy per device,
// loaded with the code object and held until the process ends.  Host code
// must not pass this name to a kernel (on the host it is only a stand-in);
// static_scratch() returns the device address.
__device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<double *>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace sho
