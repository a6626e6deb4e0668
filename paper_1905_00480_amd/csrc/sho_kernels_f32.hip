// sho_kernels_f32.hip -- single-precision projection and expansion.
//
// The paper measures its kernels in float as well as double (sec. 6,
// table 2).  An FP32 plan holds an even number 2P of bands; each lane works
// on one pair of adjacent bands (one aligned 8-byte float pair), so that
// every record of the plan, every launch shape and scratch size is that of
// an FP64 plan with P bands, and each load and store moves the same 8 bytes
// per lane as in double precision.  Tables, the x and y passes and the plane
// partials are FP32.  The sums that go through LDS atomics (the projection's
// z pass and the expansion's accumulation into each grid value) are kept in
// FP64 and rounded to float once at the end: on gfx950 a 32-bit float
// atomic add in LDS is more than an order of magnitude slower than the
// 64-bit one, and the wider sums only tighten the error.  Complex
// single-precision bands are such pairs (real, imaginary): the SHO functions
// are real, so both halves are projected and expanded alike.
//
// The passes are those of the FP64 kernels (x, y, z contractions with the
// x table read through the scalar cache; expansion by plane partials and
// owner-computes blocks).  They live in a translation unit of their own so
// that the FP64 kernels are compiled exactly as they are without them.
#include <hip/hip_runtime.h>

#include "sho_device.hpp"
#include "sho_launch.hpp"

namespace sho {
namespace f32 {

constexpr int kBlock = 64 * kWaves;
constexpr int kBatch = 6;  // loads in flight per lane and batch

#define SHO_F32_NU_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

// waves per SIMD the register allocator must allow (a pair of floats takes
// the registers of one double, so the FP64 budget carries over)
constexpr int waves_per_eu(int nf) { return nf <= 6 ? 4 : 2; }

// Two adjacent bands of one grid point (or one complex band).
struct __attribute__((aligned(8))) Pair {
  float a, b;
};

__device__ inline Pair fma2(float s, Pair v, Pair acc) {
  return Pair{fmaf(s, v.a, acc.a), fmaf(s, v.b, acc.b)};
}

__device__ inline Pair zero2() { return Pair{0.f, 0.f}; }

// Non-temporal load and store of a pair (the block expansion's read and
// write of psi: once per block, not to evict what the projection reads).
typedef float nt_float2 __attribute__((ext_vector_type(2)));
__device__ inline Pair load_nt(const Pair *p) {
  const nt_float2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float2 *>(p));
  return Pair{v.x, v.y};
}
__device__ inline void store_nt(Pair v, Pair *p) {
  const nt_float2 w = {v.a, v.b};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_float2 *>(p));
}

// ---------------------------------------------------------------- tables --

// The FP32 tables are the FP64 samples rounded once to nearest.
__global__ void k_round_tables(const double *__restrict__ src, float *__restrict__ dst,
                               int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ------------------------------------------------------------- lane state --

struct Lanes {
  int slot;  // run slot of this lane
  int TB;    // band pairs per slot
  int bl;    // pair within the tile
  bool bok;  // pair exists
  int bc;    // pair used for addressing (clamped into range)
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


struct RunState {
  const Pair *base;  // psi at the run's first point, this lane's pair
  int jx0;
  int len;
  int jy;
  int active;  // int, not bool: a struct without padding bytes stays in
               // registers when the loop carries it
};

__device__ inline RunState run_state(const KArgs &K, const Lanes &L, const Pair *psi,
                                     const BundleRec &bd) {
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

// Line records staged per wave in LDS (see the FP64 unit): moving to the
// next bundle reads its runs there instead of waiting for a global load
// issued behind the streamed psi.
constexpr int kLineStage = 64;
static_assert(kWaves * kLineStage * sizeof(LineRec) + 1024 <= kStaticLds,
              "static LDS of the streaming kernels");
__shared__ LineRec g_line_stage[kWaves][kLineStage];

__device__ inline void stage_lines(const KArgs &K, int base, LineRec *st) {
  const int lane = threadIdx.x & 63;
  const int i = min(base + lane, K.nlines - 1);
  reinterpret_cast<int4 *>(st)[lane] = reinterpret_cast<const int4 *>(K.lines)[i];
  __builtin_amdgcn_wave_barrier();
}

__device__ inline RunState run_state_staged(const KArgs &K, const Lanes &L, const Pair *psi,
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

// A complex band as one pair (a = real, b = imaginary part): v e^{i th} for
// sn = sin th, or v e^{-i th} for sn = -sin th.
__device__ inline Pair rotate(Pair v, float cs, float sn) {
  return Pair{fmaf(-sn, v.b, cs * v.a), fmaf(sn, v.a, cs * v.b)};
}

__device__ inline void load_batch(const KArgs &K, const RunState &r, int jb, Pair *v) {
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const int k = min(max(jb + u - r.jx0, 0), r.len - 1);
    v[u] = r.base[k * K.B];
  }
}

// LDS tiles hold the two bands of a pair in separate rows of TB doubles
// ([..][2][TB]), so that the lanes of one slot touch consecutive words.

// z pass for one plane: fold the slots, then C[n] += phi_nz(z) T2[nx][ny]
// into the LDS tile ([n][2][TB] doubles; float products are exact in double).
template <int NU>
__device__ inline void flush_plane(cptr<float> fz, Pair *T2, double *cacc, const Lanes &L) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  for (int s = 32; s >= L.TB; s >>= 1) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      T2[q].a += __shfl_xor(T2[q].a, s);
      T2[q].b += __shfl_xor(T2[q].b, s);
    }
  }
  if (L.slot == 0 && L.bok) {
    // the lane's word offset is made opaque here so that the per-coefficient
    // addresses are formed at the flush instead of being held live (and
    // spilled) across the whole stream of bundles
    int lane_off = L.bl;
    asm volatile("" : "+v"(lane_off));
    const int row = 2 * L.TB;
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
            double *dst = cacc + (idx * row + lane_off);
            atomicAdd(dst, f * (double)T2[q].a);
            atomicAdd(dst + L.TB, f * (double)T2[q].b);
            ++idx;
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) T2[q] = zero2();
}

// ------------------------------------------------------- projection core --

template <int NU, bool CPLX = false>
__device__ inline void project_bundles(const KArgs &K, const float *tab, const AtomRec &A,
                                       const Lanes &L, int b0, int b1,
                                       const Pair *__restrict__ psi, double *cacc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  if (b0 >= b1) return;
  const int nfp = A.tab_nfp;
  const cptr<float> tx = as_const(tab) + A.tab_off;
  const float *ty = tab + A.tab_off + (int64_t)A.mx * nfp;
  const cptr<float> tz = tx + (int64_t)(A.mx + A.my) * nfp;

  Pair T1[NF], T2[NP];
#pragma unroll
  for (int n = 0; n < NF; ++n) T1[n] = zero2();
#pragma unroll
  for (int q = 0; q < NP; ++q) T2[q] = zero2();
  LineRec *st = g_line_stage[wave_id()];
  int bi = b0;
  BundleRec bd = load_uniform(K.bundles + bi);
  int sbase = bd.run0;
  stage_lines(K, sbase, st);
  RunState rs = run_state_staged(K, L, psi, bd, st, sbase);
  int jb = bd.jlo;
  // One batch, as in the FP64 unit: request the next batch into nxt (also
  // when idle, from valid addresses), contract cur (zero weights when idle
  // or past the bundle), y pass at the bundle's end, z pass at the plane's
  // end; the loop alternates the buffers and runs both steps of a round.
  auto step = [&](Pair (&cur)[kBatch], Pair (&nxt)[kBatch], bool live) -> bool {
    BundleRec nbd = bd;
    RunState nrs = rs;
    int njb = jb + kBatch;
    const bool end = live && njb > bd.jhi;
    const bool more = live && (njb <= bd.jhi || bi + 1 < b1);
    float fy[NF];
    if (end) {
      const float *ry = ty + rs.jy * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) fy[n] = ry[n];
    }
    if (end && more) {
      nbd = load_uniform(K.bundles + bi + 1);
      nrs = run_state_staged(K, L, psi, nbd, st, sbase);
      njb = nbd.jlo;
    }
    load_batch(K, nrs, njb, nxt);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int jx = jb + u;
      const int k = jx - rs.jx0;
      const bool ok = live && jx <= bd.jhi && rs.active && k >= 0 && k < rs.len;
      const Pair xv = ok ? cur[u] : zero2();
      const cptr<float> f = tx + min(jx, (int)bd.jhi) * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = fma2(f[n], xv, T1[n]);
    }
    if (end) {
      if constexpr (CPLX) {
        // the bundle's runs share one periodic image T, which carries
        // e^{+i k.T} (cos, sin in double from the plan's table, rounded once
        // to float)
        const cptr<double> ph = as_const(K.bundle_phase) + 2 * bi;
        const float pc = (float)ph[0], ps = (float)ph[1];
#pragma unroll
        for (int n = 0; n < NF; ++n) T1[n] = rotate(T1[n], pc, ps);
      }
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const float fv = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) T2[q] = fma2(fv, T1[nx], T2[q]);
      }
#pragma unroll
      for (int n = 0; n < NF; ++n) T1[n] = zero2();
      if (!more || nbd.jz != bd.jz) flush_plane<NU>(tz + bd.jz * nfp, T2, cacc, L);
      ++bi;
    }
    bd = nbd;
    rs = nrs;
    jb = njb;
    return more;
  };
  Pair v[kBatch], w[kBatch];
  load_batch(K, rs, jb, v);
  bool more = true;
  do {
    more = step(v, w, true);
    more = step(w, v, more);
  } while (more);
}

template <int NU, bool CPLX = false>
__device__ inline void project_item(const KArgs &K, const float *tab, cptr<WorkRec> W,
                                    const AtomRec &A, const Pair *__restrict__ psi,
                                    Pair *__restrict__ c, double *cacc) {
  constexpr int NF = NU + 1;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  const int tile = blockIdx.y;
  const int TB = 1 << K.tb_shift;
  for (int t = threadIdx.x; t < 2 * NS * TB; t += blockDim.x) cacc[t] = 0.0;
  __syncthreads();
  const int w = wave_id();
  const Lanes L = lane_geometry(K, tile);
  project_bundles<NU, CPLX>(K, tab, A, L, W->wb[w], W->wb[w + 1], psi, cacc);
  __syncthreads();
  const bool split = W->split != 0;
  for (int t = threadIdx.x; t < NS * TB; t += blockDim.x) {
    const int n = t >> K.tb_shift;
    const int bb = tile * TB + (t & (TB - 1));
    if (bb >= K.B) continue;
    Pair *dst = c + (A.coeff_row + n) * K.B + bb;
    const int ia = t + (t & ~(TB - 1));  // [n][2][TB]: first float of the pair
    const Pair v{(float)(K.h3 * cacc[ia]), (float)(K.h3 * cacc[ia + TB])};
    if (split) {
      unsafeAtomicAdd(&dst->a, v.a);
      unsafeAtomicAdd(&dst->b, v.b);
    } else {
      *dst = v;
    }
  }
}

template <int NU>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NU + 1)))) void k_project(
    KArgs K, const float *__restrict__ tab, const Pair *__restrict__ psi,
    Pair *__restrict__ c) {
  extern __shared__ double cacc[];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  if (W->atom < 0) return;  // padding of an XCD-dealt launch
  const AtomRec A = load_uniform(K.atoms + W->atom);
  project_item<NU>(K, tab, W, A, psi, c, cacc);
}

template <int NUMAX, bool CPLX = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(waves_per_eu(NUMAX + 1)))) void k_project_any(
    KArgs K, const float *__restrict__ tab, const Pair *__restrict__ psi,
    Pair *__restrict__ c) {
  extern __shared__ double cacc[];
  const cptr<WorkRec> W = as_const(K.work) + blockIdx.x;
  if (W->atom < 0) return;
  const AtomRec A = load_uniform(K.atoms + W->atom);
  switch (A.nu) {
#define X(N)                                                                 \
  case N:                                                                    \
    if constexpr (N <= NUMAX) project_item<N, CPLX>(K, tab, W, A, psi, c, cacc); \
    break;
    SHO_F32_NU_CASES(X)
#undef X
  }
}

// ------------------------------------------------------------- expansion --

constexpr int kU2Tile = 32;  // band pairs per plane-partial workgroup

// Plane partials U2[jz][q][pair] = sum_nz phi_nz(z_jz) C[nx,ny,nz][pair].
template <int NU>
__global__ __launch_bounds__(256) void k_u2(EArgs E, const float *__restrict__ tab,
                                            const Pair *__restrict__ c,
                                            Pair *__restrict__ u2) {
  constexpr int NF = NU + 1;
  constexpr int NS = NF * (NF + 1) * (NF + 2) / 6;
  constexpr int NP = NF * (NF + 1) / 2;
  __shared__ Pair cs[NS * kU2Tile];
  const int a = E.nu_atoms[E.nu_begin[NU] + blockIdx.x];
  const AtomRec A = load_uniform(E.atoms + a);
  const int b0 = blockIdx.y * kU2Tile;
  {
    constexpr int U = 8;
    const int count = NS * kU2Tile;
    for (int t0 = 0; t0 < count; t0 += U * (int)blockDim.x) {
      Pair v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * (int)blockDim.x + (int)threadIdx.x;
        const int n = t / kU2Tile, bl = t % kU2Tile;
        v[u] = (t < count && b0 + bl < E.B) ? c[(A.coeff_row + n) * E.B + b0 + bl] : zero2();
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * (int)blockDim.x + (int)threadIdx.x;
        if (t < count) cs[t] = v[u];
      }
    }
  }
  __syncthreads();
  const float *tz = tab + A.tab_off + (int64_t)(A.mx + A.my) * A.tab_nfp;
  Pair *dst = u2 + E.u2_off[a];
  for (int t = threadIdx.x; t < A.mz * kU2Tile; t += blockDim.x) {
    const int bl = t % kU2Tile;
    const int jz = t / kU2Tile;
    if (b0 + bl >= E.B) continue;
    float fz[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) fz[n] = tz[(int64_t)jz * A.tab_nfp + n];
    Pair *out = dst + (int64_t)jz * NP * E.B + b0 + bl;
    int q = 0;
#pragma unroll
    for (int ny = 0; ny < NF; ++ny) {
#pragma unroll
      for (int nx = 0; nx < NF - ny; ++nx, ++q) {
        Pair acc = zero2();
#pragma unroll
        for (int nz = 0; nz < NF; ++nz) {
          if (nx + ny + nz <= NU) {
            // coefficient order: nz-major, then ny, nx fastest
            int base = 0;
#pragma unroll
            for (int k = 0; k < nz; ++k) base += (NU - k + 1) * (NU - k + 2) / 2;
#pragma unroll
            for (int j = 0; j < ny; ++j) base += NU - nz - j + 1;
            acc = fma2(fz[nz], cs[(base + nx) * kU2Tile + bl], acc);
          }
        }
        out[(int64_t)q * E.B] = acc;
      }
    }
  }
}

constexpr int kBlkWaves = 4;
constexpr int kBlkBlock = 64 * kBlkWaves;
constexpr int kBlkXStage = 256;  // floats per wave: the x-table rows of a block

constexpr int blk_group(int nu, int numax) { return (numax > 5 && nu <= 5) ? 4 : 2; }

// Adds every run of one entry (one atom plane, one image) into the LDS tile
// of the block ([row][x][2][TB] doubles).
template <int NU, int NUMAX, bool CPLX = false>
__device__ inline void add_entry(const EArgs &E, const float *tab, const EntryRec &en, int ei,
                                 const Pair *u2, int nxl, double *tile, float *xstage,
                                 int TB, int slot, int bl, int bc) {
  constexpr int NF = NU + 1;
  constexpr int NP = NF * (NF + 1) / 2;
  constexpr int G = blk_group(NU, NUMAX);
  const int nfp = en.nfp;
  const int lane = threadIdx.x & 63;
  const int slots = 64 / TB;
  const Pair *ub = u2 + en.u2 + bc;
  Pair u2v[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) u2v[q] = ub[(int64_t)q * E.B];
  if constexpr (CPLX) {
    // the entry's image T receives e^{-i k.T} times the plane partials
    const cptr<double> ph = as_const(E.entry_phase) + 2 * ei;
    const double cs = ph[0], sn = ph[1];
#pragma unroll
    for (int q = 0; q < NP; ++q) u2v[q] = rotate(u2v[q], (float)cs, -(float)sn);
  }
  const uint32_t mydesc = lane < en.nruns ? as_const(E.run_desc)[en.run_begin + lane] : 0u;
  float tx[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = lane * 4 + k;
    const int pt = i / nfp;
    tx[k] = (pt >= en.x_lo && pt < en.x_hi) ? tab[en.tab_x + i] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) xstage[lane * 4 + k] = tx[k];
  for (int g0 = 0; g0 < en.nruns; g0 += G * slots) {
    const int gend = min(g0 + G * slots, en.nruns);
    int lo = 255, hi = 0;
    for (int k = g0; k < gend; ++k) {
      const uint32_t d = __builtin_amdgcn_readlane(mydesc, k);
      lo = min(lo, (int)((d >> 8) & 0xff));
      hi = max(hi, (int)((d >> 16) & 0xff));
    }
    int rr[G], xa[G], xb[G];
    Pair U1[G][NF];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int i = g0 + j * slots + slot;
      const uint32_t d = __shfl(mydesc, min(i, gend - 1));
      rr[j] = d & 0xff;
      xa[j] = i < gend ? (int)((d >> 8) & 0xff) : 0;
      xb[j] = i < gend ? (int)((d >> 16) & 0xff) : 0;
      const float *fy = tab + en.tab_y + rr[j] * nfp;
#pragma unroll
      for (int n = 0; n < NF; ++n) U1[j][n] = zero2();
      int q = 0;
#pragma unroll
      for (int ny = 0; ny < NF; ++ny) {
        const float fv = fy[ny];
#pragma unroll
        for (int nx = 0; nx < NF - ny; ++nx, ++q) U1[j][nx] = fma2(fv, u2v[q], U1[j][nx]);
      }
    }
    for (int x = lo; x < hi; ++x) {
      const float *f = xstage + x * nfp;
      float fx[NF];
#pragma unroll
      for (int n = 0; n < NF; ++n) fx[n] = f[n];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        Pair val = zero2();
#pragma unroll
        for (int n = 0; n < NF; ++n) val = fma2(fx[n], U1[j][n], val);
        if (x >= xa[j] && x < xb[j]) {
          double *dst = tile + (((rr[j] * nxl + x) * TB) << 1) + bl;
          atomicAdd(dst, (double)val.a);
          atomicAdd(dst + TB, (double)val.b);
        }
      }
    }
  }
}

// One workgroup per (block, band-pair tile): the block's values of psi are
// read into LDS once (as doubles), every entry adds its runs, and the block
// is written back once, rounded to float.  A tile holds at most
// kBlockTileDoubles / 2 pairs, the LDS bytes of the FP64 tile, laid out as
// [row][X2][pair] (X2 the block width rounded up to a power of two) so that
// the fill and write-back split a slot with shifts and masks.
template <int NUMAX, bool CPLX = false>
__global__ __launch_bounds__(kBlkBlock) void k_expand_blocks(EArgs E,
                                                            const float *__restrict__ tab,
                                                            const Pair *__restrict__ u2,
                                                            Pair *psi) {
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
  const int nval = nrow << rs;  // pair slots, padding columns included
  const int64_t gbase = ((int64_t)(bk.z * E.ny + bk.y0) * E.nx + bk.x0) * E.B + btile * TB;
  const int64_t grow = (int64_t)E.nx * E.B;
  // slot t <-> psi index g; false past the grid's last column or for a
  // padding pair
  auto slot = [&](int64_t base, int t, int64_t &g) -> bool {
    const int r = t >> rs;
    const int x = (t >> E.tbe_shift) & ((1 << x2s) - 1);
    const int l = t & (TB - 1);
    g = base + r * grow + (int64_t)__umul24(x, E.B) + l;
    return x < nxl && btile * TB + l < E.B;
  };
  constexpr int kPer = kBlockTileDoubles / 2 / kBlkBlock;
  for (int t0 = 0; t0 < nval; t0 += kPer * kBlkBlock) {
    Pair v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      int64_t g = 0;
      v[u] = (t < nval && slot(gbase, t, g)) ? load_nt(psi + g) : zero2();
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      if (t < nval) {
        const int ia = t + (t & ~(TB - 1));
        tile[ia] = v[u].a;
        tile[ia + TB] = v[u].b;
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lslot = lane >> E.tbe_shift;
  const int bl = lane & (TB - 1);
  const int b = btile * TB + bl;
  const int bc = b < E.B ? b : E.B - 1;
  float *xstage = reinterpret_cast<float *>(lds + kBlockTileDoubles) + w * kBlkXStage;
  EntryRec en;
  if (w < bk.nentries) en = load_uniform(E.entries + bk.entry_begin + w);
  for (int i = w; i < bk.nentries; i += kBlkWaves) {
    EntryRec nxt = en;
    if (i + kBlkWaves < bk.nentries)
      nxt = load_uniform(E.entries + bk.entry_begin + i + kBlkWaves);
    switch (en.nu) {
#define X(N)                                                                        \
  case N:                                                                           \
    if constexpr (N <= NUMAX)                                                       \
      add_entry<N, NUMAX, CPLX>(E, tab, en, bk.entry_begin + i, u2, 1 << x2s, tile, xstage, TB, \
                                lslot, bl, bc);                                     \
    break;
      SHO_F32_NU_CASES(X)
#undef X
    }
    en = nxt;
  }
  __syncthreads();
  // the write-back forms its addresses again (the base is made opaque)
  int64_t gb = gbase;
  asm volatile("" : "+s"(gb));
  for (int t0 = 0; t0 < nval; t0 += kPer * kBlkBlock) {
    Pair v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      const int ia = t + (t & ~(TB - 1));
      v[u] = t < nval ? Pair{(float)tile[ia], (float)tile[ia + TB]} : zero2();
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kBlkBlock + (int)threadIdx.x;
      int64_t g = 0;
      if (t < nval && slot(gb, t, g)) store_nt(v[u], psi + g);
    }
  }
}

static dim3 grid_of(const KArgs &K) { return dim3((unsigned)K.nwork, (unsigned)K.ntiles); }

template <int NU>
static hipError_t launch_project_nu(const KArgs &K, const float *tab, const Pair *psi,
                                    Pair *c, hipStream_t s) {
  const size_t shm = 2 * lds_tile_bytes(NU + 1, 1 << K.tb_shift);
  hipLaunchKernelGGL(k_project<NU>, grid_of(K), dim3(kBlock), shm, s, K, tab, psi, c);
  return hipGetLastError();
}

template <int NUMAX>
static hipError_t launch_project_any_nu(const KArgs &K, const float *tab, const Pair *psi,
                                        Pair *c, hipStream_t s) {
  const size_t shm = 2 * lds_tile_bytes(NUMAX + 1, 1 << K.tb_shift);
  if (K.bloch)
    hipLaunchKernelGGL((k_project_any<NUMAX, true>), grid_of(K), dim3(kBlock), shm, s, K, tab,
                       psi, c);
  else
    hipLaunchKernelGGL((k_project_any<NUMAX, false>), grid_of(K), dim3(kBlock), shm, s, K, tab,
                       psi, c);
  return hipGetLastError();
}

}  // namespace f32

using f32::Pair;

hipError_t launch_tables_f32(const double *tab, float *tab32, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(f32::k_round_tables, dim3((unsigned)blocks), dim3(256), 0, s, tab,
                     tab32, n);
  return hipGetLastError();
}

hipError_t launch_project_f32(int nu, const KArgs &K, const float *tab, const float *psi,
                              float *c, hipStream_t s) {
  if (K.nwork <= 0) return hipSuccess;
  if (K.bloch) return hipErrorInvalidValue;  // Bloch plans run k_project_any
  const Pair *pp = reinterpret_cast<const Pair *>(psi);
  Pair *cp = reinterpret_cast<Pair *>(c);
  switch (nu) {
#define X(N) case N: return f32::launch_project_nu<N>(K, tab, pp, cp, s);
    SHO_F32_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_project_any_f32(int nu_max, const KArgs &K, const float *tab,
                                  const float *psi, float *c, hipStream_t s) {
  if (K.nwork <= 0) return hipSuccess;
  const Pair *pp = reinterpret_cast<const Pair *>(psi);
  Pair *cp = reinterpret_cast<Pair *>(c);
  switch (nu_max) {
#define X(N) case N: return f32::launch_project_any_nu<N>(K, tab, pp, cp, s);
    SHO_F32_NU_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand_planes_f32(const EArgs &E, const float *tab, const float *c,
                                    float *u2, hipStream_t s) {
  const Pair *cp = reinterpret_cast<const Pair *>(c);
  Pair *up = reinterpret_cast<Pair *>(u2);
  for (int nu = 0; nu <= SHO_NU_MAX; ++nu) {
    const int cnt = E.nu_begin[nu + 1] - E.nu_begin[nu];
    if (cnt <= 0) continue;
    const dim3 g((unsigned)cnt, (unsigned)E.ntiles_u2);
    switch (nu) {
#define X(N)                                                                  \
  case N:                                                                     \
    hipLaunchKernelGGL(f32::k_u2<N>, g, dim3(256), 0, s, E, tab, cp, up);     \
    break;
      SHO_F32_NU_CASES(X)
#undef X
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_blocks_f32(const EArgs &E, const float *tab, const float *u2, float *psi,
                             hipStream_t s) {
  if (E.nblocks > 0) {
    const Pair *up = reinterpret_cast<const Pair *>(u2);
    Pair *pp = reinterpret_cast<Pair *>(psi);
    const dim3 g((unsigned)E.nblocks, (unsigned)E.ntiles);
    const size_t shm =
        kBlockTileDoubles * sizeof(double) + f32::kBlkWaves * f32::kBlkXStage * sizeof(float);
    switch (E.nu_max) {
#define X(N)                                                                             \
  case N:                                                                                \
    if (E.bloch)                                                                         \
      hipLaunchKernelGGL((f32::k_expand_blocks<N, true>), g, dim3(f32::kBlkBlock), shm, s, E, \
                         tab, up, pp);                                                   \
    else                                                                                 \
      hipLaunchKernelGGL((f32::k_expand_blocks<N, false>), g, dim3(f32::kBlkBlock), shm, s, E, \
                         tab, up, pp);                                                   \
    break;
      SHO_F32_NU_CASES(X)
#undef X
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace sho
