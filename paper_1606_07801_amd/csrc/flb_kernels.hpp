// Kernels of one lattice: the fused stream-collide step (two variants that
// give bit-identical results), conversion between the stored and the
// canonical state, lattice sums, structure factor and the noise sampler.
//
// Storage (two-buffer pull scheme).  A buffer holds the post-collision
// populations of the previous step at their collision site,
//   g_i(x) = f_i*(x, t - 1),  so that  f_i(x, t) = g_i(x - v_i)
// (eq. LB).  A step gathers g_i(x - v_i) at every site x, which yields the
// pre-collision populations of x, collides them at x (site index and step
// key the noise) and stores the result at x in the other buffer.  Loads are
// unit-stride rows shifted by at most one element; stores are aligned.
#pragma once

#include "flb_device.hpp"

namespace flb {

// Neighbour offsets of a site for the pull gather, periodic in every axis.
struct Nbr {
  int64_t s, sxm, sxp, sym, syp, szm, szp;
};

__device__ __forceinline__ Nbr neighbours(int64_t x, int64_t y, int64_t z, int64_t nx, int64_t ny,
                                          int64_t nz) {
  const int64_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int64_t ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int64_t zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const int64_t row = nx * (y + ny * z);
  Nbr r;
  r.s = row + x;
  r.sxm = row + xm;
  r.sxp = row + xp;
  r.sym = nx * (ym + ny * z) + x;
  r.syp = nx * (yp + ny * z) + x;
  r.szm = nx * (y + ny * zm) + x;
  r.szp = nx * (y + ny * zp) + x;
  return r;
}

// Forms in which a state is stored (plane i holds n values, x fastest):
//   kFormPull  two-buffer storage: g_i(x) = f_i*(x, t - 1), so f_i(x, t) = g_i(x - v_i)
//   kFormAAC   single buffer after an even number of steps: A_i(x) = f_i(x, t)
//   kFormAAS   single buffer after an odd number: A_opp(i)(x) = f_i*(x, t - 1), so
//              f_i(x, t) = A_opp(i)(x - v_i), opp(i) the population moving the other way
// One AA step from form C collides every site in place and stores f_i* in the
// opposite slot (form S); one from form S gathers f_i(x) = A_opp(i)(x - v_i),
// collides and stores f_i* at A_i(x + v_i) (form C).  In both, the slots a
// site writes are exactly the slots it read, so a step runs in place.
enum StateForm : int { kFormPull = 0, kFormAAC = 1, kFormAAS = 2 };

// f_i(x, t) of one site from its stored state
template <int D, typename T>
__device__ __forceinline__ void gather(const T* __restrict__ g, int64_t n, const Nbr& b,
                                       T (&f)[2 * D + 1], int form = kFormPull) {
  if (form == kFormAAC) {
#pragma unroll
    for (int i = 0; i < 2 * D + 1; ++i) f[i] = g[i * n + b.s];
    return;
  }
  const bool sw = form == kFormAAS;  // plane of population i: opp(i)
  f[0] = g[b.s];
  f[1] = g[(sw ? 2 : 1) * n + b.sxm];
  f[2] = g[(sw ? 1 : 2) * n + b.sxp];
  if constexpr (D >= 2) {
    f[3] = g[(sw ? 4 : 3) * n + b.sym];
    f[4] = g[(sw ? 3 : 4) * n + b.syp];
  }
  if constexpr (D >= 3) {
    f[5] = g[(sw ? 6 : 5) * n + b.szm];
    f[6] = g[(sw ? 5 : 6) * n + b.szp];
  }
}

// ---------------------------------------------------------------------------
// Plain step: one site per thread, flat site index.  The reference variant.
template <int D, typename T>
__global__ void __launch_bounds__(256) k_step_plain(const T* __restrict__ g, T* __restrict__ h,
                                                    KParams<T> P, uint32_t step) {
  constexpr int Q = 2 * D + 1;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P.n) return;
  const int64_t x = s % P.nx;
  const int64_t rest = s / P.nx;
  const int64_t y = rest % P.ny;
  const int64_t z = rest / P.ny;
  const Nbr b = neighbours(x, y, z, P.nx, P.ny, P.nz);
  T f[Q];
  gather<D, T>(g, P.n, b, f);
  Collide<D, T>::run(f, P, (uint64_t)s, step);
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i * P.n + s] = f[i];
}

// Step of a lattice whose temperature and rates vary by region: site s
// collides with the constants of region[s] (a table of at most 16 entries,
// staged in LDS), streaming as in k_step_plain.
constexpr int kMaxRegions = 16;

template <int D, typename T>
__global__ void __launch_bounds__(256) k_step_regions(const T* __restrict__ g, T* __restrict__ h,
                                                      const KParams<T>* __restrict__ ptab, int nreg,
                                                      const uint8_t* __restrict__ region, int64_t n,
                                                      uint32_t step) {
  constexpr int Q = 2 * D + 1;
  __shared__ KParams<T> tab[kMaxRegions];
  for (int r = threadIdx.x; r < nreg; r += blockDim.x) tab[r] = ptab[r];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const KParams<T>& P = tab[region[s]];
  const int64_t x = s % P.nx;
  const int64_t rest = s / P.nx;
  const int64_t y = rest % P.ny;
  const int64_t z = rest / P.ny;
  const Nbr b = neighbours(x, y, z, P.nx, P.ny, P.nz);
  T f[Q];
  gather<D, T>(g, n, b, f);
  Collide<D, T>::run(f, P, (uint64_t)s, step);
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i * n + s] = f[i];
}

// Map a linear block index so that the blocks the dispatcher sends to one
// XCD (round-robin over 8) cover one contiguous range of tiles, keeping the
// shared halo lines of neighbouring tiles in one L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
  const int64_t q = G / 8, r = G % 8;
  const int64_t xcd = b % 8, k = b / 8;
  return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

template <int D, typename T, int RY, bool NT, int NP = kPlanRuntime>
__device__ __forceinline__ void flat_tile(const T* __restrict__ g, T* __restrict__ h,
                                          const KParams<T>& P, uint32_t step, int64_t s0,
                                          uint32_t lane);

// Flat step: block b covers sites b * 256 * RY ... (flat_tile).  Blocks keep
// the dispatcher's round-robin XCD placement: an XCD-contiguous assignment
// saved the halo re-fetches at tile edges (2.5 % of the reads) but measured
// slower, the concurrently active tiles then spreading over 8 distant ranges.
// NP: the noise plan (kPlanLocalGauss fixes local Gaussian noise at compile
// time; the same arithmetic, so the same bits).
template <int D, typename T, int RY, bool NT, int NP = kPlanRuntime>
__global__ void __launch_bounds__(256) k_step_flat(const T* __restrict__ g, T* __restrict__ h,
                                                   KParams<T> P, uint32_t step) {
  flat_tile<D, T, RY, NT, NP>(g, h, P, step, (int64_t)blockIdx.x * 256 * RY, threadIdx.x);
}

// Element at a 32-bit byte offset from a block-uniform base pointer: the
// base lives in scalar registers and the access needs no 64-bit vector
// address arithmetic.
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, uint32_t byte_off) {
  return *(const T*)((const char*)base + byte_off);
}
template <typename T, bool NT>
__device__ __forceinline__ void st_at(T* __restrict__ base, uint32_t byte_off, T v) {
  T* p = (T*)((char*)base + byte_off);
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Raw buffer access to a whole population array (Q planes of n values,
// Q n S < 2^32 bytes): a per-lane byte offset plus a uniform byte offset
// (plane and row) that stays in a scalar register, so the address needs no
// vector arithmetic.  0x00020000: the resource word of the gfx9 family for
// untyped 32-bit access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// NT: the non-temporal hint (cache-policy bit 1)
template <bool NT>
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, NT ? 2 : 0);
}

// Row step: a block covers blockDim.x consecutive x of RY consecutive rows
// (row = y + ny z); each thread owns one column of the tile.  All RY rows'
// populations are loaded before any is collided, so that every wave keeps
// RY * Q loads in flight; NT selects non-temporal stores (the new state is
// not re-read within this launch).
// Pre-collision populations of column x, row `row` (the pull gather).
template <int D, typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ g, const KParams<T>& P, int64_t row,
                                         uint32_t bx, uint32_t bxm, uint32_t bxp, T (&f)[2 * D + 1]) {
  const int64_t n = P.n;
  const uint32_t nx = (uint32_t)P.nx;
  const int64_t base = row * (int64_t)nx;
  f[0] = ld_at(g + base, bx);
  f[1] = ld_at(g + n + base, bxm);
  f[2] = ld_at(g + 2 * n + base, bxp);
  if constexpr (D >= 2) {
    uint32_t y, z;
    if constexpr (D == 2) {
      y = (uint32_t)row;
      z = 0;
    } else {
      y = (uint32_t)row % (uint32_t)P.ny;
      z = (uint32_t)row / (uint32_t)P.ny;
    }
    const uint32_t ny = (uint32_t)P.ny;
    const uint32_t ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    f[3] = ld_at(g + 3 * n + ((int64_t)ym + (int64_t)ny * z) * nx, bx);
    f[4] = ld_at(g + 4 * n + ((int64_t)yp + (int64_t)ny * z) * nx, bx);
    if constexpr (D >= 3) {
      const uint32_t nz = (uint32_t)P.nz;
      const uint32_t zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
      f[5] = ld_at(g + 5 * n + ((int64_t)y + (int64_t)ny * zm) * nx, bx);
      f[6] = ld_at(g + 6 * n + ((int64_t)y + (int64_t)ny * zp) * nx, bx);
    }
  }
}

// Software-pipelined rows: the next row's loads are in flight while the
// current row is collided and stored (RY rows per thread).
template <int D, typename T, int RY, bool NT>
__device__ __forceinline__ void rows_tile_pipe(const T* __restrict__ g, T* __restrict__ h,
                                               const KParams<T>& P, uint32_t step, uint32_t x,
                                               int64_t row0, int64_t nrows) {
  constexpr int Q = 2 * D + 1;
  const uint32_t nx = (uint32_t)P.nx;
  if (x >= nx) return;
  constexpr uint32_t S = sizeof(T);
  const uint32_t bx = x * S;
  const uint32_t bxm = (x == 0 ? nx - 1 : x - 1) * S, bxp = (x == nx - 1 ? 0 : x + 1) * S;
  const int64_t rend = row0 + RY < nrows ? row0 + RY : nrows;
  if (row0 >= rend) return;
  T cur[Q];
  load_row<D, T>(g, P, row0, bx, bxm, bxp, cur);
  for (int64_t row = row0; row < rend; ++row) {
    T nxt[Q];
    const bool more = row + 1 < rend;
    if (more) load_row<D, T>(g, P, row + 1, bx, bxm, bxp, nxt);
    const int64_t base = row * (int64_t)nx;
    Collide<D, T>::run(cur, P, (uint64_t)base + x, step);
#pragma unroll
    for (int i = 0; i < Q; ++i) st_at<T, NT>(h + i * P.n + base, bx, cur[i]);
    if (more) {
#pragma unroll
      for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
  }
}

// Flat-order offsets of one site of a flat tile: the site and its periodic
// neighbours along each axis (sxm = the site at x - 1, and so on), all as
// 32-bit site indices.
struct FlatSite {
  uint32_t s, sxm, sxp, sym, syp, szm, szp;
};

// Coordinates of a flat tile's first site, uniform over the workgroup (scalar
// unit).  When a row holds at least the tile's 256 RY sites a lane crosses at
// most one row end, so its coordinates follow by one compare instead of a
// per-lane division (quarter-rate integer multiplies).
struct FlatOrigin {
  uint32_t nx, ny, nz, n, nxy, x0, r0, y0, z0;
  bool wide;
};

template <int D, int RY, typename T>
__device__ __forceinline__ FlatOrigin flat_origin(const KParams<T>& P, uint32_t s0u) {
  FlatOrigin o;
  o.nx = (uint32_t)P.nx;
  o.ny = (uint32_t)P.ny;
  o.nz = (uint32_t)P.nz;
  o.n = (uint32_t)P.n;  // n * S < 2^32 (checked by the caller)
  o.nxy = o.nx * o.ny;
  o.x0 = s0u % o.nx;
  o.r0 = s0u / o.nx;
  o.y0 = D == 3 ? o.r0 % o.ny : o.r0;
  o.z0 = D == 3 ? o.r0 / o.ny : 0;
  o.wide = o.nx >= 256u * RY;
  return o;
}

// The site s = s0 + off of the tile (s < n).
template <int D>
__device__ __forceinline__ FlatSite flat_site(const FlatOrigin& o, uint32_t s, uint32_t off) {
  uint32_t x, rest, yw = 0, zw = 0;
  if (o.wide) {
    x = o.x0 + off;
    const uint32_t c = x >= o.nx ? 1u : 0u;
    x -= c ? o.nx : 0u;
    rest = o.r0 + c;
    if constexpr (D == 3) {
      yw = o.y0 + c;
      const uint32_t c2 = yw >= o.ny ? 1u : 0u;
      yw -= c2 ? o.ny : 0u;
      zw = o.z0 + c2;
    }
  } else {
    x = s % o.nx;
    rest = s / o.nx;
    if constexpr (D == 3) {
      yw = rest % o.ny;
      zw = rest / o.ny;
    }
  }
  FlatSite f;
  f.s = s;
  f.sxm = x == 0 ? s + o.nx - 1 : s - 1;
  f.sxp = x == o.nx - 1 ? s + 1 - o.nx : s + 1;
  f.sym = f.syp = f.szm = f.szp = s;
  if constexpr (D >= 2) {
    const uint32_t y = D == 2 ? rest : yw;
    f.sym = y == 0 ? s + o.nxy - o.nx : s - o.nx;
    f.syp = y == o.ny - 1 ? s + o.nx - o.nxy : s + o.nx;
  }
  if constexpr (D >= 3) {
    const uint32_t z = zw;
    f.szm = z == 0 ? s + o.n - o.nxy : s - o.nxy;
    f.szp = z == o.nz - 1 ? s + o.nxy - o.n : s + o.nxy;
  }
  return f;
}

// Flat tile: RY blocks of 256 consecutive sites s0 + j * 256 + lane of the
// row-major site order, so a lattice's sites fill every lane except in its
// last tile.  Each lane derives (x, y, z) and its periodic neighbours
// itself; all offsets are 32-bit byte offsets from the plane bases.
template <int D, typename T, int RY, bool NT, int NP>
__device__ __forceinline__ void flat_tile(const T* __restrict__ g, T* __restrict__ h,
                                          const KParams<T>& P, uint32_t step, int64_t s0,
                                          uint32_t lane) {
  constexpr int Q = 2 * D + 1;
  constexpr uint32_t S = sizeof(T);
  const FlatOrigin o = flat_origin<D, RY>(P, (uint32_t)s0);
  const uint32_t n = o.n;
  T f[RY][Q];
  uint32_t sj[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const uint32_t off = (uint32_t)j * 256u + lane;
    const uint32_t s = (uint32_t)s0 + off;
    sj[j] = s;
    if (s < n) {
      const FlatSite b = flat_site<D>(o, s, off);
      f[j][0] = ld_at(g, s * S);
      f[j][1] = ld_at(g + n, b.sxm * S);
      f[j][2] = ld_at(g + 2 * (int64_t)n, b.sxp * S);
      if constexpr (D >= 2) {
        f[j][3] = ld_at(g + 3 * (int64_t)n, b.sym * S);
        f[j][4] = ld_at(g + 4 * (int64_t)n, b.syp * S);
      }
      if constexpr (D >= 3) {
        f[j][5] = ld_at(g + 5 * (int64_t)n, b.szm * S);
        f[j][6] = ld_at(g + 6 * (int64_t)n, b.szp * S);
      }
    }
  }
  // stores through a buffer resource: the plane offsets stay scalar
  const __amdgpu_buffer_rsrc_t rh = buf_rsrc(h, (uint32_t)Q * n * S);
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    if (sj[j] < n) {
      Collide<D, T, NP>::run(f[j], P, (uint64_t)sj[j], step);
#pragma unroll
      for (int i = 0; i < Q; ++i) buf_st<NT>(f[j][i], rh, sj[j] * S, (uint32_t)i * n * S);
    }
  }
}

// Plane of the AA single buffer that population i of a site reads in form
// FORM, and the neighbour offset it reads at; the step then writes the
// population's post-collision value to the plane and offset of opp(i)'s read
// (form C -> S: the opposite plane at the site; form S -> C: plane i at the
// neighbour x + v_i), so every site writes exactly the slots it read.
template <int D>
__device__ __forceinline__ uint32_t aa_read_off(const FlatSite& b, int i, int form) {
  if (form == kFormAAC) return b.s;
  switch (i) {
    case 1: return b.sxm;
    case 2: return b.sxp;
    case 3: return b.sym;
    case 4: return b.syp;
    case 5: return b.szm;
    case 6: return b.szp;
    default: return b.s;
  }
}

__device__ __forceinline__ int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// One AA step of a flat tile in place on the single buffer a: from form
// kFormAAC (even parity) to kFormAAS, or from kFormAAS to kFormAAC.  The
// collisions are those of flat_tile on the same pre-collision values.
template <int D, typename T, int RY, bool NT, int FORM, int NP = kPlanRuntime>
__device__ __forceinline__ void flat_tile_aa(T* a, const KParams<T>& P, uint32_t step, int64_t s0, uint32_t lane) {
  constexpr int Q = 2 * D + 1;
  constexpr uint32_t S = sizeof(T);
  const FlatOrigin o = flat_origin<D, RY>(P, (uint32_t)s0);
  const uint32_t n = o.n;
  T f[RY][Q];
  FlatSite bj[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const uint32_t off = (uint32_t)j * 256u + lane;
    const uint32_t s = (uint32_t)s0 + off;
    bj[j].s = s;
    if (s < n) {
      bj[j] = flat_site<D>(o, s, off);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int pl = FORM == kFormAAC ? i : opp(i);
        f[j][i] = ld_at((const T*)a + pl * (int64_t)n, aa_read_off<D>(bj[j], i, FORM) * S);
      }
    }
  }
  const __amdgpu_buffer_rsrc_t ra = buf_rsrc(a, (uint32_t)Q * n * S);
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    if (bj[j].s < n) {
      Collide<D, T, NP>::run(f[j], P, (uint64_t)bj[j].s, step);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        // f_i* goes where opp(i) was read
        const int pl = FORM == kFormAAC ? opp(i) : i;
        buf_st<NT>(f[j][i], ra, aa_read_off<D>(bj[j], opp(i), FORM) * S, (uint32_t)pl * n * S);
      }
    }
  }
}

template <int D, typename T, int RY, bool NT, int FORM, int NP = kPlanRuntime>
__global__ void __launch_bounds__(256) k_step_flat_aa(T* a, KParams<T> P, uint32_t step) {
  flat_tile_aa<D, T, RY, NT, FORM, NP>(a, P, step, (int64_t)blockIdx.x * 256 * RY, threadIdx.x);
}

// Sum over the 64 lanes of a wave with DPP lane moves (no LDS): quad swaps,
// half-row and row mirrors leave every lane with its 16-lane row sum (the
// same bits in all 16 lanes, the additions being commutative pairwise); the
// four row sums are read from lanes 0, 16, 32, 48 and added in that order.
// A fixed order, so the result does not depend on scheduling; all 64 lanes
// must be active.  The result is uniform across the wave.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Every lane's 16-lane row sum (the first half of wave_sum_fixed).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

__device__ __forceinline__ double wave_sum_fixed(double v) {
  v = row16_sum(v);
  return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// Sum of a row of 256 lanes from its sixteen 16-lane row sums p[0..15], in
// the order of wave_sum_fixed per wave, then the four waves in order.
__device__ __forceinline__ double sum256_from_rows16(const double* p) {
  const double w0 = ((p[0] + p[1]) + p[2]) + p[3], w1 = ((p[4] + p[5]) + p[6]) + p[7];
  const double w2 = ((p[8] + p[9]) + p[10]) + p[11], w3 = ((p[12] + p[13]) + p[14]) + p[15];
  return ((w0 + w1) + w2) + w3;
}

// Two D2Q5 steps per pass (temporal blocking).  A workgroup of TW lanes
// (TW = 256 for single lattices; 128 or 64 leave fewer lanes idle on the
// uneven widths of an ensemble) owns the
// columns x0 .. x0 + w - 1 (w <= TW, one per lane) of the rows r0 .. r0 + hr - 1
// (hr <= TY).  Step t: every lane collides its column for the rows r0 - 1 ..
// r0 + hr (the owned rows plus one halo row on each side, periodic), and a
// few lanes of wave 0 collide the halo columns x0 - 1 and x0 + w for the
// owned rows.  Post-collision populations that move along x (f*_1 to the
// right, f*_2 to the left) go through LDS; those moving along y stay in the
// lane's registers.  Step t + 1: each owned site gathers
//   f_0 = f*_0(x, r), f_1 = f*_1(x - 1, r), f_2 = f*_2(x + 1, r),
//   f_3 = f*_3(x, r - 1), f_4 = f*_4(x, r + 1)
// collides with the noise of step t + 1 and stores in the storage form.
// Every collision is the per-site code of the one-step kernels on the same
// inputs, so the result is bit-identical to two single steps; halo sites are
// computed by more than one workgroup.  HBM traffic per two steps: reads
// 5 (TY + 2) / TY and writes 5 per site, against 10 and 10.
// SAMPLE: the pass also writes the FP64 density partials of the state at t
// (the input of the axis structure factor), with the layout and the
// reduction order of k_step_rows_sk for tiles of TY rows:
//   rowpart[tx * nrows + row] = sum over the tile's columns of rho(x, row)
//   colpart[ty * nx + x]      = sum over the tile's rows of rho(x, row)
template <typename T, int TY, bool NT, bool SAMPLE, int TW = 256, int NP = kPlanRuntime>
__device__ __forceinline__ void step2_tile(const T* __restrict__ g, T* __restrict__ h, const KParams<T>& P,
                                           uint32_t step, uint32_t tx, uint32_t ty,
                                           double* __restrict__ rowpart, double* __restrict__ colpart) {
  static_assert(TW == 64 || TW == 128 || TW == 256, "tile widths of 1, 2 or 4 waves");
  static_assert(2 * TY <= TW, "the halo lanes are lanes 0 .. 2 TY - 1");
  static_assert(!SAMPLE || TW == 256, "the density partials use the 256-column tiles of the sampled step");
  constexpr int Q = 5;
  constexpr uint32_t S = sizeof(T);
  __shared__ T l1[TY][TW + 2], l2[TY][TW + 2];  // [row][1 + lane]; 0: left halo (f*_1), TW + 1: right halo (f*_2)
  __shared__ double red16[SAMPLE ? TY : 1][16];  // per row, the sixteen 16-lane sums
  const uint32_t nx = (uint32_t)P.nx, ny = (uint32_t)P.ny, n = (uint32_t)P.n;
  const int lane = threadIdx.x;
  const uint32_t x0 = tx * (uint32_t)TW, r0 = ty * (uint32_t)TY;
  const int w = (int)(nx - x0 < (uint32_t)TW ? nx - x0 : (uint32_t)TW);
  const int hr = (int)(ny - r0 < (uint32_t)TY ? ny - r0 : (uint32_t)TY);
  // one collision of step t at (x, r) from the storage form g; *rho receives
  // the pre-collision density when asked for
  auto first = [&](uint32_t x, uint32_t r, T (&f)[Q], double* rho) {
    const uint32_t row = r * nx;
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const uint32_t rm = (r == 0 ? ny - 1 : r - 1) * nx, rp = (r == ny - 1 ? 0 : r + 1) * nx;
    f[0] = ld_at(g, (row + x) * S);
    f[1] = ld_at(g + n, (row + xm) * S);
    f[2] = ld_at(g + 2 * (int64_t)n, (row + xp) * S);
    f[3] = ld_at(g + 3 * (int64_t)n, (rm + x) * S);
    f[4] = ld_at(g + 4 * (int64_t)n, (rp + x) * S);
    if (rho) *rho = density_sum(f);
    Collide<2, T, NP>::run(f, P, (uint64_t)(row + x), step);
  };
  T fs[TY + 2][Q];
  const bool own = lane < w;
  const uint32_t xo = x0 + (uint32_t)(own ? lane : 0);
  // The owned columns' loads and stores go through buffer resources: the
  // column offsets per lane, the plane and row offsets in scalar registers
  // (3 % faster than 64-bit vector addresses; the halo columns, whose rows
  // differ per lane, keep the loads of `first`)
  const uint32_t nS = n * S;
  const __amdgpu_buffer_rsrc_t rg = buf_rsrc(g, 5u * nS), rh = buf_rsrc(h, 5u * nS);
  const uint32_t vx = xo * S, vxm = (xo == 0 ? nx - 1 : xo - 1) * S, vxp = (xo == nx - 1 ? 0 : xo + 1) * S;
  auto first_buf = [&](uint32_t r, T (&f)[Q], double* rho) {
    const uint32_t so = r * nx * S;
    const uint32_t sm = (r == 0 ? ny - 1 : r - 1) * nx * S, sp = (r == ny - 1 ? 0 : r + 1) * nx * S;
    f[0] = buf_ld<T>(rg, vx, so);
    f[1] = buf_ld<T>(rg, vxm, nS + so);
    f[2] = buf_ld<T>(rg, vxp, 2 * nS + so);
    f[3] = buf_ld<T>(rg, vx, 3 * nS + sm);
    f[4] = buf_ld<T>(rg, vx, 4 * nS + sp);
    if (rho) *rho = density_sum(f);
    Collide<2, T, NP>::run(f, P, (uint64_t)(r * nx + xo), step);
  };
  double col = 0;
#pragma unroll
  for (int k = 0; k < TY + 2; ++k) {
    double rho = 0;
    if (own && k <= hr + 1) {
      const int rr = (int)r0 - 1 + k;  // -1 .. r0 + hr
      const uint32_t r = rr < 0 ? (uint32_t)(rr + (int)ny) : ((uint32_t)rr >= ny ? (uint32_t)rr - ny : (uint32_t)rr);
      first_buf(r, fs[k], (SAMPLE && k >= 1 && k <= hr) ? &rho : nullptr);
      // the x-moving populations of owned rows go to LDS at once: the lane
      // keeps only f*_0, f*_3, f*_4 of its rows for the second step
      if (k >= 1 && k <= hr) {
        l1[k - 1][1 + lane] = fs[k][1];
        l2[k - 1][1 + lane] = fs[k][2];
      }
    }
    if constexpr (SAMPLE) {
      if (k >= 1 && k <= TY) {  // owned row k - 1: column sum in row order, row sum over the lanes
        if (k <= hr) col += rho;
        const double v = row16_sum(rho);  // every lane (0 where none)
        if ((lane & 15) == 0) red16[k - 1][lane >> 4] = v;
      }
    }
  }
  if constexpr (SAMPLE) {
    if (own) colpart[(int64_t)ty * nx + xo] = col;
  }

  if (lane < 2 * TY) {  // halo columns: lanes 0 .. TY-1 left (f*_1), TY .. 2TY-1 right (f*_2)
    const int k = lane < TY ? lane : lane - TY;
    if (k < hr) {
      const uint32_t xh = lane < TY ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + (uint32_t)w == nx ? 0 : x0 + (uint32_t)w);
      T fh[Q];
      first(xh, r0 + (uint32_t)k, fh, nullptr);
      if (lane < TY) l1[k][0] = fh[1];
      else l2[k][1 + w] = fh[2];
    }
  }
  __syncthreads();
  if constexpr (SAMPLE) {  // row partials: the 16-lane sums, per wave and then the waves, in order
    if (lane < TY && lane < hr) rowpart[(int64_t)tx * ny + r0 + lane] = sum256_from_rows16(red16[lane]);
  }
  if (!own) return;
  const uint32_t x = x0 + (uint32_t)lane;
#pragma unroll
  for (int k = 0; k < TY; ++k) {
    if (k < hr) {
      T f[Q];
      f[0] = fs[k + 1][0];
      f[1] = l1[k][lane];
      f[2] = l2[k][lane + 2];
      f[3] = fs[k][3];
      f[4] = fs[k + 2][4];
      const uint32_t s = (r0 + (uint32_t)k) * nx + x;
      Collide<2, T, NP>::run(f, P, (uint64_t)s, step + 1u);
#pragma unroll
      for (int i = 0; i < Q; ++i) buf_st<NT>(f[i], rh, vx, (uint32_t)i * nS + (r0 + (uint32_t)k) * nx * S);
    }
  }
}

template <typename T, int TY, bool NT, bool SAMPLE = false, int NP = kPlanRuntime>
__global__ void __launch_bounds__(256) k_step2_d2(const T* __restrict__ g, T* __restrict__ h,
                                                  KParams<T> P, uint32_t step, int tiles_x,
                                                  double* __restrict__ rowpart = nullptr,
                                                  double* __restrict__ colpart = nullptr) {
  step2_tile<T, TY, NT, SAMPLE, 256, NP>(g, h, P, step, blockIdx.x % (uint32_t)tiles_x,
                                         blockIdx.x / (uint32_t)tiles_x, rowpart, colpart);
}

// Column x of rows row0 .. row0 + RY - 1 (row0 is uniform over a wave).
template <int D, typename T, int RY, bool NT>
__device__ __forceinline__ void rows_tile(const T* __restrict__ g, T* __restrict__ h,
                                          const KParams<T>& P, uint32_t step, uint32_t x,
                                          int64_t row0, int64_t nrows) {
  constexpr int Q = 2 * D + 1;
  // the row tile and every plane/row base are uniform over the wave (scalar
  // registers); per lane only 32-bit column offsets remain
  const uint32_t nx = (uint32_t)P.nx;
  if (x >= nx) return;
  const int64_t n = P.n;
  constexpr uint32_t S = sizeof(T);
  const uint32_t bx = x * S;                                   // nx * S < 2^32
  const uint32_t bxm = (x == 0 ? nx - 1 : x - 1) * S, bxp = (x == nx - 1 ? 0 : x + 1) * S;
  T f[RY][Q];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int64_t row = row0 + r;
    if (row < nrows) {
      const int64_t base = row * (int64_t)nx;
      f[r][0] = ld_at(g + base, bx);
      f[r][1] = ld_at(g + n + base, bxm);
      f[r][2] = ld_at(g + 2 * n + base, bxp);
      if constexpr (D >= 2) {
        uint32_t y, z;
        if constexpr (D == 2) {
          y = (uint32_t)row;
          z = 0;
        } else {
          y = (uint32_t)row % (uint32_t)P.ny;
          z = (uint32_t)row / (uint32_t)P.ny;
        }
        const uint32_t ny = (uint32_t)P.ny;
        const uint32_t ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        f[r][3] = ld_at(g + 3 * n + ((int64_t)ym + (int64_t)ny * z) * nx, bx);
        f[r][4] = ld_at(g + 4 * n + ((int64_t)yp + (int64_t)ny * z) * nx, bx);
        if constexpr (D >= 3) {
          const uint32_t nz = (uint32_t)P.nz;
          const uint32_t zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
          f[r][5] = ld_at(g + 5 * n + ((int64_t)y + (int64_t)ny * zm) * nx, bx);
          f[r][6] = ld_at(g + 6 * n + ((int64_t)y + (int64_t)ny * zp) * nx, bx);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int64_t row = row0 + r;
    if (row < nrows) {
      const int64_t base = row * (int64_t)nx;
      Collide<D, T>::run(f[r], P, (uint64_t)base + x, step);
#pragma unroll
      for (int i = 0; i < Q; ++i) st_at<T, NT>(h + i * n + base, bx, f[r][i]);
    }
  }
}

template <int D, typename T, int RY, bool NT, bool PIPE = false>
__global__ void __launch_bounds__(1024) k_step_rows(const T* __restrict__ g, T* __restrict__ h,
                                                    KParams<T> P, uint32_t step, int64_t tiles_x,
                                                    int64_t nrows, int remap) {
  const int64_t G = (int64_t)gridDim.x;
  const int64_t tile = remap ? xcd_tile(blockIdx.x, G) : (int64_t)blockIdx.x;
  const int64_t tx = tile % tiles_x, tr = tile / tiles_x;
  const uint32_t x = (uint32_t)(tx * blockDim.x) + threadIdx.x;
  if constexpr (PIPE)
    rows_tile_pipe<D, T, RY, NT>(g, h, P, step, x, tr * RY, nrows);
  else
    rows_tile<D, T, RY, NT>(g, h, P, step, x, tr * RY, nrows);
}

// ---------------------------------------------------------------------------
// Canonical state <-> storage.
// out: f_i(x) = g_i(x - v_i);  in: g_i(x - v_i) = f_i(x).
template <int D, typename T>
__global__ void k_to_canonical(const T* __restrict__ g, T* __restrict__ f, int64_t nx, int64_t ny,
                               int64_t nz, int form = kFormPull) {
  constexpr int Q = 2 * D + 1;
  const int64_t n = nx * ny * nz;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const Nbr b = neighbours(x, y, z, nx, ny, nz);
    T v[Q];
    gather<D, T>(g, n, b, v, form);
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i * n + s] = v[i];
  }
}

template <int D, typename T>
__global__ void k_from_canonical(const T* __restrict__ f, T* __restrict__ g, int64_t nx, int64_t ny,
                                 int64_t nz) {
  const int64_t n = nx * ny * nz;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const Nbr b = neighbours(x, y, z, nx, ny, nz);
    g[b.s] = f[s];
    g[n + b.sxm] = f[n + s];
    g[2 * n + b.sxp] = f[2 * n + s];
    if constexpr (D >= 2) {
      g[3 * n + b.sym] = f[3 * n + s];
      g[4 * n + b.syp] = f[4 * n + s];
    }
    if constexpr (D >= 3) {
      g[5 * n + b.szm] = f[5 * n + s];
      g[6 * n + b.szp] = f[6 * n + s];
    }
  }
}

// ---------------------------------------------------------------------------
// The Gaussian map alone, on given words (2 x n in, 2 x n out).
template <typename T>
__global__ void k_gauss_map(const uint32_t* __restrict__ words, int64_t n, T* __restrict__ z) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  T z0, z1;
  gauss_pair(words[j], words[n + j], z0, z1);
  z[j] = z0;
  z[n + j] = z1;
}

// ---------------------------------------------------------------------------
// Noise sampler: Philox words and the unit variates a step would use.
template <int D, typename T>
__global__ void k_noise_sample(KParams<T> P, uint32_t step, int64_t site0, int64_t nsite,
                               uint32_t* __restrict__ words, T* __restrict__ vars) {
  constexpr int Q = 2 * D + 1;
  constexpr int NB = (Q - 1 + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsite) return;
  const uint64_t site = (uint64_t)(site0 + t);
#pragma unroll
  for (int bk = 0; bk < NB; ++bk) {
    uint32_t c0 = (uint32_t)site, c1 = (uint32_t)(site >> 32), c2 = step, c3 = (uint32_t)bk;
    philox4x32_10(c0, c1, c2, c3, P.k0, P.k1);
    if (words) {
      words[(bk * 4 + 0) * nsite + t] = c0;
      words[(bk * 4 + 1) * nsite + t] = c1;
      words[(bk * 4 + 2) * nsite + t] = c2;
      words[(bk * 4 + 3) * nsite + t] = c3;
    }
    if (vars) {
      T z[4];
      draw4(P, site, step, (uint32_t)bk, z);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int a = bk * 4 + w;
        if (a < Q - 1) vars[(int64_t)a * nsite + t] = z[w];
      }
    }
  }
}

}  // namespace flb
