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

// f_i(x, t) = g_i(x - v_i)
template <int D, typename T>
__device__ __forceinline__ void gather(const T* __restrict__ g, int64_t n, const Nbr& b,
                                       T (&f)[2 * D + 1]) {
  f[0] = g[b.s];
  f[1] = g[n + b.sxm];
  f[2] = g[2 * n + b.sxp];
  if constexpr (D >= 2) {
    f[3] = g[3 * n + b.sym];
    f[4] = g[4 * n + b.syp];
  }
  if constexpr (D >= 3) {
    f[5] = g[5 * n + b.szm];
    f[6] = g[6 * n + b.szp];
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

// Map a linear block index so that the blocks the dispatcher sends to one
// XCD (round-robin over 8) cover one contiguous range of tiles, keeping the
// shared halo lines of neighbouring tiles in one L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
  const int64_t q = G / 8, r = G % 8;
  const int64_t xcd = b % 8, k = b / 8;
  return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
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

// Row step: a block covers blockDim.x consecutive x of RY consecutive rows
// (row = y + ny z); each thread owns one column of the tile.  All RY rows'
// populations are loaded before any is collided, so that every wave keeps
// RY * Q loads in flight; NT selects non-temporal stores (the new state is
// not re-read within this launch).
template <int D, typename T, int RY, bool NT>
__global__ void __launch_bounds__(1024) k_step_rows(const T* __restrict__ g, T* __restrict__ h,
                                                    KParams<T> P, uint32_t step, int64_t tiles_x,
                                                    int64_t nrows, int remap) {
  constexpr int Q = 2 * D + 1;
  const int64_t G = (int64_t)gridDim.x;
  const int64_t tile = remap ? xcd_tile(blockIdx.x, G) : (int64_t)blockIdx.x;
  const int64_t tx = tile % tiles_x, tr = tile / tiles_x;
  // the row tile and every plane/row base are uniform over the block (scalar
  // registers); per lane only 32-bit column offsets remain
  const uint32_t nx = (uint32_t)P.nx;
  const uint32_t x = (uint32_t)(tx * blockDim.x) + threadIdx.x;
  if (x >= nx) return;
  const int64_t n = P.n;
  constexpr uint32_t S = sizeof(T);
  const uint32_t bx = x * S;                                   // nx * S < 2^32
  const uint32_t bxm = (x == 0 ? nx - 1 : x - 1) * S, bxp = (x == nx - 1 ? 0 : x + 1) * S;
  const int64_t row0 = tr * RY;
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

// ---------------------------------------------------------------------------
// Canonical state <-> storage.
// out: f_i(x) = g_i(x - v_i);  in: g_i(x - v_i) = f_i(x).
template <int D, typename T>
__global__ void k_to_canonical(const T* __restrict__ g, T* __restrict__ f, int64_t nx, int64_t ny,
                               int64_t nz) {
  constexpr int Q = 2 * D + 1;
  const int64_t n = nx * ny * nz;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const Nbr b = neighbours(x, y, z, nx, ny, nz);
    T v[Q];
    gather<D, T>(g, n, b, v);
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i * n + s] = v[i];
  }
}

template <int D, typename T>
__global__ void k_from_canonical(const T* __restrict__ f, T* __restrict__ g, int64_t nx, int64_t ny,
                                 int64_t nz) {
  constexpr int Q = 2 * D + 1;
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
// Deterministic block reductions (fixed shuffle tree, then waves in order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* lds4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds4[wave] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  return r;
}

// Lattice sums: [0] mass, [1..7] sum f_i, [8..35] sum f_i f_j (i <= j),
// [36] sum rho^2, [37] sum max(rho, 0), [38] #rho < 0, [39] #non-finite.
constexpr int kNV = 40;

template <int D, typename T>
__global__ void __launch_bounds__(256) k_moments_partial(const T* __restrict__ g, int64_t nx,
                                                         int64_t ny, int64_t nz,
                                                         double* __restrict__ part) {
  constexpr int Q = 2 * D + 1;
  constexpr int NFF = Q * (Q + 1) / 2;
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  double sf[Q], sff[NFF];
  double mass = 0, r2 = 0, rpos = 0, nneg = 0, nonfin = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) sf[i] = 0;
#pragma unroll
  for (int i = 0; i < NFF; ++i) sff[i] = 0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const Nbr b = neighbours(x, y, z, nx, ny, nz);
    T fv[Q];
    gather<D, T>(g, n, b, fv);
    double f[Q];
    double rho = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f[i] = (double)fv[i];
      rho += f[i];
      sf[i] += f[i];
      nonfin += isfinite(f[i]) ? 0.0 : 1.0;
    }
    int k = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int j = i; j < Q; ++j) sff[k++] += f[i] * f[j];
    mass += rho;
    r2 += rho * rho;
    rpos += rho > 0 ? rho : 0.0;
    nneg += rho < 0 ? 1.0 : 0.0;
  }
  double* out = part + (int64_t)blockIdx.x * kNV;
  double v;
  v = block_sum256(mass, lds);
  if (threadIdx.x == 0) out[0] = v;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    v = block_sum256(i < Q ? sf[i < Q ? i : 0] : 0.0, lds);
    if (threadIdx.x == 0) out[1 + i] = i < Q ? v : 0.0;
  }
  // sum_ff packed for the lattice's Q, padded with zeros to 28
#pragma unroll
  for (int i = 0; i < 28; ++i) {
    v = block_sum256(i < NFF ? sff[i < NFF ? i : 0] : 0.0, lds);
    if (threadIdx.x == 0) out[8 + i] = i < NFF ? v : 0.0;
  }
  v = block_sum256(r2, lds);
  if (threadIdx.x == 0) out[36] = v;
  v = block_sum256(rpos, lds);
  if (threadIdx.x == 0) out[37] = v;
  v = block_sum256(nneg, lds);
  if (threadIdx.x == 0) out[38] = v;
  v = block_sum256(nonfin, lds);
  if (threadIdx.x == 0) out[39] = v;
}

// Sum nblk rows of kNV partials: one 256-thread block per quantity, each
// thread a fixed strided subset, then the block tree (deterministic).
__global__ void __launch_bounds__(256) k_moments_final(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ out) {
  __shared__ double lds[4];
  const int q = blockIdx.x;
  double acc = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += part[(int64_t)b * kNV + q];
  acc = block_sum256(acc, lds);
  if (threadIdx.x == 0) out[q] = acc;
}

// ---------------------------------------------------------------------------
// Density of a site in FP64 (canonical gather, populations in index order).
template <int D, typename T>
__device__ __forceinline__ double site_density(const T* __restrict__ g, int64_t n, int64_t x,
                                               int64_t y, int64_t z, int64_t nx, int64_t ny,
                                               int64_t nz) {
  const Nbr b = neighbours(x, y, z, nx, ny, nz);
  T fv[2 * D + 1];
  gather<D, T>(g, n, b, fv);
  double rho = 0;
#pragma unroll
  for (int i = 0; i < 2 * D + 1; ++i) rho += (double)fv[i];
  return rho;
}

// Row sums: rowsum[row] = sum_x rho(x, row), one block per row.
template <int D, typename T>
__global__ void __launch_bounds__(256) k_row_sums(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                  int64_t nz, double* __restrict__ rowsum) {
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  const int64_t row = blockIdx.x;
  const int64_t y = row % ny, z = row / ny;
  double acc = 0;
  for (int64_t x = threadIdx.x; x < nx; x += blockDim.x)
    acc += site_density<D, T>(g, n, x, y, z, nx, ny, nz);
  const double v = block_sum256(acc, lds);
  if (threadIdx.x == 0) rowsum[row] = v;
}

// Column partials: colpart[c][x] = sum over the rows of chunk c of rho(x, row).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_col_partial(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                     int64_t nz, int64_t rows_per_chunk,
                                                     double* __restrict__ colpart) {
  const int64_t n = nx * ny * nz;
  const int64_t nrows = ny * nz;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (x >= nx) return;
  const int64_t r0 = c * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < nrows ? r0 + rows_per_chunk : nrows;
  double acc = 0;
  for (int64_t row = r0; row < r1; ++row)
    acc += site_density<D, T>(g, n, x, row % ny, row / ny, nx, ny, nz);
  colpart[c * nx + x] = acc;
}

// Axis marginals from the partials: mx[x] = sum_c colpart[c][x] and
// my[y] = sum_z rowsum[y + ny z] (one thread each, short fixed loops).
__global__ void k_marginals_xy(const double* __restrict__ colpart, int64_t nchunk,
                               const double* __restrict__ rowsum, int64_t nx, int64_t ny,
                               int64_t nz, double* __restrict__ mx, double* __restrict__ my) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nx) {
    double acc = 0;
    for (int64_t c = 0; c < nchunk; ++c) acc += colpart[c * nx + t];
    mx[t] = acc;
  } else if (t < nx + ny) {
    const int64_t y = t - nx;
    double acc = 0;
    for (int64_t z = 0; z < nz; ++z) acc += rowsum[y + ny * z];
    my[y] = acc;
  }
}

// mz[z] = sum_y rowsum[y + ny z]: one block per z (3-D lattices only).
__global__ void __launch_bounds__(256) k_marginal_z(const double* __restrict__ rowsum, int64_t ny,
                                                    double* __restrict__ mz) {
  __shared__ double lds[4];
  const int64_t z = blockIdx.x;
  double acc = 0;
  for (int64_t y = threadIdx.x; y < ny; y += blockDim.x) acc += rowsum[y + ny * z];
  acc = block_sum256(acc, lds);
  if (threadIdx.x == 0) mz[z] = acc;
}

// Axis structure factor from a marginal: one block per wave vector.
// kinfo[j] = (axis, k mod L_axis); axis < 0 marks a k = 0 entry.
// S = |sum_x (m(x) - mean) e^{-2 pi i k x / L}|^2 / N; k = 0 gives M^2 / N.
__global__ void __launch_bounds__(256) k_sk_axis(const double* __restrict__ mx,
                                                 const double* __restrict__ my,
                                                 const double* __restrict__ mz, int64_t nx,
                                                 int64_t ny, int64_t nz,
                                                 const int64_t* __restrict__ kinfo,
                                                 const int32_t* __restrict__ slot,
                                                 double* __restrict__ sval) {
  __shared__ double lds[4];
  const int j = blockIdx.x;
  const int64_t axis = kinfo[2 * j], k = kinfo[2 * j + 1];
  const double N = (double)(nx * ny * nz);
  const double* m = axis == 1 ? my : (axis == 2 ? mz : mx);
  const int64_t L = axis == 1 ? ny : (axis == 2 ? nz : nx);
  // mass from the chosen marginal
  double tot = 0;
  for (int64_t x = threadIdx.x; x < L; x += blockDim.x) tot += m[x];
  tot = block_sum256(tot, lds);
  __shared__ double mean_s;
  if (threadIdx.x == 0) mean_s = tot / (double)L;
  __syncthreads();
  const double mean = mean_s;
  if (axis < 0) {
    if (threadIdx.x == 0) sval[slot[j]] = tot * tot / N;
    return;
  }
  double re = 0, im = 0;
  for (int64_t x = threadIdx.x; x < L; x += blockDim.x) {
    const int64_t p = (k * x) % L;  // integer phase
    double s, c;
    sincospi(2.0 * (double)p / (double)L, &s, &c);
    const double v = m[x] - mean;
    re += v * c;
    im -= v * s;
  }
  re = block_sum256(re, lds);
  __syncthreads();
  im = block_sum256(im, lds);
  if (threadIdx.x == 0) sval[slot[j]] = (re * re + im * im) / N;
}

// General wave vectors: direct sum over sites.  Block (c, j) sums the sites
// of chunk c for wave vector j; partial[(j * nchunk + c) * 2 + {0, 1}].
template <int D, typename T>
__global__ void __launch_bounds__(256) k_sk_direct_partial(const T* __restrict__ g, int64_t nx,
                                                           int64_t ny, int64_t nz,
                                                           const int64_t* __restrict__ kv,
                                                           double mean, int64_t chunk,
                                                           double* __restrict__ partial) {
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  const int64_t c = blockIdx.x, j = blockIdx.y, nchunk = gridDim.x;
  const int64_t kx = kv[3 * j], ky = kv[3 * j + 1], kz = kv[3 * j + 2];
  const int64_t s0 = c * chunk, s1 = s0 + chunk < n ? s0 + chunk : n;
  double re = 0, im = 0;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const double v = site_density<D, T>(g, n, x, y, z, nx, ny, nz) - mean;
    // phase / (2 pi) = sum_a ((k_a x_a) mod L_a) / L_a, reduced mod 1
    double ph = (double)((kx * x) % nx) / (double)nx + (double)((ky * y) % ny) / (double)ny +
                (double)((kz * z) % nz) / (double)nz;
    ph -= floor(ph);
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    re += v * cs;
    im -= v * sn;
  }
  re = block_sum256(re, lds);
  __syncthreads();
  im = block_sum256(im, lds);
  if (threadIdx.x == 0) {
    partial[(j * nchunk + c) * 2] = re;
    partial[(j * nchunk + c) * 2 + 1] = im;
  }
}

// k = 0 entries hold sum_x (rho - mean) = M - N mean in `re`; S(0) = M^2 / N.
__global__ void k_sk_direct_final(const double* __restrict__ partial, int64_t nchunk, int nkg,
                                  const int32_t* __restrict__ slot,
                                  const int64_t* __restrict__ kv, double mean, double N,
                                  double* __restrict__ sval) {
  const int j = (int)((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= nkg) return;
  double re = 0, im = 0;
  for (int64_t c = 0; c < nchunk; ++c) {
    re += partial[(j * nchunk + c) * 2];
    im += partial[(j * nchunk + c) * 2 + 1];
  }
  if (kv[3 * j] == 0 && kv[3 * j + 1] == 0 && kv[3 * j + 2] == 0) {
    const double M = re + N * mean;
    sval[slot[j]] = M * M / N;
  } else {
    sval[slot[j]] = (re * re + im * im) / N;
  }
}

__global__ void k_sk_accumulate(const double* __restrict__ sval, double* __restrict__ acc, int nk) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nk) acc[j] += sval[j];
}

__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0.0;
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
