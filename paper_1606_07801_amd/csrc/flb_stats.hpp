// Statistics kernels of one lattice (lattice sums, axis marginals and the
// density structure factor), in deterministic FP64 reductions: fixed grid,
// fixed shuffle trees, partials combined in block order.  Included by the
// single translation unit that launches them.
#pragma once

#include "flb_kernels.hpp"

namespace flb {

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

// Work units of the lattice sums: segments of kMomSeg<D> consecutive sites
// of one row, kMomSeg<D> / 256 per lane.  D3Q7 keeps 40 accumulators and
// takes two sites per lane, the others four (measured at 512^3, 4096^2 and
// 2^24 sites against one, two and four: 797 against 999 us for D3Q7 with
// one, 78 against 85 us for D2Q5 with two).
template <int D> constexpr int kMomSeg = 256 * (D == 3 ? 2 : 4);

// BUF: the pull form of a state under 4 GiB, loaded through a buffer
// resource (32-bit lane offsets, row and plane offsets in scalar registers).
template <int D, typename T, bool BUF = false>
__global__ void __launch_bounds__(256) k_moments_partial(const T* __restrict__ g, int64_t nx,
                                                         int64_t ny, int64_t nz,
                                                         double* __restrict__ part, int form = kFormPull) {
  constexpr int Q = 2 * D + 1;
  constexpr int NFF = Q * (Q + 1) / 2;
  constexpr int NV = 1 + Q + NFF + 4;  // values this model has: mass, sum f, sum ff, the four others
  constexpr int SUB = kMomSeg<D> / 256;
  __shared__ double red[4][NV];
  const int64_t n = nx * ny * nz;
  const int64_t segs = (nx + kMomSeg<D> - 1) / kMomSeg<D>;
  const int64_t units = ny * nz * segs;
  double sf[Q], sff[NFF];
  double mass = 0, r2 = 0, rpos = 0, nneg = 0, nonfin = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) sf[i] = 0;
#pragma unroll
  for (int i = 0; i < NFF; ++i) sff[i] = 0;
  // a unit's row (y, z) is uniform over the block: one division per unit;
  // sites past the row's end load a valid site and add zeros, so the four
  // sites' loads carry no branch and issue together
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t r = u / segs, x0 = (u - r * segs) * kMomSeg<D>;
    const int64_t y = r % ny, z = r / ny;
    T fv[SUB][Q];
    bool ok[SUB];
    if constexpr (BUF) {
      constexpr uint32_t S = sizeof(T);
      const uint32_t nS = (uint32_t)n * S;
      const __amdgpu_buffer_rsrc_t rg = buf_rsrc(g, (uint32_t)Q * nS);
      const uint32_t ux = (uint32_t)nx, uy = (uint32_t)ny, uz = (uint32_t)nz;
      const uint32_t yy = (uint32_t)y, zz = (uint32_t)z;
      const uint32_t ym = yy == 0 ? uy - 1 : yy - 1, yp = yy == uy - 1 ? 0 : yy + 1;
      const uint32_t zm = zz == 0 ? uz - 1 : zz - 1, zp = zz == uz - 1 ? 0 : zz + 1;
      const uint32_t row = ux * (yy + uy * zz) * S;  // uniform byte offsets of the rows
      const uint32_t rym = ux * (ym + uy * zz) * S, ryp = ux * (yp + uy * zz) * S;
      const uint32_t rzm = ux * (yy + uy * zm) * S, rzp = ux * (yy + uy * zp) * S;
#pragma unroll
      for (int j = 0; j < SUB; ++j) {
        const int64_t x = x0 + j * 256 + threadIdx.x;
        ok[j] = x < nx;
        const uint32_t xs = ok[j] ? (uint32_t)x : ux - 1;
        const uint32_t vx = xs * S, vxm = (xs == 0 ? ux - 1 : xs - 1) * S, vxp = (xs == ux - 1 ? 0 : xs + 1) * S;
        fv[j][0] = buf_ld<T>(rg, vx, row);
        fv[j][1] = buf_ld<T>(rg, vxm, nS + row);
        fv[j][2] = buf_ld<T>(rg, vxp, 2 * nS + row);
        if constexpr (D >= 2) {
          fv[j][3] = buf_ld<T>(rg, vx, 3 * nS + rym);
          fv[j][4] = buf_ld<T>(rg, vx, 4 * nS + ryp);
        }
        if constexpr (D >= 3) {
          fv[j][5] = buf_ld<T>(rg, vx, 5 * nS + rzm);
          fv[j][6] = buf_ld<T>(rg, vx, 6 * nS + rzp);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < SUB; ++j) {
        const int64_t x = x0 + j * 256 + threadIdx.x;
        ok[j] = x < nx;
        const Nbr b = neighbours(ok[j] ? x : nx - 1, y, z, nx, ny, nz);
        gather<D, T>(g, n, b, fv[j], form);
      }
    }
#pragma unroll
    for (int j = 0; j < SUB; ++j) {
      double f[Q];
      double rho = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        f[i] = ok[j] ? (double)fv[j][i] : 0.0;
        rho += f[i];
        sf[i] += f[i];
        nonfin += isfinite(f[i]) ? 0.0 : 1.0;
      }
      int k = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int m = i; m < Q; ++m) sff[k++] += f[i] * f[m];
      mass += rho;
      r2 += rho * rho;
      rpos += rho > 0 ? rho : 0.0;
      nneg += rho < 0 ? 1.0 : 0.0;
    }
  }
  // block sums: every value's wave sum, then the four waves in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[NV];
  v[0] = mass;
#pragma unroll
  for (int i = 0; i < Q; ++i) v[1 + i] = sf[i];
#pragma unroll
  for (int i = 0; i < NFF; ++i) v[1 + Q + i] = sff[i];
  v[1 + Q + NFF] = r2;
  v[2 + Q + NFF] = rpos;
  v[3 + Q + NFF] = nneg;
  v[4 + Q + NFF] = nonfin;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double w = wave_sum(v[q]);
    if (lane == 0) red[wave][q] = w;
  }
  __syncthreads();
  // the kNV slots: [0] mass, [1..7] sum f_i, [8..35] sum f_i f_j, [36..39]
  if (threadIdx.x < kNV) {
    const int o = threadIdx.x;
    int q = -1;
    if (o == 0) q = 0;
    else if (o < 8) q = o - 1 < Q ? 1 + (o - 1) : -1;
    else if (o < 36) q = o - 8 < NFF ? 1 + Q + (o - 8) : -1;
    else q = 1 + Q + NFF + (o - 36);
    part[(int64_t)blockIdx.x * kNV + o] = q < 0 ? 0.0 : ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
  }
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
                                               int64_t nz, int form = kFormPull) {
  const Nbr b = neighbours(x, y, z, nx, ny, nz);
  T fv[2 * D + 1];
  gather<D, T>(g, n, b, fv, form);
  double rho = 0;
#pragma unroll
  for (int i = 0; i < 2 * D + 1; ++i) rho += (double)fv[i];
  return rho;
}

// Row sums: rowsum[row] = sum_x rho(x, row), one block per row.
template <int D, typename T>
__global__ void __launch_bounds__(256) k_row_sums(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                  int64_t nz, double* __restrict__ rowsum, int form = kFormPull) {
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  const int64_t row = blockIdx.x;
  const int64_t y = row % ny, z = row / ny;
  double acc = 0;
  for (int64_t x = threadIdx.x; x < nx; x += blockDim.x)
    acc += site_density<D, T>(g, n, x, y, z, nx, ny, nz, form);
  const double v = block_sum256(acc, lds);
  if (threadIdx.x == 0) rowsum[row] = v;
}

// Column partials: colpart[c][x] = sum over the rows of chunk c of rho(x, row).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_col_partial(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                     int64_t nz, int64_t rows_per_chunk,
                                                     double* __restrict__ colpart, int form = kFormPull) {
  const int64_t n = nx * ny * nz;
  const int64_t nrows = ny * nz;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (x >= nx) return;
  const int64_t r0 = c * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < nrows ? r0 + rows_per_chunk : nrows;
  double acc = 0;
  for (int64_t row = r0; row < r1; ++row)
    acc += site_density<D, T>(g, n, x, row % ny, row / ny, nx, ny, nz, form);
  colpart[c * nx + x] = acc;
}

// Axis marginal along x from column partials: mx[x] = sum_c colpart[c][x].
// A block covers 64 columns; its 4 waves sum interleaved chunk subsets and
// are combined in wave order (deterministic).
__global__ void __launch_bounds__(256) k_marginal_x(const double* __restrict__ colpart,
                                                    int64_t nchunk, int64_t nx,
                                                    double* __restrict__ mx) {
  __shared__ double part[4][64];
  const int lx = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t x = (int64_t)blockIdx.x * 64 + lx;
  double acc = 0;
  if (x < nx)
    for (int64_t c = grp; c < nchunk; c += 4) acc += colpart[c * nx + x];
  part[grp][lx] = acc;
  __syncthreads();
  if (grp == 0 && x < nx) mx[x] = ((part[0][lx] + part[1][lx]) + part[2][lx]) + part[3][lx];
}

// my[y] = sum_z rowsum[y + ny z]: one block per y, thread t adding
// z = t, t + 256, ... in order, then the block's fixed tree (a thread per y
// summing all of z in order left a 512^3 lattice two blocks: 126 us).
__global__ void __launch_bounds__(256) k_marginal_y(const double* __restrict__ rowsum, int64_t ny, int64_t nz,
                                                    double* __restrict__ my) {
  __shared__ double lds[4];
  const int64_t y = blockIdx.x;
  double acc = 0;
  for (int64_t z = threadIdx.x; z < nz; z += blockDim.x) acc += rowsum[y + ny * z];
  acc = block_sum256(acc, lds);
  if (threadIdx.x == 0) my[y] = acc;
}

// The reductions after a sampled pass, in one launch of 1024-thread blocks.
// Blocks [0, ncb), ncb = ceil(nx / 16), build the x marginal of 16 columns
// straight from the per-tile column partials: thread (g, c) adds the tiles
// of group g (ngroup <= 64 groups of consecutive tiles) for column c in
// order; then, per column, 4 interleaved subsets of the group sums are each
// added in order and combined in order (the additions of a group reduction
// followed by k_marginal_x).  The other blocks: rowsum[row] = sum over the x
// tiles of rowpart[t][row], in order.
__global__ void __launch_bounds__(1024) k_axis_reduce(const double* __restrict__ rowpart, int64_t ntx,
                                                      int64_t nrows, double* __restrict__ rowsum,
                                                      const double* __restrict__ colbig, int64_t ntr,
                                                      int64_t nx, int64_t ngroup, double* __restrict__ mx) {
  const int64_t ncb = (nx + 15) / 16;
  if ((int64_t)blockIdx.x >= ncb) {
    const int64_t row = ((int64_t)blockIdx.x - ncb) * blockDim.x + threadIdx.x;
    if (row >= nrows) return;
    double acc = 0;
#pragma unroll 8
    for (int64_t t = 0; t < ntx; ++t) acc += rowpart[t * nrows + row];
    rowsum[row] = acc;
    return;
  }
  __shared__ double gs[64][16];
  __shared__ double ps[4][16];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t x = (int64_t)blockIdx.x * 16 + c;
  if (g < ngroup && x < nx) {
    const int64_t t0 = g * ntr / ngroup, t1 = (g + 1) * ntr / ngroup;
    double a = 0;
#pragma unroll 8
    for (int64_t t = t0; t < t1; ++t) a += colbig[t * nx + x];
    gs[g][c] = a;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int cc = threadIdx.x & 15, sub = threadIdx.x >> 4;
    double acc = 0;
    for (int gg = sub; gg < ngroup; gg += 4) acc += gs[gg][cc];
    ps[sub][cc] = acc;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int64_t xx = (int64_t)blockIdx.x * 16 + threadIdx.x;
    if (xx < nx) mx[xx] = ((ps[0][threadIdx.x] + ps[1][threadIdx.x]) + ps[2][threadIdx.x]) + ps[3][threadIdx.x];
  }
}

// Twiddles of one axis: tw[2p] = cos(2 pi p / L), tw[2p + 1] = sin(2 pi p / L).
__global__ void k_twiddle(double* __restrict__ tw, int64_t L) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L) return;
  double s, c;
  sincospi(2.0 * (double)p / (double)L, &s, &c);
  tw[2 * p] = c;
  tw[2 * p + 1] = s;
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

// Axis structure factor from the marginals: each block takes kSkAxisK
// consecutive entries of the axis list; kinfo[j] = (axis, k mod L_axis),
// axis < 0 marking a k = 0 entry.
//   S = |sum_x (m(x) - mean) e^{-2 pi i k x / L}|^2 / N,  k = 0: M^2 / N,
// with M the mass (the sum of the x marginal) and mean = M / L of the
// entry's axis.  Each thread takes a contiguous run of x: the twiddle of its
// first x comes from the axis table (integer phase k x mod L), each next one
// by a rotation with the twiddle of k, reloaded from the table every 64
// steps (rounding stays at a few ulp); the block's entries share the loads
// of the marginal.  With acc given, S is also added to acc at its slot (the
// accumulator update of an axis-only k-list, without a launch of its own).
constexpr int kSkAxisK = 4;
constexpr int kSkAxisThreads = 256;

__global__ void __launch_bounds__(kSkAxisThreads) k_sk_axis(const double* __restrict__ mx,
                                                 const double* __restrict__ my,
                                                 const double* __restrict__ mz, int64_t nx,
                                                 int64_t ny, int64_t nz,
                                                 const int64_t* __restrict__ kinfo,
                                                 const int32_t* __restrict__ slot, int nax,
                                                 const double* __restrict__ twx,
                                                 const double* __restrict__ twy,
                                                 const double* __restrict__ twz,
                                                 double* __restrict__ sval,
                                                 double* __restrict__ acc) {
  constexpr int K = kSkAxisK, NW = kSkAxisThreads / 64;
  __shared__ double mass_w[NW];
  __shared__ double red[2 * K][NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * K;
  const double N = (double)(nx * ny * nz);
  double tot = 0;
#pragma unroll 4
  for (int64_t x = threadIdx.x; x < nx; x += blockDim.x) tot += mx[x];
  tot = wave_sum(tot);
  if (lane == 0) mass_w[wave] = tot;
  __syncthreads();
  double M = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) M += mass_w[w];
  int ax[K];
  int64_t kk[K];
  double re[K], im[K];
#pragma unroll
  for (int e = 0; e < K; ++e) {
    const int j = j0 + e;
    ax[e] = j < nax ? (int)kinfo[2 * j] : -2;
    kk[e] = j < nax ? kinfo[2 * j + 1] : 0;
    re[e] = 0.0;
    im[e] = 0.0;
  }
  for (int a = 0; a < 3; ++a) {
    bool any = false;
#pragma unroll
    for (int e = 0; e < K; ++e) any |= ax[e] == a;
    if (!any) continue;  // uniform over the block
    const double* m = a == 0 ? mx : (a == 1 ? my : mz);
    const double* tw = a == 0 ? twx : (a == 1 ? twy : twz);
    const int64_t L = a == 0 ? nx : (a == 1 ? ny : nz);
    const double mean = M / (double)L;
    const int64_t C = (L + blockDim.x - 1) / blockDim.x;
    const int64_t x0 = (int64_t)threadIdx.x * C, x1 = x0 + C < L ? x0 + C : L;
    double sr[K], si[K];
#pragma unroll
    for (int e = 0; e < K; ++e) {  // (entries of other axes read entry 0 and ignore it)
      const int64_t q = ax[e] == a ? kk[e] : 0;
      sr[e] = tw[2 * q];
      si[e] = tw[2 * q + 1];
    }
    for (int64_t xa = x0; xa < x1; xa += 64) {
      double wr[K], wi[K];
#pragma unroll
      for (int e = 0; e < K; ++e) {
        const int64_t p = L < (1ll << 31) ? (kk[e] * xa) % L
                                          : (int64_t)((unsigned __int128)kk[e] * (uint64_t)xa % (uint64_t)L);
        wr[e] = tw[2 * p];  // p < L: in the table for every entry
        wi[e] = tw[2 * p + 1];
      }
      const int64_t xb = xa + 64 < x1 ? xa + 64 : x1;
#pragma unroll 8
      for (int64_t x = xa; x < xb; ++x) {  // (unrolled: the loads of m issue together)
        const double v = m[x] - mean;
#pragma unroll
        for (int e = 0; e < K; ++e) {
          if (ax[e] != a) continue;
          re[e] += v * wr[e];
          im[e] -= v * wi[e];
          const double nr = wr[e] * sr[e] - wi[e] * si[e];
          wi[e] = wr[e] * si[e] + wi[e] * sr[e];
          wr[e] = nr;
        }
      }
    }
  }
  // block sums of the K pairs: wave sums, then the waves in order
#pragma unroll
  for (int e = 0; e < K; ++e) {
    const double r = wave_sum(re[e]), i = wave_sum(im[e]);
    if (lane == 0) {
      red[2 * e][wave] = r;
      red[2 * e + 1][wave] = i;
    }
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int e = threadIdx.x, j = j0 + e;
    if (j < nax) {
      double r = 0, i = 0;
      for (int w = 0; w < NW; ++w) {
        r += red[2 * e][w];
        i += red[2 * e + 1][w];
      }
      const double S = kinfo[2 * j] < 0 ? M * M / N : (r * r + i * i) / N;
      sval[slot[j]] = S;
      if (acc) acc[slot[j]] += S;
    }
  }
}

// General wave vectors: direct sum over sites.  Block (c, j) sums the sites
// of chunk c for wave vector j; partial[(j * nchunk + c) * 2 + {0, 1}].
template <int D, typename T>
__global__ void __launch_bounds__(256) k_sk_direct_partial(const T* __restrict__ g, int64_t nx,
                                                           int64_t ny, int64_t nz,
                                                           const int64_t* __restrict__ kv,
                                                           double mean, int64_t chunk,
                                                           double* __restrict__ partial, int form = kFormPull) {
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  const int64_t c = blockIdx.x, j = blockIdx.y, nchunk = gridDim.x;
  const int64_t kx = kv[3 * j], ky = kv[3 * j + 1], kz = kv[3 * j + 2];
  const int64_t s0 = c * chunk, s1 = s0 + chunk < n ? s0 + chunk : n;
  double re = 0, im = 0;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    const int64_t x = s % nx, rest = s / nx, y = rest % ny, z = rest / ny;
    const double v = site_density<D, T>(g, n, x, y, z, nx, ny, nz, form) - mean;
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

// ---------------------------------------------------------------------------
// Density profile along one axis: for every coordinate, the sums of rho and
// rho^2 over the sites with that coordinate, in a fixed order.
// x: chunk c of the rows gives part[(c * nx + x) * 2 + {0, 1}].
template <int D, typename T>
__global__ void __launch_bounds__(256) k_prof_cols(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                   int64_t nz, int64_t rpc, double* __restrict__ part,
                                                   int form = kFormPull) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= nx) return;
  const int64_t n = nx * ny * nz, nrows = ny * nz;
  const int64_t c = blockIdx.y, r0 = c * rpc, r1 = r0 + rpc < nrows ? r0 + rpc : nrows;
  double s = 0, s2 = 0;
  for (int64_t r = r0; r < r1; ++r) {
    const double rho = site_density<D, T>(g, n, x, r % ny, r / ny, nx, ny, nz, form);
    s += rho;
    s2 += rho * rho;
  }
  part[(c * nx + x) * 2] = s;
  part[(c * nx + x) * 2 + 1] = s2;
}

// out[x] = sum over chunks (in order) of part, out2[x] the same for rho^2
__global__ void k_prof_cols_final(const double* __restrict__ part, int64_t nchunk, int64_t nx,
                                  double* __restrict__ out, double* __restrict__ out2) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  double s = 0, s2 = 0;
  for (int64_t c = 0; c < nchunk; ++c) {
    s += part[(c * nx + x) * 2];
    s2 += part[(c * nx + x) * 2 + 1];
  }
  out[x] = s;
  out2[x] = s2;
}

// y / z: one block per row r = y + ny z sums rho and rho^2 over x into rs[2 r + {0, 1}]
template <int D, typename T>
__global__ void __launch_bounds__(256) k_prof_rows(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                   int64_t nz, double* __restrict__ rs, int form = kFormPull) {
  __shared__ double lds[4];
  const int64_t r = blockIdx.x, n = nx * ny * nz;
  double s = 0, s2 = 0;
  for (int64_t x = threadIdx.x; x < nx; x += blockDim.x) {
    const double rho = site_density<D, T>(g, n, x, r % ny, r / ny, nx, ny, nz, form);
    s += rho;
    s2 += rho * rho;
  }
  s = block_sum256(s, lds);
  __syncthreads();
  s2 = block_sum256(s2, lds);
  if (threadIdx.x == 0) {
    rs[2 * r] = s;
    rs[2 * r + 1] = s2;
  }
}

// out[c] (and out2[c] for rho^2) for c along y (axis 1) or z (axis 2)
__global__ void k_prof_yz(const double* __restrict__ rs, int64_t ny, int64_t nz, int axis,
                          double* __restrict__ out, double* __restrict__ out2) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t L = axis == 1 ? ny : nz, M = axis == 1 ? nz : ny;
  if (c >= L) return;
  double s = 0, s2 = 0;
  for (int64_t o = 0; o < M; ++o) {
    const int64_t r = axis == 1 ? c + ny * o : o + ny * c;
    s += rs[2 * r];
    s2 += rs[2 * r + 1];
  }
  out[c] = s;
  out2[c] = s2;
}

__global__ void k_add(const double* __restrict__ v, double* __restrict__ acc, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) acc[j] += v[j];
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
// Sampled step: the step of k_step_rows (same arithmetic, bit-identical
// result) for a tile of 256 columns x RY rows, which also accumulates the
// FP64 density of the pre-collision state into
//   rowpart[tx][row] = sum over the tile's columns of rho(x, row)
//   colpart[tr][x]   = sum over the tile's rows of rho(x, row)
// (fixed-order sums: down the column in row order; across the row, DPP sums
// of 16 lanes, added per wave and then over the waves in order), the inputs
// of the axis marginals.
template <int D, typename T, int RY>
__global__ void __launch_bounds__(256) k_step_rows_sk(const T* __restrict__ g, T* __restrict__ h,
                                                      KParams<T> P, uint32_t step, int64_t tiles_x,
                                                      int64_t nrows, double* __restrict__ rowpart,
                                                      double* __restrict__ colpart) {
  constexpr int Q = 2 * D + 1;
  __shared__ double red16[RY][16];  // per row, the sixteen 16-lane sums
  const int64_t tile = blockIdx.x;
  const int64_t tx = tile % tiles_x, tr = tile / tiles_x;
  const uint32_t nx = (uint32_t)P.nx;
  const int tid = threadIdx.x;
  const uint32_t x = (uint32_t)(tx * 256) + tid;
  const bool valid = x < nx;
  const int64_t row0 = tr * RY;
  const int64_t n = P.n;
  constexpr uint32_t S = sizeof(T);
  const uint32_t xs = valid ? x : 0;
  const uint32_t bx = xs * S;
  const uint32_t bxm = (xs == 0 ? nx - 1 : xs - 1) * S, bxp = (xs == nx - 1 ? 0 : xs + 1) * S;
  double col = 0;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int64_t row = row0 + r;
    double rho = 0;
    if (valid && row < nrows) {
      const int64_t base = row * (int64_t)nx;
      T f[Q];
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
      rho = density_sum(f);
      col += rho;
      Collide<D, T>::run(f, P, (uint64_t)base + x, step);
#pragma unroll
      for (int i = 0; i < Q; ++i) st_at<T, false>(h + i * n + base, bx, f[i]);
    }
    const double v = row16_sum(rho);  // every lane (0 where none)
    if ((tid & 15) == 0) red16[r][tid >> 4] = v;
  }
  if (valid) colpart[tr * (int64_t)nx + x] = col;
  __syncthreads();
  if (tid < RY && row0 + tid < nrows)
    rowpart[tx * nrows + row0 + tid] = sum256_from_rows16(red16[tid]);
}

}  // namespace flb
