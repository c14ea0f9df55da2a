// A whole small lattice resident in one workgroup's LDS for many steps.
//
// One workgroup of 1024 threads loads the canonical state f_i(x, t) into LDS,
// and for each step collides every site in registers (the per-site code of
// the HBM kernels: same arithmetic, same noise stream, bit-identical
// state), waits at a barrier and pushes the post-collision populations to
// their destinations x + v_i (eq. LB) in LDS.  After the last step it writes
// the post-collision populations at their collision sites to HBM, the
// storage form the other step kernels leave.  One launch replaces one launch
// per step, which is what bounds small lattices (a few microseconds each).
//
// The statistics flb_step samples are taken inside, on the state before each
// sampled step, with the same definitions as the HBM path (FP64, fixed-order
// reductions, so repeated runs give the same bits; the summation order
// differs from the HBM kernels, so the values agree to rounding):
//   * lattice sums (40 values) added to momacc;
//   * S(k) of the accumulator k-list added to skacc: axis entries from the
//     axis marginals, general entries by the direct sum, k = 0 as M^2 / N;
//   * population Fourier sums f_i(k) (paper's +i sign) into amp, then the
//     S_ij / time-correlator / ring update of k_corr_accumulate.
//
// Included by flb.hip only.
#pragma once

#include "flb_corr.hpp"

namespace flb {

constexpr int kResThreads = 1024;
constexpr int kResWaves = kResThreads / 64;
constexpr int kResScratch = 2 * kResThreads;  // doubles of LDS scratch
constexpr int kResMaxSites = 4 * kResThreads;
constexpr int kResMaxChunk = 1 << 16;         // steps per launch

struct ResArgs {
  const void* gin;  // storage-form buffer holding the state at step0
  void* gout;       // storage-form buffer receiving the state at step0 + nsteps
  int32_t nx, ny, nz;
  int32_t nsteps;
  int64_t step0;
  // lattice sums
  int64_t mom_every;
  double* momacc;
  // S(k) of the accumulator k-list (layout of the HBM path's k-list upload)
  int64_t sk_every;
  int32_t nax, ngen;
  const int64_t* kinfo;
  const int32_t* slot_ax;
  const int64_t* kv;
  const int32_t* slot_gen;
  double* skacc;
  // population correlators
  int64_t corr_every;
  int32_t cnk, nlag;
  int64_t corr_s0;
  const int32_t* ckinfo;
  double* amp;
  double* sij;
  double* ring;
  double* ct;
  // (cos, sin)(2 pi m / L_a) of the three axes, concatenated
  const double* tw;
};

// LDS bytes of a resident lattice: state, densities, marginals, twiddles,
// scratch (the host checks this against the device limit).
__host__ __device__ constexpr size_t res_state_bytes(size_t q_n_s) { return (q_n_s + 15) & ~(size_t)15; }
__host__ __device__ constexpr size_t res_lds_bytes(int64_t n, int q, int s, int64_t lsum) {
  return res_state_bytes((size_t)q * (size_t)n * (size_t)s) + 8 * (size_t)n + 8 * (size_t)lsum +
         16 * (size_t)lsum + 8 * (size_t)kResScratch;
}

// Largest power of two p <= cap with items * p <= kResThreads (at least 1).
__device__ __forceinline__ int res_parts(int items, int cap) {
  int p = 1;
  while (p * 2 <= cap && items * (p * 2) <= kResThreads) p *= 2;
  return p;
}

// Sum of a DFT over a line of L values m[0..L) with unit-stride phase steps:
//   sum_{x in [x0, x1)} (m[x] - mean) (cos, sgn sin)(2 pi k x / L)
__device__ __forceinline__ void res_line_dft(const double* m, int x0, int x1, int L, int k, double mean,
                                             const double* tw, double sgn, double& re, double& im) {
  int p = (int)(((int64_t)k * x0) % L);
  for (int x = x0; x < x1; ++x) {
    const double v = m[x] - mean;
    re += v * tw[2 * p];
    im += sgn * v * tw[2 * p + 1];
    p += k;
    if (p >= L) p -= L;
  }
}

template <int D, typename T, int SPT>
__device__ __forceinline__ void res_sample_moments(const T* st, int N, double* scr, double* momacc,
                                                   const int (&sites)[SPT]) {
  constexpr int Q = 2 * D + 1;
  double acc[kNV];
#pragma unroll
  for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int s = sites[j];
    if (s >= N) continue;
    double f[Q];
    double rho = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f[i] = (double)st[i * N + s];
      rho += f[i];
      acc[1 + i] += f[i];
      acc[39] += isfinite(f[i]) ? 0.0 : 1.0;
    }
    int k = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int l = i; l < Q; ++l) acc[8 + k++] += f[i] * f[l];
    acc[0] += rho;
    acc[36] += rho * rho;
    acc[37] += rho > 0 ? rho : 0.0;
    acc[38] += rho < 0 ? 1.0 : 0.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < kNV; ++v) {
    const double r = wave_sum(acc[v]);
    if (lane == 0) scr[wave * kNV + v] = r;
  }
  __syncthreads();
  if (threadIdx.x < kNV) {
    double r = 0;
    for (int w = 0; w < kResWaves; ++w) r += scr[w * kNV + threadIdx.x];
    momacc[threadIdx.x] += r;
  }
  __syncthreads();
}

// Twiddle of k.x for a general wave vector (components reduced modulo L_a),
// sign sgn on the sine: (cos, sgn sin)(2 pi sum_a k_a x_a / L_a).
template <int D>
__device__ __forceinline__ void res_twiddle(const double* tw, int nx, int ny, int nz, int kx, int ky, int kz,
                                            int x, int y, int z, double sgn, double& c, double& s) {
  int m = (int)(((int64_t)kx * x) % nx);
  c = tw[2 * m];
  s = tw[2 * m + 1];
  if constexpr (D >= 2) {
    m = (int)(((int64_t)ky * y) % ny);
    const double ar = tw[2 * (nx + m)], ai = tw[2 * (nx + m) + 1];
    const double t = c * ar - s * ai;
    s = c * ai + s * ar;
    c = t;
  }
  if constexpr (D >= 3) {
    m = (int)(((int64_t)kz * z) % nz);
    const double ar = tw[2 * (nx + ny + m)], ai = tw[2 * (nx + ny + m) + 1];
    const double t = c * ar - s * ai;
    s = c * ai + s * ar;
    c = t;
  }
  s *= sgn;
}

template <int D, typename T, int SPT>
__device__ __forceinline__ void res_sample_sk(const ResArgs& A, const T* st, double* rho, double* marg,
                                              const double* tw, double* scr, const int (&sites)[SPT]) {
  constexpr int Q = 2 * D + 1;
  const int nx = A.nx, ny = A.ny, nz = A.nz, N = nx * ny * nz;
  double part = 0;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int s = sites[j];
    if (s >= N) continue;
    double r = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) r += (double)st[i * N + s];
    rho[s] = r;
    part += r;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  part = wave_sum(part);
  if (lane == 0) scr[wave] = part;
  __syncthreads();
  double M = 0;
  for (int w = 0; w < kResWaves; ++w) M += scr[w];
  const double mean = M / (double)N;
  double* mx = marg;
  double* my = marg + nx;
  double* mz = my + ny;
  __syncthreads();  // rho complete
  if constexpr (D >= 2) {  // axis marginals from rho, each a fixed-order sum
    for (int x = threadIdx.x; x < nx; x += kResThreads) {
      double a = 0;
      for (int r = 0; r < ny * nz; ++r) a += rho[r * nx + x];
      mx[x] = a;
    }
    for (int y = threadIdx.x; y < ny; y += kResThreads) {
      double a = 0;
      for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) a += rho[(y + ny * z) * nx + x];
      my[y] = a;
    }
    if constexpr (D >= 3) {
      for (int z = threadIdx.x; z < nz; z += kResThreads) {
        double a = 0;
        for (int r = z * ny; r < (z + 1) * ny; ++r)
          for (int x = 0; x < nx; ++x) a += rho[r * nx + x];
        mz[z] = a;
      }
    }
  }
  __syncthreads();
  const int ne = A.nax + A.ngen;
  const int parts = res_parts(ne, 64);
  for (int t = threadIdx.x; t < ne * parts; t += kResThreads) {
    const int e = t / parts, p = t % parts;
    double re = 0, im = 0;
    if (e < A.nax) {
      const int axis = (int)A.kinfo[2 * e];
      if (axis >= 0) {
        const int k = (int)A.kinfo[2 * e + 1];
        const int L = axis == 0 ? nx : (axis == 1 ? ny : nz);
        const double* m = D == 1 ? rho : (axis == 0 ? mx : (axis == 1 ? my : mz));
        const double* twa = tw + 2 * (axis == 0 ? 0 : (axis == 1 ? nx : nx + ny));
        const int x0 = (int)((int64_t)L * p / parts), x1 = (int)((int64_t)L * (p + 1) / parts);
        res_line_dft(m, x0, x1, L, k, M / (double)L, twa, -1.0, re, im);
      }
    } else {
      const int64_t* kk = A.kv + 3 * (e - A.nax);
      const int kx = (int)kk[0], ky = (int)kk[1], kz = (int)kk[2];
      for (int s = p; s < N; s += parts) {
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        double c, sn;
        res_twiddle<D>(tw, nx, ny, nz, kx, ky, kz, x, y, z, -1.0, c, sn);
        const double v = rho[s] - mean;
        re += v * c;
        im += v * sn;
      }
    }
    scr[2 * t] = re;
    scr[2 * t + 1] = im;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += kResThreads) {
    double re = 0, im = 0;
    for (int p = 0; p < parts; ++p) {
      re += scr[2 * (e * parts + p)];
      im += scr[2 * (e * parts + p) + 1];
    }
    bool k0;
    int slot;
    if (e < A.nax) {
      k0 = A.kinfo[2 * e] < 0;
      slot = A.slot_ax[e];
    } else {
      const int64_t* kk = A.kv + 3 * (e - A.nax);
      k0 = kk[0] == 0 && kk[1] == 0 && kk[2] == 0;
      slot = A.slot_gen[e - A.nax];
    }
    A.skacc[slot] += k0 ? M * M / (double)N : (re * re + im * im) / (double)N;
  }
  __syncthreads();
}

template <int D, typename T>
__device__ __forceinline__ void res_sample_corr(const ResArgs& A, const T* st, const double* tw, double* scr, int64_t sidx) {
  constexpr int Q = 2 * D + 1;
  const int nx = A.nx, ny = A.ny, nz = A.nz, N = nx * ny * nz, nrows = ny * nz;
  const int nk = A.cnk;
  const int items = nk * Q;
  // rows are split between parts (whole lines for the incremental phase),
  // except in 1-D where the single line is split
  const int parts = res_parts(items, D == 1 ? 64 : (nrows < 64 ? nrows : 64));
  for (int t = threadIdx.x; t < items * parts; t += kResThreads) {
    const int kk = t / (Q * parts), i = (t / parts) % Q, p = t % parts;
    const int kx = A.ckinfo[3 * kk], ky = A.ckinfo[3 * kk + 1], kz = A.ckinfo[3 * kk + 2];
    const T* fi = st + i * N;
    double re = 0, im = 0;
    int r0 = 0, r1 = nrows, rs = 1, x0 = 0, x1 = nx;
    if (D == 1) {
      x0 = (int)((int64_t)nx * p / parts);
      x1 = (int)((int64_t)nx * (p + 1) / parts);
    } else {
      r0 = p;
      rs = parts;
    }
    for (int r = r0; r < r1; r += rs) {
      const int y = r % ny, z = r / ny;
      double rc, rsn;  // twiddle of the row's y, z part
      res_twiddle<D>(tw, nx, ny, nz, 0, ky, kz, 0, y, z, 1.0, rc, rsn);
      int px = (int)(((int64_t)kx * x0) % nx);
      const T* row = fi + r * nx;
      for (int x = x0; x < x1; ++x) {
        const double c = tw[2 * px] * rc - tw[2 * px + 1] * rsn;
        const double s = tw[2 * px] * rsn + tw[2 * px + 1] * rc;
        const double v = (double)row[x];
        re += v * c;
        im += v * s;
        px += kx;
        if (px >= nx) px -= nx;
      }
    }
    if (parts == 1) {
      A.amp[2 * t] = re;
      A.amp[2 * t + 1] = im;
    } else {
      scr[2 * t] = re;
      scr[2 * t + 1] = im;
    }
  }
  __syncthreads();
  if (parts > 1) {
    for (int u = threadIdx.x; u < items; u += kResThreads) {
      double re = 0, im = 0;
      for (int p = 0; p < parts; ++p) {
        re += scr[2 * (u * parts + p)];
        im += scr[2 * (u * parts + p) + 1];
      }
      A.amp[2 * u] = re;
      A.amp[2 * u + 1] = im;
    }
    __syncthreads();
  }
  // S_ij, time correlator and ring (the arithmetic of k_corr_accumulate)
  const int64_t ns = (int64_t)nk * Q * Q, nt = ns + (int64_t)nk * A.nlag;
  for (int64_t t = threadIdx.x; t < nt; t += kResThreads) {
    if (t < ns) {
      const int k = (int)(t / (Q * Q)), i = (int)((t / Q) % Q), j = (int)(t % Q);
      const double* a = A.amp + (int64_t)k * 2 * Q;
      const double ar = a[2 * i], ai = a[2 * i + 1], br = a[2 * j], bi = a[2 * j + 1];
      A.sij[2 * t] += ar * br + ai * bi;
      A.sij[2 * t + 1] += ai * br - ar * bi;
      if (i == 0 && j == 0) {
        double rr = 0, ri = 0;
        for (int q = 0; q < Q; ++q) {
          rr += a[2 * q];
          ri += a[2 * q + 1];
        }
        double* slot = A.ring + 2 * ((sidx % A.nlag) * (int64_t)nk + k);
        slot[0] = rr;
        slot[1] = ri;
      }
      continue;
    }
    const int64_t u = t - ns;
    const int k = (int)(u / A.nlag), l = (int)(u % A.nlag);
    if (l > sidx) continue;
    const double* a = A.amp + (int64_t)k * 2 * Q;
    double rr = 0, ri = 0;
    for (int q = 0; q < Q; ++q) {
      rr += a[2 * q];
      ri += a[2 * q + 1];
    }
    double pr = rr, pi = ri;
    if (l > 0) {
      const double* old = A.ring + 2 * (((sidx - l) % A.nlag) * (int64_t)nk + k);
      pr = old[0];
      pi = old[1];
    }
    A.ct[2 * u] += pr * rr + pi * ri;
    A.ct[2 * u + 1] += pi * rr - pr * ri;
  }
  __syncthreads();
}

template <int D, typename T, int SPT>
__global__ void __launch_bounds__(kResThreads) k_resident(KParams<T> P, ResArgs A) {
  constexpr int Q = 2 * D + 1;
  extern __shared__ __align__(16) unsigned char res_smem[];
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int N = nx * ny * nz;
  const int lsum = nx + ny + nz;
  T* st = (T*)res_smem;
  double* rho = (double*)(res_smem + res_state_bytes((size_t)Q * N * sizeof(T)));
  double* marg = rho + N;
  double* tw = marg + lsum;
  double* scr = tw + 2 * lsum;
  const int tid = threadIdx.x;
  for (int m = tid; m < 2 * lsum; m += kResThreads) tw[m] = A.tw[m];
  // canonical state f_i(x) = g_i(x - v_i); coordinates of this thread's sites
  const T* g = (const T*)A.gin;
  int sites[SPT], cx[SPT], cy[SPT], cz[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int s = tid + kResThreads * j;
    sites[j] = s;
    cx[j] = s % nx;
    cy[j] = (s / nx) % ny;
    cz[j] = s / (nx * ny);
    if (s < N) {
      const Nbr b = neighbours(cx[j], cy[j], cz[j], nx, ny, nz);
      T fv[Q];
      gather<D, T>(g, N, b, fv);
#pragma unroll
      for (int i = 0; i < Q; ++i) st[i * N + s] = fv[i];
    }
  }
  __syncthreads();
  int64_t csamp = A.corr_s0;
  T* out = (T*)A.gout;
  for (int k = 0; k < A.nsteps; ++k) {
    const int64_t t = A.step0 + k;
    if (A.mom_every > 0 && t % A.mom_every == 0) res_sample_moments<D, T, SPT>(st, N, scr, A.momacc, sites);
    if (A.corr_every > 0 && t % A.corr_every == 0) res_sample_corr<D, T>(A, st, tw, scr, csamp++);
    if (A.sk_every > 0 && t % A.sk_every == 0) res_sample_sk<D, T, SPT>(A, st, rho, marg, tw, scr, sites);
    const uint32_t t32 = (uint32_t)((uint64_t)t & 0xFFFFFFFFull);
    T f[SPT][Q];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      if (sites[j] < N) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[j][i] = st[i * N + sites[j]];
        Collide<D, T>::run(f[j], P, (uint64_t)sites[j], t32);
      }
    }
    __syncthreads();
    if (k + 1 < A.nsteps) {
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int s = sites[j];
        if (s < N) {
          const int x = cx[j], y = cy[j], z = cz[j];
          const int row = nx * (y + ny * z);
          st[s] = f[j][0];
          st[N + row + (x == nx - 1 ? 0 : x + 1)] = f[j][1];
          st[2 * N + row + (x == 0 ? nx - 1 : x - 1)] = f[j][2];
          if constexpr (D >= 2) {
            st[3 * N + nx * ((y == ny - 1 ? 0 : y + 1) + ny * z) + x] = f[j][3];
            st[4 * N + nx * ((y == 0 ? ny - 1 : y - 1) + ny * z) + x] = f[j][4];
          }
          if constexpr (D >= 3) {
            st[5 * N + nx * (y + ny * (z == nz - 1 ? 0 : z + 1)) + x] = f[j][5];
            st[6 * N + nx * (y + ny * (z == 0 ? nz - 1 : z - 1)) + x] = f[j][6];
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        if (sites[j] < N) {
#pragma unroll
          for (int i = 0; i < Q; ++i) out[(int64_t)i * N + sites[j]] = f[j][i];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace flb
