// A whole small lattice resident in one workgroup's LDS for many steps.
//
// One workgroup (256 threads for up to 1024 sites, else 1024: fewer waves
// make every barrier cheaper) loads the canonical state f_i(x, t) into LDS,
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
constexpr int kResScratch = 2 * kResThreads;  // doubles of LDS scratch
constexpr int kResMaxSites = 4 * kResThreads;
constexpr int kResMaxChunk = 1 << 16;         // steps per launch

struct ResArgs {
  const void* gin;  // buffer holding the state at step0, in form form_in
  void* gout;       // buffer receiving the state at step0 + nsteps, in form form_out
                    // (the same buffer for the single-buffer layout: the whole
                    // state is in LDS before the first store)
  int32_t form_in, form_out;
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
  int32_t sk_fft;  // bit a: axis-a entries by FFT of the marginal
  int32_t sk_dft;  // some entries need the DFT / direct-sum pass
  int32_t corr_lds;  // correlator arrays held in LDS for the launch
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
// (densities and marginals padded to even lengths: every region after the
// state starts 16-byte aligned)
__host__ __device__ constexpr size_t res_lds_bytes(int64_t n, int q, int s, int64_t lsum) {
  return res_state_bytes((size_t)q * (size_t)n * (size_t)s) + 8 * (size_t)((n + 1) & ~1ll) +
         8 * (size_t)((lsum + 1) & ~1ll) + 16 * (size_t)lsum + 8 * (size_t)kResScratch;
}

// Largest power of two p <= cap with items * p <= NT (at least 1).
template <int NT>
__device__ __forceinline__ int res_parts(int items, int cap) {
  int p = 1;
  while (p * 2 <= cap && items * (p * 2) <= NT) p *= 2;
  return p;
}

// Sum of a DFT over a line of L values m[0..L) with unit-stride phase steps:
//   sum_{x in [x0, x1)} (m[x] - mean) (cos, sgn sin)(2 pi k x / L)
__device__ __forceinline__ void res_line_dft(const double* m, int x0, int x1, int L, int k, double mean,
                                             const double* tw, double sgn, double& re, double& im) {
  int p = (int)(((unsigned)k * (unsigned)x0) % (unsigned)L);  // k, x0 < L <= 4096
  for (int x = x0; x < x1; ++x) {
    const double v = m[x] - mean;
    re += v * tw[2 * p];
    im += sgn * v * tw[2 * p + 1];
    p += k;
    if (p >= L) p -= L;
  }
}

// Lattice-sum slots a model uses: mass, sum f_i (Q), sum f_i f_j (i <= j),
// sum rho^2, sum rho^+, #rho < 0, #non-finite; the other of the 40 stay zero.
template <int D>
struct ResMom {
  static constexpr int Q = 2 * D + 1;
  static constexpr int NFF = Q * (Q + 1) / 2;
  static constexpr int NV = 1 + Q + NFF + 4;
  __device__ static constexpr int slot(int v) {
    return v == 0 ? 0 : (v <= Q ? v : (v <= Q + NFF ? 8 + (v - Q - 1) : 36 + (v - Q - NFF - 1)));
  }
};

// Adds this sample's lattice sums to mom (LDS, 40 slots).  Only waves that
// hold sites reduce (site = tid + NT j, so wave w holds sites iff 64 w < N).
template <int D, typename T, int SPT, int NT>
__device__ __forceinline__ void res_sample_moments(const T* st, int N, double* scr, double* mom,
                                                   const int (&sites)[SPT]) {
  using M = ResMom<D>;
  constexpr int Q = M::Q;
  double acc[M::NV];
#pragma unroll
  for (int v = 0; v < M::NV; ++v) acc[v] = 0.0;
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
      acc[M::NV - 1] += isfinite(f[i]) ? 0.0 : 1.0;
    }
    int k = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int l = i; l < Q; ++l) acc[1 + Q + k++] += f[i] * f[l];
    acc[0] += rho;
    acc[1 + Q + M::NFF] += rho * rho;
    acc[2 + Q + M::NFF] += rho > 0 ? rho : 0.0;
    acc[3 + Q + M::NFF] += rho < 0 ? 1.0 : 0.0;
  }
  if constexpr (NT == 256) {
    // through LDS, CV values at a time: the threads' values side by side,
    // then 32 threads per value add 8 consecutive ones, then one thread per
    // value adds the 32 partials (a few LDS rounds instead of a dependent
    // chain of lane moves per value)
    constexpr int CV = 7, PT = 32;  // CV * (256 + PT) doubles <= the scratch
    double* part = scr + CV * NT;
#pragma unroll
    for (int v0 = 0; v0 < M::NV; v0 += CV) {
#pragma unroll
      for (int c = 0; c < CV; ++c)
        if (v0 + c < M::NV) scr[c * NT + threadIdx.x] = acc[v0 + c];
      __syncthreads();
      if (threadIdx.x < CV * PT) {
        const int c = threadIdx.x / PT, q = threadIdx.x % PT;
        double a = 0;
#pragma unroll
        for (int j = 0; j < NT / PT; ++j) a += scr[c * NT + q * (NT / PT) + j];
        part[c * PT + q] = a;
      }
      __syncthreads();
      if (threadIdx.x < CV && v0 + (int)threadIdx.x < M::NV) {
        double r = 0;
        for (int q = 0; q < PT; ++q) r += part[threadIdx.x * PT + q];
        mom[M::slot(v0 + threadIdx.x)] += r;
      }
    }
    __syncthreads();
  } else {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwa = (N + 63) / 64 < NT / 64 ? (N + 63) / 64 : NT / 64;
    if (wave < nwa) {
#pragma unroll
      for (int v = 0; v < M::NV; ++v) {
        const double r = wave_sum_fixed(acc[v]);
        if (lane == 0) scr[wave * M::NV + v] = r;
      }
    }
    __syncthreads();
    if (threadIdx.x < M::NV) {
      double r = 0;
      for (int w = 0; w < nwa; ++w) r += scr[w * M::NV + threadIdx.x];
      mom[M::slot(threadIdx.x)] += r;
    }
    __syncthreads();
  }
}

// In-place radix-2 FFT of a line: X (2 L doubles, complex) receives
// sum_x (m[x] - mean) e^{-2 pi i k x / L} at index k.  L a power of two;
// tw holds (cos, sin)(2 pi j / L).  Whole-workgroup barriers between stages.
template <int NT>
__device__ __forceinline__ void res_fft_line(double* X, const double* m, int L, double mean, const double* tw) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  for (int x = threadIdx.x; x < L; x += NT) {
    const int r = (int)(__brev((unsigned)x) >> (32 - lg));
    X[2 * r] = m[x] - mean;
    X[2 * r + 1] = 0.0;
  }
  __syncthreads();
  for (int half = 1; half < L; half *= 2) {
    const int stride = L / (2 * half);
    for (int b = threadIdx.x; b < L / 2; b += NT) {
      const int j = b & (half - 1);
      const int i0 = (b - j) * 2 + j, i1 = i0 + half;
      const double c = tw[2 * j * stride], sn = -tw[2 * j * stride + 1];
      const double xr = X[2 * i1], xi = X[2 * i1 + 1];
      const double tr = c * xr - sn * xi, ti = c * xi + sn * xr;
      const double ur = X[2 * i0], ui = X[2 * i0 + 1];
      X[2 * i0] = ur + tr;
      X[2 * i0 + 1] = ui + ti;
      X[2 * i1] = ur - tr;
      X[2 * i1 + 1] = ui - ti;
    }
    __syncthreads();
  }
}

// Twiddle of k.x for a general wave vector (components reduced modulo L_a),
// sign sgn on the sine: (cos, sgn sin)(2 pi sum_a k_a x_a / L_a).
template <int D>
__device__ __forceinline__ void res_twiddle(const double* tw, int nx, int ny, int nz, int kx, int ky, int kz,
                                            int x, int y, int z, double sgn, double& c, double& s) {
  int m = (int)(((unsigned)kx * (unsigned)x) % (unsigned)nx);  // all below 4096
  c = tw[2 * m];
  s = tw[2 * m + 1];
  if constexpr (D >= 2) {
    m = (int)(((unsigned)ky * (unsigned)y) % (unsigned)ny);
    const double ar = tw[2 * (nx + m)], ai = tw[2 * (nx + m) + 1];
    const double t = c * ar - s * ai;
    s = c * ai + s * ar;
    c = t;
  }
  if constexpr (D >= 3) {
    m = (int)(((unsigned)kz * (unsigned)z) % (unsigned)nz);
    const double ar = tw[2 * (nx + ny + m)], ai = tw[2 * (nx + ny + m) + 1];
    const double t = c * ar - s * ai;
    s = c * ai + s * ar;
    c = t;
  }
  s *= sgn;
}

// LDS tables and accumulators that live for one launch (after the scratch):
//   mom[40]      lattice sums of this launch's samples
//   skl[ne]      S(k) sums of this launch's samples (ne padded to even)
//   ent[ne]      k-list entries: (code, kx, ky, kz); code -1: k = 0, a >= 0:
//                along axis a, -2: general
//   eslot[ne]    output slot of each entry (ne padded to a multiple of 4)
//   cki[cnk]     correlator wave vectors (kx, ky, kz, 0)
//   corr         if corr_lds: amp (2 Q cnk) | sij (2 Q Q cnk) | ct, ring (2 cnk nlag each)
__host__ __device__ constexpr size_t res_extra_bytes(int ne, int cnk, int q, int nlag, bool corr_lds) {
  return 8 * (size_t)kNV + 8 * (size_t)((ne + 1) & ~1) + 16 * (size_t)ne + 4 * (size_t)((ne + 3) & ~3) +
         16 * (size_t)cnk +
         (corr_lds ? 16 * ((size_t)q * cnk + (size_t)q * q * cnk + 2 * (size_t)cnk * nlag) : 0);
}

struct ResLocal {
  double* mom;
  double* skl;
  int4* ent;
  int* eslot;
  int4* cki;
  double *amp, *sij, *ct, *ring;  // LDS or HBM
};

template <int D, typename T, int SPT, int NT>
__device__ __forceinline__ void res_sample_sk(const ResArgs& A, const ResLocal& R, const T* st, double* rho,
                                              double* marg, const double* tw, double* scr,
                                              const int (&sites)[SPT]) {
  constexpr int Q = 2 * D + 1;
  const int nx = A.nx, ny = A.ny, nz = A.nz, N = nx * ny * nz;
  const int ne = A.nax + A.ngen;
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
  part = wave_sum_fixed(part);
  if (lane == 0) scr[wave] = part;
  __syncthreads();
  double M = 0;
  for (int w = 0; w < NT / 64; ++w) M += scr[w];
  const double mean = M / (double)N;
  for (int e = threadIdx.x; e < ne; e += NT)  // k = 0: the squared mass
    if (R.ent[e].x == -1) R.skl[e] += M * M / (double)N;
  double* mx = marg;
  double* my = marg + nx;
  double* mz = my + ny;
  __syncthreads();  // every thread has read the mass partials
  if constexpr (D >= 2) {  // axis marginals from rho, each a fixed-order sum
    for (int x = threadIdx.x; x < nx; x += NT) {
      double a = 0;
      for (int r = 0; r < ny * nz; ++r) a += rho[r * nx + x];
      mx[x] = a;
    }
    for (int y = threadIdx.x; y < ny; y += NT) {
      double a = 0;
      for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) a += rho[(y + ny * z) * nx + x];
      my[y] = a;
    }
    if constexpr (D >= 3) {
      for (int z = threadIdx.x; z < nz; z += NT) {
        double a = 0;
        for (int r = z * ny; r < (z + 1) * ny; ++r)
          for (int x = 0; x < nx; ++x) a += rho[r * nx + x];
        mz[z] = a;
      }
    }
    __syncthreads();
  }
  // axes whose entries come from an FFT of the marginal (bit a of sk_fft:
  // power-of-two extent that fits the scratch)
  for (int a = 0; a < D; ++a) {
    if (!(A.sk_fft & (1 << a))) continue;
    const int L = a == 0 ? nx : (a == 1 ? ny : nz);
    const double* m = D == 1 ? rho : (a == 0 ? mx : (a == 1 ? my : mz));
    res_fft_line<NT>(scr, m, L, M / (double)L, tw + 2 * (a == 0 ? 0 : (a == 1 ? nx : nx + ny)));
    for (int e = threadIdx.x; e < ne; e += NT) {
      const int4 en = R.ent[e];
      if (en.x != a) continue;
      const int k = a == 0 ? en.y : (a == 1 ? en.z : en.w);
      R.skl[e] += (scr[2 * k] * scr[2 * k] + scr[2 * k + 1] * scr[2 * k + 1]) / (double)N;
    }
    __syncthreads();
  }
  if (!A.sk_dft) return;
  // the remaining entries: DFT of the marginal along one axis, or the direct
  // sum over the sites for a general wave vector
  const int parts = res_parts<NT>(ne, 64);
  for (int t = threadIdx.x; t < ne * parts; t += NT) {
    const int e = t / parts, p = t % parts;
    const int4 en = R.ent[e];
    double re = 0, im = 0;
    if (en.x >= 0 && !(A.sk_fft & (1 << en.x))) {
      const int a = en.x;
      const int L = a == 0 ? nx : (a == 1 ? ny : nz);
      const int k = a == 0 ? en.y : (a == 1 ? en.z : en.w);
      const double* m = D == 1 ? rho : (a == 0 ? mx : (a == 1 ? my : mz));
      const double* twa = tw + 2 * (a == 0 ? 0 : (a == 1 ? nx : nx + ny));
      const int x0 = L * p / parts, x1 = L * (p + 1) / parts;
      res_line_dft(m, x0, x1, L, k, M / (double)L, twa, -1.0, re, im);
    } else if (en.x == -2) {
      for (int s = p; s < N; s += parts) {
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        double c, sn;
        res_twiddle<D>(tw, nx, ny, nz, en.y, en.z, en.w, x, y, z, -1.0, c, sn);
        const double v = rho[s] - mean;
        re += v * c;
        im += v * sn;
      }
    }
    scr[2 * t] = re;
    scr[2 * t + 1] = im;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += NT) {
    const int4 en = R.ent[e];
    if (en.x == -1 || (en.x >= 0 && (A.sk_fft & (1 << en.x)))) continue;
    double re = 0, im = 0;
    for (int p = 0; p < parts; ++p) {
      re += scr[2 * (e * parts + p)];
      im += scr[2 * (e * parts + p) + 1];
    }
    R.skl[e] += (re * re + im * im) / (double)N;
  }
  __syncthreads();
}

template <int D, typename T, int NT>
__device__ __forceinline__ void res_sample_corr(const ResArgs& A, const ResLocal& R, const T* st,
                                                const double* tw, double* scr, int64_t sidx, int rpos) {
  constexpr int Q = 2 * D + 1;
  const int nx = A.nx, ny = A.ny, nz = A.nz, N = nx * ny * nz, nrows = ny * nz;
  const int nk = A.cnk;
  const int items = nk * Q;
  // rows are split between parts (whole lines for the incremental phase),
  // except in 1-D where the single line is split
  const int parts = res_parts<NT>(items, D == 1 ? 64 : (nrows < 64 ? nrows : 64));
  for (int t = threadIdx.x; t < items * parts; t += NT) {
    const int kk = t / (Q * parts), i = (t / parts) % Q, p = t % parts;
    const int4 kv = R.cki[kk];
    const T* fi = st + i * N;
    double re = 0, im = 0;
    int r0 = 0, r1 = nrows, rs = 1, x0 = 0, x1 = nx;
    if (D == 1) {
      x0 = nx * p / parts;
      x1 = nx * (p + 1) / parts;
    } else {
      r0 = p;
      rs = parts;
    }
    for (int r = r0; r < r1; r += rs) {
      const int y = r % ny, z = r / ny;
      double rc, rsn;  // twiddle of the row's y, z part
      res_twiddle<D>(tw, nx, ny, nz, 0, kv.y, kv.z, 0, y, z, 1.0, rc, rsn);
      int px = (int)(((unsigned)kv.x * (unsigned)x0) % (unsigned)nx);
      const T* row = fi + r * nx;
      for (int x = x0; x < x1; ++x) {
        const double c = tw[2 * px] * rc - tw[2 * px + 1] * rsn;
        const double s = tw[2 * px] * rsn + tw[2 * px + 1] * rc;
        const double v = (double)row[x];
        re += v * c;
        im += v * s;
        px += kv.x;
        if (px >= nx) px -= nx;
      }
    }
    if (parts == 1) {
      R.amp[2 * t] = re;
      R.amp[2 * t + 1] = im;
    } else {
      scr[2 * t] = re;
      scr[2 * t + 1] = im;
    }
  }
  __syncthreads();
  if (parts > 1) {
    for (int u = threadIdx.x; u < items; u += NT) {
      double re = 0, im = 0;
      for (int p = 0; p < parts; ++p) {
        re += scr[2 * (u * parts + p)];
        im += scr[2 * (u * parts + p) + 1];
      }
      R.amp[2 * u] = re;
      R.amp[2 * u + 1] = im;
    }
    __syncthreads();
  }
  // S_ij, time correlator and ring (the arithmetic of k_corr_accumulate); a
  // C entry with l >= 1 reads ring slot (sidx - l) mod nlag, never the slot
  // rpos = sidx mod nlag written here.  Indices fit 32 bits (nk Q Q <= 50176,
  // nk nlag <= 2^20).
  const int nlag = A.nlag;
  const int ns = nk * Q * Q, nt = ns + nk * nlag;
  for (int t = threadIdx.x; t < nt; t += NT) {
    if (t < ns) {
      const int k = t / (Q * Q), i = (t / Q) % Q, j = t % Q;
      const double* a = R.amp + k * 2 * Q;
      const double ar = a[2 * i], ai = a[2 * i + 1], br = a[2 * j], bi = a[2 * j + 1];
      R.sij[2 * t] += ar * br + ai * bi;
      R.sij[2 * t + 1] += ai * br - ar * bi;
      if (i == 0 && j == 0) {
        double rr = 0, ri = 0;
        for (int q = 0; q < Q; ++q) {
          rr += a[2 * q];
          ri += a[2 * q + 1];
        }
        double* slot = R.ring + 2 * (rpos * nk + k);
        slot[0] = rr;
        slot[1] = ri;
      }
      continue;
    }
    const int u = t - ns;
    const int k = u / nlag, l = u % nlag;
    if (l > sidx) continue;
    const double* a = R.amp + k * 2 * Q;
    double rr = 0, ri = 0;
    for (int q = 0; q < Q; ++q) {
      rr += a[2 * q];
      ri += a[2 * q + 1];
    }
    double pr = rr, pi = ri;
    if (l > 0) {
      const int slot = rpos - l < 0 ? rpos - l + nlag : rpos - l;
      const double* old = R.ring + 2 * (slot * nk + k);
      pr = old[0];
      pi = old[1];
    }
    R.ct[2 * u] += pr * rr + pi * ri;
    R.ct[2 * u + 1] += pi * rr - pr * ri;
  }
  __syncthreads();
}

template <int D, typename T, int SPT, int NT>
__global__ void __launch_bounds__(NT) k_resident(KParams<T> P, ResArgs A) {
  constexpr int Q = 2 * D + 1;
  extern __shared__ __align__(16) unsigned char res_smem[];
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int N = nx * ny * nz;
  const int lsum = nx + ny + nz;
  const int ne = A.sk_every > 0 ? A.nax + A.ngen : 0;
  const int cnk = A.corr_every > 0 ? A.cnk : 0;
  T* st = (T*)res_smem;
  double* rho = (double*)(res_smem + res_state_bytes((size_t)Q * N * sizeof(T)));
  double* marg = rho + ((N + 1) & ~1);
  double* tw = marg + ((lsum + 1) & ~1);
  double* scr = tw + 2 * lsum;
  ResLocal R;
  R.mom = scr + kResScratch;
  R.skl = R.mom + kNV;
  R.ent = (int4*)(R.skl + ((ne + 1) & ~1));
  R.eslot = (int*)(R.ent + ne);
  R.cki = (int4*)(R.eslot + ((ne + 3) & ~3));
  const int nsij = 2 * Q * Q * cnk, nct = 2 * cnk * A.nlag;
  if (A.corr_lds) {
    R.amp = (double*)(R.cki + cnk);
    R.sij = R.amp + 2 * Q * cnk;
    R.ct = R.sij + nsij;
    R.ring = R.ct + nct;
  } else {
    R.amp = A.amp;
    R.sij = A.sij;
    R.ct = A.ct;
    R.ring = A.ring;
  }
  const int tid = threadIdx.x;
  for (int m = tid; m < 2 * lsum; m += NT) tw[m] = A.tw[m];
  for (int v = tid; v < kNV; v += NT) R.mom[v] = 0.0;
  for (int e = tid; e < ne; e += NT) {
    R.skl[e] = 0.0;
    int4 en;
    if (e < A.nax) {
      const int a = (int)A.kinfo[2 * e], k = (int)A.kinfo[2 * e + 1];
      en = make_int4(a, a == 0 ? k : 0, a == 1 ? k : 0, a == 2 ? k : 0);
      R.eslot[e] = A.slot_ax[e];
    } else {
      const int64_t* kk = A.kv + 3 * (e - A.nax);
      const int nnz = (kk[0] != 0) + (kk[1] != 0) + (kk[2] != 0);
      const int a = nnz == 0 ? -1 : (nnz > 1 ? -2 : (kk[0] != 0 ? 0 : (kk[1] != 0 ? 1 : 2)));
      en = make_int4(a, (int)kk[0], (int)kk[1], (int)kk[2]);
      R.eslot[e] = A.slot_gen[e - A.nax];
    }
    R.ent[e] = en;
  }
  for (int k = tid; k < cnk; k += NT)
    R.cki[k] = make_int4(A.ckinfo[3 * k], A.ckinfo[3 * k + 1], A.ckinfo[3 * k + 2], 0);
  if (A.corr_lds) {
    for (int m = tid; m < nsij; m += NT) R.sij[m] = A.sij[m];
    for (int m = tid; m < nct; m += NT) {
      R.ct[m] = A.ct[m];
      R.ring[m] = A.ring[m];
    }
  }
  // canonical state f_i(x) = g_i(x - v_i); coordinates of this thread's sites
  const T* g = (const T*)A.gin;
  int sites[SPT], cx[SPT], cy[SPT], cz[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int s = tid + NT * j;
    sites[j] = s;
    cx[j] = s % nx;
    cy[j] = (s / nx) % ny;
    cz[j] = s / (nx * ny);
    if (s < N) {
      const Nbr b = neighbours(cx[j], cy[j], cz[j], nx, ny, nz);
      T fv[Q];
      gather<D, T>(g, N, b, fv, A.form_in);
#pragma unroll
      for (int i = 0; i < Q; ++i) st[i * N + s] = fv[i];
    }
  }
  __syncthreads();
  // steps until the next sample of each kind (0: this step), counted down
  // instead of a 64-bit modulo per step
  int64_t cm = A.mom_every > 0 ? (A.mom_every - A.step0 % A.mom_every) % A.mom_every : -1;
  int64_t cc = cnk > 0 ? (A.corr_every - A.step0 % A.corr_every) % A.corr_every : -1;
  int64_t cs = ne > 0 ? (A.sk_every - A.step0 % A.sk_every) % A.sk_every : -1;
  int64_t csamp = A.corr_s0;
  int rpos = cnk > 0 ? (int)(A.corr_s0 % A.nlag) : 0;
  T* out = (T*)A.gout;
  for (int k = 0; k < A.nsteps; ++k) {
    const int64_t t = A.step0 + k;
    if (cm == 0) {
      res_sample_moments<D, T, SPT, NT>(st, N, scr, R.mom, sites);
      cm = A.mom_every;
    }
    if (cc == 0) {
      res_sample_corr<D, T, NT>(A, R, st, tw, scr, csamp++, rpos);
      rpos = rpos + 1 == A.nlag ? 0 : rpos + 1;
      cc = A.corr_every;
    }
    if (cs == 0) {
      res_sample_sk<D, T, SPT, NT>(A, R, st, rho, marg, tw, scr, sites);
      cs = A.sk_every;
    }
    --cm;
    --cc;
    --cs;
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
    } else if (A.form_out == kFormPull) {
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        if (sites[j] < N) {
#pragma unroll
          for (int i = 0; i < Q; ++i) out[(int64_t)i * N + sites[j]] = f[j][i];
        }
      }
    } else {
      // single buffer: form S keeps f_i* in the opposite slot at the site,
      // form C pushes it to slot i of the neighbour x + v_i
      const bool sw = A.form_out == kFormAAS;
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int s = sites[j];
        if (s < N) {
          const Nbr b = neighbours(cx[j], cy[j], cz[j], nx, ny, nz);
          out[s] = f[j][0];
          out[(int64_t)(sw ? 2 : 1) * N + (sw ? s : b.sxp)] = f[j][1];
          out[(int64_t)(sw ? 1 : 2) * N + (sw ? s : b.sxm)] = f[j][2];
          if constexpr (D >= 2) {
            out[(int64_t)(sw ? 4 : 3) * N + (sw ? s : b.syp)] = f[j][3];
            out[(int64_t)(sw ? 3 : 4) * N + (sw ? s : b.sym)] = f[j][4];
          }
          if constexpr (D >= 3) {
            out[(int64_t)(sw ? 6 : 5) * N + (sw ? s : b.szp)] = f[j][5];
            out[(int64_t)(sw ? 5 : 6) * N + (sw ? s : b.szm)] = f[j][6];
          }
        }
      }
    }
    __syncthreads();
  }
  // flush this launch's sums
  if (A.mom_every > 0)
    for (int v = tid; v < kNV; v += NT) A.momacc[v] += R.mom[v];
  for (int e = tid; e < ne; e += NT) A.skacc[R.eslot[e]] += R.skl[e];
  if (A.corr_lds) {
    for (int m = tid; m < nsij; m += NT) A.sij[m] = R.sij[m];
    for (int m = tid; m < nct; m += NT) {
      A.ct[m] = R.ct[m];
      A.ring[m] = R.ring[m];
    }
  }
}

}  // namespace flb
