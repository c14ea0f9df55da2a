// Population correlators of the equilibrium analysis (Sec. IV):
//   Fourier sums   f_i(k, t) = sum_x exp(+2 pi i k.x / L) f_i(x, t)   (paper's sign)
//   structure      S_ij(k)  += f_i(k, t) conj(f_j(k, t))              (eqs. fkfk, FourierTest)
//   time           C(k, l)  += rho(k, t_s) conj(rho(k, t_{s+l}))       (eq. TimeCorrEqn)
// with rho(k) = sum_i f_i(k) and t_s the s-th sampled step.  All sums in FP64,
// in a fixed order, so repeated runs give identical bits.
//
// Included by flb.hip only (non-template kernels).
#pragma once

#include "flb_stats.hpp"

namespace flb {

constexpr int kCorrKC = 4;  // wave vectors per workgroup in the amplitude pass

// Partial Fourier sums of the canonical populations.  Workgroup (sb, kg)
// takes the sites s = sb*256 + tid + m*nsb*256 and the wave vectors
// kg*KC .. kg*KC+KC-1; kinfo holds (k_x mod L_x, k_y mod L_y, k_z mod L_z).
// tw is the concatenated twiddle table of the axes, (cos, sin)(2 pi m / L_a).
// part[(sb * nk + k) * 2Q + 2i + {0, 1}] = (re, im) of the workgroup's sum.
template <int D, typename T>
__global__ void __launch_bounds__(256) k_amp_partial(const T* __restrict__ g, int64_t nx, int64_t ny,
                                                     int64_t nz, const double* __restrict__ tw,
                                                     const int32_t* __restrict__ kinfo, int nk, int nsb,
                                                     double* __restrict__ part, int form = kFormPull) {
  constexpr int Q = 2 * D + 1;
  constexpr int KC = kCorrKC;
  __shared__ double lds[4];
  const int64_t n = nx * ny * nz;
  const int sb = blockIdx.x;
  const int k0 = blockIdx.y * KC;
  const double* twx = tw;
  const double* twy = tw + 2 * nx;
  const double* twz = tw + 2 * (nx + ny);
  int64_t kx[KC], ky[KC], kz[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int k = k0 + c < nk ? k0 + c : k0;
    kx[c] = kinfo[3 * k];
    ky[c] = kinfo[3 * k + 1];
    kz[c] = kinfo[3 * k + 2];
  }
  double re[KC][Q], im[KC][Q];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int i = 0; i < Q; ++i) re[c][i] = im[c][i] = 0.0;
  for (int64_t s = (int64_t)sb * 256 + threadIdx.x; s < n; s += (int64_t)nsb * 256) {
    const int64_t x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
    const Nbr b = neighbours(x, y, z, nx, ny, nz);
    T fv[Q];
    gather<D, T>(g, n, b, fv, form);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      double cr = twx[2 * ((kx[c] * x) % nx)], ci = twx[2 * ((kx[c] * x) % nx) + 1];
      if constexpr (D >= 2) {
        const int64_t m = (ky[c] * y) % ny;
        const double ar = twy[2 * m], ai = twy[2 * m + 1];
        const double tr = cr * ar - ci * ai;
        ci = cr * ai + ci * ar;
        cr = tr;
      }
      if constexpr (D >= 3) {
        const int64_t m = (kz[c] * z) % nz;
        const double ar = twz[2 * m], ai = twz[2 * m + 1];
        const double tr = cr * ar - ci * ai;
        ci = cr * ai + ci * ar;
        cr = tr;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        re[c][i] += (double)fv[i] * cr;
        im[c][i] += (double)fv[i] * ci;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double r = block_sum256(re[c][i], lds);
      const double m = block_sum256(im[c][i], lds);
      if (threadIdx.x == 0 && k0 + c < nk) {
        double* o = part + ((int64_t)sb * nk + k0 + c) * 2 * Q + 2 * i;
        o[0] = r;
        o[1] = m;
      }
    }
  }
}

// amp[k * 2Q + j] = sum over sb (in order) of part[(sb * nk + k) * 2Q + j].
__global__ void k_amp_final(const double* __restrict__ part, int nsb, int nk, int q2,
                            double* __restrict__ amp) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)nk * q2) return;
  double acc = 0;
  for (int sb = 0; sb < nsb; ++sb) acc += part[(int64_t)sb * nk * q2 + j];
  amp[j] = acc;
}

// Accumulate one sample s (0-based) from amp (nk x Q complex):
//   sij[(k*Q + i)*Q + j] += a_i conj(a_j)
//   ct[k*nlag + l]       += r(s - l) conj(r(s)),  l <= min(s, nlag - 1)
//   ring[(s mod nlag) * nk + k] = r(s)
// Threads [0, nk*Q*Q) do S_ij, threads [nk*Q*Q, nk*Q*Q + nk*nlag) do C.  A
// C thread with l >= 1 reads ring slot (s - l) mod nlag, never the slot
// (s mod nlag) that the k-th S_ij thread (i = j = 0) overwrites.
__global__ void k_corr_accumulate(const double* __restrict__ amp, int nk, int Q, int nlag, int64_t s,
                                  double* __restrict__ sij, double* __restrict__ ring,
                                  double* __restrict__ ct) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = (int64_t)nk * Q * Q;
  auto rho_of = [&](int k, double& rr, double& ri) {
    rr = 0;
    ri = 0;
    for (int i = 0; i < Q; ++i) {
      rr += amp[(int64_t)k * 2 * Q + 2 * i];
      ri += amp[(int64_t)k * 2 * Q + 2 * i + 1];
    }
  };
  if (t < ns) {
    const int k = (int)(t / (Q * Q));
    const int i = (int)((t / Q) % Q), j = (int)(t % Q);
    const double* a = amp + (int64_t)k * 2 * Q;
    const double ar = a[2 * i], ai = a[2 * i + 1], br = a[2 * j], bi = a[2 * j + 1];
    sij[2 * t] += ar * br + ai * bi;
    sij[2 * t + 1] += ai * br - ar * bi;
    if (i == 0 && j == 0) {
      double rr, ri;
      rho_of(k, rr, ri);
      double* slot = ring + 2 * ((s % nlag) * (int64_t)nk + k);
      slot[0] = rr;
      slot[1] = ri;
    }
    return;
  }
  const int64_t u = t - ns;
  if (u >= (int64_t)nk * nlag) return;
  const int k = (int)(u / nlag), l = (int)(u % nlag);
  if (l > s) return;
  double rr, ri;
  rho_of(k, rr, ri);
  double pr = rr, pi = ri;
  if (l > 0) {
    const double* old = ring + 2 * (((s - l) % nlag) * (int64_t)nk + k);
    pr = old[0];
    pi = old[1];
  }
  ct[2 * u] += pr * rr + pi * ri;
  ct[2 * u + 1] += pi * rr - pr * ri;
}

}  // namespace flb
