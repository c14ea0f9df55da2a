// C ABI of the fluctuating lattice Boltzmann library (declared in flb.h):
// parameter validation, lattice handles, launch configuration of the step,
// lattice sums, structure factor and the noise sampler.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flb.h"
#include "flb_internal.hpp"
#include "flb_kernels.hpp"
#include "flb_stats.hpp"
#include "flb_corr.hpp"
#include "flb_resident.hpp"

using namespace flb;

static_assert(kNV == kNVals, "lattice-sum count");

// ---------------------------------------------------------------------------
// errors
namespace flb {
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FLB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace flb

#define HIP_TRY(expr)                                \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

// ---------------------------------------------------------------------------
// constants of the product side (Sec. II closed forms)
namespace flb {

double default_theta(int d) { return d == 3 ? 0.25 : 1.0 / 3.0; }

int check_params(const flb_params* p) {
  if (!p) return fail(FLB_EINVAL, "params is NULL");
  if (p->model < 1 || p->model > 3) return fail(FLB_EINVAL, "model must be 1 (D1Q3), 2 (D2Q5) or 3 (D3Q7)");
  if (p->precision != 4 && p->precision != 8) return fail(FLB_EINVAL, "precision must be 4 or 8");
  const int d = p->model;
  for (int a = 0; a < 3; ++a) {
    if (p->n[a] < 1) return fail(FLB_EINVAL, "box size n[%d] = %lld must be >= 1", a, (long long)p->n[a]);
    if (a >= d && p->n[a] != 1) return fail(FLB_EINVAL, "n[%d] must be 1 for a %d-D model", a, d);
  }
  const double n = (double)p->n[0] * (double)p->n[1] * (double)p->n[2];
  if (n * (2 * d + 1) * p->precision > 9.0e18) return fail(FLB_EINVAL, "lattice too large");
  // the row kernel indexes columns and rows in 32 bits
  if (p->n[0] * p->precision >= (1ll << 32) || p->n[1] * p->n[2] >= (1ll << 31))
    return fail(FLB_EINVAL, "rows of n[0] values must be under 4 GiB and n[1] * n[2] below 2^31");
  const double th = p->theta == 0.0 ? default_theta(d) : p->theta;
  if (!(th > 0.0 && th < 1.0 / d)) return fail(FLB_EINVAL, "theta = %g outside (0, 1/%d)", th, d);
  if (!(p->omega[0] > 0.0 && p->omega[0] < 2.0)) return fail(FLB_EINVAL, "omega_j = %g outside (0, 2)", p->omega[0]);
  for (int a = 1; a < 3; ++a)
    if (p->omega[a] != 0.0 && !(p->omega[a] > 0.0 && p->omega[a] < 2.0))
      return fail(FLB_EINVAL, "omega[%d] = %g outside (0, 2)", a, p->omega[a]);
  if (p->noise < 0 || p->noise > 2) return fail(FLB_EINVAL, "noise must be 0 (local), 1 (global) or 2 (off)");
  if (p->noise_law < 0 || p->noise_law > 1) return fail(FLB_EINVAL, "noise_law must be 0 (Gauss) or 1 (uniform)");
  if (p->layout != FLB_LAYOUT_TWO_BUFFER && p->layout != FLB_LAYOUT_AA)
    return fail(FLB_EINVAL, "layout must be FLB_LAYOUT_TWO_BUFFER or FLB_LAYOUT_AA");
  if (p->layout == FLB_LAYOUT_AA) {
    if (p->kernel != FLB_KERNEL_AUTO && p->kernel != FLB_KERNEL_FLAT && p->kernel != FLB_KERNEL_RESIDENT)
      return fail(FLB_EINVAL, "the AA layout steps with the flat or resident kernels (kernel 0, 3 or 4)");
    if (n * (2 * d + 1) * p->precision >= 4294967296.0)
      return fail(FLB_EINVAL, "the AA layout needs Q * N * precision < 2^32 (the flat kernel's 32-bit offsets)");
    if (p->tile_rows > 8) return fail(FLB_EINVAL, "AA layout (flat kernel): tile_rows <= 8");
  }
  if (p->kernel < 0 || p->kernel > 5)
    return fail(FLB_EINVAL, "kernel must be 0 (auto), 1 (plain), 2 (rows), 3 (flat), 4 (resident) or 5 (two-step)");
  if (p->kernel == FLB_KERNEL_TWO_STEP &&
      (d != 2 || p->tile_rows > 16 || n * (2 * d + 1) * p->precision >= 4294967296.0))
    return fail(FLB_EINVAL, "two-step kernel: D2Q5 only, tile_rows <= 16, Q * N * precision < 2^32");
  if (p->kernel == FLB_KERNEL_FLAT && (p->tile_rows > 8 || n * (2 * d + 1) * p->precision >= 4294967296.0))
    return fail(FLB_EINVAL, "flat kernel: tile_rows <= 8 and Q * N * precision < 2^32");
  if (p->tile_x != 0 && (p->tile_x < 64 || p->tile_x > 1024 || p->tile_x % 64 != 0))
    return fail(FLB_EINVAL, "tile_x must be a multiple of 64 in [64, 1024]");
  if (p->nt_store != 0 && p->nt_store != 1) return fail(FLB_EINVAL, "nt_store must be 0 or 1");
  if (p->pipeline != 0 && p->pipeline != 1) return fail(FLB_EINVAL, "pipeline must be 0 or 1");
  if (p->tile_rows != 0 && p->tile_rows != 1 && p->tile_rows != 2 && p->tile_rows != 4 &&
      p->tile_rows != 8 && p->tile_rows != 16)
    return fail(FLB_EINVAL, "tile_rows must be 1, 2, 4, 8 or 16");
  return FLB_OK;
}

template <typename T>
KParams<T> make_kparams(const flb_params& p, double rho_eq) {
  const int d = p.model;
  const double th = p.theta == 0.0 ? default_theta(d) : p.theta;
  const double oj = p.omega[0];
  const double on = p.omega[1] != 0.0 ? p.omega[1] : oj;
  const double os = p.omega[2] != 0.0 ? p.omega[2] : oj;
  const double law = p.noise_law == FLB_LAW_UNIFORM ? std::sqrt(3.0) : 1.0;
  KParams<T> k;
  k.nx = p.n[0];
  k.ny = p.n[1];
  k.nz = p.n[2];
  k.n = p.n[0] * p.n[1] * p.n[2];
  k.rho_eq = (T)rho_eq;
  // folded products of the collision (in double, rounded once)
  const double a = 1.0 / std::sqrt(th), b = 1.0 / std::sqrt(2.0 * th), e = 1.0 / std::sqrt(6.0 * th);
  const double c0 = std::sqrt(d * th / (1.0 - d * th)), c1 = std::sqrt((1.0 - d * th) / (d * th));
  const double w1 = th / 2.0;
  const double sj = law * std::sqrt(oj * (2.0 - oj)), sn = law * std::sqrt(on * (2.0 - on));
  const double ss = law * std::sqrt(os * (2.0 - os));
  k.nA = (T)(w1 * a * sj);
  k.nB = (T)(w1 * b * sn);
  k.nC = (T)(w1 * c1 * ss);
  k.nE = (T)(w1 * e * sn);
  k.kj = (T)(w1 * a * a * oj);
  k.kn = (T)(w1 * b * b * on);
  k.ke = (T)(w1 * e * e * on);
  k.ks = (T)(w1 * c1 * c1 * os);
  k.ks0 = (T)(w1 * c1 * c0 * os);
  k.k0 = (uint32_t)(p.seed & 0xFFFFFFFFull);
  k.k1 = (uint32_t)(p.seed >> 32);
  k.noise = p.noise;
  k.law = p.noise_law;
  return k;
}
template KParams<float> make_kparams<float>(const flb_params&, double);
template KParams<double> make_kparams<double>(const flb_params&, double);

}  // namespace flb

// ---------------------------------------------------------------------------
// workspace layout
namespace flb {

WorkLayout work_layout(const flb_params& p) {
  WorkLayout L{};
  const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2];
  const int64_t nrows = ny * nz;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.red_part = take(sizeof(double) * kRedBlocks * kNV);
  L.red_out = take(sizeof(double) * kNV);
  if (p.model >= 2) {
    L.rowsum = take(sizeof(double) * nrows);
    L.colpart = take(sizeof(double) * std::min<int64_t>(kColChunks, nrows) * nx);
    L.marg = take(sizeof(double) * (nx + ny + nz));
    L.rowpart = take(sizeof(double) * ((nx + 255) / 256) * nrows);
    L.colbig = take(sizeof(double) * ((nrows + kSampleRows - 1) / kSampleRows) * nx);
  }
  L.tw = take(sizeof(double) * 2 * (nx + ny + nz));
  L.skpart = take(sizeof(double) * 2 * (size_t)kMaxK * kSkChunks);
  for (int s = 0; s < 2; ++s) {
    L.kinfo[s] = take(sizeof(int64_t) * 2 * kMaxK);
    L.kv[s] = take(sizeof(int64_t) * 3 * kMaxK);
    L.slot_ax[s] = take(sizeof(int32_t) * kMaxK);
    L.slot_gen[s] = take(sizeof(int32_t) * kMaxK);
    L.sval[s] = take(sizeof(double) * kMaxK);
  }
  L.skacc = take(sizeof(double) * kMaxK);
  L.momacc = take(sizeof(double) * kNVals);
  L.total = o;
  return L;
}

}  // namespace flb

namespace flb {

// the two buffers of the pull scheme; the single buffer of the AA layout
char* lat_buffer(flb_lattice* h, int which) { return h->aa ? h->pop : h->pop + (size_t)which * h->plane; }

// form of the stored state: pull storage, or the AA parity (cur counts steps mod 2)
int state_form(const flb_lattice* h) { return !h->aa ? kFormPull : (h->cur ? kFormAAS : kFormAAC); }

// ---------------------------------------------------------------------------
// step launch
template <int D, typename T>
int launch_step_t(flb_lattice* h, const T* g, T* out, uint32_t step, hipStream_t st) {
  if (h->reg_n > 0) {
    k_step_regions<D, T><<<(unsigned)((h->n + 255) / 256), 256, 0, st>>>(
        g, out, (const KParams<T>*)h->reg_tab, h->reg_n, h->reg_map, h->n, step);
    return 0;
  }
  const KParams<T> P = make_kparams<T>(h->p, h->rho_eq);
  if (h->aa) {  // in place on the single buffer, from the current parity's form
    T* a = out;
    const int ry = h->p.tile_rows ? h->p.tile_rows : (D == 2 ? 2 : 1);
    const int64_t nb = (h->n + 256 * ry - 1) / (256 * ry);
    const bool nt = h->p.nt_store != 0;
    const bool even = state_form(h) == kFormAAC;
    const bool lg = h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
#define FLB_AA1(NTV, FV)                                                                                        \
  (lg ? (void)(k_step_flat_aa<D, T, RYV, NTV, FV, kPlanLocalGauss><<<(unsigned)nb, 256, 0, st>>>(a, P, step)) \
      : (void)(k_step_flat_aa<D, T, RYV, NTV, FV><<<(unsigned)nb, 256, 0, st>>>(a, P, step)))
#define FLB_AA(RYV_)                                                                      \
  {                                                                                       \
    constexpr int RYV = RYV_;                                                             \
    if (even) { if (nt) FLB_AA1(true, kFormAAC); else FLB_AA1(false, kFormAAC); }         \
    else { if (nt) FLB_AA1(true, kFormAAS); else FLB_AA1(false, kFormAAS); }              \
  }
    switch (ry) {
      case 1: FLB_AA(1) break;
      case 2: FLB_AA(2) break;
      case 4: FLB_AA(4) break;
      default: FLB_AA(8) break;
    }
#undef FLB_AA
#undef FLB_AA1
    return FLB_OK;
  }
  // single steps of a two-step lattice take the flat kernel (2 rows per tile)
  const int kern = h->p.kernel == FLB_KERNEL_AUTO ? FLB_KERNEL_ROWS
                   : (h->p.kernel == FLB_KERNEL_TWO_STEP ? FLB_KERNEL_FLAT : h->p.kernel);
  if (kern == FLB_KERNEL_PLAIN) {
    const int64_t nb = (h->n + 255) / 256;
    k_step_plain<D, T><<<dim3((unsigned)nb), dim3(256), 0, st>>>(g, out, P, step);
  } else if (kern == FLB_KERNEL_FLAT) {
    const int ry = h->p.kernel == FLB_KERNEL_TWO_STEP ? 2 : (h->p.tile_rows ? h->p.tile_rows : 2);
    const int64_t nb = (h->n + 256 * ry - 1) / (256 * ry);
    const bool nt = h->p.nt_store != 0;
    // local Gaussian noise (the default) takes the instances with that noise plan fixed at compile time
    const bool lg = h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
#define FLB_FLAT(RYV)                                                                                             \
  (lg ? (nt ? (void)(k_step_flat<D, T, RYV, true, kPlanLocalGauss><<<(unsigned)nb, 256, 0, st>>>(g, out, P, step))  \
            : (void)(k_step_flat<D, T, RYV, false, kPlanLocalGauss><<<(unsigned)nb, 256, 0, st>>>(g, out, P, step))) \
      : (nt ? (void)(k_step_flat<D, T, RYV, true><<<(unsigned)nb, 256, 0, st>>>(g, out, P, step))                   \
            : (void)(k_step_flat<D, T, RYV, false><<<(unsigned)nb, 256, 0, st>>>(g, out, P, step))))
    switch (ry) {
      case 1: FLB_FLAT(1); break;
      case 2: FLB_FLAT(2); break;
      case 4: FLB_FLAT(4); break;
      default: FLB_FLAT(8); break;
    }
#undef FLB_FLAT
  } else {
    const int bx = h->p.tile_x ? h->p.tile_x : 256;
    const int ry = D == 1 ? 1 : (h->p.tile_rows ? h->p.tile_rows : 4);
    const int64_t nrows = P.ny * P.nz;
    const int64_t tiles_x = (P.nx + bx - 1) / bx;
    const int64_t tiles_r = (nrows + ry - 1) / ry;
    const int64_t G = tiles_x * tiles_r;
    const int remap = 1;
    dim3 grid((unsigned)G), block((unsigned)bx);
    const bool nt = h->p.nt_store != 0;
    const bool pipe = h->p.pipeline != 0;
#define FLB_ROWS(RYV)                                                                                    \
  (pipe ? (nt ? (void)(k_step_rows<D, T, RYV, true, true><<<grid, block, 0, st>>>(g, out, P, step, tiles_x, nrows, remap))   \
              : (void)(k_step_rows<D, T, RYV, false, true><<<grid, block, 0, st>>>(g, out, P, step, tiles_x, nrows, remap)))  \
        : (nt ? (void)(k_step_rows<D, T, RYV, true><<<grid, block, 0, st>>>(g, out, P, step, tiles_x, nrows, remap))         \
              : (void)(k_step_rows<D, T, RYV, false><<<grid, block, 0, st>>>(g, out, P, step, tiles_x, nrows, remap))))
    switch (ry) {
      case 1: FLB_ROWS(1); break;
      case 2: FLB_ROWS(2); break;
      case 4: FLB_ROWS(4); break;
      case 8: FLB_ROWS(8); break;
      default: FLB_ROWS(16); break;
    }
#undef FLB_ROWS
  }
  return FLB_OK;
}

int launch_step(flb_lattice* h, const void* g, void* out, uint32_t step, hipStream_t st) {
  if (h->s == 4) {
    switch (h->d) {
      case 1: return launch_step_t<1, float>(h, (const float*)g, (float*)out, step, st);
      case 2: return launch_step_t<2, float>(h, (const float*)g, (float*)out, step, st);
      default: return launch_step_t<3, float>(h, (const float*)g, (float*)out, step, st);
    }
  }
  switch (h->d) {
    case 1: return launch_step_t<1, double>(h, (const double*)g, (double*)out, step, st);
    case 2: return launch_step_t<2, double>(h, (const double*)g, (double*)out, step, st);
    default: return launch_step_t<3, double>(h, (const double*)g, (double*)out, step, st);
  }
}

// canonical conversions
template <typename T>
void launch_convert_t(int d, bool to_canon, const T* src, T* dst, int64_t nx, int64_t ny, int64_t nz,
                      hipStream_t st, int form) {
  const int64_t n = nx * ny * nz;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  if (to_canon) {
    if (d == 1) k_to_canonical<1, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz, form);
    else if (d == 2) k_to_canonical<2, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz, form);
    else k_to_canonical<3, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz, form);
  } else {
    if (d == 1) k_from_canonical<1, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz);
    else if (d == 2) k_from_canonical<2, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz);
    else k_from_canonical<3, T><<<nb, 256, 0, st>>>(src, dst, nx, ny, nz);
  }
}

// to_canon: the canonical state from src stored in `form`; else the pull
// storage form from canonical src
void launch_convert(flb_lattice* h, bool to_canon, const void* src, void* dst, int form = kFormPull) {
  if (h->s == 4)
    launch_convert_t<float>(h->d, to_canon, (const float*)src, (float*)dst, h->p.n[0], h->p.n[1], h->p.n[2], h->stream,
                            form);
  else
    launch_convert_t<double>(h->d, to_canon, (const double*)src, (double*)dst, h->p.n[0], h->p.n[1], h->p.n[2],
                             h->stream, form);
}

// lattice sums into work.red_out (device)
template <int D, typename T>
void launch_moments_t(flb_lattice* h, const T* g) {
  const int64_t units = h->p.n[1] * h->p.n[2] * ((h->p.n[0] + kMomSeg<D> - 1) / kMomSeg<D>);
  const int64_t nb = std::min<int64_t>(units, kRedBlocks);
  double* part = (double*)(h->work + h->wl.red_part);
  double* out = (double*)(h->work + h->wl.red_out);
  // pull-form states under 4 GiB take the buffer-resource loads
  if (state_form(h) == kFormPull && h->plane < (1ull << 32) && (int64_t)h->Q * h->n * (int64_t)h->s < (1ll << 32))
    k_moments_partial<D, T, true><<<(unsigned)nb, 256, 0, h->stream>>>(g, h->p.n[0], h->p.n[1], h->p.n[2], part);
  else
    k_moments_partial<D, T><<<(unsigned)nb, 256, 0, h->stream>>>(g, h->p.n[0], h->p.n[1], h->p.n[2], part,
                                                                  state_form(h));
  k_moments_final<<<kNV, 256, 0, h->stream>>>(part, (int)nb, out);
}

void launch_moments(flb_lattice* h) {
  const void* g = lat_buffer(h, h->cur);
  if (h->s == 4) {
    if (h->d == 1) launch_moments_t<1, float>(h, (const float*)g);
    else if (h->d == 2) launch_moments_t<2, float>(h, (const float*)g);
    else launch_moments_t<3, float>(h, (const float*)g);
  } else {
    if (h->d == 1) launch_moments_t<1, double>(h, (const double*)g);
    else if (h->d == 2) launch_moments_t<2, double>(h, (const double*)g);
    else launch_moments_t<3, double>(h, (const double*)g);
  }
}

// kernel constants of every region (theta, rates, the lattice's noise set-up
// and global-noise density) into the device table; synchronous
template <typename T>
int rebuild_regions_t(flb_lattice* h) {
  KParams<T> tab[kMaxRegions];
  for (int r = 0; r < h->reg_n; ++r) {
    flb_params q = h->p;
    q.theta = h->reg_theta[r];
    for (int a = 0; a < 3; ++a) q.omega[a] = h->reg_omega[r][a];
    tab[r] = make_kparams<T>(q, h->rho_eq);
  }
  HIP_TRY(hipMemcpyAsync(h->reg_tab, tab, sizeof(KParams<T>) * h->reg_n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FLB_OK;
}

int rebuild_regions(flb_lattice* h) { return h->s == 4 ? rebuild_regions_t<float>(h) : rebuild_regions_t<double>(h); }

// resident small lattice: `c` steps in one launch, sampling inside
int64_t multiples_in(int64_t t0, int64_t c, int64_t every) {
  if (every <= 0 || c <= 0) return 0;
  const int64_t first = (t0 + every - 1) / every * every, last = t0 + c - 1;
  return first > last ? 0 : (last - first) / every + 1;
}

// LDS bytes of a resident launch with the current sampling set-up, and
// whether the correlator arrays go to LDS; false when even the tables do not
// fit (flb_step then uses the HBM kernels).
bool resident_lds(const flb_lattice* h, size_t* lds, int* corr_lds) {
  const int ne = h->sample_every > 0 ? h->nk[1] : 0;
  const int cnk = h->corr_mem && h->corr_every > 0 ? h->corr_nk : 0;
  const size_t with = h->res_lds + res_extra_bytes(ne, cnk, h->Q, h->corr_nlag, cnk > 0);
  const size_t without = h->res_lds + res_extra_bytes(ne, cnk, h->Q, h->corr_nlag, false);
  if (with <= (size_t)h->res_lds_max) {
    *lds = with;
    *corr_lds = cnk > 0;
    return true;
  }
  if (without <= (size_t)h->res_lds_max) {
    *lds = without;
    *corr_lds = 0;
    return true;
  }
  return false;
}

template <int D, typename T, int SPT, int NT>
void launch_resident_spt(flb_lattice* h, const ResArgs& A, size_t lds) {
  static bool attr = false;  // raise the dynamic LDS limit once per instantiation
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_resident<D, T, SPT, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              h->res_lds_max);
    (void)hipGetLastError();
    attr = true;
  }
  k_resident<D, T, SPT, NT><<<1, NT, lds, h->stream>>>(make_kparams<T>(h->p, h->rho_eq), A);
}

// Up to kResSmall sites: four waves (one per SIMD) with up to four sites per
// thread; beyond, sixteen waves.
constexpr int kResSmall = 1024;

template <int D, typename T>
void launch_resident_t(flb_lattice* h, const ResArgs& A, size_t lds) {
  if (h->n <= 256) launch_resident_spt<D, T, 1, 256>(h, A, lds);
  else if (h->n <= 512) launch_resident_spt<D, T, 2, 256>(h, A, lds);
  else if (h->n <= kResSmall) launch_resident_spt<D, T, 4, 256>(h, A, lds);
  else if (h->n <= 2 * kResThreads) launch_resident_spt<D, T, 2, kResThreads>(h, A, lds);
  else launch_resident_spt<D, T, 4, kResThreads>(h, A, lds);
}

void launch_resident(flb_lattice* h, int c, size_t lds, int corr_lds) {
  char* w = h->work;
  ResArgs A{};
  A.gin = lat_buffer(h, h->cur);
  A.gout = lat_buffer(h, (h->cur + c) & 1);
  A.form_in = state_form(h);
  A.form_out = !h->aa ? kFormPull : (((h->cur + c) & 1) ? kFormAAS : kFormAAC);
  A.nx = (int32_t)h->p.n[0];
  A.ny = (int32_t)h->p.n[1];
  A.nz = (int32_t)h->p.n[2];
  A.nsteps = c;
  A.step0 = h->step;
  A.mom_every = h->mom_every;
  A.momacc = (double*)(w + h->wl.momacc);
  A.sk_every = h->sample_every;
  A.nax = h->nax[1];
  A.ngen = h->ngen[1];
  A.kinfo = (const int64_t*)(w + h->wl.kinfo[1]);
  A.slot_ax = (const int32_t*)(w + h->wl.slot_ax[1]);
  A.kv = (const int64_t*)(w + h->wl.kv[1]);
  A.slot_gen = (const int32_t*)(w + h->wl.slot_gen[1]);
  A.skacc = (double*)(w + h->wl.skacc);
  A.sk_fft = 0;
  A.sk_dft = 0;
  if (h->sample_every > 0) {  // axes with entries, power-of-two extent that fits the FFT scratch
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < h->nk[1]; ++j) {
        int nnz = 0, ax = -1;
        for (int a = 0; a < 3; ++a) {
          const int64_t La = h->p.n[a];
          if ((((int64_t)h->klist[1][3 * j + a] % La) + La) % La != 0) {
            ++nnz;
            ax = a;
          }
        }
        const int64_t L = nnz == 1 ? h->p.n[ax] : 0;
        const bool fft = nnz == 1 && L >= 2 && (L & (L - 1)) == 0 && 2 * L <= kResScratch;
        if (pass == 0 && fft) A.sk_fft |= 1 << ax;
        if (pass == 1 && nnz > 0 && !(nnz == 1 && (A.sk_fft & (1 << ax)))) A.sk_dft = 1;
      }
  }
  A.corr_lds = corr_lds;
  A.corr_every = h->corr_mem ? h->corr_every : 0;
  if (h->corr_mem) {
    char* m = h->corr_mem;
    A.cnk = h->corr_nk;
    A.nlag = h->corr_nlag;
    A.corr_s0 = h->corr_count;
    A.ckinfo = (const int32_t*)(m + h->corr_off[0]);
    A.amp = (double*)(m + h->corr_off[3]);
    A.sij = (double*)(m + h->corr_off[4]);
    A.ring = (double*)(m + h->corr_off[5]);
    A.ct = (double*)(m + h->corr_off[6]);
  }
  A.tw = (const double*)(w + h->wl.tw);
  if (h->s == 4) {
    if (h->d == 1) launch_resident_t<1, float>(h, A, lds);
    else if (h->d == 2) launch_resident_t<2, float>(h, A, lds);
    else launch_resident_t<3, float>(h, A, lds);
  } else {
    if (h->d == 1) launch_resident_t<1, double>(h, A, lds);
    else if (h->d == 2) launch_resident_t<2, double>(h, A, lds);
    else launch_resident_t<3, double>(h, A, lds);
  }
  h->mom_count += multiples_in(h->step, c, h->mom_every);
  h->sk_count += multiples_in(h->step, c, h->sample_every);
  h->corr_count += multiples_in(h->step, c, A.corr_every);
  h->cur = (h->cur + c) & 1;
  h->step += c;
}

// two D2Q5 steps in one pass (steps t and t + 1): g holds the state at t,
// out receives the state at t + 2
template <typename T>
void launch_step2_t(flb_lattice* h, const T* g, T* out, uint32_t step) {
  const KParams<T> P = make_kparams<T>(h->p, h->rho_eq);
  const int ty = h->p.tile_rows ? h->p.tile_rows : 8;
  const int tiles_x = (int)((h->p.n[0] + 255) / 256);
  const bool nt = h->p.nt_store != 0;
  // local Gaussian noise (the default) takes the instances with the noise plan fixed at compile time
  const bool lg = h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
#define FLB_TWO(TYV)                                                                                    \
  {                                                                                                     \
    const unsigned nb = (unsigned)(tiles_x * ((h->p.n[1] + TYV - 1) / TYV));                             \
    if (lg && nt) k_step2_d2<T, TYV, true, false, kPlanLocalGauss><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x); \
    else if (lg) k_step2_d2<T, TYV, false, false, kPlanLocalGauss><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x); \
    else if (nt) k_step2_d2<T, TYV, true><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x);          \
    else k_step2_d2<T, TYV, false><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x);                 \
  }
  switch (ty) {
    case 1: case 2: FLB_TWO(2) break;
    case 4: FLB_TWO(4) break;
    case 16: FLB_TWO(16) break;
    default: FLB_TWO(8) break;
  }
#undef FLB_TWO
}

// the same pass writing the density partials of the state at t (tiles of
// kSampleRows rows, as the sampled one-step kernel)
template <typename T>
void launch_step2_sampled_t(flb_lattice* h, const T* g, T* out, uint32_t step) {
  const KParams<T> P = make_kparams<T>(h->p, h->rho_eq);
  const int tiles_x = (int)((h->p.n[0] + 255) / 256);
  const unsigned nb = (unsigned)(tiles_x * ((h->p.n[1] + kSampleRows - 1) / kSampleRows));
  double* rp = (double*)(h->work + h->wl.rowpart);
  double* cp = (double*)(h->work + h->wl.colbig);
  const bool lg = h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
  if (lg && h->p.nt_store)
    k_step2_d2<T, kSampleRows, true, true, kPlanLocalGauss><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x, rp, cp);
  else if (lg)
    k_step2_d2<T, kSampleRows, false, true, kPlanLocalGauss><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x, rp, cp);
  else if (h->p.nt_store)
    k_step2_d2<T, kSampleRows, true, true><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x, rp, cp);
  else
    k_step2_d2<T, kSampleRows, false, true><<<nb, 256, 0, h->stream>>>(g, out, P, step, tiles_x, rp, cp);
}

void launch_step2(flb_lattice* h, const void* g, void* out, uint32_t step) {
  if (h->s == 4) launch_step2_t<float>(h, (const float*)g, (float*)out, step);
  else launch_step2_t<double>(h, (const double*)g, (double*)out, step);
}

void launch_step2_sampled(flb_lattice* h, const void* g, void* out, uint32_t step) {
  if (h->s == 4) launch_step2_sampled_t<float>(h, (const float*)g, (float*)out, step);
  else launch_step2_sampled_t<double>(h, (const double*)g, (double*)out, step);
}

// a statistic is sampled on the state before step t
bool sample_due(const flb_lattice* h, int64_t t) {
  return (h->mom_every > 0 && t % h->mom_every == 0) ||
         (h->corr_mem && h->corr_every > 0 && t % h->corr_every == 0) ||
         (h->sample_every > 0 && t % h->sample_every == 0);
}

// Bytes of partial sums the density profile along `axis` needs.
size_t profile_part_bytes(const flb_lattice* h, int axis) {
  const int64_t nx = h->p.n[0], nrows = h->p.n[1] * h->p.n[2];
  return axis == 0 ? sizeof(double) * 2 * (size_t)std::min<int64_t>(kColChunks, nrows) * (size_t)nx
                   : sizeof(double) * 2 * (size_t)nrows;
}

// density profile along `axis` into out (sums of rho) and out2 (sums of rho^2)
template <int D, typename T>
void launch_profile_t(flb_lattice* h, int axis, double* part, double* out, double* out2) {
  const T* g = (const T*)lat_buffer(h, h->cur);
  const int64_t nx = h->p.n[0], ny = h->p.n[1], nz = h->p.n[2], nrows = ny * nz;
  if (axis == 0) {
    const int64_t nchunk = std::min<int64_t>(kColChunks, nrows), rpc = (nrows + nchunk - 1) / nchunk;
    k_prof_cols<D, T><<<dim3((unsigned)((nx + 255) / 256), (unsigned)nchunk), 256, 0, h->stream>>>(g, nx, ny, nz, rpc,
                                                                                                    part, state_form(h));
    k_prof_cols_final<<<(unsigned)((nx + 255) / 256), 256, 0, h->stream>>>(part, nchunk, nx, out, out2);
  } else {
    k_prof_rows<D, T><<<(unsigned)nrows, 256, 0, h->stream>>>(g, nx, ny, nz, part, state_form(h));
    const int64_t L = h->p.n[axis];
    k_prof_yz<<<(unsigned)((L + 255) / 256), 256, 0, h->stream>>>(part, ny, nz, axis, out, out2);
  }
}

// population correlators: Fourier sums of the current state, then one
// accumulation step (S_ij, time correlator, ring of rho(k))
template <int D, typename T>
void launch_amp_t(flb_lattice* h, const T* g) {
  const int Q = h->Q;
  char* m = h->corr_mem;
  const dim3 grid((unsigned)h->corr_nsb, (unsigned)((h->corr_nk + kCorrKC - 1) / kCorrKC));
  k_amp_partial<D, T><<<grid, 256, 0, h->stream>>>(g, h->p.n[0], h->p.n[1], h->p.n[2],
                                                    (const double*)(m + h->corr_off[1]),
                                                    (const int32_t*)(m + h->corr_off[0]), h->corr_nk,
                                                    h->corr_nsb, (double*)(m + h->corr_off[2]), state_form(h));
  const int64_t nv = (int64_t)h->corr_nk * 2 * Q;
  k_amp_final<<<(unsigned)((nv + 255) / 256), 256, 0, h->stream>>>((const double*)(m + h->corr_off[2]),
                                                                   h->corr_nsb, h->corr_nk, 2 * Q,
                                                                   (double*)(m + h->corr_off[3]));
}

void launch_amp(flb_lattice* h) {
  const void* g = lat_buffer(h, h->cur);
  if (h->s == 4) {
    if (h->d == 1) launch_amp_t<1, float>(h, (const float*)g);
    else if (h->d == 2) launch_amp_t<2, float>(h, (const float*)g);
    else launch_amp_t<3, float>(h, (const float*)g);
  } else {
    if (h->d == 1) launch_amp_t<1, double>(h, (const double*)g);
    else if (h->d == 2) launch_amp_t<2, double>(h, (const double*)g);
    else launch_amp_t<3, double>(h, (const double*)g);
  }
}

void launch_profile(flb_lattice* h, int axis, double* part, double* out, double* out2) {
  if (h->s == 4) {
    if (h->d == 1) launch_profile_t<1, float>(h, axis, part, out, out2);
    else if (h->d == 2) launch_profile_t<2, float>(h, axis, part, out, out2);
    else launch_profile_t<3, float>(h, axis, part, out, out2);
  } else {
    if (h->d == 1) launch_profile_t<1, double>(h, axis, part, out, out2);
    else if (h->d == 2) launch_profile_t<2, double>(h, axis, part, out, out2);
    else launch_profile_t<3, double>(h, axis, part, out, out2);
  }
}

void corr_sample(flb_lattice* h) {
  launch_amp(h);
  char* m = h->corr_mem;
  const int Q = h->Q;
  const int64_t nt = (int64_t)h->corr_nk * Q * Q + (int64_t)h->corr_nk * h->corr_nlag;
  k_corr_accumulate<<<(unsigned)((nt + 255) / 256), 256, 0, h->stream>>>(
      (const double*)(m + h->corr_off[3]), h->corr_nk, Q, h->corr_nlag, h->corr_count,
      (double*)(m + h->corr_off[4]), (double*)(m + h->corr_off[5]), (double*)(m + h->corr_off[6]));
  h->corr_count += 1;
}

}  // namespace flb

// ---------------------------------------------------------------------------
// structure factor
namespace {

// Split a k-list into axis entries (one nonzero component, or zero, for
// D >= 2) and general entries, reduced modulo the box.
void classify_k(const flb_lattice* h, const int32_t* kvec, int nk, KStage* st, int* nax, int* ngen) {
  int na = 0, ng = 0;
  for (int j = 0; j < nk; ++j) {
    int64_t k[3];
    int nnz = 0, ax = -1;
    for (int a = 0; a < 3; ++a) {
      const int64_t L = h->p.n[a];
      k[a] = ((int64_t)kvec[3 * j + a] % L + L) % L;
      if (k[a] != 0) {
        ++nnz;
        ax = a;
      }
    }
    if (h->d >= 2 && nnz <= 1) {
      st->kinfo[2 * na] = nnz == 0 ? -1 : ax;
      st->kinfo[2 * na + 1] = nnz == 0 ? 0 : k[ax];
      st->slot_ax[na++] = j;
    } else {
      st->kv[3 * ng] = k[0];
      st->kv[3 * ng + 1] = k[1];
      st->kv[3 * ng + 2] = k[2];
      st->slot_gen[ng++] = j;
    }
  }
  *nax = na;
  *ngen = ng;
}

// Axis marginals from rowsum / colpart (nchunk chunks), then the axis DFTs.
// mx_ready: the x marginal is already in place (k_axis_reduce).
void axis_sk(flb_lattice* h, int set, int64_t nchunk, bool mx_ready) {
  const int64_t nx = h->p.n[0], ny = h->p.n[1], nz = h->p.n[2];
  hipStream_t st = h->stream;
  char* w = h->work;
  double* rowsum = (double*)(w + h->wl.rowsum);
  double* colpart = (double*)(w + h->wl.colpart);
  double* mx = (double*)(w + h->wl.marg);
  double* my = mx + nx;
  double* mz = my + ny;
  const double* tw = (const double*)(w + h->wl.tw);
  if (!mx_ready) k_marginal_x<<<(unsigned)((nx + 63) / 64), 256, 0, st>>>(colpart, nchunk, nx, mx);
  // with one plane the row sums are the y marginal
  if (nz > 1) k_marginal_y<<<(unsigned)ny, 256, 0, st>>>(rowsum, ny, nz, my);
  if (h->d == 3) k_marginal_z<<<(unsigned)nz, 256, 0, st>>>(rowsum, ny, mz);
  // an axis-only accumulator list is accumulated here (sk_accumulate skips it)
  double* acc = set == 1 && h->ngen[1] == 0 ? (double*)(w + h->wl.skacc) : nullptr;
  k_sk_axis<<<(unsigned)((h->nax[set] + kSkAxisK - 1) / kSkAxisK), kSkAxisThreads, 0, st>>>(
      mx, nz > 1 ? my : rowsum, mz, nx, ny, nz, (const int64_t*)(w + h->wl.kinfo[set]),
      (const int32_t*)(w + h->wl.slot_ax[set]), h->nax[set], tw, tw + 2 * nx, tw + 2 * (nx + ny),
      (double*)(w + h->wl.sval[set]), acc);
}

// S(k) of the current state for k-list `set`.  from_step: the axis
// partials were written by the sampled step (colbig / rowpart) and only need
// to be reduced.
template <int D, typename T>
void launch_sk_t(flb_lattice* h, int set, bool from_step) {
  const T* g = (const T*)flb::lat_buffer(h, h->cur);
  const int64_t nx = h->p.n[0], ny = h->p.n[1], nz = h->p.n[2];
  hipStream_t st = h->stream;
  char* w = h->work;
  double* sval = (double*)(w + h->wl.sval[set]);
  if (h->nax[set] > 0) {
    const int64_t nrows = ny * nz;
    const int64_t nchunk = std::min<int64_t>(kColChunks, nrows);
    const int64_t rpc = (nrows + nchunk - 1) / nchunk;
    double* rowsum = (double*)(w + h->wl.rowsum);
    double* colpart = (double*)(w + h->wl.colpart);
    static_assert(kColChunks <= 64, "k_axis_reduce holds at most 64 group sums per column");
    if (from_step) {  // row sums and the x marginal from the pass's partials, one launch
      const int64_t ntx = (nx + 255) / 256, ntr = (nrows + kSampleRows - 1) / kSampleRows;
      const int64_t nblk = (nx + 15) / 16 + (nrows + 1023) / 1024;
      k_axis_reduce<<<(unsigned)nblk, 1024, 0, st>>>((const double*)(w + h->wl.rowpart), ntx, nrows, rowsum,
                                                    (const double*)(w + h->wl.colbig), ntr, nx, nchunk,
                                                    (double*)(w + h->wl.marg));
    } else {
      k_row_sums<D, T><<<(unsigned)nrows, 256, 0, st>>>(g, nx, ny, nz, rowsum, state_form(h));
      k_col_partial<D, T><<<dim3((unsigned)((nx + 255) / 256), (unsigned)nchunk), 256, 0, st>>>(g, nx, ny, nz, rpc, colpart,
                                                                                               state_form(h));
    }
    axis_sk(h, set, nchunk, from_step);
  }
  if (h->ngen[set] > 0 && !from_step) {
    const int64_t nchunk = std::min<int64_t>(kSkChunks, (h->n + 255) / 256);
    const int64_t chunk = (h->n + nchunk - 1) / nchunk;
    double* part = (double*)(w + h->wl.skpart);
    k_sk_direct_partial<D, T><<<dim3((unsigned)nchunk, (unsigned)h->ngen[set]), 256, 0, st>>>(
        g, nx, ny, nz, (const int64_t*)(w + h->wl.kv[set]), h->rho_eq, chunk, part, state_form(h));
    k_sk_direct_final<<<(unsigned)((h->ngen[set] + 63) / 64), 64, 0, st>>>(
        part, nchunk, h->ngen[set], (const int32_t*)(w + h->wl.slot_gen[set]),
        (const int64_t*)(w + h->wl.kv[set]), h->rho_eq, (double)h->n, sval);
  }
}

void launch_sk(flb_lattice* h, int set, bool from_step = false) {
  if (h->s == 4) {
    if (h->d == 1) launch_sk_t<1, float>(h, set, from_step);
    else if (h->d == 2) launch_sk_t<2, float>(h, set, from_step);
    else launch_sk_t<3, float>(h, set, from_step);
  } else {
    if (h->d == 1) launch_sk_t<1, double>(h, set, from_step);
    else if (h->d == 2) launch_sk_t<2, double>(h, set, from_step);
    else launch_sk_t<3, double>(h, set, from_step);
  }
}

// The sampled step (D >= 2): step + axis partials of the pre-collision state.
template <int D, typename T>
void launch_step_sampled_t(flb_lattice* h, const T* g, T* out, uint32_t step) {
  const KParams<T> P = make_kparams<T>(h->p, h->rho_eq);
  const int64_t nrows = P.ny * P.nz;
  const int64_t tiles_x = (P.nx + 255) / 256;
  const int64_t G = tiles_x * ((nrows + kSampleRows - 1) / kSampleRows);
  k_step_rows_sk<D, T, kSampleRows><<<(unsigned)G, 256, 0, h->stream>>>(
      g, out, P, step, tiles_x, nrows, (double*)(h->work + h->wl.rowpart), (double*)(h->work + h->wl.colbig));
}

void launch_step_sampled(flb_lattice* h, const void* g, void* out, uint32_t step) {
  if (h->s == 4) {
    if (h->d == 2) launch_step_sampled_t<2, float>(h, (const float*)g, (float*)out, step);
    else launch_step_sampled_t<3, float>(h, (const float*)g, (float*)out, step);
  } else {
    if (h->d == 2) launch_step_sampled_t<2, double>(h, (const double*)g, (double*)out, step);
    else launch_step_sampled_t<3, double>(h, (const double*)g, (double*)out, step);
  }
}

// Adds the last sample of k-list 1 to the accumulator (an axis-only list
// was added by k_sk_axis already).
void sk_accumulate(flb_lattice* h) {
  char* w = h->work;
  if (h->ngen[1] > 0)
    k_sk_accumulate<<<(h->nk[1] + 255) / 256, 256, 0, h->stream>>>((const double*)(w + h->wl.sval[1]),
                                                                   (double*)(w + h->wl.skacc), h->nk[1]);
  h->sk_count += 1;
}

// Upload a k-list into set `set` of the workspace; synchronises.
int upload_k(flb_lattice* h, const int32_t* kvec, int nk, int set) {
  KStage* st = h->stage;
  int na = 0, ng = 0;
  classify_k(h, kvec, nk, st, &na, &ng);
  char* w = h->work;
  HIP_TRY(hipMemcpyAsync(w + h->wl.kinfo[set], st->kinfo, sizeof(int64_t) * 2 * std::max(na, 1), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(w + h->wl.slot_ax[set], st->slot_ax, sizeof(int32_t) * std::max(na, 1), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(w + h->wl.kv[set], st->kv, sizeof(int64_t) * 3 * std::max(ng, 1), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(w + h->wl.slot_gen[set], st->slot_gen, sizeof(int32_t) * std::max(ng, 1), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->nk[set] = nk;
  h->nax[set] = na;
  h->ngen[set] = ng;
  h->klist[set].assign(kvec, kvec + 3 * nk);
  return FLB_OK;
}

// Check mode: the non-finite count of the lattice sums of the current
// state (synchronises); FLB_ENONFINITE when there are any.
int check_finite(flb_lattice* h) {
  launch_moments(h);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->stage->red, h->work + h->wl.red_out, sizeof(double) * kNV, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int64_t bad = (int64_t)h->stage->red[kNV - 1];
  if (bad > 0)
    return fail(FLB_ENONFINITE, "%lld non-finite populations after step %lld", (long long)bad, (long long)h->step);
  return FLB_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of flb_profile_noalloc: one array per GPU (the module's
// device global), whose device address is looked up once per device and kept.
// In host code the array's name is not a device address: only the looked-up
// pointer is ever passed to kernels.
namespace {

constexpr size_t kScratchBytes = (size_t)FLB_PROFILE_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on device `dev` (current), looked up on the
// first call on that device.
int scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FLB_EDEVICE, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FLB_OK;
}

}  // namespace

// the step loop of flb_step (defined with the exported functions)
static int step_unchecked(flb_lattice* h, int64_t nsteps);

// ---------------------------------------------------------------------------
// exported functions
extern "C" {

int flb_version(void) { return FLB_ABI_VERSION; }

const char* flb_last_error(void) { return flb::g_err.c_str(); }

int flb_lattice_constants(int32_t model, double theta, double* w, double* m) {
  if (model < 1 || model > 3) return fail(FLB_EINVAL, "model must be 1, 2 or 3");
  const int d = model, Q = 2 * d + 1;
  const double th = theta == 0.0 ? default_theta(d) : theta;
  if (!(th > 0.0 && th < 1.0 / d)) return fail(FLB_EINVAL, "theta outside (0, 1/d)");
  if (w) {
    w[0] = 1.0 - d * th;
    for (int i = 1; i < Q; ++i) w[i] = th / 2.0;
  }
  if (m) {
    const double a = 1.0 / std::sqrt(th), b = 1.0 / std::sqrt(2.0 * th), e = 1.0 / std::sqrt(6.0 * th);
    const double c0 = std::sqrt(d * th / (1.0 - d * th)), c1 = std::sqrt((1.0 - d * th) / (d * th));
    std::vector<double> M((size_t)Q * Q, 0.0);
    auto at = [&](int r, int i) -> double& { return M[(size_t)r * Q + i]; };
    for (int i = 0; i < Q; ++i) at(0, i) = 1.0;
    for (int ax = 0; ax < d; ++ax) {  // current moments
      at(1 + ax, 1 + 2 * ax) = a;
      at(1 + ax, 2 + 2 * ax) = -a;
    }
    int r = 1 + d;
    if (d >= 2) {  // v_x^2 - v_y^2
      for (int i = 1; i <= 2; ++i) at(r, i) = b;
      for (int i = 3; i <= 4; ++i) at(r, i) = -b;
      ++r;
    }
    if (d == 3) {  // v_x^2 + v_y^2 - 2 v_z^2
      for (int i = 1; i <= 4; ++i) at(r, i) = e;
      for (int i = 5; i <= 6; ++i) at(r, i) = -2.0 * e;
      ++r;
    }
    at(r, 0) = -c0;  // trace
    for (int i = 1; i < Q; ++i) at(r, i) = c1;
    std::memcpy(m, M.data(), sizeof(double) * Q * Q);
  }
  return Q;
}

int flb_required_bytes(const flb_params* p, size_t* pop_bytes, size_t* work_bytes) {
  int rc = check_params(p);
  if (rc) return rc;
  const size_t n = (size_t)(p->n[0] * p->n[1] * p->n[2]);
  const size_t Q = 2 * p->model + 1;
  if (pop_bytes) *pop_bytes = (p->layout == FLB_LAYOUT_AA ? 1 : 2) * Q * n * (size_t)p->precision;
  if (work_bytes) *work_bytes = work_layout(*p).total;
  return FLB_OK;
}

int flb_create(const flb_params* p, void* d_pop, size_t pop_bytes, void* d_work, size_t work_bytes,
               void* hip_stream, flb_lattice** out) {
  if (!out) return fail(FLB_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need_pop = 0, need_work = 0;
  int rc = flb_required_bytes(p, &need_pop, &need_work);
  if (rc) return rc;
  if (!d_pop) return fail(FLB_EINVAL, "d_pop is NULL");
  if (((uintptr_t)d_pop) % 256) return fail(FLB_EINVAL, "d_pop must be 256-byte aligned");
  if (pop_bytes < need_pop) return fail(FLB_ENOMEM, "pop_bytes %zu < required %zu", pop_bytes, need_pop);
  if (d_work && work_bytes < need_work) return fail(FLB_ENOMEM, "work_bytes %zu < required %zu", work_bytes, need_work);
  if (d_work && ((uintptr_t)d_work) % 256) return fail(FLB_EINVAL, "d_work must be 256-byte aligned");
  flb_lattice* h = new (std::nothrow) flb_lattice();
  if (!h) return fail(FLB_ENOMEM, "handle allocation failed");
  h->p = *p;
  h->d = p->model;
  h->Q = 2 * p->model + 1;
  h->n = p->n[0] * p->n[1] * p->n[2];
  h->s = (size_t)p->precision;
  h->plane = (size_t)h->Q * h->n * h->s;
  h->pop = (char*)d_pop;
  h->aa = p->layout == FLB_LAYOUT_AA;
  h->cur = 0;
  h->stream = (hipStream_t)hip_stream;
  h->step = 0;
  h->mass0 = 0;
  h->rho_eq = 0;
  h->sk_count = 0;
  h->batch_refs = 0;
  h->wl = work_layout(*p);
  h->nk[0] = h->nk[1] = 0;
  h->nax[0] = h->nax[1] = h->ngen[0] = h->ngen[1] = 0;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipGetDevice");
  }
  {  // one workgroup keeps the whole lattice in LDS when it fits
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess)
      lds_max = 0;
    (void)hipGetLastError();
    const size_t need = res_lds_bytes(h->n, h->Q, (int)h->s, p->n[0] + p->n[1] + p->n[2]);
    const bool fits = h->n <= kResMaxSites && need <= (size_t)lds_max;
    if (p->kernel == FLB_KERNEL_RESIDENT && !fits) {
      delete h;
      return fail(FLB_EINVAL, "resident kernel: the lattice needs %zu bytes of LDS (limit %d) or has more than %d sites",
                  need, lds_max, kResMaxSites);
    }
    h->resident = fits && (p->kernel == FLB_KERNEL_AUTO || p->kernel == FLB_KERNEL_RESIDENT);
    h->res_lds = need;
    h->res_lds_max = lds_max;
  }
  if (d_work) {
    h->work = (char*)d_work;
    h->own_work = false;
  } else {
    e = hipMalloc((void**)&h->work, h->wl.total);
    if (e != hipSuccess) {
      delete h;
      return fail(FLB_ENOMEM, "workspace allocation of %zu bytes failed: %s", h->wl.total, hipGetErrorString(e));
    }
    h->own_work = true;
  }
  h->sample_every = 0;
  h->sample_fused = false;
  h->mom_every = 0;
  h->mom_count = 0;
  h->corr_every = 0;
  h->corr_nk = h->corr_nlag = h->corr_nsb = 0;
  h->corr_count = 0;
  h->check_every = 0;
  h->corr_mem = nullptr;
  h->prof_mem = nullptr;
  h->reg_n = 0;
  h->reg_map = nullptr;
  h->reg_tab = nullptr;
  {  // twiddle tables of the structure factor and of the resident kernel
    double* tw = (double*)(h->work + h->wl.tw);
    const int64_t L3[3] = {p->n[0], p->n[1], p->n[2]};
    int64_t off = 0;
    for (int a = 0; a < 3; ++a) {
      k_twiddle<<<(unsigned)((L3[a] + 255) / 256), 256, 0, h->stream>>>(tw + 2 * off, L3[a]);
      off += L3[a];
    }
  }
  e = hipHostMalloc((void**)&h->stage, sizeof(KStage), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (h->own_work) (void)hipFree(h->work);
    delete h;
    return hip_fail(e, "hipHostMalloc");
  }
  *out = h;
  return FLB_OK;
}

int flb_destroy(flb_lattice* h) {
  if (!h) return FLB_OK;
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->own_work) (void)hipFree(h->work);
  if (h->corr_mem) (void)hipFree(h->corr_mem);
  if (h->prof_mem) (void)hipFree(h->prof_mem);
  if (h->reg_map) (void)hipFree(h->reg_map);
  if (h->reg_tab) (void)hipFree(h->reg_tab);
  (void)hipHostFree(h->stage);
  delete h;
  return FLB_OK;
}

int flb_set_populations(flb_lattice* h, const void* src, int src_on_device, int64_t step) {
  flb::TraceRange trace_("flb_set_populations");
  if (!h || !src) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (step < 0) return fail(FLB_EINVAL, "step must be >= 0");
  DeviceGuard g(h->device);
  if (h->aa) {  // the canonical state is the AA layout's even-parity form
    h->cur = 0;
    HIP_TRY(hipMemcpyAsync(h->pop, src, h->plane, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           h->stream));
  } else {
    // stage the canonical state in the spare buffer, then pull it back into
    // storage form in the current buffer
    const int spare = 1 - h->cur;
    HIP_TRY(hipMemcpyAsync(lat_buffer(h, spare), src, h->plane,
                           src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    launch_convert(h, false, lat_buffer(h, spare), lat_buffer(h, h->cur));
    HIP_TRY(hipGetLastError());
  }
  launch_moments(h);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->stage->red, h->work + h->wl.red_out, sizeof(double) * kNV, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->mass0 = h->stage->red[0];
  h->rho_eq = h->mass0 / (double)h->n;
  if (h->reg_n > 0) {
    const int rc = rebuild_regions(h);
    if (rc) return rc;
  }
  h->step = step;
  return FLB_OK;
}

int flb_get_populations(flb_lattice* h, void* dst, int dst_on_device) {
  flb::TraceRange trace_("flb_get_populations");
  if (!h || !dst) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  if (h->aa) {
    if (state_form(h) == kFormAAC) {  // already canonical
      HIP_TRY(hipMemcpyAsync(dst, h->pop, h->plane, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             h->stream));
    } else if (dst_on_device) {  // gather straight into the caller's buffer
      launch_convert(h, true, h->pop, dst, kFormAAS);
      HIP_TRY(hipGetLastError());
    } else {  // no spare buffer in this layout: a temporary one
      void* tmp = nullptr;
      HIP_TRY(hipMalloc(&tmp, h->plane));
      launch_convert(h, true, h->pop, tmp, kFormAAS);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, h->plane, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) return hip_fail(e, "AA-layout readback");
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return FLB_OK;
  }
  const int spare = 1 - h->cur;
  launch_convert(h, true, lat_buffer(h, h->cur), lat_buffer(h, spare));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(dst, lat_buffer(h, spare), h->plane,
                         dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FLB_OK;
}

int flb_step(flb_lattice* h, int64_t nsteps) {
  flb::TraceRange trace_("flb_step");
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  if (h->check_every <= 0 || nsteps == 0) return step_unchecked(h, nsteps);
  // check mode: run up to each multiple of check_every, check, go on
  const int64_t end = h->step + nsteps;
  while (h->step < end) {
    const int64_t next = std::min(end, (h->step / h->check_every + 1) * h->check_every);
    int rc = step_unchecked(h, next - h->step);
    if (rc) return rc;
    rc = check_finite(h);
    if (rc) return rc;
  }
  return FLB_OK;
}

int flb_set_check(flb_lattice* h, int64_t every) {
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (every < 0) return fail(FLB_EINVAL, "every must be >= 0");
  h->check_every = every;
  return FLB_OK;
}

}  // extern "C"

static int step_unchecked(flb_lattice* h, int64_t nsteps) {
  size_t lds = 0;
  int corr_lds = 0;
  if (h->resident && h->reg_n == 0 && resident_lds(h, &lds, &corr_lds)) {
    for (int64_t k = 0; k < nsteps;) {
      const int c = (int)std::min<int64_t>(nsteps - k, kResMaxChunk);
      launch_resident(h, c, lds, corr_lds);
      k += c;
    }
    HIP_TRY(hipGetLastError());
    return FLB_OK;
  }
  const bool two = h->p.kernel == FLB_KERNEL_TWO_STEP && h->reg_n == 0;
  const bool two_sk = two && (h->p.tile_rows ? h->p.tile_rows : 8) == kSampleRows;
  for (int64_t k = 0; k < nsteps; ++k) {
    const int nxt = 1 - h->cur;
    const uint32_t t32 = (uint32_t)(h->step & 0xFFFFFFFF);
    if (h->mom_every > 0 && h->step % h->mom_every == 0) {  // lattice sums of the state before this step
      launch_moments(h);
      k_add<<<1, 64, 0, h->stream>>>((const double*)(h->work + h->wl.red_out), (double*)(h->work + h->wl.momacc), kNV);
      h->mom_count += 1;
    }
    if (h->corr_every > 0 && h->step % h->corr_every == 0) corr_sample(h);  // state before this step
    const bool sample = h->sample_every > 0 && h->step % h->sample_every == 0;
    if (two_sk && sample && h->sample_fused && k + 1 < nsteps && !sample_due(h, h->step + 1)) {
      // a sampled pair: the pass also writes the density partials of the state at t
      launch_step2_sampled(h, lat_buffer(h, h->cur), lat_buffer(h, nxt), t32);
      launch_sk(h, 1, true);
      sk_accumulate(h);
      h->cur = nxt;
      h->step += 2;
      ++k;
      continue;
    }
    if (two && !sample && k + 1 < nsteps && !sample_due(h, h->step + 1)) {
      // steps t and t + 1 in one pass; nothing is sampled on the state between
      launch_step2(h, lat_buffer(h, h->cur), lat_buffer(h, nxt), t32);
      h->cur = nxt;
      h->step += 2;
      ++k;
      continue;
    }
    if (sample && h->sample_fused && h->reg_n == 0) {
      launch_step_sampled(h, lat_buffer(h, h->cur), lat_buffer(h, nxt), t32);
      launch_sk(h, 1, true);
      sk_accumulate(h);
    } else {
      if (sample) {  // S(k) of the state before this step, then the step
        launch_sk(h, 1);
        sk_accumulate(h);
      }
      launch_step(h, lat_buffer(h, h->cur), lat_buffer(h, nxt), t32, h->stream);
    }
    h->cur = nxt;
    h->step += 1;
  }
  HIP_TRY(hipGetLastError());
  return FLB_OK;
}

extern "C" {

int flb_get_step(flb_lattice* h, int64_t* step) {
  if (!h || !step) return fail(FLB_EINVAL, "NULL argument");
  *step = h->step;
  return FLB_OK;
}

int flb_moments(flb_lattice* h, flb_moments_t* out) {
  flb::TraceRange trace_("flb_moments");
  if (!h || !out) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  launch_moments(h);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->stage->red, h->work + h->wl.red_out, sizeof(double) * kNV, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const double* r = h->stage->red;
  std::memset(out, 0, sizeof *out);
  out->step = h->step;
  out->nsite = h->n;
  out->mass = r[0];
  out->mass0 = h->mass0;
  out->rho_eq = h->rho_eq;
  for (int i = 0; i < 7; ++i) out->sum_f[i] = r[1 + i];
  for (int i = 0; i < 28; ++i) out->sum_ff[i] = r[8 + i];
  out->sum_rho2 = r[36];
  out->sum_rho_pos = r[37];
  out->n_negative = (int64_t)r[38];
  out->nonfinite = (int64_t)r[39];
  return FLB_OK;
}

int flb_structure_factor(flb_lattice* h, const int32_t* kvec, int32_t nk, int32_t mode, double* S_out) {
  flb::TraceRange trace_("flb_structure_factor");
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (mode < 0 || mode > 3) return fail(FLB_EINVAL, "unknown mode %d", mode);
  DeviceGuard g(h->device);
  char* w = h->work;
  if (mode == FLB_SK_SNAPSHOT || mode == FLB_SK_RESET) {
    if (!kvec || nk < 1 || nk > kMaxK) return fail(FLB_EINVAL, "need 1 <= nk <= %d wave vectors", kMaxK);
    if (mode == FLB_SK_SNAPSHOT && !S_out) return fail(FLB_EINVAL, "S_out is NULL");
  }
  if (mode == FLB_SK_SNAPSHOT) {
    int rc = upload_k(h, kvec, nk, 0);
    if (rc) return rc;
    launch_sk(h, 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h->stage->out, w + h->wl.sval[0], sizeof(double) * nk, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::memcpy(S_out, h->stage->out, sizeof(double) * nk);
    return FLB_OK;
  }
  if (mode == FLB_SK_RESET) {
    int rc = upload_k(h, kvec, nk, 1);
    if (rc) return rc;
    k_fill_zero<<<(kMaxK + 255) / 256, 256, 0, h->stream>>>((double*)(w + h->wl.skacc), kMaxK);
    HIP_TRY(hipGetLastError());
    h->sk_count = 0;
    return FLB_OK;
  }
  if (h->nk[1] == 0) return fail(FLB_ESTATE, "structure factor accumulator has no k-list (call RESET)");
  if (mode == FLB_SK_SAMPLE) {
    if (kvec && (nk != h->nk[1] || std::memcmp(kvec, h->klist[1].data(), sizeof(int32_t) * 3 * nk) != 0))
      return fail(FLB_EINVAL, "SAMPLE k-list differs from the one given at RESET");
    launch_sk(h, 1);
    sk_accumulate(h);
    HIP_TRY(hipGetLastError());
    return FLB_OK;
  }
  // READ
  if (!S_out) return fail(FLB_EINVAL, "S_out is NULL");
  if (h->sk_count == 0) return fail(FLB_ESTATE, "no samples accumulated");
  HIP_TRY(hipMemcpyAsync(h->stage->out, w + h->wl.skacc, sizeof(double) * h->nk[1], hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int j = 0; j < h->nk[1]; ++j) S_out[j] = h->stage->out[j] / (double)h->sk_count;
  return FLB_OK;
}

int flb_set_sampling(flb_lattice* h, int64_t every, const int32_t* kvec, int32_t nk) {
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (every < 0) return fail(FLB_EINVAL, "every must be >= 0");
  if (every == 0) {
    h->sample_every = 0;
    return FLB_OK;
  }
  DeviceGuard g(h->device);
  const int rc = flb_structure_factor(h, kvec, nk, FLB_SK_RESET, nullptr);
  if (rc) return rc;
  h->sample_every = every;
  // the sampled step kernels write the pull storage form: two buffers only
  h->sample_fused = h->d >= 2 && h->ngen[1] == 0 && !h->aa;
  return FLB_OK;
}

int flb_set_moment_sampling(flb_lattice* h, int64_t every) {
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (every < 0) return fail(FLB_EINVAL, "every must be >= 0");
  DeviceGuard g(h->device);
  if (every > 0) {
    k_fill_zero<<<1, 64, 0, h->stream>>>((double*)(h->work + h->wl.momacc), kNV);
    HIP_TRY(hipGetLastError());
    h->mom_count = 0;
  }
  h->mom_every = every;
  return FLB_OK;
}

int flb_sampled_moments(flb_lattice* h, flb_moments_t* sum, int64_t* nsamples) {
  flb::TraceRange trace_("flb_sampled_moments");
  if (!h || !sum || !nsamples) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  HIP_TRY(hipMemcpyAsync(h->stage->red, h->work + h->wl.momacc, sizeof(double) * kNV, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const double* r = h->stage->red;
  std::memset(sum, 0, sizeof *sum);
  sum->step = h->step;
  sum->nsite = h->n;
  sum->mass = r[0];
  sum->mass0 = h->mass0;
  sum->rho_eq = h->rho_eq;
  for (int i = 0; i < 7; ++i) sum->sum_f[i] = r[1 + i];
  for (int i = 0; i < 28; ++i) sum->sum_ff[i] = r[8 + i];
  sum->sum_rho2 = r[36];
  sum->sum_rho_pos = r[37];
  sum->n_negative = (int64_t)r[38];
  sum->nonfinite = (int64_t)r[39];
  *nsamples = h->mom_count;
  return FLB_OK;
}

int flb_set_correlation(flb_lattice* h, int64_t every, const int32_t* kvec, int32_t nk, int32_t nlag) {
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (every < 0) return fail(FLB_EINVAL, "every must be >= 0");
  DeviceGuard g(h->device);
  if (every == 0) {
    h->corr_every = 0;
    return FLB_OK;
  }
  if (!kvec || nk < 1 || nk > kMaxK) return fail(FLB_EINVAL, "need 1 <= nk <= %d wave vectors", kMaxK);
  if (nlag < 1 || nlag > kMaxLag) return fail(FLB_EINVAL, "need 1 <= nlag <= %d", kMaxLag);
  if ((int64_t)nk * nlag > kMaxKLag) return fail(FLB_EINVAL, "nk * nlag must be <= %d", kMaxKLag);
  const int Q = h->Q;
  const int64_t nsb = std::min<int64_t>((h->n + 255) / 256, kCorrBlocks);
  const int64_t L = h->p.n[0] + h->p.n[1] + h->p.n[2];
  size_t sz[7] = {sizeof(int32_t) * 3 * (size_t)nk,
                  sizeof(double) * 2 * (size_t)L,
                  sizeof(double) * 2 * (size_t)Q * (size_t)nk * (size_t)nsb,
                  sizeof(double) * 2 * (size_t)Q * (size_t)nk,
                  sizeof(double) * 2 * (size_t)Q * Q * (size_t)nk,
                  sizeof(double) * 2 * (size_t)nk * (size_t)nlag,
                  sizeof(double) * 2 * (size_t)nk * (size_t)nlag};
  size_t off[7], total = 0;
  for (int j = 0; j < 7; ++j) {
    off[j] = total;
    total += (sz[j] + 255) & ~(size_t)255;
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->corr_mem) {
    (void)hipFree(h->corr_mem);
    h->corr_mem = nullptr;
  }
  h->corr_every = 0;
  void* mem = nullptr;
  const hipError_t e = hipMalloc(&mem, total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (correlation buffers)");
  h->corr_mem = (char*)mem;
  std::memcpy(h->corr_off, off, sizeof off);
  std::vector<int32_t> kin(3 * (size_t)nk);
  for (int j = 0; j < nk; ++j)
    for (int a = 0; a < 3; ++a) {
      const int64_t La = h->p.n[a];
      kin[3 * j + a] = (int32_t)(((int64_t)kvec[3 * j + a] % La + La) % La);
    }
  HIP_TRY(hipMemcpyAsync(h->corr_mem + off[0], kin.data(), sz[0], hipMemcpyHostToDevice, h->stream));
  double* tw = (double*)(h->corr_mem + off[1]);
  for (int a = 0, base = 0; a < 3; base += (int)h->p.n[a], ++a)
    k_twiddle<<<(unsigned)((h->p.n[a] + 255) / 256), 256, 0, h->stream>>>(tw + 2 * base, h->p.n[a]);
  for (int j = 4; j < 7; ++j) {
    const int64_t nd = (int64_t)(sz[j] / sizeof(double));
    k_fill_zero<<<(unsigned)((nd + 255) / 256), 256, 0, h->stream>>>((double*)(h->corr_mem + off[j]), nd);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->stream));  // the host k-list buffer goes out of scope
  h->corr_nk = nk;
  h->corr_nlag = nlag;
  h->corr_nsb = (int)nsb;
  h->corr_count = 0;
  h->corr_every = every;
  return FLB_OK;
}

int flb_correlation(flb_lattice* h, double* sij, double* ct, int64_t* nsamples) {
  flb::TraceRange trace_("flb_correlation");
  if (!h || !nsamples) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (!h->corr_mem) return fail(FLB_ESTATE, "no correlation sampling was set up");
  DeviceGuard g(h->device);
  const int Q = h->Q;
  if (sij)
    HIP_TRY(hipMemcpyAsync(sij, h->corr_mem + h->corr_off[4], sizeof(double) * 2 * Q * Q * (size_t)h->corr_nk,
                           hipMemcpyDeviceToHost, h->stream));
  if (ct)
    HIP_TRY(hipMemcpyAsync(ct, h->corr_mem + h->corr_off[6],
                           sizeof(double) * 2 * (size_t)h->corr_nk * (size_t)h->corr_nlag,
                           hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  *nsamples = h->corr_count;
  return FLB_OK;
}

int flb_fourier_amplitudes(flb_lattice* h, double* amp) {
  flb::TraceRange trace_("flb_fourier_amplitudes");
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (!h->corr_mem) return fail(FLB_ESTATE, "no correlation k-list was set up");
  if (!amp) return fail(FLB_EINVAL, "amp is NULL");
  DeviceGuard g(h->device);
  launch_amp(h);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(amp, h->corr_mem + h->corr_off[3], sizeof(double) * 2 * h->Q * (size_t)h->corr_nk,
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FLB_OK;
}


int flb_set_regions(flb_lattice* h, const uint8_t* region, int32_t nregions, const double* theta,
                    const double* omega) {
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  DeviceGuard g(h->device);
  if (nregions == 0) {
    h->reg_n = 0;
    return FLB_OK;
  }
  if (h->aa) return fail(FLB_EINVAL, "regions step with the per-site two-buffer kernel: not with the AA layout");
  if (!region || !theta || !omega) return fail(FLB_EINVAL, "NULL argument");
  if (nregions < 1 || nregions > kMaxRegions) return fail(FLB_EINVAL, "need 1 <= nregions <= %d", kMaxRegions);
  for (int r = 0; r < nregions; ++r) {
    if (!(theta[r] > 0.0 && theta[r] < 1.0 / h->d))
      return fail(FLB_EINVAL, "region %d: theta = %g outside (0, 1/%d)", r, theta[r], h->d);
    if (!(omega[3 * r] > 0.0 && omega[3 * r] < 2.0))
      return fail(FLB_EINVAL, "region %d: omega_j = %g outside (0, 2)", r, omega[3 * r]);
    for (int a = 1; a < 3; ++a)
      if (omega[3 * r + a] != 0.0 && !(omega[3 * r + a] > 0.0 && omega[3 * r + a] < 2.0))
        return fail(FLB_EINVAL, "region %d: omega[%d] = %g outside (0, 2)", r, a, omega[3 * r + a]);
  }
  for (int64_t s = 0; s < h->n; ++s)
    if (region[s] >= nregions) return fail(FLB_EINVAL, "site %lld has region %d >= %d", (long long)s, region[s], nregions);
  if (!h->reg_map) {
    void* m = nullptr;
    hipError_t e = hipMalloc(&m, (size_t)h->n);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (region map)");
    h->reg_map = (uint8_t*)m;
    e = hipMalloc(&m, sizeof(KParams<double>) * kMaxRegions);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (region table)");
    h->reg_tab = (char*)m;
  }
  HIP_TRY(hipMemcpyAsync(h->reg_map, region, (size_t)h->n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int r = 0; r < nregions; ++r) {
    h->reg_theta[r] = theta[r];
    for (int a = 0; a < 3; ++a) h->reg_omega[r][a] = omega[3 * r + a];
  }
  h->reg_n = nregions;
  return rebuild_regions(h);
}

int flb_profile(flb_lattice* h, int32_t axis, double* sum_rho, double* sum_rho2) {
  flb::TraceRange trace_("flb_profile");
  if (!h || !sum_rho || !sum_rho2) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (axis < 0 || axis >= h->d) return fail(FLB_EINVAL, "axis %d outside [0, %d)", axis, h->d);
  DeviceGuard g(h->device);
  const int64_t nx = h->p.n[0], ny = h->p.n[1], nz = h->p.n[2], nrows = ny * nz;
  const int64_t L = h->p.n[axis];
  const size_t part_d = std::max<size_t>(2 * (size_t)std::min<int64_t>(kColChunks, nrows) * nx, 2 * (size_t)nrows);
  const size_t bytes = sizeof(double) * (part_d + 2 * (size_t)std::max(nx, std::max(ny, nz)));
  if (!h->prof_mem) {
    void* mem = nullptr;
    const hipError_t e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (profile buffers)");
    h->prof_mem = (char*)mem;
  }
  double* part = (double*)h->prof_mem;
  double* out = part + part_d;
  launch_profile(h, axis, part, out, out + L);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(sum_rho, out, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(sum_rho2, out + L, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FLB_OK;
}

int flb_profile_noalloc(flb_lattice* h, int32_t axis, double* d_sum_rho, double* d_sum_rho2) {
  flb::TraceRange trace_("flb_profile_noalloc");
  if (!h || !d_sum_rho || !d_sum_rho2) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is a member of a batch");
  if (axis < 0 || axis >= h->d) return fail(FLB_EINVAL, "axis %d outside [0, %d)", axis, h->d);
  const size_t need = profile_part_bytes(h, axis);
  if (need > kScratchBytes)
    return fail(FLB_EINVAL, "profile along axis %d needs %zu bytes of partial sums, above the static scratch of %zu",
                axis, need, kScratchBytes);
  DeviceGuard g(h->device);
  void* part = nullptr;
  const int rc = scratch_for(h->device, &part);
  if (rc) return rc;
  launch_profile(h, axis, (double*)part, d_sum_rho, d_sum_rho2);
  HIP_TRY(hipGetLastError());
  return FLB_OK;
}

int flb_sync(flb_lattice* h) {
  flb::TraceRange trace_("flb_sync");
  if (!h) return fail(FLB_EINVAL, "NULL handle");
  DeviceGuard g(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FLB_OK;
}

// one thread per value, 256 per block: the grid stays below 2^23 blocks
constexpr int64_t kMaxSample = (1ll << 31) - 256;

int flb_noise_sample(int32_t model, int32_t precision, int32_t law, uint64_t seed, int64_t step,
                     int64_t site0, int64_t nsite, void* d_words, void* d_vars, void* hip_stream) {
  if (model < 1 || model > 3) return fail(FLB_EINVAL, "model must be 1, 2 or 3");
  if (precision != 4 && precision != 8) return fail(FLB_EINVAL, "precision must be 4 or 8");
  if (law < 0 || law > 1) return fail(FLB_EINVAL, "law must be 0 or 1");
  if (nsite < 0 || site0 < 0 || step < 0) return fail(FLB_EINVAL, "negative size, site or step");
  if (nsite > kMaxSample) return fail(FLB_EINVAL, "nsite above 2^31 - 256");
  if (nsite == 0) return FLB_OK;
  flb_params p{};
  p.model = model;
  p.precision = precision;
  p.n[0] = 1;
  p.n[1] = 1;
  p.n[2] = 1;
  p.omega[0] = 1.0;
  p.seed = seed;
  p.noise = FLB_NOISE_LOCAL;
  p.noise_law = law;
  hipStream_t st = (hipStream_t)hip_stream;
  const unsigned nb = (unsigned)((nsite + 255) / 256);
  const uint32_t t32 = (uint32_t)(step & 0xFFFFFFFF);
  if (precision == 4) {
    KParams<float> P = make_kparams<float>(p, 0.0);
    if (model == 1) k_noise_sample<1, float><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (float*)d_vars);
    else if (model == 2) k_noise_sample<2, float><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (float*)d_vars);
    else k_noise_sample<3, float><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (float*)d_vars);
  } else {
    KParams<double> P = make_kparams<double>(p, 0.0);
    if (model == 1) k_noise_sample<1, double><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (double*)d_vars);
    else if (model == 2) k_noise_sample<2, double><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (double*)d_vars);
    else k_noise_sample<3, double><<<nb, 256, 0, st>>>(P, t32, site0, nsite, (uint32_t*)d_words, (double*)d_vars);
  }
  HIP_TRY(hipGetLastError());
  return FLB_OK;
}

int flb_gauss_map(int32_t precision, const void* d_words, int64_t n, void* d_z, void* hip_stream) {
  if (precision != 4 && precision != 8) return fail(FLB_EINVAL, "precision must be 4 or 8");
  if (n < 0) return fail(FLB_EINVAL, "negative size");
  if (n > kMaxSample) return fail(FLB_EINVAL, "n above 2^31 - 256");
  if (n == 0) return FLB_OK;
  if (!d_words || !d_z) return fail(FLB_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (precision == 4) k_gauss_map<float><<<nb, 256, 0, st>>>((const uint32_t*)d_words, n, (float*)d_z);
  else k_gauss_map<double><<<nb, 256, 0, st>>>((const uint32_t*)d_words, n, (double*)d_z);
  HIP_TRY(hipGetLastError());
  return FLB_OK;
}

}  // extern "C"
