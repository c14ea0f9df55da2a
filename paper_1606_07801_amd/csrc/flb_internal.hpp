// Declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "../../include/flb.h"
#include "flb_device.hpp"

namespace flb {

constexpr int kRedBlocks = 1024;  // blocks of the lattice-sum reduction
constexpr int kMaxK = 1024;       // wave vectors per structure-factor list
constexpr int kMaxLag = 65536;     // lags of the time correlator
constexpr int kMaxKLag = 1 << 20;  // wave vectors x lags (ring and correlator: 16 B each)
constexpr int kCorrBlocks = 256;   // site blocks of the Fourier-sum pass
constexpr int kSkChunks = 256;    // site chunks of the direct structure factor
constexpr int kColChunks = 64;    // row chunks of the column marginals
constexpr int kNVals = 40;        // lattice sums (see k_moments_partial)
constexpr int kSampleRows = 8;    // rows per tile of the sampled step (and of a sampled two-step pass)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the workspace regions.
struct WorkLayout {
  size_t red_part, red_out, rowsum, colpart, marg, skpart, total;
  size_t tw;              // twiddle tables of the three axes (2 (nx + ny + nz) doubles)
  size_t rowpart, colbig; // partials of the sampled step (tiles of 256 x kSampleRows)
  size_t momacc;          // accumulated lattice sums of sampled states (kNVals doubles)
  // two k-list sets: [0] snapshot, [1] accumulator
  size_t kinfo[2], kv[2], slot_ax[2], slot_gen[2], sval[2];
  size_t skacc;
};
WorkLayout work_layout(const flb_params& p);

// Pinned host staging of one lattice.
struct KStage {
  int64_t kinfo[2 * kMaxK];
  int64_t kv[3 * kMaxK];
  int32_t slot_ax[kMaxK];
  int32_t slot_gen[kMaxK];
  double out[kMaxK];
  double red[kNVals];
};

}  // namespace flb

struct flb_lattice {
  flb_params p;
  int d, Q;
  int64_t n;
  size_t s;           // bytes per real
  size_t plane;       // bytes of one buffer (Q * n * s)
  char* pop;          // two buffers, or one (AA layout)
  bool aa;            // single-buffer AA layout
  int cur;            // buffer holding the current state; AA: steps since set, mod 2
  char* work;
  bool own_work;
  flb::WorkLayout wl;
  hipStream_t stream;
  int device;
  int64_t step;
  double mass0, rho_eq;
  flb::KStage* stage;
  // structure-factor lists: [0] snapshot, [1] accumulator
  int nk[2], nax[2], ngen[2];
  std::vector<int32_t> klist[2];
  int64_t sk_count;
  int batch_refs;     // > 0 while a batch holds the lattice
  int64_t sample_every;  // > 0: accumulate S(k) of the accumulator k-list every this many steps
  bool sample_fused;     // the sampled step kernel produces the marginals
  int64_t mom_every;     // > 0: accumulate the lattice sums every this many steps
  int64_t mom_count;     // samples in the lattice-sum accumulator
  // population correlators (flb_set_correlation); one library allocation
  // holding k-list | twiddles | partials | amplitudes | S_ij | ring | C
  int64_t corr_every;    // > 0: sample every this many steps
  int corr_nk, corr_nlag, corr_nsb;
  int64_t corr_count;    // samples accumulated
  int64_t check_every;   // > 0: flb_step checks the state for non-finite values
  char* corr_mem;
  size_t corr_off[7];
  // small lattices: one workgroup steps the whole lattice in LDS
  bool resident;
  size_t res_lds;        // its LDS bytes
  int res_lds_max;       // the device's LDS bytes per workgroup
  char* prof_mem;        // density-profile buffers (library-allocated on first use)
  // temperature and rates by region (flb_set_regions); reg_n = 0: uniform
  int reg_n;
  uint8_t* reg_map;      // region of every site (device, library-allocated)
  char* reg_tab;         // kernel constants of every region (device)
  double reg_theta[16], reg_omega[16][3];
};

namespace flb {

// A roctx range around one API call (host side: the call's enqueue time;
// rocprofv3 --marker-trace records it beside the kernels it launched).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
double default_theta(int d);
int check_params(const flb_params* p);
template <typename T>
KParams<T> make_kparams(const flb_params& p, double rho_eq);

}  // namespace flb
