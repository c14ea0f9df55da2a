// Batched ensembles: many lattices of uneven size and dimension advanced by
// one work-list launch per step (lattices in HBM) and one
// LDS-resident launch per chunk of steps (small D1Q3 lattices), the chunk
// captured once into a HIP graph and replayed.  Every member's arithmetic,
// noise keys and storage order are those of flb_step on the member alone,
// so results are bit-identical to stepping each lattice by itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "flb_internal.hpp"
#include "flb_kernels.hpp"

using namespace flb;

namespace flb {

// One member as the device sees it.  step0 / cur0 describe the state at the
// start of the current chunk and are advanced on the device at its end, so a
// captured chunk can be replayed.
template <typename T>
struct BatchRep {
  char* pop;        // the member's two population buffers
  int64_t plane;    // bytes of one buffer
  KParams<T> P;
  int64_t tiles_x;  // tiles of kBatchTX columns
  int64_t nrows;    // ny * nz
  int64_t step0;    // steps completed at the start of the chunk
  int32_t cur0;     // buffer holding the state at the start of the chunk (AA layout: its parity)
  int32_t depth;    // 2: D2Q5 member stepped in two-step passes (one buffer swap per pass)
  int32_t aa;       // single-buffer AA layout (stepped in place, depth 1)
};

// Buffer holding a member's state k steps into a chunk: one swap per step,
// or per two-step pass (a trailing single step of an odd chunk swaps once).
template <typename T>
__device__ __forceinline__ int member_parity(const BatchRep<T>& R, int k) {
  return R.depth == 2 ? (R.cur0 + (k + 1) / 2) & 1 : (R.cur0 + k) & 1;
}

// A work item is a tile of kBatchTX columns x `rows` rows (a multiple of
// kBatchRY), run by one kBatchTX-thread workgroup in sub-tiles of kBatchRY
// rows; taller items spread the item's descriptor loads over more sites.
constexpr int kBatchTX = 256;
constexpr int kBatchRY = 2;
// Flat work items: rows of 256 sites per lane and the store kind per model.
// D3Q7 members take one row and ordinary (cached) stores: at the member
// sizes of an ensemble or a request stream (up to ~1e8 sites) that measured
// 35 against 47 us per step at 153^3 and 622 against 703 us at 390^3
// (two rows, non-temporal stores); the others keep two rows and
// non-temporal stores, as fast either way.
template <int D> constexpr int kFlatRY = D == 3 ? 1 : 2;
template <int D> constexpr bool kFlatNT = D != 3;

// Work list: item w is tile item_tile[w] of member item_rep[w]; with a grid
// smaller than the list the workgroups persist and stride over it.
// Flat work list: item w covers sites item_tile[w] * 256 * kFlatRY<D> ... of
// member item_rep[w] (flat_tile), so narrow lattices keep every lane busy.
template <int D, typename T, int NP = kPlanRuntime>
__global__ void __launch_bounds__(256) k_batch_flat(const BatchRep<T>* __restrict__ reps,
                                                    const int32_t* __restrict__ item_rep,
                                                    const int32_t* __restrict__ item_tile,
                                                    int nitems, int k) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int r = __builtin_amdgcn_readfirstlane(item_rep[w]);
    const int64_t tile = __builtin_amdgcn_readfirstlane(item_tile[w]);
    const BatchRep<T>& R = reps[r];
    const KParams<T> P = R.P;
    const uint32_t step = (uint32_t)((uint64_t)(R.step0 + k) & 0xFFFFFFFFull);
    const int par = member_parity(R, k);
    if (R.aa) {  // in place, from the form of this step's parity
      if (par == 0)
        flat_tile_aa<D, T, kFlatRY<D>, kFlatNT<D>, kFormAAC, NP>((T*)R.pop, P, step, tile * 256 * kFlatRY<D>,
                                                                 threadIdx.x);
      else
        flat_tile_aa<D, T, kFlatRY<D>, kFlatNT<D>, kFormAAS, NP>((T*)R.pop, P, step, tile * 256 * kFlatRY<D>,
                                                                 threadIdx.x);
      continue;
    }
    const T* g = (const T*)(R.pop + par * R.plane);
    T* h = (T*)(R.pop + (par ^ 1) * R.plane);
    flat_tile<D, T, kFlatRY<D>, kFlatNT<D>, NP>(g, h, P, step, tile * 256 * kFlatRY<D>, threadIdx.x);
  }
}

// Two-step work list (D2Q5 members at depth 2): item w is the tile
// item_tile[w] = ty * tiles_x + tx (TW columns x kBatchTwoTY rows) of member
// item_rep[w]; steps k and k + 1 of the chunk in one pass.
constexpr int kBatchTwoTY = 8;

template <typename T, int TW, int NP = kPlanRuntime>
__global__ void __launch_bounds__(TW) k_batch_two(const BatchRep<T>* __restrict__ reps,
                                                  const int32_t* __restrict__ item_rep,
                                                  const int32_t* __restrict__ item_tile, int nitems, int k) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int r = __builtin_amdgcn_readfirstlane(item_rep[w]);
    const uint32_t tile = __builtin_amdgcn_readfirstlane(item_tile[w]);
    const BatchRep<T>& R = reps[r];
    const KParams<T> P = R.P;
    const uint32_t step = (uint32_t)((uint64_t)(R.step0 + k) & 0xFFFFFFFFull);
    const int par = member_parity(R, k);
    const T* g = (const T*)(R.pop + par * R.plane);
    T* h = (T*)(R.pop + (par ^ 1) * R.plane);
    const uint32_t tx2 = (uint32_t)((P.nx + TW - 1) / TW);
    step2_tile<T, kBatchTwoTY, true, false, TW, NP>(g, h, P, step, tile % tx2, tile / tx2, nullptr, nullptr);
  }
}

template <int D, typename T, int SUB>
__global__ void __launch_bounds__(kBatchTX) k_batch_rows(const BatchRep<T>* __restrict__ reps,
                                                         const int32_t* __restrict__ item_rep,
                                                         const int32_t* __restrict__ item_tile,
                                                         int nitems, int k) {
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int r = __builtin_amdgcn_readfirstlane(item_rep[w]);
    const int64_t tile = __builtin_amdgcn_readfirstlane(item_tile[w]);
    const BatchRep<T>& R = reps[r];
    const KParams<T> P = R.P;
    const uint32_t step = (uint32_t)((uint64_t)(R.step0 + k) & 0xFFFFFFFFull);
    const int par = member_parity(R, k);
    const T* g = (const T*)(R.pop + par * R.plane);
    T* h = (T*)(R.pop + (par ^ 1) * R.plane);
    const int64_t tx = tile % R.tiles_x, tr = tile / R.tiles_x;
    const uint32_t x = (uint32_t)(tx * kBatchTX) + threadIdx.x;
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub)
      rows_tile<D, T, kBatchRY, true>(g, h, P, step, x, (tr * SUB + sub) * kBatchRY, R.nrows);
  }
}

// A whole D1Q3 lattice in one workgroup's LDS for c steps.  The LDS holds
// the canonical pre-collision state; a step reads each site, collides it in
// registers, and after a barrier pushes the populations to their
// destinations.  The last step stores the post-collision populations at
// their collision sites in the member's other-parity buffer, the storage form
// flb_step leaves.
template <typename T, int SPT, int NP = kPlanRuntime>
__global__ void __launch_bounds__(256) k_batch_lds_d1(const BatchRep<T>* __restrict__ reps,
                                                      const int32_t* __restrict__ lds_rep, int c) {
  extern __shared__ unsigned char smem_raw[];
  T* s0 = (T*)smem_raw;
  const int r = __builtin_amdgcn_readfirstlane(lds_rep[blockIdx.x]);
  const BatchRep<T>& R = reps[r];
  const KParams<T> P = R.P;
  const int L = (int)P.nx;
  T* s1 = s0 + L;
  T* s2 = s1 + L;
  const int tid = threadIdx.x;
  // pull storage: f_i(x) = g_i(x - v_i); AA layout (one buffer, read whole
  // into LDS before anything is stored): the form of the parity
  const T* g = (const T*)(R.pop + (R.aa ? 0 : R.cur0 * R.plane));
  const bool cin = R.aa && R.cur0 == 0, swin = R.aa && R.cur0 == 1;
  for (int x = tid; x < L; x += 256) {
    s0[x] = g[x];
    s1[x] = cin ? g[L + x] : g[(swin ? 2 : 1) * L + (x == 0 ? L - 1 : x - 1)];
    s2[x] = cin ? g[2 * L + x] : g[(swin ? 1 : 2) * L + (x == L - 1 ? 0 : x + 1)];
  }
  __syncthreads();
  T* out = (T*)(R.pop + (R.aa ? 0 : ((R.cur0 + c) & 1) * R.plane));
  const bool cout_ = R.aa && ((R.cur0 + c) & 1) == 0, swout = R.aa && !cout_;
  for (int k = 0; k < c; ++k) {
    const uint32_t step = (uint32_t)((uint64_t)(R.step0 + k) & 0xFFFFFFFFull);
    T f[SPT][3];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int x = tid + 256 * j;
      if (x < L) {
        f[j][0] = s0[x];
        f[j][1] = s1[x];
        f[j][2] = s2[x];
        Collide<1, T, NP>::run(f[j], P, (uint64_t)x, step);
      }
    }
    __syncthreads();
    if (k + 1 < c) {
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int x = tid + 256 * j;
        if (x < L) {
          s0[x] = f[j][0];
          s1[x == L - 1 ? 0 : x + 1] = f[j][1];
          s2[x == 0 ? L - 1 : x - 1] = f[j][2];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const int x = tid + 256 * j;
        if (x < L) {  // pull storage at x; AA form S: opposite slots at x; form C: pushed
          out[x] = f[j][0];
          out[(swout ? 2 : 1) * L + (cout_ ? (x == L - 1 ? 0 : x + 1) : x)] = f[j][1];
          out[(swout ? 1 : 2) * L + (cout_ ? (x == 0 ? L - 1 : x - 1) : x)] = f[j][2];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void k_batch_advance(BatchRep<T>* __restrict__ reps, int n, int c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    reps[i].cur0 = member_parity(reps[i], c);
    reps[i].step0 += c;
  }
}

}  // namespace flb

struct flb_batch {
  flb_batch_opts o;
  hipStream_t stream;
  bool own_stream;
  int device;
  int ncu;
  std::vector<flb_lattice*> members;
  int precision;  // 0 until the first member
  bool dirty;
  // device table: reps, then the item lists and the LDS member list
  char* d_table;
  size_t table_cap;
  // per class: d = 1..3 row tiles, d + 3 flat tiles, 7 two-step tiles and 8
  // flat tiles of the depth-2 members (their odd trailing step); item_rep, item_tile
  size_t off_items[9][2];
  int nitems[9];
  size_t off_lds;
  int nlds, lds_spt;
  size_t lds_bytes;
  int nreps;
  int sub;  // sub-tiles of kBatchRY rows per work item
  bool two_lg;  // every depth-2 member has local Gaussian noise (compile-time noise plan)
  bool flat_lg;  // every flat-item member has local Gaussian noise
  bool lds_lg;   // every LDS member has local Gaussian noise
  hipGraphExec_t exec;
  int exec_chunk;
  // the LDS members run on a second stream, forked from and joined to the
  // batch's stream around the HBM members' passes (in a captured graph: a
  // parallel branch)
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
};

namespace {

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int spt_for(int64_t L) {
  const int64_t need = (L + 255) / 256;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

void drop_graph(flb_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->exec_chunk = 0;
}

// Rebuild the device table from the members' host state (stream idle).
template <typename T>
int rebuild_t(flb_batch* b) {
  const int n = (int)b->members.size();
  std::vector<BatchRep<T>> reps(n);
  std::vector<int32_t> items[9][2];
  std::vector<int32_t> lds;
  int64_t lmax = 0;
  const int64_t lds_max = b->o.lds_max_bytes < 0 ? -1 : (b->o.lds_max_bytes ? b->o.lds_max_bytes : 65536);
  bool two_lg = true, flat_lg = true, lds_lg = true;
  for (int i = 0; i < n; ++i) {
    flb_lattice* h = b->members[i];
    BatchRep<T>& R = reps[i];
    std::memset(&R, 0, sizeof R);
    R.pop = h->pop;
    R.plane = (int64_t)h->plane;
    R.P = make_kparams<T>(h->p, h->rho_eq);
    R.tiles_x = (h->p.n[0] + kBatchTX - 1) / kBatchTX;
    R.nrows = h->p.n[1] * h->p.n[2];
    R.step0 = h->step;
    R.cur0 = h->cur;
    R.aa = h->aa ? 1 : 0;
    const int64_t state_bytes = (int64_t)h->Q * h->n * (int64_t)sizeof(T);
    const bool lg = h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
    if (h->d == 1 && lds_max > 0 && state_bytes <= lds_max && h->n <= 256 * 16) {
      lds_lg = lds_lg && lg;
      lds.push_back(i);
      lmax = std::max<int64_t>(lmax, h->n);
      continue;
    }
    const int64_t item_rows = (int64_t)kBatchRY * b->sub;
    // AA members step in place with the flat items (their layout has no
    // second buffer for a two-step pass)
    const bool flat = (b->o.tiling == 0 || h->aa) && (int64_t)h->plane < (1ll << 32);
    if (b->o.depth == 2 && h->d == 2 && !h->aa && (int64_t)h->plane < (1ll << 32)) {
      R.depth = 2;
      two_lg = two_lg && h->p.noise == FLB_NOISE_LOCAL && h->p.noise_law == FLB_LAW_GAUSS;
      const int64_t tw = b->o.width;
      const int64_t t2 = ((h->p.n[0] + tw - 1) / tw) * ((h->p.n[1] + kBatchTwoTY - 1) / kBatchTwoTY);
      const int64_t tf = (h->n + 256 * kBatchRY - 1) / (256 * kBatchRY);
      if (t2 >= (1ll << 31) || tf >= (1ll << 31)) return fail(FLB_EINVAL, "member %d has too many tiles", i);
      for (int64_t t = 0; t < t2; ++t) {
        items[7][0].push_back(i);
        items[7][1].push_back((int32_t)t);
      }
      R.tiles_x = -1;
      for (int64_t t = 0; t < tf; ++t) {
        items[8][0].push_back(i);
        items[8][1].push_back((int32_t)t);
      }
      flat_lg = flat_lg && lg;  // their odd trailing step takes the flat items
      continue;
    }
    R.depth = 1;
    if (flat) R.tiles_x = -1;  // marks a flat member
    const int64_t fry = h->d == 3 ? kFlatRY<3> : kFlatRY<1>;
    const int64_t ntile = flat ? (h->n + 256 * fry - 1) / (256 * fry)
                               : R.tiles_x * ((R.nrows + item_rows - 1) / item_rows);
    if (ntile >= (1ll << 31)) return fail(FLB_EINVAL, "member %d has too many tiles", i);
    const int cls = h->d + (flat ? 3 : 0);
    if (flat) flat_lg = flat_lg && lg;
    for (int64_t t = 0; t < ntile; ++t) {
      items[cls][0].push_back(i);
      items[cls][1].push_back((int32_t)t);
    }
  }
  size_t o = align256(sizeof(BatchRep<T>) * std::max(n, 1));
  for (int d = 1; d <= 8; ++d) {
    b->nitems[d] = (int)items[d][0].size();
    b->off_items[d][0] = o;
    o += align256(sizeof(int32_t) * std::max<size_t>(items[d][0].size(), 1));
    b->off_items[d][1] = o;
    o += align256(sizeof(int32_t) * std::max<size_t>(items[d][1].size(), 1));
  }
  b->off_lds = o;
  o += align256(sizeof(int32_t) * std::max<size_t>(lds.size(), 1));
  if (o > b->table_cap) {
    if (b->d_table) HIP_TRY(hipFree(b->d_table));
    b->d_table = nullptr;
    hipError_t e = hipMalloc((void**)&b->d_table, o);
    if (e != hipSuccess) return fail(FLB_ENOMEM, "batch table allocation of %zu bytes failed", o);
    b->table_cap = o;
  }
  HIP_TRY(hipMemcpy(b->d_table, reps.data(), sizeof(BatchRep<T>) * n, hipMemcpyHostToDevice));
  for (int d = 1; d <= 8; ++d)
    for (int k = 0; k < 2; ++k)
      if (!items[d][k].empty())
        HIP_TRY(hipMemcpy(b->d_table + b->off_items[d][k], items[d][k].data(),
                          sizeof(int32_t) * items[d][k].size(), hipMemcpyHostToDevice));
  if (!lds.empty())
    HIP_TRY(hipMemcpy(b->d_table + b->off_lds, lds.data(), sizeof(int32_t) * lds.size(), hipMemcpyHostToDevice));
  b->nlds = (int)lds.size();
  b->lds_spt = spt_for(lmax);
  b->lds_bytes = (size_t)(3 * lmax * (int64_t)sizeof(T));
  b->nreps = n;
  b->two_lg = two_lg;
  b->flat_lg = flat_lg;
  b->lds_lg = lds_lg;
  b->dirty = false;
  drop_graph(b);
  return FLB_OK;
}

template <typename T>
int enqueue_chunk_t(flb_batch* b, int c) {
  const BatchRep<T>* reps = (const BatchRep<T>*)b->d_table;
  hipStream_t st = b->stream;
  // the LDS members share nothing with the others until the step advance:
  // with HBM members present they run on the side stream, concurrently
  bool hbm = false;
  for (int d = 1; d <= 8; ++d) hbm |= b->nitems[d] > 0;
  const bool fork = b->nlds > 0 && hbm;
  if (fork) {
    HIP_TRY(hipEventRecord(b->ev_fork, st));
    HIP_TRY(hipStreamWaitEvent(b->side, b->ev_fork, 0));
  }
  if (b->nlds > 0) {
    const int32_t* lr = (const int32_t*)(b->d_table + b->off_lds);
    const dim3 grid(b->nlds), block(256);
    hipStream_t ls = fork ? b->side : st;
#define FLB_LDS(SV)                                                                                  \
  (b->lds_lg ? (void)(k_batch_lds_d1<T, SV, kPlanLocalGauss><<<grid, block, b->lds_bytes, ls>>>(reps, lr, c)) \
             : (void)(k_batch_lds_d1<T, SV><<<grid, block, b->lds_bytes, ls>>>(reps, lr, c)))
    switch (b->lds_spt) {
      case 1: FLB_LDS(1); break;
      case 2: FLB_LDS(2); break;
      case 4: FLB_LDS(4); break;
      case 8: FLB_LDS(8); break;
      default: FLB_LDS(16); break;
    }
#undef FLB_LDS
    if (fork) HIP_TRY(hipEventRecord(b->ev_join, b->side));
  }
  if (b->nitems[7] > 0) {  // depth-2 members: two-step passes, a single flat step for an odd chunk
    const int32_t* ir2 = (const int32_t*)(b->d_table + b->off_items[7][0]);
    const int32_t* it2 = (const int32_t*)(b->d_table + b->off_items[7][1]);
    const int32_t* ir1 = (const int32_t*)(b->d_table + b->off_items[8][0]);
    const int32_t* it1 = (const int32_t*)(b->d_table + b->off_items[8][1]);
    for (int k = 0; k < c; k += 2) {
      if (k + 1 < c) {
        const int ni = b->nitems[7];
        const int grid = b->o.workers > 0 ? std::max(1, std::min(ni, b->o.workers)) : ni;
#define FLB_BTWO(TWV)                                                                         \
  (b->two_lg ? (void)(k_batch_two<T, TWV, kPlanLocalGauss><<<grid, TWV, 0, st>>>(reps, ir2, it2, ni, k)) \
             : (void)(k_batch_two<T, TWV><<<grid, TWV, 0, st>>>(reps, ir2, it2, ni, k)))
        if (b->o.width == 64) FLB_BTWO(64);
        else if (b->o.width == 128) FLB_BTWO(128);
        else FLB_BTWO(256);
#undef FLB_BTWO
      } else {
        const int ni = b->nitems[8];
        const int grid = b->o.workers > 0 ? std::max(1, std::min(ni, b->o.workers)) : ni;
        if (b->flat_lg) k_batch_flat<2, T, kPlanLocalGauss><<<grid, 256, 0, st>>>(reps, ir1, it1, ni, k);
        else k_batch_flat<2, T><<<grid, 256, 0, st>>>(reps, ir1, it1, ni, k);
      }
    }
  }
  for (int k = 0; k < c; ++k) {
    for (int d = 4; d <= 6; ++d) {  // flat members
      const int ni = b->nitems[d];
      if (ni == 0) continue;
      const int grid = b->o.workers > 0 ? std::max(1, std::min(ni, b->o.workers)) : ni;
      const int32_t* ir = (const int32_t*)(b->d_table + b->off_items[d][0]);
      const int32_t* it = (const int32_t*)(b->d_table + b->off_items[d][1]);
      if (b->flat_lg) {
        if (d == 4) k_batch_flat<1, T, kPlanLocalGauss><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
        else if (d == 5) k_batch_flat<2, T, kPlanLocalGauss><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
        else k_batch_flat<3, T, kPlanLocalGauss><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
      } else {
        if (d == 4) k_batch_flat<1, T><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
        else if (d == 5) k_batch_flat<2, T><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
        else k_batch_flat<3, T><<<grid, 256, 0, st>>>(reps, ir, it, ni, k);
      }
    }
    for (int d = 1; d <= 3; ++d) {
      const int ni = b->nitems[d];
      if (ni == 0) continue;
      // workers == 0: one workgroup per item, the dispatcher balances; else a
      // persistent grid of `workers` workgroups strides over the items
      const int grid = b->o.workers > 0 ? std::max(1, std::min(ni, b->o.workers)) : ni;
      const int32_t* ir = (const int32_t*)(b->d_table + b->off_items[d][0]);
      const int32_t* it = (const int32_t*)(b->d_table + b->off_items[d][1]);
#define FLB_BATCH_ROWS(SUBV)                                                                   \
  do {                                                                                         \
    if (d == 1) k_batch_rows<1, T, SUBV><<<grid, kBatchTX, 0, st>>>(reps, ir, it, ni, k);      \
    else if (d == 2) k_batch_rows<2, T, SUBV><<<grid, kBatchTX, 0, st>>>(reps, ir, it, ni, k); \
    else k_batch_rows<3, T, SUBV><<<grid, kBatchTX, 0, st>>>(reps, ir, it, ni, k);             \
  } while (0)
      switch (b->sub) {
        case 1: FLB_BATCH_ROWS(1); break;
        case 2: FLB_BATCH_ROWS(2); break;
        case 4: FLB_BATCH_ROWS(4); break;
        default: FLB_BATCH_ROWS(8); break;
      }
#undef FLB_BATCH_ROWS
    }
  }
  if (fork) HIP_TRY(hipStreamWaitEvent(st, b->ev_join, 0));
  k_batch_advance<T><<<(b->nreps + 255) / 256, 256, 0, st>>>((BatchRep<T>*)b->d_table, b->nreps, c);
  return FLB_OK;
}

int enqueue_chunk(flb_batch* b, int c) {
  return b->precision == 4 ? enqueue_chunk_t<float>(b, c) : enqueue_chunk_t<double>(b, c);
}

int capture(flb_batch* b, int c) {
  drop_graph(b);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_chunk(b, c);
  hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->exec_chunk = c;
  return FLB_OK;
}

}  // namespace

extern "C" {

int flb_batch_create(const flb_batch_opts* opts, flb_batch** out) {
  if (!out) return fail(FLB_EINVAL, "out is NULL");
  *out = nullptr;
  flb_batch_opts o{};
  if (opts) o = *opts;
  if (o.chunk < 0 || o.chunk > 4096) return fail(FLB_EINVAL, "chunk must be in [0, 4096]");
  if (o.workers < 0) return fail(FLB_EINVAL, "workers must be >= 0");
  if (o.lds_max_bytes > 65536) return fail(FLB_EINVAL, "lds_max_bytes must be <= 65536");
  if (o.tiling < 0 || o.tiling > 1) return fail(FLB_EINVAL, "tiling must be 0 (flat) or 1 (rows)");
  if (o.item_rows != 0 && o.item_rows != 2 && o.item_rows != 4 && o.item_rows != 8 && o.item_rows != 16)
    return fail(FLB_EINVAL, "item_rows must be 2, 4, 8 or 16");
  if (o.depth < 0 || o.depth > 2) return fail(FLB_EINVAL, "depth must be 0 (default), 1 or 2");
  if (o.depth == 0) o.depth = 2;
  if (o.width != 0 && o.width != 64 && o.width != 128 && o.width != 256)
    return fail(FLB_EINVAL, "width must be 0 (default), 64, 128 or 256");
  if (o.width == 0) o.width = 256;
  if (o.chunk == 0) o.chunk = 16;
  flb_batch* b = new (std::nothrow) flb_batch();
  if (!b) return fail(FLB_ENOMEM, "batch allocation failed");
  b->o = o;
  b->precision = 0;
  b->dirty = true;
  b->d_table = nullptr;
  b->table_cap = 0;
  b->exec = nullptr;
  b->exec_chunk = 0;
  b->nlds = 0;
  b->nreps = 0;
  b->sub = o.item_rows ? o.item_rows / kBatchRY : 1;
  b->two_lg = false;
  b->flat_lg = false;
  b->lds_lg = false;
  for (int d = 0; d < 9; ++d) b->nitems[d] = 0;
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "device query");
  }
  if (o.hip_stream) {
    b->stream = (hipStream_t)o.hip_stream;
    b->own_stream = false;
  } else {
    // a stream of our own (the null stream cannot be captured); default priority
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete b;
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    b->own_stream = true;
  }
  b->side = nullptr;
  b->ev_fork = b->ev_join = nullptr;
  e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);  // default priority
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return hip_fail(e, "side stream / events");
  }
  *out = b;
  return FLB_OK;
}

int flb_batch_admit(flb_batch* b, flb_lattice* h) {
  if (!b || !h) return fail(FLB_EINVAL, "NULL argument");
  if (h->batch_refs > 0) return fail(FLB_ESTATE, "lattice is already in a batch");
  if (h->device != b->device) return fail(FLB_EINVAL, "lattice and batch are on different devices");
  if (h->reg_n > 0) return fail(FLB_EINVAL, "a lattice with regions (flb_set_regions) is stepped alone");
  // a batch step takes no statistics: refuse rather than leave them unsampled
  if (h->sample_every > 0 || h->mom_every > 0 || h->corr_every > 0)
    return fail(FLB_ESTATE, "lattice samples statistics while stepping (flb_set_sampling / "
                            "flb_set_moment_sampling / flb_set_correlation); stop that before admitting it");
  if (b->precision && (int)h->s != b->precision)
    return fail(FLB_EINVAL, "batch holds precision %d, lattice has %d", b->precision, (int)h->s);
  DevGuard g(b->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->members.push_back(h);
  b->precision = (int)h->s;
  h->batch_refs += 1;
  b->dirty = true;
  return FLB_OK;
}

int flb_batch_retire(flb_batch* b, flb_lattice* h) {
  if (!b || !h) return fail(FLB_EINVAL, "NULL argument");
  auto it = std::find(b->members.begin(), b->members.end(), h);
  if (it == b->members.end()) return fail(FLB_EINVAL, "lattice is not a member of this batch");
  DevGuard g(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->members.erase(it);
  h->batch_refs -= 1;
  if (b->members.empty()) b->precision = 0;
  b->dirty = true;
  return FLB_OK;
}

int flb_batch_step(flb_batch* b, int64_t nsteps) {
  flb::TraceRange trace_("flb_batch_step");
  if (!b) return fail(FLB_EINVAL, "NULL batch");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  if (b->members.empty() || nsteps == 0) return FLB_OK;
  DevGuard g(b->device);
  if (b->dirty) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int rc = b->precision == 4 ? rebuild_t<float>(b) : rebuild_t<double>(b);
    if (rc) return rc;
  }
  const int c = b->o.chunk;
  const int64_t chunks = nsteps / c;
  const int rem = (int)(nsteps % c);
  if (chunks > 0) {
    if (b->o.use_graph) {
      if (!b->exec || b->exec_chunk != c) {
        const int rc = capture(b, c);
        if (rc) return rc;
      }
      for (int64_t i = 0; i < chunks; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    } else {
      for (int64_t i = 0; i < chunks; ++i) {
        const int rc = enqueue_chunk(b, c);
        if (rc) return rc;
      }
    }
  }
  if (rem) {
    const int rc = enqueue_chunk(b, rem);
    if (rc) return rc;
  }
  HIP_TRY(hipGetLastError());
  // buffer swaps of each member, chunk by chunk (depth-2 D2Q5 members swap once per pass)
  for (flb_lattice* h : b->members) {
    const bool two = b->o.depth == 2 && h->d == 2 && !h->aa && (int64_t)h->plane < (1ll << 32);
    const int64_t swaps = two ? chunks * ((c + 1) / 2) + (rem + 1) / 2 : nsteps;
    h->step += nsteps;
    h->cur = (int)((h->cur + swaps) & 1);
  }
  return FLB_OK;
}

int flb_batch_size(flb_batch* b, int32_t* n) {
  if (!b || !n) return fail(FLB_EINVAL, "NULL argument");
  *n = (int32_t)b->members.size();
  return FLB_OK;
}

int flb_batch_sync(flb_batch* b) {
  flb::TraceRange trace_("flb_batch_sync");
  if (!b) return fail(FLB_EINVAL, "NULL batch");
  DevGuard g(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream));
  return FLB_OK;
}

int flb_batch_destroy(flb_batch* b) {
  if (!b) return FLB_OK;
  DevGuard g(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (flb_lattice* h : b->members) h->batch_refs -= 1;
  drop_graph(b);
  if (b->d_table) (void)hipFree(b->d_table);
  (void)hipStreamSynchronize(b->side);
  (void)hipEventDestroy(b->ev_fork);
  (void)hipEventDestroy(b->ev_join);
  (void)hipStreamDestroy(b->side);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return FLB_OK;
}

}  // extern "C"
