/*
 * flb.h - C ABI of the MI355X (gfx950) fluctuating lattice Boltzmann library
 * for the diffusion equation (Wagner & Strand, "A Fluctuating Lattice
 * Boltzmann Method for the Diffusion Equation", arXiv:1606.07801).
 *
 * The method (paper Sec. II):
 *   f_i(x + v_i, t + 1) = f_i(x, t) + Omega_i                         eq. (LB)
 *   Omega_i = sum_j Lambda_ij (f_j^0 - f_j) + xi_i                    eq. (collision)
 * with f_i^0 = rho w_i (eq. f0def), a collision matrix that is diagonal in
 * the orthonormal moment basis m_i^a (Sec. II, Gram-Schmidt under
 * sum_i m_i^a w_i m_i^b = delta^ab), relaxation rate omega_a = 1/tau^a per
 * isotropy class, and noise on the non-conserved moments only, with variance
 *   <xi^a xi^a> = rho_n (2 tau^a - 1) / (tau^a)^2                     eqs. (xilocal), (xiglobal)
 * where rho_n is the local density clamped at zero (Sec. IV, closing the
 * algorithm), the global mean density, or zero (noise off).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Lattices: D1Q3, D2Q5, D3Q7 on a periodic box n[0] x n[1] x n[2]
 *   (unused sizes are 1).  Velocity order: 0, +x, -x, +y, -y, +z, -z.
 * - Canonical state: the pre-collision populations f_i(x, t) in SoA layout
 *   f[i][z][y][x] (x fastest), in the lattice's precision (4 = float32,
 *   8 = float64).  The site index is s = x + n0 (y + n1 z).
 * - Noise: Philox4x32-10 keyed by the 64-bit seed (low word, high word),
 *   counter (s low word, s high word, t mod 2^32, block) with t the number
 *   of steps completed before the collision and block = (a - 1) / 4 for
 *   moment a >= 1; moment a takes word (a - 1) mod 4 of its block.  Words map
 *   to u = (2 (r >> 9) + 1) 2^-24, and pairs of u to normals by Box-Muller
 *   (R = sqrt(-2 ln u0), z0 = R cos 2 pi u1, z1 = R sin 2 pi u1).  The
 *   uniform law uses xi = sqrt(3 var) (2u - 1) (the paper's flat law, Sec. IV).
 * - Memory: the caller owns every device buffer and the HIP stream; the
 *   library owns the opaque handle, an optional workspace it allocates when
 *   the caller passes none, and small pinned staging.  Calls on one handle
 *   are not thread-safe; each handle issues all of its work on its stream.
 * - Errors: every function returns 0 (FLB_OK) or a negative FLB_E* code and
 *   leaves a message for flb_last_error() (thread-local).  Nothing throws
 *   across the ABI.  A failed call leaves the handle's state unchanged,
 *   except FLB_EDEVICE, after which the handle should be destroyed.
 */
#ifndef FLB_H
#define FLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLB_ABI_VERSION 1

enum {
  FLB_OK = 0,
  FLB_EINVAL = -1,      /* invalid argument or parameter */
  FLB_ENOMEM = -2,      /* buffer too small, or allocation failed */
  FLB_EDEVICE = -3,     /* HIP runtime error */
  FLB_ESTATE = -4,      /* call not valid in the handle's current state */
  FLB_ENONFINITE = -5   /* non-finite populations detected (check mode, flb_set_check) */
};

enum { FLB_D1Q3 = 1, FLB_D2Q5 = 2, FLB_D3Q7 = 3 };
enum { FLB_NOISE_LOCAL = 0, FLB_NOISE_GLOBAL = 1, FLB_NOISE_OFF = 2 };
enum { FLB_LAW_GAUSS = 0, FLB_LAW_UNIFORM = 1 };
/* Storage scheme of the populations (eq. LB's streaming).  TWO_BUFFER: two
 * buffers of Q N values, pull streaming from one into the other.  AA: one
 * buffer, stepped in place: a step from the canonical form (even steps
 * since flb_set_populations) collides every site and stores f_i* in the
 * slot of the opposite velocity at the same site; the next gathers the
 * incoming populations from those slots and stores the post-collision values
 * at the neighbours' own slots, which gives the canonical form again.  Each
 * site writes exactly the slots it read.  Half the memory, the same traffic,
 * results bit-identical to TWO_BUFFER.  AA lattices step with the flat or
 * resident kernels (kernel AUTO, FLAT or RESIDENT; Q N precision < 2^32),
 * take S(k) samples in a pass of their own, have no regions, and
 * flb_get_populations into host memory at odd parity allocates a temporary
 * device buffer of Q N precision bytes (a device destination needs none). */
enum { FLB_LAYOUT_TWO_BUFFER = 0, FLB_LAYOUT_AA = 1 };
/* kernel variants of the step (all give bit-identical results).  RESIDENT:
 * one workgroup keeps the whole lattice in LDS and runs up to 65536 steps per
 * launch, with the sampled statistics taken inside; for lattices of at most
 * 4096 sites whose state, densities and twiddles fit the device's LDS per
 * workgroup (EINVAL at flb_create otherwise).  AUTO picks RESIDENT when it
 * fits, else ROWS. */
enum { FLB_KERNEL_AUTO = 0, FLB_KERNEL_PLAIN = 1, FLB_KERNEL_ROWS = 2, FLB_KERNEL_FLAT = 3,
       FLB_KERNEL_RESIDENT = 4, FLB_KERNEL_TWO_STEP = 5 };
/* TWO_STEP (D2Q5 only; Q N precision < 2^32): pairs of steps between which
 * nothing is sampled run as one pass over the lattice (tiles of 256 columns
 * x tile_rows rows, 2..16, default 8, with a one-site halo recomputed by
 * the neighbouring tiles), halving the populations' trips through HBM; the
 * other steps take the flat kernel.  Bit-identical to single steps. */

typedef struct flb_lattice flb_lattice; /* opaque */
typedef struct flb_batch flb_batch;     /* opaque */

typedef struct {
  int32_t model;      /* FLB_D1Q3 / FLB_D2Q5 / FLB_D3Q7 */
  int32_t precision;  /* 4 = float32 populations, 8 = float64 */
  int64_t n[3];       /* box sizes (n[1], n[2] = 1 below 2-D / 3-D); each >= 1 */
  double theta;       /* lattice temperature; 0 -> 1/3 (D1Q3, D2Q5), 1/4 (D3Q7);
                         must satisfy 0 < theta < 1/d */
  double omega[3];    /* relaxation rates of the current (j), traceless (n) and
                         trace (s) moments, each in (0, 2); omega[1], omega[2]
                         = 0 -> omega[0].  D = (1/omega_j - 1/2) theta. */
  uint64_t seed;      /* Philox key */
  int32_t noise;      /* FLB_NOISE_* */
  int32_t noise_law;  /* FLB_LAW_* */
  int32_t layout;     /* FLB_LAYOUT_* */
  int32_t kernel;     /* FLB_KERNEL_* */
  int32_t tile_x;     /* rows kernel: threads per block along x (64..1024, multiple
                         of 64); 0 -> default */
  int32_t tile_rows;  /* rows kernel: rows per thread (1, 2, 4, 8, 16); flat: sites per lane
                         in units of 256; two-step: rows per tile; 0 -> default */
  int32_t nt_store;   /* rows kernel: 1 = non-temporal stores of the new state */
  int32_t pipeline;   /* rows kernel: 1 = rows software-pipelined (next row's loads in
                         flight while the current row is collided), 0 = all rows of a
                         tile loaded first */
} flb_params;

typedef struct {
  int64_t step;          /* steps completed */
  int64_t nsite;
  double mass;           /* sum_x rho */
  double mass0;          /* mass when the populations were last set */
  double rho_eq;         /* mass0 / nsite: the global-noise density */
  double sum_f[7];       /* sum_x f_i (first Q used) */
  double sum_ff[28];     /* sum_x f_i f_j, i <= j, packed row-major upper triangle */
  double sum_rho2;       /* sum_x rho^2 */
  double sum_rho_pos;    /* sum_x max(rho, 0) */
  int64_t n_negative;    /* number of sites with rho < 0 */
  int64_t nonfinite;     /* number of non-finite populations */
} flb_moments_t;

/* flb_structure_factor modes */
enum {
  FLB_SK_SNAPSHOT = 0, /* S_out[n] = |rho(k_n)|^2 / N of the current state */
  FLB_SK_SAMPLE = 1,   /* add the current state's values to the accumulator (async) */
  FLB_SK_READ = 2,     /* S_out[n] = accumulated mean over samples */
  FLB_SK_RESET = 3     /* clear the accumulator and adopt kvec as its k-list */
};

/* Library ABI version (FLB_ABI_VERSION). */
int flb_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* flb_last_error(void);

/* The library's own equilibrium weights w (Q values) and moment basis m
 * (Q x Q, row a = moment, column i = population) for a model and theta
 * (0 -> default), paper Sec. II.  Host pointers; either may be NULL.
 * Returns Q (> 0) or FLB_EINVAL. */
int flb_lattice_constants(int32_t model, double theta, double* w, double* m);

/* Bytes of caller-provided device memory a lattice needs: pop_bytes for the
 * populations (two buffers of Q * N * precision bytes, one for the AA layout) and
 * work_bytes for the workspace (reductions, structure-factor marginals and
 * accumulators).  Validates the parameters. */
int flb_required_bytes(const flb_params* p, size_t* pop_bytes, size_t* work_bytes);

/* Create a lattice on the current HIP device.  d_pop (>= pop_bytes, 256-byte
 * aligned) holds the populations; d_work (>= work_bytes) the workspace, or
 * NULL to let the library allocate it.  hip_stream is a hipStream_t (NULL =
 * the null stream).  The populations are undefined until
 * flb_set_populations.  On success *out receives the handle. */
int flb_create(const flb_params* p, void* d_pop, size_t pop_bytes, void* d_work,
               size_t work_bytes, void* hip_stream, flb_lattice** out);

/* Load the canonical state (Q x N values of the lattice's precision; host or
 * device memory per src_on_device) and set the step counter to `step`.
 * Records mass0 and rho_eq (the global-noise density) from the new state.
 * Synchronises the handle's stream. */
int flb_set_populations(flb_lattice* h, const void* src, int src_on_device, int64_t step);

/* Copy the canonical state f_i(x, t) into dst (host or device memory).
 * Synchronises the handle's stream.  FLB_ESTATE while the lattice is a
 * member of a batch (as for every call that reads or writes its state). */
int flb_get_populations(flb_lattice* h, void* dst, int dst_on_device);

/* Advance nsteps >= 0 time steps: eq. (LB) with eq. (collision) at every
 * site.  Asynchronous on the handle's stream. */
int flb_step(flb_lattice* h, int64_t nsteps);

/* Check mode (off by default): with every > 0, flb_step stops after each
 * step t with t % every == 0 and after its last step, reads the state's
 * lattice sums back (synchronising the stream) and, if any population is
 * not finite, returns FLB_ENONFINITE with the lattice left at that step
 * (flb_last_error names the step and the count).  every = 0 turns it off. */
int flb_set_check(flb_lattice* h, int64_t every);

/* Steps completed so far. */
int flb_get_step(flb_lattice* h, int64_t* step);

/* Lattice sums of the current state in FP64 (Sec. IV: mass, <f_i>,
 * <f_i f_j>, plus the density variance, clamped mass, negative-density and
 * non-finite counts).  Deterministic order.  Synchronises the stream. */
int flb_moments(flb_lattice* h, flb_moments_t* out);

/* Density structure factor S(k) = |sum_x (rho(x) - rho_mean)
 * exp(-2 pi i sum_a k_a x_a / n_a)|^2 / N for k != 0 and M^2 / N for k = 0
 * (Sec. IV, Fourier test with the k = 0 correction).  kvec: nk x 3 host int32
 * wave numbers (k_x, k_y, k_z), any integers (taken modulo n_a); 1 <= nk <=
 * 1024.  Modes FLB_SK_*.  SNAPSHOT and READ write nk doubles to S_out (host)
 * and synchronise; SAMPLE and RESET are asynchronous and ignore S_out.
 * SAMPLE needs the same kvec as the last RESET.  Axis wave vectors (one
 * nonzero component) are evaluated from FP64 axis marginals; general ones
 * by a direct FP64 sum. */
int flb_structure_factor(flb_lattice* h, const int32_t* kvec, int32_t nk, int32_t mode,
                         double* S_out);

/* Sample the structure factor while stepping: from now on, flb_step
 * accumulates S(k) of the state before every step t with t % every == 0 into
 * the accumulator (read with FLB_SK_READ), for the k-list kvec (nk x 3, as
 * for flb_structure_factor).  Resets the accumulator.  When every wave vector
 * lies on an axis (or is zero) and the lattice is 2-D or 3-D, the sampled
 * step itself accumulates the density marginals (no extra pass over the
 * populations).  every = 0 stops sampling (kvec may be NULL). */
int flb_set_sampling(flb_lattice* h, int64_t every, const int32_t* kvec, int32_t nk);

/* Accumulate the lattice sums (as flb_moments) of the state before every
 * step t with t % every == 0 while stepping, on the device (no
 * synchronisation); every = 0 stops.  Starting resets the accumulator.  These
 * are the space-time sums of Sec. IV (means of f_i and of f_i f_j, eq. dijexp). */
int flb_set_moment_sampling(flb_lattice* h, int64_t every);

/* The accumulated sums (every field summed over the samples; step, nsite,
 * mass0 and rho_eq as for flb_moments) and the number of samples.
 * Synchronises the stream. */
int flb_sampled_moments(flb_lattice* h, flb_moments_t* sum, int64_t* nsamples);

/* ---- Population correlators (Sec. IV: Fourier test and equilibrium dynamics)
 *
 * With the paper's sign, f_i(k, t) = sum_x exp(+2 pi i k.x / L) f_i(x, t),
 * k.x / L = sum_a k_a x_a / L_a, and rho(k) = sum_i f_i(k).  While stepping,
 * at every step t with t % every == 0 (state before that step's collision)
 * the library adds
 *   S_ij(k)  += f_i(k, t) conj(f_j(k, t))         = f_i(k) f_j(-k), eqs. fkfk / FourierTest
 *   C(k, l)  += rho(k, t_s) conj(rho(k, t_{s+l}))  l = 0 .. nlag-1, eq. TimeCorrEqn
 * where t_s is the s-th sample since the last flb_set_correlation; the lag-l
 * sum has (nsamples - l) terms (none while nsamples <= l).  FP64 sums in a
 * fixed order.
 *
 * flb_set_correlation: kvec is nk x 3 int32 wave numbers (host memory,
 * components beyond the lattice's dimension ignored, any integer, taken
 * modulo the box), 1 <= nk <= 1024, 1 <= nlag <= 65536, nk * nlag <= 2^20.
 * The library allocates the buffers (device memory, about
 * 16 (nk (Q (Q + 1 + 256)) + 2 nk nlag) bytes) on this call, replaces any
 * earlier ones, zeroes the sums and synchronises the stream; they are freed
 * by flb_destroy.  every = 0 stops sampling and keeps the sums. */
int flb_set_correlation(flb_lattice* h, int64_t every, const int32_t* kvec, int32_t nk, int32_t nlag);

/* Copy the sums to host memory: sij is nk x Q x Q complex as (re, im)
 * doubles, index ((k Q + i) Q + j); ct is nk x nlag complex, index (k nlag + l).
 * Either may be NULL.  *nsamples = samples taken.  Synchronises the stream.
 * FLB_ESTATE if flb_set_correlation was never called. */
int flb_correlation(flb_lattice* h, double* sij, double* ct, int64_t* nsamples);

/* Fourier sums f_i(k) of the current state for the k-list of the last
 * flb_set_correlation, written to host memory as nk x Q complex (re, im)
 * doubles, index (k Q + i).  Synchronises the stream. */
int flb_fourier_amplitudes(flb_lattice* h, double* amp);

/* Temperature and rates varying in space (Sec. IV, non-homogeneous systems:
 * two domains of different theta, or of different current relaxation time
 * and hence diffusion constant).  region (host, n[0] n[1] n[2] bytes, x
 * fastest) gives every site's region r < nregions <= 16; theta[r] (each in
 * (0, 1/d); 0 is not allowed here) and omega[3 r .. 3 r + 2] (omega_j,
 * omega_n, omega_s as in flb_params, 0 for n and s meaning omega_j) set the
 * equilibrium weights, moment basis and rates with which that site collides
 * (eq. f0def with the local theta, eq. collision); streaming is unchanged.
 * The lattice's own theta and omega are then unused; seed, noise mode and
 * law still apply.  nregions = 0 returns to the uniform lattice (region may
 * be NULL).  Copies the map to library-allocated device memory (freed by
 * flb_destroy); synchronises.  Stepping uses a per-site kernel; a lattice
 * with regions cannot join a batch (FLB_EINVAL). */
int flb_set_regions(flb_lattice* h, const uint8_t* region, int32_t nregions, const double* theta,
                    const double* omega);

/* Density profile along one axis (Sec. IV, non-equilibrium dynamics: the
 * diffusion front is averaged over the other directions, and its variance
 * compared with eq. rhoth).  For every coordinate c along `axis` (0 = x,
 * 1 = y, 2 = z; below the model's dimension), sum_rho[c] and sum_rho2[c] are
 * the FP64 sums of rho and rho^2 over the sites with that coordinate, for
 * the current state, in a fixed order.  Host arrays of n[axis] doubles.
 * The library allocates its device buffers on the first call (freed by
 * flb_destroy).  Synchronises the stream. */
int flb_profile(flb_lattice* h, int32_t axis, double* sum_rho, double* sum_rho2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * density profile of flb_profile with no allocation and no
 * synchronisation.  d_sum_rho and d_sum_rho2 are device arrays of n[axis]
 * doubles, written asynchronously on the handle's stream (read them after
 * flb_sync or a later event); the values are those flb_profile returns.
 * The partial sums go to a static device array of
 * FLB_PROFILE_NOALLOC_MAX_BYTES that the library holds on every GPU it runs
 * on until the process ends, shared by all calls on that GPU: calls that
 * overlap on one GPU (on different streams or threads) race, and every call
 * overwrites what the previous one left there.  The partials need
 * 16 min(64, n[1] n[2]) n[0] bytes along axis 0 and 16 n[1] n[2] bytes along
 * axes 1 and 2; above the maximum the call returns FLB_EINVAL and launches
 * nothing.  The first call on a device looks up the array's address there. */
#define FLB_PROFILE_NOALLOC_MAX_BYTES (16u << 20)
int flb_profile_noalloc(flb_lattice* h, int32_t axis, double* d_sum_rho, double* d_sum_rho2);

/* Block until the handle's stream has finished. */
int flb_sync(flb_lattice* h);

/* Destroy the handle (and the workspace if the library allocated it).
 * Caller memory is never freed.  NULL is accepted. */
int flb_destroy(flb_lattice* h);

/* The device noise stream, for checking it against other implementations:
 * for sites site0 .. site0 + nsite - 1 of a `model` lattice at step `step`,
 * write the Philox words (uint32, nblock x 4 x nsite, nblock = 1 for D1Q3 and
 * D2Q5 and 2 for D3Q7) to d_words and the Q - 1 unit-variance variates of
 * `law` (Q - 1 x nsite, of `precision`) to d_vars.  Device pointers; either
 * may be NULL.  nsite <= 2^31 - 256.  Asynchronous on hip_stream. */
int flb_noise_sample(int32_t model, int32_t precision, int32_t law, uint64_t seed,
                     int64_t step, int64_t site0, int64_t nsite, void* d_words, void* d_vars,
                     void* hip_stream);

/* The Gaussian map of the noise stream on given words, for checking it
 * exhaustively: for j < n, with u_a = (2 (r_a >> 9) + 1) 2^-24 the uniform of
 * word r_a = d_words[a * n + j] (a = 0, 1), write the Box-Muller pair
 *   d_z[j] = sqrt(-2 ln u_0) cos(2 pi u_1),  d_z[n + j] = sqrt(-2 ln u_0) sin(2 pi u_1)
 * in `precision` (4 or 8), computed exactly as the step kernels compute it
 * (the paper's noise is Gaussian in the fluctuating-hydrodynamics limit;
 * Sec. IV discusses the flat law it replaces).  d_words: 2 x n uint32,
 * d_z: 2 x n reals, device pointers; n <= 2^31 - 256.  Asynchronous on
 * hip_stream. */
int flb_gauss_map(int32_t precision, const void* d_words, int64_t n, void* d_z, void* hip_stream);

/* ---- batched ensembles (one launch advances many lattices) ---------------
 * A batch holds references to lattices created with flb_create (all float32
 * or all float64, all on one device).  flb_batch_step advances every member
 * by nsteps with results bit-identical to flb_step on each member alone.
 * The lattices that live in global memory are advanced by work-list
 * launches (one workgroup per work item by default: a tile of one member,
 * one launch per step, or per two steps for D2Q5 members at depth 2; with
 * `workers` > 0 a persistent grid strides over the items), and small D1Q3
 * lattices run whole chunks of steps inside one workgroup's LDS, in a launch
 * of their own on a second stream of the batch (forked from the batch's
 * stream at the chunk start and joined before the chunk's step advance, so
 * it overlaps the other members' passes; in a captured graph, a parallel
 * branch).  Chunks of `chunk` steps are captured once into a HIP graph and
 * replayed.  Members may be admitted and retired between calls; flb_batch_sync
 * (or work ordered after it on the batch's stream) sees every member done. */
typedef struct {
  int32_t chunk;        /* steps per graph (>= 1); 0 -> 16 */
  int32_t use_graph;    /* 1 = capture chunks in a HIP graph, 0 = eager launches */
  int32_t lds_max_bytes;/* largest D1Q3 state run LDS-resident; 0 -> 64 KiB, -1 = never */
  int32_t workers;      /* 0: one workgroup per work item; > 0: a persistent grid of
                           this many workgroups striding over the items */
  int32_t item_rows;    /* row tiling: rows per work item, 2, 4, 8, 16; 0 -> 2 */
  int32_t tiling;       /* work items of the HBM kernel: 0 = 512 consecutive sites of a
                           member (lanes filled across row ends), 1 = 256 x item_rows
                           row tiles */
  int32_t depth;        /* temporal blocking of D2Q5 members in HBM: 2 = two steps per
                           pass (width x 8 tiles with a one-site halo; a chunk of odd
                           length ends with one single step), 1 = one step per pass;
                           0 -> 2.  Results are bit-identical either way. */
  int32_t width;        /* depth 2: columns per two-step tile, 64, 128 or 256 (narrower
                           tiles leave fewer lanes idle on uneven widths, at more halo
                           work); 0 -> 256.  Bit-identical either way. */
  void* hip_stream;     /* stream of all batch work (NULL = a stream of its own) */
} flb_batch_opts;

int flb_batch_create(const flb_batch_opts* opts, flb_batch** out);
/* Add a lattice; it must not be stepped on its own while it is a member.
 * FLB_ESTATE if it is in a batch already or samples statistics while
 * stepping (a batch step takes none: stop flb_set_sampling,
 * flb_set_moment_sampling and flb_set_correlation first); FLB_EINVAL for a
 * lattice with regions, of another precision or on another device. */
int flb_batch_admit(flb_batch* b, flb_lattice* h);
/* Remove a lattice (its state stays valid and can be read or stepped alone). */
int flb_batch_retire(flb_batch* b, flb_lattice* h);
/* Advance every member by nsteps.  Asynchronous on the batch stream. */
int flb_batch_step(flb_batch* b, int64_t nsteps);
int flb_batch_size(flb_batch* b, int32_t* n);
int flb_batch_sync(flb_batch* b);
int flb_batch_destroy(flb_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* FLB_H */
