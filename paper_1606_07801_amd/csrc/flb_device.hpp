// Device-side building blocks of the fluctuating lattice Boltzmann step for
// gfx950: the Philox noise stream, the uniform and Gaussian mappings, and the
// per-site collision of the D1Q3 / D2Q5 / D3Q7 models.
//
// The collision follows eq. (collision) of Wagner & Strand (arXiv:1606.07801)
// in moment space (Sec. II): the density rho = M^0 is conserved, every other
// moment relaxes with its class rate omega_a = 1/tau^a towards its
// equilibrium value 0 and receives noise of variance
// rho_n (2 tau^a - 1)/(tau^a)^2 = rho_n omega_a (2 - omega_a)
// (eqs. xilocal / xiglobal), with rho_n the local density clamped at zero
// (Sec. IV) or the global mean density.  The post-collision populations are
// formed in the equivalent increment form
//   f_i* = f_i + sum_{a>=1} w_i m_i^a (xi^a - omega_a M^a),   i >= 1,
//   f_0* = rho - sum_{i>=1} f_i*,
// which uses f_i = sum_a w_i m_i^a M^a (completeness of the basis) and makes
// each site's post-collision sum round to rho (the density and the residual
// are formed in double for float populations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flb_tables.hpp"

// No implicit multiply-add contraction in the kernels: every kernel variant
// (and every context a collision is inlined into) must round each site's
// arithmetic identically, and which mul/add pairs the compiler fuses depends
// on the surrounding code.  Fused operations are written out where wanted.
#pragma clang fp contract(off)

namespace flb {

enum NoiseMode : int { kNoiseLocal = 0, kNoiseGlobal = 1, kNoiseOff = 2 };
enum NoiseLaw : int { kLawGauss = 0, kLawUniform = 1 };
// Noise plan of a kernel instance: read from the parameters at run time, or
// fixed at compile time to local noise with the Gaussian law (the default
// configuration), which drops the run-time selections from the collision.
// Both give the same arithmetic, so the same bits.
enum NoisePlan : int { kPlanRuntime = 0, kPlanLocalGauss = 1 };

// Everything a step kernel needs about one lattice, passed by value.
template <typename T>
struct KParams {
  int64_t nx, ny, nz, n;   // box and site count
  T rho_eq;                // density of the global noise mode
  // The collision's constants, folded with the back-transform weight
  // w1 = theta/2 of the moving populations.  Basis scales (Sec. II):
  // a = 1/sqrt(theta) (currents), b = 1/sqrt(2 theta) and e = 1/sqrt(6 theta)
  // (traceless moments), c1 = sqrt((1 - d theta)/(d theta)) on the moving
  // populations and -c0 = -sqrt(d theta/(1 - d theta)) on f_0 (trace).
  // Rates om per class (j: currents, n: traceless, s: trace) and noise
  // factors sq = sqrt(om (2 - om)) (times sqrt(3) for the flat law).
  T nA, nB, nC, nE;        // noise scales w1 a sq_j, w1 b sq_n, w1 c1 sq_s, w1 e sq_n
  T kj, kn, ke, ks, ks0;   // w1 a^2 om_j, w1 b^2 om_n, w1 e^2 om_n, w1 c1^2 om_s, w1 c1 c0 om_s
  uint32_t k0, k1;         // Philox key (seed low / high word)
  int32_t noise;           // NoiseMode
  int32_t law;             // NoiseLaw
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Ten rounds of two 32x32->64-bit
// products on counter words 0 and 2; the high halves are mixed with words 1
// and 3 and the key, the key advances by two Weyl increments between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    // three-input XOR in one instruction (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
}

// u = (2 (r >> 9) + 1) 2^-24: an odd multiple of 2^-24, exact in float.
template <typename T>
__device__ __forceinline__ T word_to_uniform(uint32_t r) {
  return (T)((r >> 9) * 2u + 1u) * (T)5.9604644775390625e-08;  // 2^-24
}

// The same value in two instructions: one funnel shift places r's top 23
// bits under the exponent field of 1.0, giving x = 1 + (r >> 9) 2^-23 in
// [1, 2), and x - (1 - 2^-24) = (2 (r >> 9) + 1) 2^-24 is representable, so
// the subtraction is exact.
template <>
__device__ __forceinline__ float word_to_uniform<float>(uint32_t r) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
}

// Box-Muller pair from two Philox words: with u0, u1 their uniforms,
// z0 = R cos(2 pi u1), z1 = R sin(2 pi u1), R = sqrt(-2 ln u0).
//
// Float: the hardware instructions are used directly.  u0 and u1 lie in
// [2^-24, 1), where v_log_f32 (base-2 logarithm) and v_sqrt_f32 are within
// about one ulp and v_sin_f32 / v_cos_f32, which take their argument in
// revolutions (sin 2 pi x), are within 1.3e-7 absolute (measured against
// FP64 references over all odd multiples of 2^-25 in (0, 1)).  This keeps the
// step's ALU cost below its memory cost.
__device__ __forceinline__ void gauss_pair(uint32_t r0, uint32_t r1, float& z0, float& z1) {
  const float u0 = word_to_uniform<float>(r0), u1 = word_to_uniform<float>(r1);
  const float R = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u0));  // -2 ln 2
  z0 = R * __builtin_amdgcn_cosf(u1);
  z1 = R * __builtin_amdgcn_sinf(u1);
}

// Double: both functions take u = n 2^-24 with n odd in [1, 2^24) as the
// integer n, which reduces their arguments exactly; a short series around a
// tabulated breakpoint (flb_tables.hpp) finishes each.  Errors are a few ulp
// of the result (the exhaustive GPU test over all 2^23 values of each
// argument bounds them).

// ln(n 2^-24), table-driven in the manner of Tang (ACM TOMS 16(4), 1990):
// n 2^-24 = 2^-k m with m in [1/2, 1); the seven bits after n's leading one
// select c_i = (257 + 2 i)/512, the middle of m's subinterval, and
// ln(n 2^-24) = ln c_i + log1p(v) - k ln 2 with v = (m - c_i)/c_i, |v| <= 2^-8.
// The last subinterval uses its right end c_127 = 1 (ln c = 0) and the top
// binade (k = 0) has no ln 2 term, so values near u = 1 keep their relative
// accuracy.
__device__ __forceinline__ double ln_odd24(uint32_t n) {
  const uint32_t k = (uint32_t)__builtin_clz(n) - 8u;
  const uint32_t m = n << k;                                              // m 2^24, leading one at bit 23
  const uint32_t i = (m >> 16) & (uint32_t)(kBmTab - 1);
  const uint32_t c = i == (uint32_t)(kBmTab - 1) ? 512u : 257u + 2u * i;   // 512 c_i
  const int32_t dm = (int32_t)m - (int32_t)(c << 15);                     // (m - c_i) 2^24, |dm| <= 2^16
  const double2 t = kLnTab[i];
  const double v = (double)dm * t.x;
  // log1p(v) = v - v^2/2 + v^3/3 - ... - v^8/8; the rest is below 2^-75
  double q = fma(v, -0.125, 1.0 / 7.0);
  q = fma(v, q, -1.0 / 6.0);
  q = fma(v, q, 0.2);
  q = fma(v, q, -0.25);
  q = fma(v, q, 1.0 / 3.0);
  q = fma(v, q, -0.5);
  const double lp = fma(v * v, q, v);
  return fma(-(double)k, 0.69314718055994530942, t.y + lp);
}

// sin and cos of 2 pi n 2^-24: the top two bits of n give the quadrant, the
// next seven the breakpoint phi_i = 2 pi (2 i + 1)/1024 and the last fifteen
// the offset d = 2 pi (low15 - 2^14) 2^-24, |d| <= pi 2^-9.
__device__ __forceinline__ void sincos_odd24(uint32_t n, double& s, double& c) {
  const uint32_t quad = n >> 22;
  const uint32_t i = (n >> 15) & (uint32_t)(kBmTab - 1);
  const int32_t b = (int32_t)(n & 0x7FFFu) - 0x4000;
  const double d = (double)b * 0x1.921fb54442d18p-22;                    // 2 pi 2^-24
  const double d2 = d * d;
  const double sd = fma(d * d2, fma(d2, 1.0 / 120.0, -1.0 / 6.0), d);     // sin d; next term < 2^-63
  const double cm = d2 * fma(d2, fma(d2, -1.0 / 720.0, 1.0 / 24.0), -0.5);  // cos d - 1; next < 2^-74
  const double2 t = kScTab[i];
  const double S = fma(t.x, cm, fma(t.y, sd, t.x));                        // sin(phi_i + d)
  const double C = fma(t.y, cm, fma(-t.x, sd, t.y));                       // cos(phi_i + d)
  // quarter turns: (sin, cos) -> (cos, -sin) per quadrant
  const double sv = (quad & 1u) ? C : S, cv = (quad & 1u) ? S : C;
  s = (quad & 2u) ? -sv : sv;
  c = ((quad + 1u) & 2u) ? -cv : cv;
}

// Square root of a in [2^-24, 64]: the reciprocal square root estimate
// refined by Goldschmidt iterations -- the operations of the compiler's
// general sqrt in its order, so the same result, without its rescaling of
// arguments below 2^-767 and its special cases (zero, infinity), which this
// range never meets.
__device__ __forceinline__ double sqrt_mid(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, hh = y * 0.5;
  const double r = fma(-hh, g, 0.5);
  g = fma(g, r, g);
  hh = fma(hh, r, hh);
  double d = fma(-g, g, a);
  g = fma(d, hh, g);
  d = fma(-g, g, a);
  return fma(d, hh, g);
}

__device__ __forceinline__ void gauss_pair(uint32_t r0, uint32_t r1, double& z0, double& z1) {
  // -2 ln u lies in [1.19e-7, 33.3] for the uniforms of the stream
  const double R = sqrt_mid(-2.0 * ln_odd24(((r0 >> 9) << 1) | 1u));
  double s, c;
  sincos_odd24(((r1 >> 9) << 1) | 1u, s, c);
  z0 = R * c;
  z1 = R * s;
}

// Variates for one Philox block: four unit-variance values.
template <typename T, int NP = kPlanRuntime>
__device__ __forceinline__ void draw4(const KParams<T>& P, uint64_t site, uint32_t step,
                                      uint32_t block, T (&z)[4]) {
  uint32_t c0 = (uint32_t)site, c1 = (uint32_t)(site >> 32), c2 = step, c3 = block;
  philox4x32_10(c0, c1, c2, c3, P.k0, P.k1);
  if (NP == kPlanLocalGauss || P.law == kLawGauss) {
    gauss_pair(c0, c1, z[0], z[1]);
    gauss_pair(c2, c3, z[2], z[3]);
  } else {  // flat law on (-1, 1); the sqrt(3) lives in sq_*
    z[0] = (T)2 * word_to_uniform<T>(c0) - (T)1;
    z[1] = (T)2 * word_to_uniform<T>(c1) - (T)1;
    z[2] = (T)2 * word_to_uniform<T>(c2) - (T)1;
    z[3] = (T)2 * word_to_uniform<T>(c3) - (T)1;
  }
}

// Noise terms of one Philox block for the collision: X_k = S_k sqrt(rn) z_k
// with z_k the block's k-th unit variate (Gaussian: z_0, z_1 from the pair
// (c0, c1) as cos and sin, z_2, z_3 from (c2, c3); flat: 2 u_k - 1), S_k the
// folded scale of the moment that takes it and rn the density of the noise
// amplitude.  c holds the block's Philox output words.
//
// Float, Gaussian law: the amplitude enters the Box-Muller radius,
// sqrt(rn) sqrt(-2 ln u0) = sqrt(rn (-2 ln 2) log2 u0), one root per pair
// instead of two roots and a product (the same value up to rounding).
__device__ __forceinline__ void scaled_pair(uint32_t r0, uint32_t r1, float rk, float Sa, float Sb,
                                            float& Xa, float& Xb) {
  const float u0 = word_to_uniform<float>(r0), u1 = word_to_uniform<float>(r1);
  const float R = __builtin_amdgcn_sqrtf(rk * __builtin_amdgcn_logf(u0));  // rk = -2 ln 2 rn
  Xa = (Sa * R) * __builtin_amdgcn_cosf(u1);
  Xb = (Sb * R) * __builtin_amdgcn_sinf(u1);
}
__device__ __forceinline__ void scaled_pair(uint32_t r0, uint32_t r1, double sr, double Sa, double Sb,
                                            double& Xa, double& Xb) {
  double z0, z1;
  gauss_pair(r0, r1, z0, z1);  // sr = sqrt(rn)
  Xa = (Sa * sr) * z0;
  Xb = (Sb * sr) * z1;
}
__device__ __forceinline__ float amp_root(float rn) { return __builtin_amdgcn_sqrtf(rn); }
__device__ __forceinline__ double amp_root(double rn) { return sqrt(rn); }

template <typename T, int NP = kPlanRuntime>
__device__ __forceinline__ void noise_terms(const KParams<T>& P, const uint32_t (&c)[4], T rn, T Sa, T Sb,
                                            T Sc, T Sd, T (&X)[4]) {
  if (NP == kPlanLocalGauss || P.law == kLawGauss) {
    if constexpr (sizeof(T) == 4) {
      const T rk = rn * (T)-1.38629436111989061;  // -2 ln 2
      scaled_pair(c[0], c[1], rk, Sa, Sb, X[0], X[1]);
      scaled_pair(c[2], c[3], rk, Sc, Sd, X[2], X[3]);
    } else {
      const T sr = amp_root(rn);
      scaled_pair(c[0], c[1], sr, Sa, Sb, X[0], X[1]);
      scaled_pair(c[2], c[3], sr, Sc, Sd, X[2], X[3]);
    }
  } else {  // flat law on (-1, 1); the sqrt(3) lives in the scales
    const T sr = amp_root(rn);
    X[0] = (Sa * sr) * ((T)2 * word_to_uniform<T>(c[0]) - (T)1);
    X[1] = (Sb * sr) * ((T)2 * word_to_uniform<T>(c[1]) - (T)1);
    X[2] = (Sc * sr) * ((T)2 * word_to_uniform<T>(c[2]) - (T)1);
    X[3] = (Sd * sr) * ((T)2 * word_to_uniform<T>(c[3]) - (T)1);
  }
}

// Philox output words of block `block` at (site, step).
template <typename T>
__device__ __forceinline__ void noise_words(const KParams<T>& P, uint64_t site, uint32_t step, uint32_t block,
                                            uint32_t (&c)[4]) {
  c[0] = (uint32_t)site;
  c[1] = (uint32_t)(site >> 32);
  c[2] = step;
  c[3] = block;
  philox4x32_10(c[0], c[1], c[2], c[3], P.k0, P.k1);
}

// Density of the noise amplitude: the local density clamped at zero, or the
// global mean density.
template <typename T, int NP>
__device__ __forceinline__ T noise_density(const KParams<T>& P, T rho) {
  if (NP == kPlanLocalGauss || P.noise == kNoiseLocal) return rho > (T)0 ? rho : (T)0;
  return P.rho_eq;
}

// Site density sum_i f_i in index order, in double.  For float populations
// this is the correctly rounded sum of the stored values, so that the clamp
// at zero of the noise amplitude (where sqrt(rho) is not Lipschitz) is
// decided on the exact density.
template <typename T, int Q>
__device__ __forceinline__ double density_sum(const T (&f)[Q]) {
  double r = (double)f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) r += (double)f[i];
  return r;
}

// Rest population after the collision, f_0* = rho - sum_{i>=1} f_i*.  For
// float populations the residual is formed in double and rounded once, so
// the stored populations of a site sum to rho within half an ulp of f_0*
// without a systematic bias (exact mass conservation up to that rounding).
template <int N>
__device__ __forceinline__ float rest_of(double rho, const float (&fi)[N]) {
  double s = (double)fi[0];
#pragma unroll
  for (int i = 1; i < N; ++i) s += (double)fi[i];
  return (float)(rho - s);
}
template <int N>
__device__ __forceinline__ double rest_of(double rho, const double (&fi)[N]) {
  double s = fi[0];
#pragma unroll
  for (int i = 1; i < N; ++i) s += fi[i];
  return rho - s;
}

// ---------------------------------------------------------------------------
// Per-site collision.  f holds the pre-collision populations of one site in
// the velocity order 0, +x, -x, +y, -y, +z, -z and is overwritten with the
// post-collision populations.
template <int D, typename T, int NP = kPlanRuntime>
struct Collide;

// In every model the moving populations change by
//   f_i* = f_i + w1 sum_{a >= 1} m_i^a (xi^a - om_a M^a),
// written with the folded products of KParams.  A moment M^a = m S^a, with
// m its basis scale (a, b, e or c1) and S^a an integer combination of the
// moving populations (f_1 - f_2, f_1 + f_2 - f_3 - f_4, ...), contributes
// w1 m (xi^a - om_a M^a) = X^a - k_a S^a with k_a = w1 m^2 om_a and X^a its
// noise term (noise_terms); the trace moment's entry -c0 on f_0 adds
// ks0 f_0.  The rest population takes the residual (rest_of).
template <typename T, int NP>
struct Collide<1, T, NP> {
  static constexpr int Q = 3;
  __device__ __forceinline__ static void run(T (&f)[3], const KParams<T>& P, uint64_t site,
                                             uint32_t step) {
    constexpr bool fixed = NP == kPlanLocalGauss;
    const bool on = fixed || P.noise != kNoiseOff;
    // the words depend on (site, step) only: drawn first, they overlap the
    // loads of f still in flight
    uint32_t c[4];
    if (on) noise_words(P, site, step, 0u, c);
    const double rho_d = density_sum(f);
    const T rho = (T)rho_d;
    T X[4] = {0, 0, 0, 0};
    if (on) noise_terms<T, NP>(P, c, noise_density<T, NP>(P, rho), P.nA, P.nC, P.nC, P.nC, X);
    // current (j) and trace (s) moments
    const T Cj = fma(-P.kj, f[1] - f[2], X[0]);
    const T Cs = fma(-P.ks, f[1] + f[2], fma(P.ks0, f[0], X[1]));
    const T f1 = f[1] + (Cs + Cj);
    const T f2 = f[2] + (Cs - Cj);
    f[1] = f1;
    f[2] = f2;
    const T mv[2] = {f1, f2};
    f[0] = rest_of(rho_d, mv);
  }
};

template <typename T, int NP>
struct Collide<2, T, NP> {
  static constexpr int Q = 5;
  __device__ __forceinline__ static void run(T (&f)[5], const KParams<T>& P, uint64_t site,
                                             uint32_t step) {
    constexpr bool fixed = NP == kPlanLocalGauss;
    const bool on = fixed || P.noise != kNoiseOff;
    uint32_t c[4];
    if (on) noise_words(P, site, step, 0u, c);  // independent of f: overlaps its loads
    const double rho_d = density_sum(f);
    const T rho = (T)rho_d;
    T X[4] = {0, 0, 0, 0};
    if (on) noise_terms<T, NP>(P, c, noise_density<T, NP>(P, rho), P.nA, P.nA, P.nB, P.nC, X);
    const T sx = f[1] + f[2], sy = f[3] + f[4];
    const T Cx = fma(-P.kj, f[1] - f[2], X[0]);                // currents
    const T Cy = fma(-P.kj, f[3] - f[4], X[1]);
    const T Pn = fma(-P.kn, sx - sy, X[2]);                    // traceless
    const T Ps = fma(-P.ks, sx + sy, fma(P.ks0, f[0], X[3]));  // trace
    const T Hx = Pn + Ps, Hy = Ps - Pn;
    const T f1 = f[1] + (Hx + Cx);
    const T f2 = f[2] + (Hx - Cx);
    const T f3 = f[3] + (Hy + Cy);
    const T f4 = f[4] + (Hy - Cy);
    f[1] = f1;
    f[2] = f2;
    f[3] = f3;
    f[4] = f4;
    const T mv[4] = {f1, f2, f3, f4};
    f[0] = rest_of(rho_d, mv);
  }
};

template <typename T, int NP>
struct Collide<3, T, NP> {
  static constexpr int Q = 7;
  __device__ __forceinline__ static void run(T (&f)[7], const KParams<T>& P, uint64_t site,
                                             uint32_t step) {
    constexpr bool fixed = NP == kPlanLocalGauss;
    const bool on = fixed || P.noise != kNoiseOff;
    uint32_t c[4], cc[4];
    if (on) {  // independent of f: overlaps its loads
      noise_words(P, site, step, 0u, c);
      noise_words(P, site, step, 1u, cc);
    }
    const double rho_d = density_sum(f);
    const T rho = (T)rho_d;
    T X[4] = {0, 0, 0, 0}, XX[4] = {0, 0, 0, 0};
    if (on) {
      const T rn = noise_density<T, NP>(P, rho);
      noise_terms<T, NP>(P, c, rn, P.nA, P.nA, P.nA, P.nB, X);
      noise_terms<T, NP>(P, cc, rn, P.nE, P.nC, P.nC, P.nC, XX);
    }
    const T sx = f[1] + f[2], sy = f[3] + f[4], sz = f[5] + f[6];
    const T Cx = fma(-P.kj, f[1] - f[2], X[0]);                      // currents
    const T Cy = fma(-P.kj, f[3] - f[4], X[1]);
    const T Cz = fma(-P.kj, f[5] - f[6], X[2]);
    const T P1 = fma(-P.kn, sx - sy, X[3]);                          // traceless
    const T P2 = fma(-P.ke, (sx + sy) - (T)2 * sz, XX[0]);
    const T Ps = fma(-P.ks, (sx + sy) + sz, fma(P.ks0, f[0], XX[1]));  // trace
    const T Hx = (P1 + P2) + Ps;
    const T Hy = (P2 - P1) + Ps;
    const T Hz = Ps - (T)2 * P2;
    const T f1 = f[1] + (Hx + Cx);
    const T f2 = f[2] + (Hx - Cx);
    const T f3 = f[3] + (Hy + Cy);
    const T f4 = f[4] + (Hy - Cy);
    const T f5 = f[5] + (Hz + Cz);
    const T f6 = f[6] + (Hz - Cz);
    f[1] = f1;
    f[2] = f2;
    f[3] = f3;
    f[4] = f4;
    f[5] = f5;
    f[6] = f6;
    const T mv[6] = {f1, f2, f3, f4, f5, f6};
    f[0] = rest_of(rho_d, mv);
  }
};

}  // namespace flb
