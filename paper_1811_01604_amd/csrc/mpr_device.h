// Device-side building blocks of the MPR checkerboard sweep for gfx950.
//
// Storage: each chain keeps its grid as two "half-grids", one per
// checkerboard colour c = (x + y) & 1.  Row y of colour c holds the sites
// x = 2h + s, s = (y + c) & 1, at index y * S + h (S = padded half-row
// stride, even).  A site's four neighbours all have the other colour: left
// and right at h + s - 1 and h + s of the same row, up and down at h of rows
// y - 1 and y + 1.  Sampled (fixed) sites carry their angle with the sign
// bit set, so the mask costs no extra bytes; |v| is the angle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpr {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// Chain phases of the per-chain state machine (Algorithm 2).
enum : int32_t { PH_RELAX = 0, PH_EQ = 1, PH_DONE = 2, PH_TABLE = 3 };

// Per-site diagnostic flags.
enum : uint32_t { F_KEPT = 1, F_ACCEPTED = 2, F_WRAPPED = 4, F_UPDATED = 8, F_FP64 = 16 };

constexpr int kMaxFit = 64;

// Static description of one chain (one image x one realization).
struct ChainDesc {
    // In double-precision chains h, acc and m2 point to doubles.
    float *h[2];          // colour half-grids, ny * S each
    float *acc[2];        // equilibrium sums (K > 1), or null
    float *m2[2];         // sums of squared deviations from the running mean
                          // of the equilibrium states (K > 1, spread wanted), or null
    float *h2[2];         // second pair of half-grids (single-precision chains): the
                          // fused tile sweep reads h and writes h2, and the pointers
                          // are swapped after the sweep, so h always holds the state
    int32_t nx, ny, S;    // grid size and half-row stride
    uint32_t image_id;    // Philox counter word 3
    uint32_t chain;       // Philox counter word 2
    int32_t pad;
    int64_t P;            // number of gap sites
    int64_t ngp;          // number of bonds
};

// Mutable per-chain state; the sweep kernels read the parameters and add
// to the accumulators, the control kernel does the rest.
struct ChainState {
    int32_t phase;
    uint32_t sweep;        // sweep counter t (Philox counter word 1)
    float inv_T;           // 1 / T
    float dscale;          // 2 pi q / a: proposal half-width scale in q*phi units
    double T;
    double a_cur;          // a used by the next sweep
    double a_relax;        // a of the relaxation rule
    unsigned long long e_fx;   // sum over bonds of 1 - cos(q (phi_i - phi_j)), units of 2^-27
    unsigned long long acc;    // accepted proposals in the current sweep
    double k;              // last energy slope
    double A_last;
    double e_sum;          // table mode: sum of (1 + e) over measured sweeps
    int32_t relax_sweeps;
    int32_t not_converged;
    int32_t eq_left;
    float inv_k;           // 1 / k and 1 / (k - 1) for the k-th equilibrium state
    float inv_km1;         // of the next sweep (k = 1: 1 and 0)
    int32_t swapped;       // 1 while the chain's h and h2 are exchanged (fused sweeps
                           // toggle it), so that a resumed run can rebuild its descriptor
    double inv_k_d;        // the same in double (double-precision chains)
    double inv_km1_d;
    double ring[kMaxFit];  // last n_fit values of 1 + e
};

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplications and a Weyl key schedule.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    // round 1 in plain xors: counter words 1-3 are usually uniform over a
    // launch, so the compiler keeps their part on the scalar unit
    {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    // rounds 2-10: each three-way xor is one v_bitop3_b32 (truth table 0x96)
#pragma unroll
    for (int i = 1; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        U4 n;
        n.x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
        n.y = (uint32_t)p1;
        n.z = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24-bit dyadic uniform in [0, 1), exact in float and double.
__device__ __forceinline__ float unit24(uint32_t w)
{
    return (float)(w >> 8) * 5.9604644775390625e-08f;
}

// Set bits of the wave mask m in the lanes below this one (a lane's rank
// among the lanes whose bit is set).
__device__ __forceinline__ int rank_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ------------------------------------------------------------- sign bit
__device__ __forceinline__ bool is_fixed(float v) { return (__float_as_uint(v) >> 31) != 0u; }
// fabsf clears the sign bit (also of -0.0) and folds into instruction modifiers
__device__ __forceinline__ float angle_of(float v) { return fabsf(v); }
__device__ __forceinline__ float mark_fixed(float a) { return __uint_as_float(__float_as_uint(a) | 0x80000000u); }

// Sweep parameters shared by a launch.
struct SweepConsts {
    double q64;                 // coupling exponent (the single-precision kernels assume 1/2)
    uint32_t seed_lo, seed_hi;  // Philox key
};

// ------------------------------------------------- double-precision path
// Result of one site's update.
struct SiteOut {
    float phi;       // new angle
    float e_bonds;   // sum over the site's bonds of 1 - cos(q (phi_new - phi_j))
    float e_before;  // the same sum before the update
    uint32_t flags;
    bool accepted;   // flags & F_ACCEPTED, kept apart so that unused flag bits fold away
};

// atan2 in double precision in few registers (the library routine needs
// 60): octant reduction to t = min/max in [0, 1]; t > tan(pi/12) maps to
// t' = (sqrt3 t - 1) / (t + sqrt3) with atan t = pi/6 + atan t'; atan on
// |t'| <= tan(pi/12) by its Taylor series to degree 29 (truncation below
// 1e-19 relative).  Within 4 ulp of the correctly rounded value on 2e6
// random and boundary arguments.  (0, 0) is excluded by the caller.
__device__ __forceinline__ double atan2_fp64(double y, double x)
{
#pragma clang fp contract(off)
    const double ax = fabs(x), ay = fabs(y);
    const bool swap = ay > ax;
    const double t = swap ? ax / ay : ay / ax;
    const bool big = t > 0.26794919243112270;
    const double tr = big ? (t * 1.7320508075688772 - 1.0) / (t + 1.7320508075688772) : t;
    const double z = tr * tr;
    double p = -1.0 / 29.0;
#pragma unroll
    for (int k = 13; k >= 1; --k) p = p * z + ((k & 1) ? -1.0 : 1.0) / (double)(2 * k + 1);
    double a = (big ? 0.52359877559829887 : 0.0) + (tr + tr * (z * p));
    if (swap) a = 1.5707963267948966 - a;
    if (x < 0.0) a = 3.1415926535897931 - a;
    return y < 0.0 ? -a : a;
}

// ------------------------------------------------ single-precision math
// Minimax polynomials fitted for this library (least squares with Lawson
// reweighting on Chebyshev nodes):
//   sin x, |x| <= pi/2: x (1 + x^2 P(x^2)), relative error 5e-9;
//   cos x, |x| <= pi/2: Q(x^2) of degree 8, absolute error 5e-8;
//   atan t, |t| <= 1:   t (1 + t^2 R(t^2)), relative error 1.5e-8.
__device__ __forceinline__ float sin_poly(float x)
{
    const float x2 = x * x;
    float p = fmaf(x2, 2.601902224e-06f, -1.980741799e-04f);
    p = fmaf(p, x2, 8.333025500e-03f);
    p = fmaf(p, x2, -1.666665673e-01f);
    return fmaf(p * x2, x, x);
}

// The same polynomials taking a full angle d and returning 2 sin(d/2) and
// cos(d/2) from d2 = d * d: every coefficient is the |x| <= pi/2 one divided
// by a power of two (cosine: 9.999999404e-01, -4.999990463e-01,
// 4.166358337e-02, -1.385370386e-03, 2.315392157e-05 for x^0 .. x^8), so the
// results equal 2 sin_poly(d/2) and the cosine polynomial at d/2 bit for bit,
// without the halving and doubling.
__device__ __forceinline__ float sin2_half_poly(float d, float d2)
{
    float p = fmaf(d2, 2.601902224e-06f / 256.0f, -1.980741799e-04f / 64.0f);
    p = fmaf(p, d2, 8.333025500e-03f / 16.0f);
    p = fmaf(p, d2, -1.666665673e-01f / 4.0f);
    return fmaf(p * d2, d, d);
}

__device__ __forceinline__ float cos_half_poly(float d2)
{
    float p = fmaf(d2, 2.315392157e-05f / 256.0f, -1.385370386e-03f / 64.0f);
    p = fmaf(p, d2, 4.166358337e-02f / 16.0f);
    p = fmaf(p, d2, -4.999990463e-01f / 4.0f);
    return fmaf(p, d2, 9.999999404e-01f);
}

// atan2(y, x) in (-pi, pi]: octant reduction to t = min/max in [0, 1].
__device__ __forceinline__ float atan2_poly(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float t2 = t * t;
    float p = fmaf(t2, 2.849767916e-03f, -1.606814750e-02f);
    p = fmaf(p, t2, 4.269074649e-02f);
    p = fmaf(p, t2, -7.504229993e-02f);
    p = fmaf(p, t2, 1.064090431e-01f);
    p = fmaf(p, t2, -1.420363635e-01f);
    p = fmaf(p, t2, 1.999261826e-01f);
    p = fmaf(p, t2, -3.333307207e-01f);
    float a = fmaf(p * t2, t, t);
    a = ay > ax ? 1.57079637f - a : a;
    a = x < 0.0f ? 3.14159274f - a : a;
    return y < 0.0f ? -a : a;
}

// Algorithm 1 for one site, q = 1/2, in single precision (computed for
// sampled sites too; the caller discards those results).
//   phi        current angle; th = phi / 2
//   n0..n3     neighbour angles (left, right, up, down), valid bits in `valid`
//   u, r       the site's two uniforms
// With D_j = th - th_j (exact in float when the angles are close), the
// local field relative to the spin is A = sum cos D_j = |h| cos(th - Psi)
// and B = sum sin D_j = |h| sin(th - Psi), computed from sin and cos of D_j/2
// so that both stay accurate for nearly aligned spins.  Over-relaxation:
// th' = th + 2 d with d = Psi - th = atan2(-B, A), kept if th' leaves
// [0, pi).  With Bs = |h| sin(th' - Psi) (= -B, or B when kept) and the
// proposal th'' = th' + delta, the energy change is
//   H(th'') - H(th') = 2 A sin^2(delta/2) + Bs sin(delta)        (no wrap)
//                    = 2 A cos^2(delta/2) - Bs sin(delta)        (wrapped by pi)
// with no cancellation.  The reflection keeps the energy, so the site's
// bond energy afterwards is sum (1 - cos D_j) plus Delta H if accepted.
// need64 is set for a decision whose margin |ln r + dH/T| lies inside a
// bound on its rounding error, a reflection or proposal within 4e-6 of the
// ends of [0, pi), and a weak field (|h| < 1/4: neighbours split between
// both ends of [0, 2 pi), where Psi is ill-conditioned in single precision).
__device__ __forceinline__ SiteOut update_site(float phi, float n0, float n1, float n2, float n3,
                                               uint32_t valid, float u, float r, float inv_T, float dscale,
                                               bool or_only, bool *need64)
{
    const float th = 0.5f * phi;
    const float nb[4] = {n0, n1, n2, n3};
    float A2 = 0.0f, B = 0.0f, S1 = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool v = (valid >> j) & 1u;
        const float dj = v ? th - 0.5f * nb[j] : 0.0f;
        const float d2 = dj * dj;
        const float s2 = sin2_half_poly(dj, d2);  // 2 sin(D_j / 2)
        const float cj = cos_half_poly(d2);
        B = fmaf(s2, cj, B);        // sin D_j
        A2 = fmaf(s2, s2, A2);      // 2 (1 - cos D_j)
        S1 += fabsf(dj);
    }
    const float A_small = 0.5f * A2;
    const float A = (float)__popc(valid & 15u) - A_small;
    const float d1 = atan2_poly(-B, A);
    const float raw1 = fmaf(2.0f, d1, th);
    const float pi_f = 3.14159274f;
    const float tb = 4.0e-6f;
    bool close = (A * A + B * B) < 0.0625f || fabsf(raw1) < tb || fabsf(raw1 - pi_f) < tb;
    const bool kept = !(raw1 >= 0.0f && raw1 < pi_f);
    const float th1 = kept ? th : raw1;
    SiteOut o;
    o.e_before = A_small;
    if (or_only) {
        *need64 = close;
        o.phi = 2.0f * th1;
        o.e_bonds = A_small;
        o.flags = F_UPDATED | (kept ? F_KEPT : 0u);
        o.accepted = false;
        return o;
    }
    const float Bs = kept ? B : -B;
    const float delta = (u - 0.5f) * dscale;
    const float dd2 = delta * delta;
    const float sh2 = sin2_half_poly(delta, dd2), ch = cos_half_poly(dd2);  // 2 sin(delta/2), cos(delta/2)
    const float sd = sh2 * ch;
    const float raw2 = th1 + delta;
    const bool wrapped = raw2 < 0.0f || raw2 >= pi_f;
    close = close || fabsf(raw2) < tb || fabsf(raw2 - pi_f) < tb || r == 0.0f;
    const float th2 = raw2 < 0.0f ? raw2 + pi_f : (raw2 >= pi_f ? raw2 - pi_f : raw2);
    const float w2 = wrapped ? 2.0f * (ch * ch) : 0.5f * (sh2 * sh2);
    const float dH = fmaf(A, w2, wrapped ? -Bs * sd : Bs * sd);
    const float x = dH * inv_T;
    const float lr = __builtin_amdgcn_logf(r) * 0.693147182f;  // r >= 2^-24 here: no denormals
    const float m = -x - lr;
    // Rounding-error bound of m: B carries a relative error ~6e-7 of
    // sum |D_j|, A an absolute one ~1e-6; the rest is relative:
    //   err(dH) <= 2e-6 ((S1 + (|A| + |B|) |sd|) |sd| + w2 + |dH|),
    //   band = err(dH) / T + 1e-6 (|x| + |ln r|) + 1e-6.
    const float t_err = fmaf(fmaf(fabsf(A) + fabsf(B), fabsf(sd), S1), fabsf(sd), w2);
    const float band = fmaf(t_err, 2.0e-6f * inv_T, fmaf(3.0e-6f, fabsf(x), fmaf(1.0e-6f, fabsf(lr), 1.0e-6f)));
    *need64 = close || !(fabsf(m) > band);
    const bool acc = m > 0.0f;
    o.phi = 2.0f * (acc ? th2 : th1);
    o.e_bonds = acc ? A_small + dH : A_small;
    o.flags = F_UPDATED | (kept ? F_KEPT : 0u) | (wrapped ? F_WRAPPED : 0u) | (acc ? F_ACCEPTED : 0u);
    o.accepted = acc;
    return o;
}

// Sum over the bonds of a site of 1 - cos D_j (q = 1/2, th = phi / 2), in
// the same operations and order as update_site, so that a sampled site's
// energy equals the value update_site would report for it.
__device__ __forceinline__ float bond_energy_half(float th, float n0, float n1, float n2, float n3, uint32_t valid)
{
    const float nb[4] = {n0, n1, n2, n3};
    float A2 = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool v = (valid >> j) & 1u;
        const float dj = v ? th - 0.5f * nb[j] : 0.0f;
        const float s2 = sin2_half_poly(dj, dj * dj);
        A2 = fmaf(s2, s2, A2);
    }
    return 0.5f * A2;
}

// Loads and stores through global-address-space pointers (the chain
// descriptors hold generic ones, which would otherwise give flat accesses).
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) v2f gv2f;
__device__ __forceinline__ float gld(const float *p) { return *(const gfloat *)p; }
__device__ __forceinline__ void gst(float *p, float v) { *(gfloat *)p = v; }

// The same through a uniform base pointer and a 32-bit element index, so
// that the address is the base plus a zero-extended 32-bit byte offset (the
// scalar-base form of a global access, with no 64-bit address arithmetic per
// lane).  The caller keeps the byte offset below 2^32 (a single-precision
// half-grid is smaller than 4 GiB).
__device__ __forceinline__ const gfloat *gaddr(const float *base, uint32_t i)
{
    return (const gfloat *)((const char *)base + (uint64_t)(i << 2));
}
__device__ __forceinline__ float gldi(const float *base, uint32_t i) { return *gaddr(base, i); }
__device__ __forceinline__ float2 gldi2(const float *base, uint32_t i)
{
    const v2f v = *(const gv2f *)gaddr(base, i);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gsti(float *base, uint32_t i, float v) { *(gfloat *)gaddr(base, i) = v; }
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f gv4f;
// 16-byte load and store at element i (a multiple of 4) of a uniform base.
__device__ __forceinline__ v4f gldi4(const float *base, uint32_t i) { return *(const gv4f *)gaddr(base, i); }
__device__ __forceinline__ void gsti4(float *base, uint32_t i, v4f v) { *(gv4f *)gaddr(base, i) = v; }

// Adds the k-th equilibrium state phi of a site to its running sum acc and,
// when m2 is given, to the sum of squared deviations from the running mean
// (Welford's update with the mean taken from the sum: mean_{k-1} = acc
// inv_km1 before, mean_k = acc inv_k after; k = 1 adds exactly zero).
__device__ __forceinline__ void accumulate_state(float *acc, float *m2, float phi, float inv_k, float inv_km1)
{
    const float s0 = gld(acc);
    const float s1 = s0 + phi;
    gst(acc, s1);
    if (m2) gst(m2, fmaf(phi - s0 * inv_km1, phi - s1 * inv_k, gld(m2)));
}

// accumulate_state at element i of uniform base pointers.
__device__ __forceinline__ void accumulate_state_i(float *acc, float *m2, uint32_t i, float phi, float inv_k,
                                                   float inv_km1)
{
    const float s0 = gldi(acc, i);
    const float s1 = s0 + phi;
    gsti(acc, i, s1);
    if (m2) gsti(m2, i, fmaf(phi - s0 * inv_km1, phi - s1 * inv_k, gldi(m2, i)));
}

// Bond energies of a site in fixed point: units of 2^-27, rounded, so that
// integer sums over sites do not depend on their order (a site has at most
// 4 bonds of at most 2 each, so a value stays below 2^30).
constexpr float kEnergyScale = 134217728.0f;
constexpr double kEnergyUnit = 1.0 / 134217728.0;

__device__ __forceinline__ uint32_t energy_fx(float e) { return (uint32_t)fmaf(e, kEnergyScale, 0.5f); }

// Sum over the bonds of one site of 1 - cos(q (phi_i - phi_j)) = 2 sin^2(D/2),
// D = q (phi_i - phi_j), straight from the angles.
__device__ __forceinline__ float site_energy(float phi, const float nb[4], uint32_t valid, float q)
{
    float e = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool v = (valid >> j) & 1u;
        const float sj = sin_poly(v ? 0.5f * q * (phi - nb[j]) : 0.0f);
        e = fmaf(2.0f * sj, sj, e);
    }
    return e;
}

// ------------------------------------------------ double-precision chains
// The double-precision variant of the sweep (the paper's DP runs, Section 4,
// Tables 2 and 3): half-grids of doubles, the sign bit again marking the
// sampled sites, and every step of update_site carried out in double
// precision, so that no decision needs a second look.
__device__ __forceinline__ bool is_fixed_d(double v) { return __double_as_longlong(v) < 0; }
__device__ __forceinline__ double mark_fixed_d(double a)
{
    return __longlong_as_double(__double_as_longlong(a) | (long long)0x8000000000000000ull);
}

// 2 sin(d/2) and cos(d/2) for |d| <= pi from d2 = d * d: their Taylor
// series in d, with coefficients (-1)^k / (4^k (2k+1)!) and
// (-1)^k / (4^k (2k)!) rounded to double; the first omitted terms are below
// 1e-18 and 2e-17 (relative and absolute).
__device__ __forceinline__ double sin2_half_d(double d, double d2)
{
    double p = -3.135923479699833e-23;
    p = fma(p, d2, 4.289943320229371e-20);
    p = fma(p, d2, -4.667458332409556e-17);
    p = fma(p, d2, 3.920664999224027e-14);
    p = fma(p, d2, -2.446494959515793e-11);
    p = fma(p, d2, 1.076457782186949e-08);
    p = fma(p, d2, -3.1001984126984127e-06);
    p = fma(p, d2, 0.0005208333333333333);
    p = fma(p, d2, -0.041666666666666664);
    return fma(d * d2, p, d);
}

__device__ __forceinline__ double cos_half_d(double d2)
{
    double p = -2.1211603623510776e-28;
    p = fma(p, d2, 3.919904349624791e-25);
    p = fma(p, d2, -5.958254611429682e-22);
    p = fma(p, d2, 7.292903644389931e-19);
    p = fma(p, d2, -7.001187498614334e-16);
    p = fma(p, d2, 5.096864498991235e-13);
    p = fma(p, d2, -2.691144455467372e-10);
    p = fma(p, d2, 9.68812003968254e-08);
    p = fma(p, d2, -2.170138888888889e-05);
    p = fma(p, d2, 0.0026041666666666665);
    p = fma(p, d2, -0.125);
    return fma(p, d2, 1.0);
}

// Result of one double-precision site update.
struct SiteOutD {
    double phi;       // new angle
    double e_bonds;   // sum over the site's bonds of 1 - cos(q (phi_new - phi_j))
    double e_before;  // the same sum before the update
    uint32_t flags;
    bool accepted;
};

// Algorithm 1 for one site in double precision, for 0 < q <= 1/2: the steps
// of update_site in the variable th = q phi in [0, 2 pi q) (reflection
// th' = th + 2 atan2(-B, A), kept when it leaves that range), with the
// proposal, wrap and acceptance test in the form of their plain definition:
// phi'' = phi' + 2 pi (u - 1/2) / a taken mod 2 pi, accepted when Delta H <= 0
// or exp(-Delta H / T) > r.  The energy change uses the cancellation-free
// form Delta H = 2 A sin^2(d / 2) + B_s sin d for the move d = th'' - th' in
// th (q delta phi, shifted by -+2 pi q when the proposal wraps; |d| <= pi).
// Sums over the valid neighbours of a site with th = q phi, D_j = th - q phi_j:
// A2 = sum 2 (1 - cos D_j) and, with WITH_B, B = sum sin D_j.  The update and
// the bond energy of a sampled site both take A2 from here, so that the two
// round alike.
template <bool WITH_B>
__device__ __forceinline__ void neighbour_sums_d(double th, double q, const double nb[4], uint32_t valid, double &A2,
                                                 double &B)
{
    A2 = 0.0;
    B = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool v = (valid >> j) & 1u;
        const double dj = v ? th - q * nb[j] : 0.0;
        const double d2 = dj * dj;
        const double s2 = sin2_half_d(dj, d2);         // 2 sin(D_j / 2)
        if (WITH_B) B = fma(s2, cos_half_d(d2), B);  // sin D_j
        A2 = fma(s2, s2, A2);                          // 2 (1 - cos D_j)
    }
}

// Bond energy sum_j (1 - cos D_j) of a site: the e_before of update_site_d
// (for sampled sites, which are not updated).
__device__ __forceinline__ double bond_energy_d(double phi, double n0, double n1, double n2, double n3,
                                                uint32_t valid, double q)
{
    const double nb[4] = {n0, n1, n2, n3};
    double A2, B;
    neighbour_sums_d<false>(q * phi, q, nb, valid, A2, B);
    return 0.5 * A2;
}

__device__ __forceinline__ SiteOutD update_site_d(double phi, double n0, double n1, double n2, double n3,
                                                  uint32_t valid, double u, double r, double a, double T, double q,
                                                  bool or_only)
{
    const double period = kTwoPi * q;  // range of th
    const double th = q * phi;
    const double nb[4] = {n0, n1, n2, n3};
    double A2, B;
    neighbour_sums_d<true>(th, q, nb, valid, A2, B);
    const double A_small = 0.5 * A2;
    const int nnb = __popc(valid & 15u);
    const double A = (double)nnb - A_small;
    SiteOutD o;
    o.e_before = A_small;
    double p1 = phi;
    bool kept = true;
    if (nnb > 0 && (A != 0.0 || B != 0.0)) {
        const double raw1 = fma(2.0, atan2_fp64(-B, A), th);
        if (raw1 >= 0.0 && raw1 < period) {
            p1 = raw1 / q;
            kept = false;
        }
    }
    uint32_t f = F_UPDATED | F_FP64 | (kept ? F_KEPT : 0u);
    if (or_only) {
        o.phi = p1;
        o.e_bonds = A_small;
        o.flags = f;
        o.accepted = false;
        return o;
    }
    const double Bs = kept ? B : -B;  // |h| sin(th' - Psi)
    const double dphi = kTwoPi * (u - 0.5) / a;
    const double raw2 = p1 + dphi;
    const bool wrapped = raw2 < 0.0 || raw2 >= kTwoPi;
    double p2 = raw2 < 0.0 ? raw2 + kTwoPi : (raw2 >= kTwoPi ? raw2 - kTwoPi : raw2);
    if (p2 >= kTwoPi || p2 < 0.0) p2 = 0.0;
    const double d = q * dphi + (raw2 < 0.0 ? period : (raw2 >= kTwoPi ? -period : 0.0));
    const double dd2 = d * d;
    const double sh2 = sin2_half_d(d, dd2);   // 2 sin(d/2)
    const double sd = sh2 * cos_half_d(dd2);  // sin d
    const double dH = fma(A, 0.5 * (sh2 * sh2), Bs * sd);
    const bool acc = (dH <= 0.0) || (exp(-dH / T) > r);
    if (wrapped) f |= F_WRAPPED;
    if (acc) f |= F_ACCEPTED;
    o.phi = acc ? p2 : p1;
    o.e_bonds = acc ? A_small + dH : A_small;
    o.flags = f;
    o.accepted = acc;
    return o;
}

typedef double v2d __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) v2d gv2d;
__device__ __forceinline__ double gldd(const double *p) { return *(const gdouble *)p; }
__device__ __forceinline__ double2 gldd2(const double *p)
{
    const v2d v = *(const gv2d *)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstd(double *p, double v) { *(gdouble *)p = v; }
__device__ __forceinline__ void gstd2(double *p, double2 v)
{
    v2d w;
    w.x = v.x;
    w.y = v.y;
    *(gv2d *)p = w;
}

// accumulate_state for double-precision chains.
__device__ __forceinline__ void accumulate_state_d(double *acc, double *m2, double phi, double inv_k, double inv_km1)
{
    const double s0 = gldd(acc);
    const double s1 = s0 + phi;
    gstd(acc, s1);
    if (m2) gstd(m2, fma(phi - s0 * inv_km1, phi - s1 * inv_k, gldd(m2)));
}

// Bond energies of a double-precision site in fixed point, units of 2^-30
// (at most 8 per site, so a chain of up to 2^30 sites of one colour sums
// below 2^63).
constexpr double kEnergyScale64 = 1073741824.0;
constexpr double kEnergyUnit64 = 1.0 / 1073741824.0;
__device__ __forceinline__ unsigned long long energy_fx_d(double e)
{
    return (unsigned long long)fma(e, kEnergyScale64, 0.5);
}

}  // namespace mpr
