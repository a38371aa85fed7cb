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
    float *h[2];          // colour half-grids, ny * S each
    float *acc[2];        // equilibrium sums (K > 1), or null
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
    unsigned long long e_fx;   // sum over bonds of |u_i - u_j|^2 in units of 2^-31
    unsigned long long acc;    // accepted proposals in the current sweep
    double k;              // last energy slope
    double A_last;
    double e_sum;          // table mode: sum of (1 + e) over measured sweeps
    int32_t relax_sweeps;
    int32_t not_converged;
    int32_t eq_left;
    int32_t pad;
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
#pragma unroll
    for (int i = 0; i < 10; ++i) {
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
    return c;
}

// 24-bit dyadic uniform in [0, 1), exact in float and double.
__device__ __forceinline__ float unit24(uint32_t w)
{
    return (float)(w >> 8) * 5.9604644775390625e-08f;
}

// ------------------------------------------------------------- sign bit
__device__ __forceinline__ bool is_fixed(float v) { return (__float_as_uint(v) >> 31) != 0u; }
__device__ __forceinline__ float angle_of(float v) { return __uint_as_float(__float_as_uint(v) & 0x7FFFFFFFu); }
__device__ __forceinline__ float mark_fixed(float a) { return __uint_as_float(__float_as_uint(a) | 0x80000000u); }

// Sweep parameters shared by a launch.
struct SweepConsts {
    float q;          // coupling exponent
    float two_pi_q;   // period of q*phi
    double q64;
    uint32_t seed_lo, seed_hi;
};

// ------------------------------------------------- double-precision path
// The whole update of one site in double precision, in the same steps and
// order as the plain definition: local q-field, reflection with the keep
// rule, wrapped proposal, Delta H as the difference of the two local
// energies, and the acceptance test.  Used when the single-precision
// decision is too close to call.
__device__ __noinline__ float update_site_fp64(double phi, const float nb[4], uint32_t valid,
                                               double u, double r, double a, double T,
                                               double q, uint32_t *flags)
{
#pragma clang fp contract(off)
    double sx = 0.0, sy = 0.0;
    int nnb = 0;
    for (int j = 0; j < 4; ++j) {
        if (valid & (1u << j)) {
            const double v = (double)nb[j];
            sx += cos(q * v);
            sy += sin(q * v);
            ++nnb;
        }
    }
    double p1;
    uint32_t f = F_UPDATED | F_FP64;
    if (nnb == 0 || (sx == 0.0 && sy == 0.0)) {
        p1 = phi;
        f |= F_KEPT;
    } else {
        const double psi = atan2(sy, sx);
        p1 = (2.0 * psi - q * phi) / q;
        if (!(p1 >= 0.0 && p1 < kTwoPi)) {
            p1 = phi;
            f |= F_KEPT;
        }
    }
    const double raw = p1 + kTwoPi * (u - 0.5) / a;
    double p2 = raw;
    if (p2 < 0.0) p2 += kTwoPi;
    else if (p2 >= kTwoPi) p2 -= kTwoPi;
    if (p2 >= kTwoPi || p2 < 0.0) p2 = 0.0;
    if (raw < 0.0 || raw >= kTwoPi) f |= F_WRAPPED;
    double h2 = 0.0, h1 = 0.0;
    for (int j = 0; j < 4; ++j)
        if (valid & (1u << j)) h2 -= cos(q * (p2 - (double)nb[j]));
    for (int j = 0; j < 4; ++j)
        if (valid & (1u << j)) h1 -= cos(q * (p1 - (double)nb[j]));
    const double dH = h2 - h1;
    const bool acc = (dH <= 0.0) || (exp(-dH / T) > r);
    if (acc) f |= F_ACCEPTED;
    *flags = f;
    return (float)(acc ? p2 : p1);
}

// --------------------------------------------------- single-site update
struct SiteOut {
    float phi;       // new angle
    uint32_t flags;
};

// Algorithm 1 for one gap site in single precision.
//   phi        current angle of the site
//   nb[4]      neighbour angles (left, right, up, down), valid bits in `valid`
//   nc, ns     cos / sin of q * neighbour angle (0 for missing neighbours)
//   u, r       the site's two uniforms
// Over-relaxation reflects theta = q*phi about Psi = arg(h), h = sum of the
// neighbour unit vectors: theta' = 2 Psi - theta, kept when it leaves
// [0, 2 pi q).  The Metropolis energy change of theta'' = theta' + delta is
// evaluated without cancellation: with d = theta' - Psi,
//   H(theta'') - H(theta') = |h| (cos d - cos(d + delta))
//                          = 2 |h| sin(d + delta/2) sin(delta/2)
// when the proposal does not wrap, and directly otherwise.  Decisions whose
// margin |ln r + Delta H / T| is inside a bound on the rounding error, and
// reflections or proposals that land within rounding of the domain's ends,
// are redone in double precision.
__device__ __forceinline__ SiteOut update_site(float phi, const float nb[4], uint32_t valid,
                                               const float nc[4], const float ns[4],
                                               float u, float r, const ChainState &st,
                                               const SweepConsts &sc, bool or_only)
{
    const float hx = (nc[0] + nc[1]) + (nc[2] + nc[3]);
    const float hy = (ns[0] + ns[1]) + (ns[2] + ns[3]);
    const float th = sc.q * phi;
    const float psi = atan2f(hy, hx);
    const float raw1 = 2.0f * psi - th;
    const bool degenerate = (hx == 0.0f && hy == 0.0f);
    bool kept = degenerate || !(raw1 >= 0.0f && raw1 < sc.two_pi_q);
    const float tb = 4.0e-6f;
    bool close = fabsf(raw1) < tb || fabsf(raw1 - sc.two_pi_q) < tb;
    const float th1 = kept ? th : raw1;
    const float d1 = kept ? (th - psi) : (psi - th);
    SiteOut o;
    if (or_only) {
        o.phi = th1 / sc.q;
        o.flags = F_UPDATED | (kept ? F_KEPT : 0u);
        if (close) {
            // Decide the keep rule in double precision as well.
            double sx = 0.0, sy = 0.0;
            for (int j = 0; j < 4; ++j)
                if (valid & (1u << j)) {
                    sx += cos(sc.q64 * (double)nb[j]);
                    sy += sin(sc.q64 * (double)nb[j]);
                }
            const double p1 = (2.0 * atan2(sy, sx) - sc.q64 * (double)phi) / sc.q64;
            const bool k64 = !(p1 >= 0.0 && p1 < kTwoPi);
            o.phi = k64 ? phi : (float)p1;
            o.flags = F_UPDATED | F_FP64 | (k64 ? F_KEPT : 0u);
        }
        return o;
    }
    const float delta = (u - 0.5f) * st.dscale;
    const float raw2 = th1 + delta;
    const bool wrapped = raw2 < 0.0f || raw2 >= sc.two_pi_q;
    close = close || fabsf(raw2) < tb || fabsf(raw2 - sc.two_pi_q) < tb;
    float th2 = raw2 < 0.0f ? raw2 + sc.two_pi_q : (raw2 >= sc.two_pi_q ? raw2 - sc.two_pi_q : raw2);
    if (th2 >= sc.two_pi_q || th2 < 0.0f) th2 = 0.0f;
    const float hmag = sqrtf(hx * hx + hy * hy);
    float dH;
    if (!wrapped) {
        const float hd = 0.5f * delta;
        dH = 2.0f * hmag * sinf(d1 + hd) * sinf(hd);
    } else {
        dH = hmag * (cosf(d1) - cosf(th2 - psi));
    }
    const float x = dH * st.inv_T;
    const float lr = logf(r);
    const float m = -x - lr;
    const bool acc = (r == 0.0f) || (m > 0.0f);
    // Rounding-error bound of m (generous): errors of the neighbour sums and
    // of Psi enter through d times |delta| (times 2 for a wrapped proposal);
    // the rest is relative to Delta H, ln r and their ratio.
    const float err_dH = 8.0e-6f * (1.0f + hmag) * (fabsf(delta) + (wrapped ? 2.0f : 0.0f))
                         + 8.0e-6f * fabsf(dH) * (1.0f + 1.0f / fmaxf(hmag, 1.0e-3f));
    const float err_m = err_dH * st.inv_T + 1.0e-6f * (fabsf(x) + fabsf(lr)) + 1.0e-30f;
    if (close || fabsf(m) <= err_m || degenerate) {
        o.phi = update_site_fp64((double)phi, nb, valid, (double)u, (double)r, st.a_cur, st.T,
                                 sc.q64, &o.flags);
        return o;
    }
    o.phi = (acc ? th2 : th1) / sc.q;
    o.flags = F_UPDATED | (kept ? F_KEPT : 0u) | (wrapped ? F_WRAPPED : 0u) | (acc ? F_ACCEPTED : 0u);
    return o;
}

// Bond energy sum of one site in fixed point: sum over its bonds of
// |u_i - u_j|^2 = 2 (1 - cos(q (phi_i - phi_j))), scaled by 2^31 and
// truncated, so that integer sums over sites do not depend on their order.
__device__ __forceinline__ unsigned long long site_energy_fx(float ci, float si, const float *nc,
                                                             const float *ns, uint32_t valid)
{
    float e = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (valid & (1u << j)) {
            const float dx = ci - nc[j];
            const float dy = si - ns[j];
            e = fmaf(dx, dx, fmaf(dy, dy, e));
        }
    }
    return (unsigned long long)((double)e * 2147483648.0);
}

}  // namespace mpr
