/*
 * FP64 CPU oracle for MPR gap filling (arXiv:1811.01604).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code, header or constant table with the HIP path.
 *
 * Everything is double precision, single threaded, on the full grid stored
 * row-major (index y*nx + x, x fastest).  sampled[i] != 0 marks a sampled
 * (fixed) site, 0 marks a gap.  Each function names the passage it follows.
 *
 * Readings of points the paper leaves open:
 *  - Over-relaxation for q = 1/2.  The printed reflection uses the q = 1
 *    local field and does not conserve the q = 1/2 energy.  Here the spin is
 *    reflected in the variable q*phi about the direction Psi of the q-field
 *    sum_j (cos q phi_j, sin q phi_j): phi' = (2 Psi - q phi) / q.  When that
 *    leaves [0, 2pi) the spin is kept, which is the only energy-conserving
 *    choice and keeps the map an involution.
 *  - One sweep updates colour 0 ((x+y) even) and then colour 1; the
 *    Metropolis energy difference is taken against the over-relaxed value.
 *  - Open boundaries; N_GP = nx(ny-1) + ny(nx-1).
 *  - Random numbers: Philox4x32-10 with key = seed, counter =
 *    (y*nx + (x & ~2), sweep, chain, stream); the site at x uses words
 *    (0,1) if ((x>>1)&1) == 0, else words (2,3); a 32-bit word w becomes
 *    (w >> 8) * 2^-24.  The first word of the pair proposes, the second
 *    accepts.  Initial gap angles use sweep = 0xFFFFFFFF.
 *  - The stopping slope is the derivative, at the newest point, of the
 *    least-squares polynomial (degree d, default 1) through the last n_fit
 *    specific energies.
 *  - If the acceptance ratio does not fall below the target, a is unchanged.
 *  - e(T, L) comes from unconditional runs started from phi = pi, with the
 *    relaxation-phase rule for a, averaged over the measured sweeps; the
 *    temperature is read off a monotone fit of log(1 + e) against log T.
 *  - Besides the mean, the statistics of the M realizations reported are
 *    their sample standard deviation (denominator M - 1) after the back
 *    transform, which is linear in phi, and their quantiles: linear
 *    interpolation between order statistics (Hyndman and Fan's definition
 *    7), back-transformed like the mean.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_TWO_PI 6.283185307179586476925286766559
#define O_PI 3.1415926535897932384626433832795

enum { O_OK = 0, O_ERR_ARG = 1, O_ERR_DEGENERATE = 2 };

/* Mode bits for a half-sweep. */
enum { O_MODE_FULL = 0, O_MODE_OR_ONLY = 1 };

/* Per-site flag bits written by a half-sweep. */
enum { O_FLAG_KEPT = 1, O_FLAG_ACCEPTED = 2, O_FLAG_WRAPPED = 4, O_FLAG_UPDATED = 8 };

typedef struct {
    double q;            /* coupling, 1/2 in the paper */
    int32_t R, K;        /* independent chains, equilibrium states per chain */
    int32_t n_f, n_fit, sg_degree;
    double a_targ, k_a;
    int32_t i_max;
    int32_t fixed_relax; /* <0: stopping rule; >=0: exactly this many relaxation sweeps */
    int32_t eq_a_mode;   /* 0: a = 1 in the equilibrium phase; 1: keep the final a */
    int32_t pad;
    uint64_t seed;
    uint32_t stream;
    uint32_t pad2;
} oracle_params;

typedef struct {
    int32_t relax_sweeps;
    int32_t not_converged;
    double a_final;
    double A_last;
    double k_last;
} oracle_chain_stats;

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10: Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11.  The paper's GPU code draws from the same
 * generator family (Section 3.3, random numbers). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The two uniforms [0,1) that site (x, y) uses in a given sweep. */
void oracle_site_uniforms(uint64_t seed, int nx, int x, int y, uint32_t sweep,
                          uint32_t chain, uint32_t stream, double *u, double *r)
{
    uint32_t ctr[4] = {(uint32_t)y * (uint32_t)nx + ((uint32_t)x & ~2u), sweep, chain, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    int sel = (x >> 1) & 1;
    *u = (double)(w[2 * sel] >> 8) * (1.0 / 16777216.0);
    *r = (double)(w[2 * sel + 1] >> 8) * (1.0 / 16777216.0);
}

/* Samples kept for fitting when a fraction `hold` of them is held out for
 * validation (the choice of q, which the paper leaves open): the sample at
 * index i = y*nx + x is held out when (w >> 8) 2^-24 < hold for word w = word 0
 * of Philox4x32-10 with counter (i, 0xFFFFFFFE, 0, 0x40000000), key = seed. */
void oracle_holdout_mask(int nx, int ny, const uint8_t *sampled, uint64_t seed, double hold, uint8_t *fit)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    long n = (long)nx * ny;
    for (long i = 0; i < n; ++i) {
        fit[i] = 0;
        if (!sampled[i]) continue;
        uint32_t ctr[4] = {(uint32_t)i, 0xFFFFFFFEu, 0u, 0x40000000u}, w[4];
        oracle_philox4x32_10(ctr, key, w);
        fit[i] = ((double)(w[0] >> 8) * (1.0 / 16777216.0) < hold) ? 0 : 1;
    }
}

/* ------------------------------------------------------------ data map */
/* Equation (map), Algorithm 2 step 3.1: phi = 2 pi (z - z_min)/(z_max - z_min)
 * at the sampled sites; z_min, z_max over the samples.  Gaps get 0. */
int oracle_map_to_angles(int nx, int ny, const double *z, const uint8_t *sampled,
                         double *phi, double *zmin_zmax)
{
    if (nx <= 0 || ny <= 0) return O_ERR_ARG;
    long n = (long)nx * ny, count = 0;
    double zmin = INFINITY, zmax = -INFINITY;
    for (long i = 0; i < n; ++i) {
        if (!sampled[i]) continue;
        if (!isfinite(z[i])) return O_ERR_ARG;
        if (z[i] < zmin) zmin = z[i];
        if (z[i] > zmax) zmax = z[i];
        ++count;
    }
    if (count < 2 || !(zmax > zmin)) return O_ERR_DEGENERATE;
    for (long i = 0; i < n; ++i)
        phi[i] = sampled[i] ? O_TWO_PI * ((z[i] - zmin) / (zmax - zmin)) : 0.0;
    zmin_zmax[0] = zmin;
    zmin_zmax[1] = zmax;
    return O_OK;
}

/* ------------------------------------------------------------- energies */
/* Equation (Hamiltonian_mod) with J absorbed into T: H = -sum_<ij> cos(q(phi_i - phi_j))
 * over the nearest-neighbour bonds of the grid (open boundaries). */
double oracle_energy(int nx, int ny, const double *phi, double q)
{
    double H = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            if (x + 1 < nx) H -= cos(q * (phi[i] - phi[i + 1]));
            if (y + 1 < ny) H -= cos(q * (phi[i] - phi[i + nx]));
        }
    return H;
}

long oracle_bond_count(int nx, int ny)
{
    return (long)nx * (ny - 1) + (long)ny * (nx - 1);
}

/* Equation (mpr-sse): e_s = -(1/N_SP) sum over sample-sample nearest-neighbour
 * pairs of cos(q(phi_i - phi_j)); each unordered pair counted once. */
int oracle_sample_energy(int nx, int ny, const double *phi, const uint8_t *sampled,
                         double q, double *e_s, long *n_sp)
{
    double s = 0.0;
    long n = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            if (!sampled[i]) continue;
            if (x + 1 < nx && sampled[i + 1]) { s -= cos(q * (phi[i] - phi[i + 1])); ++n; }
            if (y + 1 < ny && sampled[i + nx]) { s -= cos(q * (phi[i] - phi[i + nx])); ++n; }
        }
    *n_sp = n;
    if (n == 0) return O_ERR_DEGENERATE;
    *e_s = s / (double)n;
    return O_OK;
}

/* Energy of the bonds of site (x, y) if its angle were v. */
static double local_energy(int nx, int ny, const double *phi, int x, int y, double v, double q)
{
    long i = (long)y * nx + x;
    double h = 0.0;
    if (x > 0) h -= cos(q * (v - phi[i - 1]));
    if (x + 1 < nx) h -= cos(q * (v - phi[i + 1]));
    if (y > 0) h -= cos(q * (v - phi[i - nx]));
    if (y + 1 < ny) h -= cos(q * (v - phi[i + nx]));
    return h;
}

/* x mod 2 pi into [0, 2 pi); x is within one period of that range here. */
static double wrap_2pi(double x)
{
    if (x < 0.0) x += O_TWO_PI;
    else if (x >= O_TWO_PI) x -= O_TWO_PI;
    if (x >= O_TWO_PI || x < 0.0) x = 0.0;
    return x;
}

/* ------------------------------------------------------- hybrid update */
/* Algorithm 1 applied to the gap sites of one checkerboard colour (Section
 * 3.3: the two sub-grids are updated one after the other; a site's
 * neighbours all belong to the other colour, so the order within a colour
 * does not matter).  For each gap site of the colour:
 *   step 1: over-relaxation, equation (over-relax) in the q-aware reading;
 *   step 2-3: proposal phi'' = phi' + 2 pi (u - 1/2)/a  (mod 2 pi);
 *   step 4: Delta H = H(phi'') - H(phi') with the other sites fixed;
 *   step 5-6: accept when min(1, exp(-Delta H / T)) > r.
 * Returns the number of accepted proposals.  flags (nullable) gets per-site
 * bits O_FLAG_*.  mode O_MODE_OR_ONLY stops after step 1. */
long oracle_half_sweep(int nx, int ny, double *phi, const uint8_t *sampled, int colour,
                       double T, double a, double q, uint64_t seed, uint32_t sweep,
                       uint32_t chain, uint32_t stream, int mode, uint8_t *flags)
{
    long accepted = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (((x + y) & 1) != colour) continue;
            long i = (long)y * nx + x;
            if (flags) flags[i] = 0;
            if (sampled[i]) continue;
            /* step 1: local q-field and reflection */
            double sx = 0.0, sy = 0.0;
            int nnb = 0;
            if (x > 0) { sx += cos(q * phi[i - 1]); sy += sin(q * phi[i - 1]); ++nnb; }
            if (x + 1 < nx) { sx += cos(q * phi[i + 1]); sy += sin(q * phi[i + 1]); ++nnb; }
            if (y > 0) { sx += cos(q * phi[i - nx]); sy += sin(q * phi[i - nx]); ++nnb; }
            if (y + 1 < ny) { sx += cos(q * phi[i + nx]); sy += sin(q * phi[i + nx]); ++nnb; }
            double cur = phi[i];
            double p1;
            int kept = 0;
            if (nnb == 0 || (sx == 0.0 && sy == 0.0)) {
                p1 = cur;
                kept = 1;
            } else {
                double psi = atan2(sy, sx);
                p1 = (2.0 * psi - q * cur) / q;
                if (!(p1 >= 0.0 && p1 < O_TWO_PI)) {
                    p1 = cur;
                    kept = 1;
                }
            }
            uint8_t f = O_FLAG_UPDATED | (kept ? O_FLAG_KEPT : 0);
            if (mode == O_MODE_OR_ONLY) {
                phi[i] = p1;
                if (flags) flags[i] = f;
                continue;
            }
            /* steps 2-6 */
            double u, r;
            oracle_site_uniforms(seed, nx, x, y, sweep, chain, stream, &u, &r);
            double raw = p1 + O_TWO_PI * (u - 0.5) / a;
            double p2 = wrap_2pi(raw);
            if (raw < 0.0 || raw >= O_TWO_PI) f |= O_FLAG_WRAPPED;
            double dH = local_energy(nx, ny, phi, x, y, p2, q) - local_energy(nx, ny, phi, x, y, p1, q);
            int acc = (dH <= 0.0) || (exp(-dH / T) > r);
            phi[i] = acc ? p2 : p1;
            if (acc) {
                ++accepted;
                f |= O_FLAG_ACCEPTED;
            }
            if (flags) flags[i] = f;
        }
    return accepted;
}

/* ------------------------------------------------------------ SG slope */
/* Derivative at the newest point of the least-squares polynomial of degree
 * `degree` through (j, e[j]), j = 0..n-1 (Algorithm 2 step 5.4: slope of the
 * energy evolution from a Savitzky-Golay fit of the last n_fit values).
 * Solved from the normal equations in the centred abscissa s = j - (n-1)/2. */
double oracle_sg_slope(const double *e, int n, int degree)
{
    if (n < 2) return 0.0;
    if (degree < 1) degree = 1;
    if (degree > n - 1) degree = n - 1;
    if (degree > 8) degree = 8;
    int m = degree + 1;
    double A[9][10];
    double c = 0.5 * (n - 1);
    for (int k = 0; k < m; ++k) {
        for (int l = 0; l < m; ++l) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += pow(j - c, k + l);
            A[k][l] = s;
        }
        double b = 0.0;
        for (int j = 0; j < n; ++j) b += pow(j - c, k) * e[j];
        A[k][m] = b;
    }
    /* Gaussian elimination with partial pivoting */
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int l = 0; l <= m; ++l) {
                double t = A[col][l];
                A[col][l] = A[piv][l];
                A[piv][l] = t;
            }
        for (int r = col + 1; r < m; ++r) {
            double f = A[r][col] / A[col][col];
            for (int l = col; l <= m; ++l) A[r][l] -= f * A[col][l];
        }
    }
    double coef[9];
    for (int r = m - 1; r >= 0; --r) {
        double s = A[r][m];
        for (int l = r + 1; l < m; ++l) s -= A[r][l] * coef[l];
        coef[r] = s / A[r][r];
    }
    double send = (n - 1) - c, d = 0.0;
    for (int k = 1; k < m; ++k) d += k * coef[k] * pow(send, k - 1);
    return d;
}

/* ----------------------------------------------------------- simulation */
/* Algorithm 2 steps 2, 5 and 6 for one image, repeated for R independent
 * chains; each chain relaxes with its own stopping test and then contributes
 * K equilibrium states, so M = R*K realizations in all (R = 1, K = M is the
 * paper's layout).  phi holds the sample angles (gaps ignored).  phi_init
 * (nullable) supplies the starting gap angles instead of U(0, 2 pi).
 * phi_sum receives the sum of the M realizations at the gap sites (0 at the
 * samples).  e_trace (nullable, R x trace_len) receives e after each
 * relaxation sweep.  phi_last (nullable) receives the final state of the last
 * chain.  phi_states (nullable, M x nx*ny) receives every equilibrium state,
 * state r*K + k of chain r after its k-th equilibrium sweep.  a_trace and
 * acc_trace (nullable, R x trace_len) receive, for every sweep t of a chain
 * (relaxation and equilibrium, t < trace_len), the a the sweep's proposals
 * used and the number of proposals it accepted. */
int oracle_simulate(int nx, int ny, const double *phi, const uint8_t *sampled, double T,
                    const oracle_params *p, const double *phi_init, double *phi_sum,
                    double *phi_sq_sum, double *phi_states, oracle_chain_stats *stats, double *e_trace,
                    int trace_len, double *phi_last, double *a_trace, double *acc_trace)
{
    if (nx <= 0 || ny <= 0 || p->R < 1 || p->K < 0 || !(T > 0.0) || p->n_f < 1 || p->n_fit < 2)
        return O_ERR_ARG;
    if ((long)nx * ny < 2) return O_ERR_DEGENERATE;
    long n = (long)nx * ny, P = 0;
    for (long i = 0; i < n; ++i) if (!sampled[i]) ++P;
    double n_gp = (double)oracle_bond_count(nx, ny);
    for (long i = 0; i < n; ++i) phi_sum[i] = 0.0;
    if (phi_sq_sum)
        for (long i = 0; i < n; ++i) phi_sq_sum[i] = 0.0;
    double *s = (double *)malloc(sizeof(double) * n);
    int cap = (p->fixed_relax >= 0 ? p->fixed_relax : p->i_max + 1) + 1;
    double *eh = (double *)malloc(sizeof(double) * (size_t)cap);
    for (int r = 0; r < p->R; ++r) {
        /* step 2: initial state */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = (long)y * nx + x;
                if (sampled[i]) {
                    s[i] = phi[i];
                } else if (phi_init) {
                    s[i] = phi_init[i];
                } else {
                    double u, rr;
                    oracle_site_uniforms(p->seed, nx, x, y, 0xFFFFFFFFu, (uint32_t)r, p->stream, &u, &rr);
                    s[i] = O_TWO_PI * u;
                }
            }
        double a = 1.0, k = -1.0, A = 0.0;
        int t = 0;
        if (P > 0) {
            /* step 5: relaxation */
            for (;;) {
                if (p->fixed_relax >= 0) {
                    if (t >= p->fixed_relax) break;
                } else if (!(k < 0.0 && t <= p->i_max)) {
                    break;
                }
                long acc = oracle_half_sweep(nx, ny, s, sampled, 0, T, a, p->q, p->seed, (uint32_t)t,
                                             (uint32_t)r, p->stream, O_MODE_FULL, NULL);
                acc += oracle_half_sweep(nx, ny, s, sampled, 1, T, a, p->q, p->seed, (uint32_t)t,
                                         (uint32_t)r, p->stream, O_MODE_FULL, NULL);
                if (a_trace && t < trace_len) a_trace[(long)r * trace_len + t] = a;
                if (acc_trace && t < trace_len) acc_trace[(long)r * trace_len + t] = (double)acc;
                A = (double)acc / (double)P;
                if (A < p->a_targ) a = 1.0 + (double)(t + 1) / p->k_a;
                double e = oracle_energy(nx, ny, s, p->q) / n_gp;
                eh[t] = e;
                if (e_trace && t < trace_len) e_trace[(long)r * trace_len + t] = e;
                if (t >= p->n_fit && t % p->n_f == 0)
                    k = oracle_sg_slope(eh + (t + 1 - p->n_fit), p->n_fit, p->sg_degree);
                ++t;
            }
        }
        stats[r].relax_sweeps = t;
        stats[r].not_converged = (p->fixed_relax < 0 && P > 0 && k < 0.0) ? 1 : 0;
        stats[r].a_final = a;
        stats[r].A_last = A;
        stats[r].k_last = k;
        /* step 6: equilibrium states */
        double a_eq = p->eq_a_mode ? a : 1.0;
        for (int j = 0; j < p->K; ++j) {
            if (P > 0) {
                long acc = oracle_half_sweep(nx, ny, s, sampled, 0, T, a_eq, p->q, p->seed, (uint32_t)t,
                                             (uint32_t)r, p->stream, O_MODE_FULL, NULL);
                acc += oracle_half_sweep(nx, ny, s, sampled, 1, T, a_eq, p->q, p->seed, (uint32_t)t,
                                         (uint32_t)r, p->stream, O_MODE_FULL, NULL);
                if (a_trace && t < trace_len) a_trace[(long)r * trace_len + t] = a_eq;
                if (acc_trace && t < trace_len) acc_trace[(long)r * trace_len + t] = (double)acc;
            }
            ++t;
            for (long i = 0; i < n; ++i)
                if (!sampled[i]) {
                    phi_sum[i] += s[i];
                    if (phi_sq_sum) phi_sq_sum[i] += s[i] * s[i];
                }
            if (phi_states) memcpy(phi_states + ((long)r * p->K + j) * n, s, sizeof(double) * n);
        }
        if (phi_last && r == p->R - 1) memcpy(phi_last, s, sizeof(double) * n);
    }
    free(s);
    free(eh);
    return O_OK;
}

/* Algorithm 2 steps 6.3 and 7 with the mean as the statistic:
 * z_hat = G^{-1}(phi_sum / M) at the gaps, with G^{-1} in the convex form
 * z_min (1 - t) + z_max t, t = phi / (2 pi); samples are copied. */
void oracle_predict(int nx, int ny, const double *z, const uint8_t *sampled, const double *phi_sum,
                    int M, const double *zmin_zmax, double *z_hat)
{
    long n = (long)nx * ny;
    for (long i = 0; i < n; ++i) {
        if (sampled[i]) {
            z_hat[i] = z[i];
        } else {
            double t = (phi_sum[i] / (double)M) / O_TWO_PI;
            z_hat[i] = zmin_zmax[0] * (1.0 - t) + zmin_zmax[1] * t;
        }
    }
}

/* Algorithm 2 step 7, the realizations' spread: the sample standard
 * deviation over the M states of z = G^{-1}(phi), with G^{-1} linear in phi:
 * z_std = (z_max - z_min) / (2 pi) * sqrt((S2 - S1^2 / M) / (M - 1)) for the
 * sums S1 of phi and S2 of phi^2 (negative rounding residue clipped to 0);
 * 0 at sampled sites and for M = 1. */
void oracle_spread(int nx, int ny, const uint8_t *sampled, const double *phi_sum, const double *phi_sq_sum,
                   int M, const double *zmin_zmax, double *z_std)
{
    long n = (long)nx * ny;
    double scale = (zmin_zmax[1] - zmin_zmax[0]) / O_TWO_PI;
    for (long i = 0; i < n; ++i) {
        double v = 0.0;
        if (!sampled[i] && M > 1) {
            double m2 = phi_sq_sum[i] - phi_sum[i] * phi_sum[i] / (double)M;
            v = scale * sqrt((m2 > 0.0 ? m2 : 0.0) / (double)(M - 1));
        }
        z_std[i] = v;
    }
}

/* The p-quantile of v[0..M-1] (sorted in place): linear interpolation
 * between the order statistics v_(floor h) and v_(floor h + 1), h = (M - 1) p
 * (Hyndman and Fan 1996, definition 7). */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static double quantile_sorted(const double *v, int M, double p)
{
    double h = (double)(M - 1) * p;
    int lo = (int)floor(h);
    if (lo >= M - 1) return v[M - 1];
    return v[lo] + (h - (double)lo) * (v[lo + 1] - v[lo]);
}

/* Algorithm 2 step 7, quantiles of the M realizations: at each gap site the
 * p-quantile of the M states of phi (states[m * nx*ny + i]), back-transformed
 * like the mean, z = z_min (1 - t) + z_max t with t = phi_p / (2 pi) (G^{-1}
 * is increasing, so this is the p-quantile of the back-transformed states);
 * sampled sites get their data value.  out[k * nx*ny + i] for probs[k]. */
int oracle_quantiles(int nx, int ny, const double *z, const uint8_t *sampled, const double *states, int M,
                     const double *probs, int nq, const double *zmin_zmax, double *out)
{
    if (nx <= 0 || ny <= 0 || M < 1 || nq < 1) return O_ERR_ARG;
    for (int k = 0; k < nq; ++k)
        if (!(probs[k] >= 0.0 && probs[k] <= 1.0)) return O_ERR_ARG;
    long n = (long)nx * ny;
    double *v = (double *)malloc(sizeof(double) * M);
    for (long i = 0; i < n; ++i) {
        if (sampled[i]) {
            for (int k = 0; k < nq; ++k) out[k * n + i] = z[i];
            continue;
        }
        for (int m = 0; m < M; ++m) v[m] = states[(long)m * n + i];
        qsort(v, (size_t)M, sizeof(double), cmp_double);
        for (int k = 0; k < nq; ++k) {
            double t = quantile_sorted(v, M, probs[k]) / O_TWO_PI;
            out[k * n + i] = zmin_zmax[0] * (1.0 - t) + zmin_zmax[1] * t;
        }
    }
    free(v);
    return O_OK;
}

/* ---------------------------------------------------------- temperature */
/* Equation (ene): e(T, L) = <H> / N_GP from unconditional simulations (every
 * site free) at each temperature of the grid T[0..nT-1], the grid size fixed.
 * Start phi = pi, n_burn sweeps, then the mean of H/N_GP over n_meas sweeps;
 * the acceptance-driven rule for a runs throughout.  Chain index = T index. */
int oracle_energy_table(int nx, int ny, double q, int nT, const double *Tg, int n_burn,
                        int n_meas, double a_targ, double k_a, uint64_t seed, uint32_t stream,
                        double *e_out)
{
    if (nx <= 0 || ny <= 0 || nT < 1 || n_meas < 1 || n_burn < 0) return O_ERR_ARG;
    if ((long)nx * ny < 2) return O_ERR_DEGENERATE;
    long n = (long)nx * ny;
    double n_gp = (double)oracle_bond_count(nx, ny);
    double *s = (double *)malloc(sizeof(double) * n);
    uint8_t *free_mask = (uint8_t *)calloc((size_t)n, 1);
    for (int k = 0; k < nT; ++k) {
        for (long i = 0; i < n; ++i) s[i] = O_PI;
        double a = 1.0, acc_e = 0.0;
        for (int t = 0; t < n_burn + n_meas; ++t) {
            long acc = oracle_half_sweep(nx, ny, s, free_mask, 0, Tg[k], a, q, seed, (uint32_t)t,
                                         (uint32_t)k, stream, O_MODE_FULL, NULL);
            acc += oracle_half_sweep(nx, ny, s, free_mask, 1, Tg[k], a, q, seed, (uint32_t)t,
                                     (uint32_t)k, stream, O_MODE_FULL, NULL);
            double A = (double)acc / (double)n;
            if (A < a_targ) a = 1.0 + (double)(t + 1) / k_a;
            if (t >= n_burn) acc_e += oracle_energy(nx, ny, s, q) / n_gp;
        }
        e_out[k] = acc_e / (double)n_meas;
    }
    free(s);
    free(free_mask);
    return O_OK;
}

/* The temperature grid: nT points evenly spaced in log T over [T_lo, T_hi]. */
void oracle_temperature_grid(int nT, double T_lo, double T_hi, double *Tg)
{
    for (int k = 0; k < nT; ++k)
        Tg[k] = (nT == 1) ? T_lo : exp(log(T_lo) + (log(T_hi) - log(T_lo)) * (double)k / (double)(nT - 1));
}

/* T_hat = argmin_T |e_s - e(T, L)| (Section 2.3, Algorithm 2 step 4.2) read
 * off the table: y = log(1 + e) is made non-decreasing in T by pooling
 * adjacent violators, then log T is interpolated linearly in y.  Outside the
 * table's range the end temperature is returned and *clamped is set. */
int oracle_invert_temperature(int nT, const double *Tg, const double *e, double e_s,
                              double *T_hat, int *clamped)
{
    if (nT < 2) return O_ERR_ARG;
    double *y = (double *)malloc(sizeof(double) * nT);
    double *w = (double *)malloc(sizeof(double) * nT);
    int *len = (int *)malloc(sizeof(int) * nT);
    int nb = 0;
    for (int k = 0; k < nT; ++k) {
        double v = 1.0 + e[k];
        y[nb] = log(v > 1e-300 ? v : 1e-300);
        w[nb] = 1.0;
        len[nb] = 1;
        ++nb;
        while (nb > 1 && y[nb - 2] > y[nb - 1]) {
            double ww = w[nb - 2] + w[nb - 1];
            y[nb - 2] = (w[nb - 2] * y[nb - 2] + w[nb - 1] * y[nb - 1]) / ww;
            w[nb - 2] = ww;
            len[nb - 2] += len[nb - 1];
            --nb;
        }
    }
    double *yf = (double *)malloc(sizeof(double) * nT);
    for (int b = 0, k = 0; b < nb; ++b)
        for (int j = 0; j < len[b]; ++j) yf[k++] = y[b];
    double v = 1.0 + e_s;
    double ys = log(v > 1e-300 ? v : 1e-300);
    *clamped = 0;
    if (ys <= yf[0]) {
        *T_hat = Tg[0];
        *clamped = 1;
    } else if (ys >= yf[nT - 1]) {
        *T_hat = Tg[nT - 1];
        *clamped = 1;
    } else {
        int k = 0;
        while (!(yf[k + 1] >= ys && yf[k + 1] > yf[k])) ++k;
        double x0 = log(Tg[k]), x1 = log(Tg[k + 1]);
        *T_hat = exp(x0 + (ys - yf[k]) * (x1 - x0) / (yf[k + 1] - yf[k]));
    }
    free(y);
    free(w);
    free(len);
    free(yf);
    return O_OK;
}
