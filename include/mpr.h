/*
 * mpr.h - C ABI of the MI355X (gfx950) library for gap filling with the
 * modified planar rotator (MPR) model: Zukovic, Borovsky, Lach and
 * Hristopulos, "GPU-accelerated simulation of massive spatial data based on
 * the modified planar rotator model", arXiv:1811.01604.
 *
 * Problem (Section 2.1): an nx x ny grid of which some sites are sampled
 * (values z known) and the rest are gaps; the library predicts the gaps.
 * The calls follow the steps of Algorithm 2:
 *   mpr_map_to_angles        step 3   (equation "map")
 *   mpr_estimate_temperature step 4   (equations "mpr-sse" and "ene")
 *   mpr_simulate             steps 2, 5, 6 (Algorithm 1 sweeps, the stopping
 *                            rule, the equilibrium states)
 *   mpr_predict              steps 6.3 and 7 (back-transform of the mean)
 *
 * Conventions
 *  - Grids are row-major with x fastest: element (x, y) of image b is at
 *    index imgs[b].offset + y * imgs[b].nx + x of every per-site buffer.
 *  - (dev) pointers are device pointers on the context's device; (host)
 *    pointers are host memory.  The caller owns every buffer, including the
 *    device workspace sized by mpr_workspace_size.  The library does not
 *    allocate device memory in these calls (the mpr_diag_* calls excepted).
 *    Every call checks its (dev) pointers with hipPointerGetAttributes and
 *    refuses one that is not device memory of the context's device (or
 *    managed memory) with MPR_ERR_ARG; it cannot check their extent, which
 *    is the caller's to size as each call states.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued on it and every call synchronises the stream before it
 *    returns.
 *  - Sampled flags are uint8: nonzero = sampled (fixed), 0 = gap.
 *  - Every call returns MPR_OK (0) or an error code (mpr_simulate also
 *    MPR_INCOMPLETE, see mpr_params.sweep_limit); mpr_last_error gives a
 *    text for the most recent failure on the context.  No C++ exception
 *    crosses the boundary.  A context is used by one host thread at a time.
 */
#ifndef MPR_H
#define MPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPR_OK = 0,
    MPR_ERR_ARG = 1,         /* invalid argument (null pointer, bad size, non-finite sample) */
    MPR_ERR_DEGENERATE = 2,  /* data the method cannot handle, see each call */
    MPR_ERR_WORKSPACE = 3,   /* workspace smaller than mpr_workspace_size */
    MPR_ERR_HIP = 4,         /* a HIP runtime call failed */
    MPR_INCOMPLETE = 5       /* not an error: mpr_simulate stopped at params.sweep_limit with
                                chains still running (outputs not written; resume later) */
};

/* Flags of mpr_params.tile_rows (and the tile argument of
 * mpr_diag_half_sweep): the compacted sweep shape, and the fused tile sweep
 * (a whole sweep per launch on tiles of 8, 12, 16, 24, 32 or 48 rows x 128 columns
 * staged in LDS with a two-site halo; single precision only). */
#define MPR_TILE_COMPACT 0x100
#define MPR_TILE_FUSED 0x200
/* With MPR_TILE_FUSED (8, 12, 16, 24 or 32 rows): the fused sweeps of a chain
 * set whose tiles the GPU holds at once run many per cooperative launch, with
 * a grid barrier between sweeps (small fills; a set too large for that, or a
 * call that records states, runs the same rows one launch per sweep). */
#define MPR_TILE_PERSIST 0x400

typedef struct mpr_ctx mpr_ctx;

/* One image of a (possibly ragged) batch. */
typedef struct {
    int32_t nx, ny;   /* grid size; nx * ny >= 2 */
    int64_t offset;   /* element offset of the image in per-site buffers */
    uint32_t id;      /* random-stream id of the image (Philox counter word 3,
                         must be < 2^31); results depend on it, not on the
                         image's position in the batch */
    uint32_t reserved;
} mpr_image;

/* Simulation parameters (Algorithm 2 step 1.1, Section 2.3).  The paper
 * leaves the defaults to earlier work; mpr_default_params fills the values
 * this library uses. */
typedef struct {
    double q;             /* coupling exponent: 1/2 (Section 2.2), or 0 < q < 1/2 with
                             fp64 = 1 (the single-precision sweep is written for 1/2;
                             see mpr_select_q); other values: MPR_ERR_ARG */
    int32_t R;            /* independent chains per image */
    int32_t K;            /* equilibrium states per chain; M = R * K realizations */
    int32_t n_f;          /* slope checked every n_f sweeps ... */
    int32_t n_fit;        /* ... from the last n_fit energies (2..64) */
    int32_t sg_degree;    /* degree of the Savitzky-Golay fit (1..4) */
    int32_t i_max;        /* cap on relaxation sweeps (relaxation runs while t <= i_max) */
    double a_targ;        /* target acceptance ratio */
    double k_a;           /* a(i+1) = 1 + (i+1)/k_a when the acceptance ratio < a_targ */
    int32_t fixed_relax;  /* -1: stopping rule; >= 0: exactly this many relaxation sweeps */
    int32_t eq_a_mode;    /* 0: a = 1 in the equilibrium states (Algorithm 2 step 6.2);
                             1: keep the final relaxation a */
    /* e(T, L) table for the temperature (equation "ene"): table_nT
     * temperatures log-spaced over [table_T_lo, table_T_hi], unconditional
     * runs from phi = pi with table_burn + table_meas sweeps each. */
    int32_t table_nT;
    int32_t table_burn;
    int32_t table_meas;
    int32_t tile_rows;    /* sweep block shape: 1, 2, 4 or 8 half-rows x (256 / rows)
                             site pairs, or 2, 4 or 8 half-rows | MPR_TILE_COMPACT for
                             (1024 / rows) sites with the gap sites compacted onto
                             lanes, or 8, 12, 16, 24, 32 or 48 rows | MPR_TILE_FUSED for the fused
                             tile sweep (single precision; a double-precision run
                             takes the default shape instead); 0 = autotune
                             (results do not depend on it) */
    double table_T_lo, table_T_hi;
    uint64_t seed;        /* Philox key */
    int32_t sweeps_per_launch;  /* sweeps per captured graph between done-checks;
                                   0 = chosen from the measured sweep time */
    int32_t spread;       /* 1: also keep, per chain and site, the squared deviations
                             of the equilibrium states from their running mean (K > 1;
                             needed for mpr_simulate's phi_m2 then; more workspace) */
    int32_t fp64;         /* 1: the chains of mpr_simulate store and update their angles
                             in double precision (the paper's DP runs, Section 4, Tables
                             2 and 3); twice the workspace per chain; every block shape
                             (the e(T, L) table chains of q < 1/2 take the plain ones).
                             Inputs and outputs stay float; sums are taken in double and
                             rounded once.  The temperature estimate is unaffected. */
    int32_t table_side_cap;  /* 0: the e(T, L) table of an nx x ny image is built on nx x ny;
                                >= 2: on min(nx, cap) x min(ny, cap), so that the images larger
                                than cap share one table (e(T, L) approaches its L -> infinity
                                limit with an error of order 1/L; it trades that bias for a
                                table cost bounded by cap^2 sites).  1 is invalid. */
    int32_t warm_min_states; /* a call with phi_init (a warm start) needs K >= this many
                                equilibrium states per chain, else MPR_ERR_ARG: all chains
                                start from the same angles, and the realizations average out
                                that start only over enough equilibrium sweeps (with K = 1 the
                                state right after the stopping rule fires stays correlated with
                                it).  Default 100: on 2048^2 fields with 50% cloud gaps, 32
                                images, the warm start's MAE over the plain start's is
                                1.012 (95% interval up to 1.023) with K = 25 and 1.0045 (up
                                to 1.013) with K = 50, within 1.006 with K = 100.  0 turns
                                the check off (parity tests that start the oracle and the
                                library from the same angles). */
    int32_t sweep_limit;     /* > 0: mpr_simulate runs at most this many sweeps in this call
                                and returns MPR_INCOMPLETE if a chain is still running; the
                                workspace then holds the whole state of the run (a checkpoint:
                                its first mpr_workspace_size bytes, which may be copied to the
                                host and later back into any workspace); 0: run to the end */
    int32_t resume;          /* 1: mpr_simulate continues the run held in the workspace (left
                                by a call that returned MPR_INCOMPLETE, with the same images and
                                parameters apart from sweep_limit, resume, tile_rows and
                                sweeps_per_launch) instead of starting its chains; phi_init is
                                ignored.  Results equal those of an uninterrupted run bit for
                                bit (random numbers are keyed by sweep, not by call). */
    int32_t barrier_timeout_us; /* > 0: the longest a block of the persistent sweep
                                (MPR_TILE_PERSIST) waits at its grid barrier, in microseconds,
                                before the call gives up with MPR_ERR_HIP (every block then
                                leaves at its next barrier; the workspace contents are lost);
                                0: 2 seconds.  Results do not depend on it. */
} mpr_params;

/* Per chain results of mpr_simulate (R per image, image-major). */
typedef struct {
    int32_t relax_sweeps;   /* relaxation sweeps performed */
    int32_t not_converged;  /* 1 if i_max stopped the relaxation */
    double a_final;         /* a at the end of the relaxation */
    double A_last;          /* acceptance ratio of the last relaxation sweep */
    double k_last;          /* last energy slope */
} mpr_chain_stats;

/* Context on HIP device `device`.  Returns MPR_ERR_HIP if the device cannot
 * be used.  The context caches e(T, L) tables by grid size and parameters. */
int32_t mpr_create(mpr_ctx **ctx, int32_t device);
void mpr_destroy(mpr_ctx *ctx);
/* Text of the last error on ctx (valid until the next call on ctx). */
const char *mpr_last_error(const mpr_ctx *ctx);
/* Defaults: q=0.5, R=1, K=100, n_f=5, n_fit=20, sg_degree=1, i_max=20000,
 * a_targ=0.3, k_a=3, fixed_relax=-1, eq_a_mode=0, table 32 points over
 * [1e-5, 10], 200 + 400 sweeps, seed 3000, tile_rows=0 and
 * sweeps_per_launch=0 (automatic). */
void mpr_default_params(mpr_params *p);

/* Device workspace bytes needed by mpr_estimate_temperature and
 * mpr_simulate for this batch; < 0 on invalid arguments. */
int64_t mpr_workspace_size(const mpr_image *imgs, int32_t n_images, const mpr_params *p);

/* Equation (map): phi = 2 pi (z - z_min) / (z_max - z_min) at the sampled
 * sites, with z_min, z_max over the image's samples; gaps get 0.
 *   z        (dev, float)  data; gap values are ignored
 *   sampled  (dev, uint8)
 *   phi      (dev, float, out)
 *   zmin_zmax (host, double[2 * n_images], out)
 * The map is evaluated in double precision and rounded once, so sampled
 * angles are exactly 0 at z_min and the float nearest 2 pi at z_max.
 * Errors: MPR_ERR_ARG for a non-finite sampled z; MPR_ERR_DEGENERATE if an
 * image has fewer than 2 samples or z_max == z_min. */
int32_t mpr_map_to_angles(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                          const float *z, const uint8_t *sampled, float *phi,
                          double *zmin_zmax, void *stream);

/* Section 2.3, Algorithm 2 step 4: the sample specific energy e_s (equation
 * "mpr-sse", each unordered sample-sample nearest-neighbour pair once) and
 * T_hat with e(T_hat, L) = e_s.  e(T, L) (equation "ene") comes from
 * unconditional simulations on the image's grid size with this library's
 * own sweep, tabulated per mpr_params table_* fields, made monotone and
 * interpolated in (log T, log(1 + e)).  Tables are cached in ctx.
 *   phi, sampled (dev)  angles from mpr_map_to_angles
 *   workspace (dev)     ws_bytes >= mpr_workspace_size
 *   e_s, T_hat (host, double[n_images], out)
 *   t_clamped (host, int32[n_images], out, nullable): 1 when e_s lies
 *             outside the table and T_hat is the end temperature.
 * Errors: MPR_ERR_DEGENERATE when an image has no sample-sample pair. */
int32_t mpr_estimate_temperature(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                                 const float *phi, const uint8_t *sampled,
                                 const mpr_params *p, void *workspace, int64_t ws_bytes,
                                 double *e_s, double *T_hat, int32_t *t_clamped,
                                 void *stream);

/* Algorithm 2 steps 2, 5 and 6 with Algorithm 1 sweeps on the GPU, for all
 * images and R chains per image at once: every half-sweep is one launch over
 * the blocks of all chains of the (ragged) batch, and groups of sweeps are
 * replayed as a captured HIP graph.  Unless tile_rows is set, the first
 * sweeps of a new batch shape time each block shape and the fastest is kept
 * for that shape (cached in ctx).  Each chain starts from U(0, 2 pi)
 * gap angles (or phi_init), relaxes with the hybrid update until the energy
 * slope is >= 0 or i_max (or fixed_relax sweeps), then runs K equilibrium
 * sweeps.  Random numbers are Philox4x32-10 keyed by (seed; site, sweep,
 * chain, image id), so results do not depend on launch shapes or batch
 * composition.
 *   phi, sampled (dev)  sample angles (gap entries ignored)
 *   T_hat (host, double[n_images])
 *   phi_init (dev, float, nullable)  starting gap angles, reduced into [0, 2 pi)
 *           (sign cleared); needs K >= p->warm_min_states
 *   phi_sum (dev, float, out)  sum of the M = R*K states at gap sites, 0 at samples
 *   phi_m2 (dev, float, out, nullable)  sum over the M states of (phi - mean)^2
 *           at gap sites, 0 at samples (the realizations' spread; Algorithm 2
 *           step 7 returns statistics of the M realizations).  With K > 1 it
 *           needs p->spread = 1 (each chain keeps a running sum of squared
 *           deviations, Welford's update); chains are combined with the
 *           spread of their means.
 *   phi_states (dev, float, out, nullable)  every equilibrium state: state
 *           m = r*K + k (chain r after its k-th equilibrium sweep) of the site at
 *           packed position j is phi_states[m * N + j], N = max over images of
 *           offset + nx*ny (all sites of the image, samples included); M*N floats.
 *           Adds a pass over each chain's grid per equilibrium sweep.
 *   stats (host, mpr_chain_stats[n_images * R], out, nullable)
 * An image without gaps is left unchanged (phi_sum 0).
 * Errors: MPR_ERR_WORKSPACE if ws_bytes is too small; MPR_ERR_ARG for phi_m2
 * with K > 1 and p->spread = 0. */
int32_t mpr_simulate(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                     const float *phi, const uint8_t *sampled, const double *T_hat,
                     const mpr_params *p, const float *phi_init, void *workspace,
                     int64_t ws_bytes, float *phi_sum, float *phi_m2, float *phi_states,
                     mpr_chain_stats *stats, void *stream);

/* mpr_simulate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments without the workspace, which is instead a static
 * device array of mpr_simulate_noalloc_max_bytes() (64 MiB) that each GPU
 * the library runs on holds until the process ends.  Every sweep is
 * launched directly (no graph is instantiated); results equal
 * mpr_simulate's bit for bit.  The call allocates nothing (no hipMalloc,
 * hipFree or graph instantiation); the context was created earlier.
 * All calls on one GPU share its array: calls that overlap in time on the
 * same GPU (other threads, other contexts) race and must be serialised by
 * the caller.  The call returns after its work is complete.
 * Errors: as mpr_simulate, and MPR_ERR_WORKSPACE when the batch needs more
 * than mpr_simulate_noalloc_max_bytes() (mpr_workspace_size of the batch). */
int32_t mpr_simulate_noalloc(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                             const float *phi, const uint8_t *sampled, const double *T_hat,
                             const mpr_params *p, const float *phi_init, float *phi_sum,
                             float *phi_m2, float *phi_states, mpr_chain_stats *stats,
                             void *stream);
int64_t mpr_simulate_noalloc_max_bytes(void);

/* Algorithm 2 steps 6.3 and 7 with the mean as the statistic:
 * z_hat = z_min (1 - t) + z_max t with t = (phi_sum / M) / (2 pi) at gaps
 * (double precision, rounded once); sampled sites are copied bit-exactly.
 * All buffers (dev) except zmin_zmax (host). */
int32_t mpr_predict(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                    const float *z, const uint8_t *sampled, const float *phi_sum,
                    const double *zmin_zmax, int32_t M, float *z_hat, void *stream);

/* Learnable coupling exponent.  The paper fixes q = 1/2 (Section 2.2: any
 * q <= 1/2 keeps 0 and 2 pi apart) and gives no rule to choose it; this call
 * chooses q for one image from the candidates q_grid[0..nq-1] (each in
 * (0, 1/2], nq <= 64) by hold-out validation: the samples whose site uniform
 * (Philox4x32-10, key seed, counter (y nx + x, 0xFFFFFFFE, 0, 0x40000000),
 * word 0) is below `holdout` (0 < holdout < 1) are hidden; for each q the
 * remaining samples give T_hat(q) (mpr_estimate_temperature with p->q = q),
 * mpr_simulate (R, K of p; double-precision chains for q < 1/2) and
 * mpr_predict fill the hidden sites, scored by their mean absolute error.
 *   z, sampled (dev, the image at img->offset)
 *   val_mae (host, double[nq], out): the error for each candidate
 *   T_hat (host, double[nq], out, nullable): the temperature for each
 *   q_best (host, out): the candidate with the smallest error (on a tie, the
 *         larger q)
 *   workspace: mpr_select_q_workspace_size bytes (dev).
 * Errors: MPR_ERR_ARG for bad arguments or K < 1; MPR_ERR_DEGENERATE when no
 * sample is held out or too few remain. */
int64_t mpr_select_q_workspace_size(const mpr_image *img, const mpr_params *p, const double *q_grid,
                                    int32_t nq);
int32_t mpr_select_q(mpr_ctx *ctx, const mpr_image *img, const float *z, const uint8_t *sampled,
                     const mpr_params *p, const double *q_grid, int32_t nq, double holdout,
                     void *workspace, int64_t ws_bytes, double *val_mae, double *T_hat,
                     double *q_best, void *stream);

/* Quantiles of the prediction (Algorithm 2 step 7, statistics of the M
 * realizations): at each gap site the probs[k]-quantile of the M states of
 * phi_states (as written by mpr_simulate; M <= 256), by linear interpolation
 * between the order statistics around h = (M - 1) p (Hyndman and Fan's
 * definition 7), back-transformed like the mean, z = z_min (1 - t) + z_max t
 * with t = phi_p / (2 pi) (double precision, rounded once); sampled sites get
 * their data value z.  z_q[k * N + j] (N as for phi_states) for 1 <= nq <= 64
 * probabilities in [0, 1].
 *   z, sampled, phi_states, z_q (out): dev; probs, zmin_zmax: host.
 * Errors: MPR_ERR_ARG for M or nq out of range or p outside [0, 1]. */
int32_t mpr_quantiles(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images, const float *z,
                      const uint8_t *sampled, const float *phi_states, int32_t M,
                      const double *probs, int32_t nq, const double *zmin_zmax, float *z_q,
                      void *stream);

/* Spread of the prediction (Algorithm 2 step 7, statistics of the M
 * realizations besides their mean): z_std = standard deviation over the M
 * states of G^{-1}(phi) = (z_max - z_min) / (2 pi) sqrt(phi_m2 / (M - 1)) at
 * gap sites; 0 at sampled sites and when M = 1.
 *   sampled, phi_m2 (from mpr_simulate), z_std (out): dev; zmin_zmax: host. */
int32_t mpr_spread(mpr_ctx *ctx, const mpr_image *imgs, int32_t n_images,
                   const uint8_t *sampled, const float *phi_m2, const double *zmin_zmax,
                   int32_t M, float *z_std, void *stream);

/* ------------------------------------------------------------------ */
/* Warm start: a residual CNN that predicts starting gap angles from the
 * sampled ones (replacing the U(0, 2 pi) start of Algorithm 2 step 2.2;
 * the chain then runs to the same stopping rule).  Architecture: input
 * (cos q phi, sin q phi, 1) at sampled sites, 0 at gaps, zero-padded to 32
 * channels; stem conv + ReLU; 8 blocks h <- h + conv(ReLU(conv(h))); head
 * conv whose channels 0, 1 estimate (cos q phi, sin q phi).  All convs are
 * 3x3, 32 -> 32 channels, zero padding; bfloat16 weights and activations,
 * float accumulation on the matrix cores.
 *
 * Tensors: x, y, dy are NHWC bfloat16 (n x h x w x 32) device buffers;
 * phi, target and sampled are n x h x w (target: 2 floats per site, the
 * (cos q phi, sin q phi) to learn).  params (float, mpr_cnn_param_count())
 * holds per layer W[tap][c_in][c_out] (tap = 3 (dy+1) + (dx+1)) then
 * b[c_out], 18 layers (stem, 8 x 2 block convs, head); grads has the same
 * layout.  packed (mpr_cnn_packed_bytes()) holds the bfloat16 copies the
 * kernels read; refresh it with mpr_cnn_pack after every parameter change. */
int64_t mpr_cnn_param_count(void);
int64_t mpr_cnn_packed_bytes(void);
/* Device workspace for forward (training = 0: inference, 1: keep the
 * activations for mpr_cnn_backward) on n images of h x w; < 0 if invalid. */
int64_t mpr_cnn_workspace_size(int32_t n, int32_t h, int32_t w, int32_t training);
int32_t mpr_cnn_pack(mpr_ctx *ctx, const float *params, void *packed, void *stream);
int32_t mpr_cnn_encode(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *phi,
                       const uint8_t *sampled, void *x, void *stream);
int32_t mpr_cnn_forward(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params,
                        const void *packed, const void *x, void *ws, int64_t ws_bytes,
                        int32_t training, void *y, void *stream);
/* Mean over the n_gaps gap sites of the squared (cos, sin) error of y's
 * channels 0, 1 (host *loss), and its gradient dy (all 32 channels; zero at
 * sampled sites).  ws needs 8 bytes per 256 sites. */
int32_t mpr_cnn_loss(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *y,
                     const float *target, const uint8_t *sampled, int64_t n_gaps, void *dy,
                     void *ws, int64_t ws_bytes, double *loss, void *stream);
/* Gradients of every layer from dy, using the activations a training
 * forward pass left in ws (same ws, same x). */
int32_t mpr_cnn_backward(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params,
                         const void *packed, const void *x, const void *dy, void *ws,
                         int64_t ws_bytes, float *grads, void *stream);
/* One Adam step (bias-corrected; step counts from 1) on params with moment
 * buffers m, v (float, zero-initialised by the caller). */
int32_t mpr_cnn_opt_step(mpr_ctx *ctx, float *params, const float *grads, float *m, float *v,
                         int64_t step, double lr, double beta1, double beta2, double eps,
                         void *stream);
/* Starting angles at gap sites: phi = atan2(max(s, 0), c) / q, capped below
 * 2 pi (the gap entries of phi_init for mpr_simulate; 0 at samples). */
int32_t mpr_cnn_decode(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *y,
                       const uint8_t *sampled, float *phi_init, void *stream);
/* The warm start in one call: mpr_cnn_encode, mpr_cnn_forward (inference)
 * and mpr_cnn_decode with the same results bit for bit, the encoding done
 * while the stem stages its input and the decoding in the head's epilogue
 * (no x or y tensor).  phi, sampled, phi_init: n x h x w (dev); workspace:
 * mpr_cnn_workspace_size(n, h, w, 0) bytes (dev). */
int32_t mpr_cnn_infer(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params,
                      const void *packed, const float *phi, const uint8_t *sampled, void *ws,
                      int64_t ws_bytes, float *phi_init, void *stream);
/* Diagnostics: one conv layer (wpack in the forward or dgrad layout of
 * mpr_cnn_pack; bias, add, ref nullable: out = ReLU?(conv + bias + add),
 * zeroed where ref <= 0), and one layer's weight and bias gradients
 * (grads: 9*32*32 + 32 floats; gout multiplied by (gref > 0) when gref is
 * given; ws >= 256*4*(9*32*32+32)*4 bytes). */
int32_t mpr_cnn_diag_conv(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *in,
                          const void *wpack, const float *bias, const void *add, const void *ref,
                          int32_t relu, void *out, void *stream);
int32_t mpr_cnn_diag_wgrad(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *in,
                           const void *gout, const void *gref, float *grads, void *ws,
                           int64_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Profiling.  While enabled, mpr_simulate and mpr_estimate_temperature
 * bracket every sweep's two half-sweep launches with HIP events on the
 * caller's stream, and count the work done: chain-sweeps, gap-site updates
 * and the method's useful HBM bytes (4 bytes per site read + 4 per gap site
 * written, per chain-sweep).  mpr_profile_read returns the totals since the
 * last mpr_profile_enable(ctx, 1). */
typedef struct {
    double sweep_kernel_ms;   /* summed event time of the half-sweep launches */
    int64_t sweep_launches;   /* half-sweep launches timed */
    int64_t chain_sweeps;     /* sweeps summed over chains that were active */
    int64_t site_updates;     /* gap-site updates summed over those sweeps */
    double useful_bytes;      /* sum of (4 nx ny + 4 P) over those sweeps */
    int32_t last_tile;        /* block shape of the last simulation's sweeps, as
                                 mpr_params.tile_rows (rows | MPR_TILE_COMPACT) */
    int32_t reserved;
} mpr_profile;

int32_t mpr_profile_enable(mpr_ctx *ctx, int32_t on);
int32_t mpr_profile_read(mpr_ctx *ctx, mpr_profile *out);

/* ------------------------------------------------------------------ */
/* Diagnostics: the production kernels on one grid, for parity testing.
 * These calls allocate scratch device memory and synchronise. */

/* Philox4x32-10 of n counters (dev, uint32[4n]) with key `seed`, into out
 * (dev, uint32[4n]). */
int32_t mpr_diag_philox(mpr_ctx *ctx, const uint32_t *ctr, uint64_t seed, int64_t n,
                        uint32_t *out, void *stream);

/* One half-sweep (Algorithm 1 on the gap sites of one checkerboard colour,
 * colour = (x + y) & 1) of an nx x ny grid in place.
 *   phi (dev, float, in/out), sampled (dev, uint8)
 *   mode 0: full hybrid update; 1: over-relaxation only
 *   tile: block shape as mpr_params.tile_rows (0 = 4 half-rows, plain);
 *         every shape gives the same results
 *   flags (dev, uint8, out, nullable): per site bit 0 = reflection kept the
 *         spin, bit 1 = proposal accepted, bit 2 = proposal wrapped,
 *         bit 3 = site updated, bit 4 = decided by the double-precision path
 *   accepted (host, int64, out, nullable)
 *   bond_energy (host, double, out, nullable): for colour 1, the sweep's own
 *         accumulation of H + N_GP = sum over bonds of (1 - cos(q dphi))
 *         after the update (every bond has one colour-1 end)
 * (sweep, chain, stream_id) select the random numbers as in mpr_simulate. */
int32_t mpr_diag_half_sweep(mpr_ctx *ctx, int32_t nx, int32_t ny, float *phi,
                            const uint8_t *sampled, int32_t colour, double T, double a,
                            double q, uint64_t seed, uint32_t sweep, uint32_t chain,
                            uint32_t stream_id, int32_t mode, int32_t tile, uint8_t *flags,
                            int64_t *accepted, double *bond_energy, void *stream);

/* mpr_diag_half_sweep for a grid of double angles (phi: dev, double,
 * in/out) through the double-precision sweep of mpr_params.fp64: the same
 * arguments (tile: any shape, plain or MPR_TILE_COMPACT), flags bit 4 set at every updated
 * site, and bond_energy summed in fixed point of 2^-30. */
int32_t mpr_diag_half_sweep_fp64(mpr_ctx *ctx, int32_t nx, int32_t ny, double *phi,
                                 const uint8_t *sampled, int32_t colour, double T, double a,
                                 double q, uint64_t seed, uint32_t sweep, uint32_t chain,
                                 uint32_t stream_id, int32_t mode, int32_t tile, uint8_t *flags,
                                 int64_t *accepted, double *bond_energy, void *stream);

/* H + N_GP of an nx x ny grid of angles (dev, float) as the simulation
 * accumulates it: sum over bonds of (1 - cos(q (phi_i - phi_j))) in fixed
 * point; returned in double (host). */
int32_t mpr_diag_energy(mpr_ctx *ctx, int32_t nx, int32_t ny, const float *phi, double q,
                        double *h_plus_ngp, void *stream);

/* Plain device copy of `bytes` (multiple of 16, 16-byte aligned pointers):
 * the known-size reference for calibrating HBM byte counters. */
int32_t mpr_diag_copy(mpr_ctx *ctx, const void *src, void *dst, int64_t bytes, void *stream);

/* The device stopping-rule slope: derivative at the newest point of the
 * degree-`degree` least-squares polynomial through e[0..n-1] (host). */
int32_t mpr_diag_sg_slope(mpr_ctx *ctx, const double *e, int32_t n, int32_t degree,
                          double *slope);

#ifdef __cplusplus
}
#endif

#endif /* MPR_H */
