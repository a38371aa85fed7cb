// MI355X (gfx950) implementation of the C ABI in include/mpr.h: MPR gap
// filling with the checkerboard hybrid Monte Carlo sweep (arXiv:1811.01604,
// Algorithms 1 and 2, Section 3.3).
//
// Kernels
//   init_chains       gap angles U(0, 2 pi) from Philox (Algorithm 2 step 2.2)
//                     or a warm start; samples stored with the sign bit set
//   half_sweep        Algorithm 1 on the gap sites of one colour for every
//                     chain; the colour-1 pass also sums all bond energies
//                     (every bond has exactly one colour-1 end) and both
//                     passes count accepted proposals
//   control           Algorithm 2 steps 5.2-5.5 and 6 per chain: a-rule,
//                     e(i+1), Savitzky-Golay slope, phase changes
//   finalize          sum of the M states per gap site
//   map_*, predict    equation (map) and its inverse
//   sample_energy     equation (mpr-sse)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/mpr.h"
#include "mpr_device.h"

static_assert(sizeof(mpr_params) == 128, "mpr_params layout");

using namespace mpr;

namespace {

constexpr int kBlock = 256;
constexpr int kMapBlocks = 512;          // partial-result blocks per image at most (map, e_s)
constexpr int kHoldoutBlocks = 64;       // partial-result blocks of the hold-out error
constexpr size_t kScratchBytes = 8u << 20;
constexpr uint32_t kTableStream = 0x80000000u;
constexpr uint32_t kInitSweep = 0xFFFFFFFFu;
// Layout of the context's device scratch: fixed slots, then a region for
// per-call partial results.
constexpr int64_t kDoneOffset = 0;       // done-chain counter
constexpr int64_t kTicketOffset = 256;   // last-block ticket of the redo kernel with the control fused
constexpr int64_t kGenOffset = 512;      // barrier generation of the persistent sweep
constexpr int64_t kAbortOffset = 768;    // barrier time-out word of the persistent sweep
constexpr int64_t kSlotsOffset = 16384;  // per-chain sweep sums of the persistent sweep (32 bytes a chain)
constexpr int64_t kWorkOffset = 1024;    // three work counters (profiling)
constexpr int64_t kEnergyOffset = 2048;  // diag energy accumulator
constexpr int64_t kSlopeOffset = 4096;   // diag slope input / output
constexpr int64_t kVarOffset = 65536;    // per-call partials
constexpr int64_t kHostWordsBytes = 1024;      // pinned mirror of the control words
constexpr int64_t kHostStageBytes = 64 << 10;  // pinned host block (control words + staging)
static_assert(kAbortOffset + 4 <= kHostWordsBytes && kGenOffset + 4 <= kHostWordsBytes,
              "the control words are read back in one copy");
constexpr int kCompactSites = 4 * kBlock;  // sites per block of the compacted sweep shapes
constexpr int kRecordSegs = 32;            // blocks per chain of record_states_kernel
constexpr int kWarmMinStates = 100;        // default of mpr_params.warm_min_states

// Workspace of mpr_simulate_noalloc, for callers that cannot allocate: one
// copy per device, held by the library's code object until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns on each device, kept per device by static_ws_addr.
constexpr int64_t kStaticWorkspaceBytes = (int64_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char static_workspace[kStaticWorkspaceBytes];

// Sites whose single-precision decision is too close to call are not written
// by the sweep kernels: they set the site's bit in their block's mask (one
// bit per site of the block, site = 2 pair + slot) and the block's bit in a
// bitmap, and redo_fp64_kernel redoes them in double precision afterwards.
// Keeping the double-precision code out of the sweep kernels keeps them at
// fewer than 64 registers.
struct Redo {
    uint32_t *mask;    // words_per_block per sweep block (flattened block index)
    uint32_t *blocks;  // one bit per sweep block
};

__device__ __forceinline__ void defer_redo(const Redo &rd, uint32_t gb, int words, uint32_t idx)
{
    atomicOr(&rd.mask[(size_t)gb * words + (idx >> 5)], 1u << (idx & 31u));
    atomicOr(&rd.blocks[gb >> 5], 1u << (gb & 31u));
}

// Parameters of the control kernel.
struct CtlParams {
    double a_targ, k_a, q;
    double e_unit;        // energy fixed-point unit of the sweep kernels
    int32_t angle_bytes;  // bytes per stored angle (4 or 8), for the work counters
    int32_t n_f, n_fit, i_max, fixed_relax, eq_a_mode, K, burn, meas;
    double w[kMaxFit];  // Savitzky-Golay derivative weights, oldest first
};

struct ImgDev {
    int64_t offset;
    int32_t nx, ny;
};

}  // namespace

// ====================================================================== kernels

// Slope of the energy series from the ring buffer: sum_j w_j e(t+1-n_fit+j).
__device__ double ring_slope(const double *ring, uint32_t t, int n_fit, const double *w)
{
    double s = 0.0;
    for (int j = 0; j < n_fit; ++j) {
        // e(t + 1 - n_fit + j) was stored at slot (t + 1 - n_fit + j) mod n_fit
        const uint32_t idx = (t + 1u + (uint32_t)j) % (uint32_t)n_fit;
        s += w[j] * ring[idx];
    }
    return s;
}

// (fp64: the chains hold doubles; a gap starts at 2 pi u in double, as in
// the plain definition.)
__global__ void init_chains_kernel(const ChainDesc *__restrict__ descs, const int64_t *__restrict__ offsets,
                                   const float *__restrict__ phi, const uint8_t *__restrict__ sampled,
                                   const float *__restrict__ phi_init, uint32_t seed_lo, uint32_t seed_hi,
                                   int table_mode, int fp64)
{
    const ChainDesc d = descs[blockIdx.y];
    const int64_t n = (int64_t)d.nx * d.ny;
    const int64_t off = offsets[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / d.nx);
        const int x = (int)(i - (int64_t)y * d.nx);
        const int c = (x + y) & 1;
        const int h = x >> 1;
        double v;
        bool fixed = false;
        if (table_mode) {
            v = kPi;
        } else if (sampled[off + i]) {
            v = (double)fabsf(phi[off + i]);
            fixed = true;
        } else if (phi_init) {
            // a given start is reduced into [0, 2 pi) with its sign bit clear
            // (a set sign bit marks a sampled site; -0.0 included)
            v = (double)phi_init[off + i];
            if (!(v >= 0.0 && v < kTwoPi)) {
                v -= kTwoPi * floor(v / kTwoPi);
                if (!(v >= 0.0 && v < kTwoPi)) v = 0.0;
            }
            v = fabs(v);
            if (!fp64 && (float)v >= 6.28318548f) v = 6.28318501;  // the largest float below 2 pi
        } else {
            U4 ctr = {(uint32_t)y * (uint32_t)d.nx + ((uint32_t)x & ~2u), kInitSweep, d.chain, d.image_id};
            const U4 w = philox4x32_10(ctr, seed_lo, seed_hi);
            const uint32_t word = ((x >> 1) & 1) ? w.z : w.x;
            v = kTwoPi * (double)unit24(word);
        }
        const int64_t j = (int64_t)y * d.S + h;
        // select by value: indexing the descriptor with c would put it in memory
        float *hp = c ? d.h[1] : d.h[0];
        float *ap = c ? d.acc[1] : d.acc[0];
        float *mp = c ? d.m2[1] : d.m2[0];
        if (fp64) {
            ((double *)hp)[j] = fixed ? mark_fixed_d(v) : v;
            if (ap) ((double *)ap)[j] = 0.0;
            if (mp) ((double *)mp)[j] = 0.0;
        } else {
            const float hv = fixed ? mark_fixed((float)v) : (float)v;
            hp[j] = hv;
            float *h2 = c ? d.h2[1] : d.h2[0];
            if (h2) h2[j] = hv;
            if (ap) ap[j] = 0.0f;
            if (mp) mp[j] = 0.0f;
        }
    }
}

// A full row-major grid of double angles (gaps: the starting state) into the
// half-grids of one double-precision chain, samples marked.
__global__ void split_fp64_kernel(const ChainDesc *__restrict__ descs, const double *__restrict__ phi,
                                  const uint8_t *__restrict__ sampled)
{
    const ChainDesc d = descs[0];
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / d.nx);
        const int x = (int)(i - (int64_t)y * d.nx);
        const double v = fabs(phi[i]);
        double *hp = (double *)(((x + y) & 1) ? d.h[1] : d.h[0]);
        hp[(int64_t)y * d.S + (x >> 1)] = sampled[i] ? mark_fixed_d(v) : v;
    }
}

// Chain of a flattened block index: start[c] <= b < start[c + 1].  The
// search runs on block-uniform values, so it stays in scalar registers.
__device__ __forceinline__ int find_chain(const int64_t *__restrict__ start, int n, int64_t b)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The blocks of a sweep launch, laid end to end over the chains it covers
// (the chains not yet done): launch chain k < n owns blocks start[k] <= b <
// start[k + 1] and is chain id[k] of the chain set.
struct BlockMap {
    const int64_t *start;
    const int32_t *id;
    int32_t n;
    int32_t pad;
};

// Chain of block b, and the block's index within that chain.
__device__ __forceinline__ int chain_of_block(const BlockMap &bm, int64_t b, int *local)
{
    const int k = find_chain(bm.start, bm.n, b);
    *local = (int)(b - bm.start[k]);
    return bm.id[k];
}

// Half-sweep of colour `colour` for every chain of a (possibly ragged)
// batch in one launch.  The blocks of all chains are laid end to end
// (start[] = prefix sums of blocks per chain).  A 256-thread block covers
// ROWS half-rows x (256 / ROWS) site pairs; each thread takes the two
// neighbouring sites h0 = 2k and h0 + 1 of one half-row, which share one
// Philox call.  Results do not depend on ROWS: random numbers are keyed by
// site and energies are summed in fixed point.
template <bool DIAG, int ROWS>
__device__ __forceinline__ void half_sweep_body(const ChainDesc *__restrict__ descs,
                                                ChainState *__restrict__ states,
                                                BlockMap bm, int colour,
                                                SweepConsts sc, int or_only, Redo rd, uint8_t *__restrict__ flags)
{
    constexpr int PX = kBlock / ROWS;
    int lb;
    const int c = chain_of_block(bm, (int64_t)blockIdx.x, &lb);
    ChainState *stp = states + c;
    const int phase = stp->phase;
    if (phase == PH_DONE) return;
    const ChainDesc d = descs[c];
    const int nbx = ((d.S >> 1) + PX - 1) / PX;
    const int by = lb / nbx;
    const int bx = lb - by * nbx;
    const int y = by * ROWS + (int)(threadIdx.x / PX);
    const int h0 = 2 * (bx * PX + (int)(threadIdx.x % PX));
    const uint32_t sweep = stp->sweep;
    const float inv_T = stp->inv_T, dscale = stp->dscale;
    const bool want_energy = (colour == 1) && (phase != PH_EQ);
    const bool want_acc = phase != PH_EQ;
    uint32_t e_thread = 0u, acc_thread = 0u;

    if (y < d.ny) {
        const int s = (y + colour) & 1;
        const int W = (d.nx - s + 1) >> 1;
        const int Wo = (d.nx + s) >> 1;
        if (h0 < W) {
            const bool two = (h0 + 1) < W;
            // select by value: indexing d.h with a runtime colour would put
            // the descriptor in memory
            float *mine = colour ? d.h[1] : d.h[0];
            const float *oth = colour ? d.h[0] : d.h[1];
            const int row = y * d.S;
            const bool vL = h0 + s - 1 >= 0, vM = h0 + s < Wo, vR = h0 + s + 1 < Wo;
            const bool vU = y > 0, vD = y + 1 < d.ny;
            // every load is issued, from a clamped in-row position when the
            // neighbour is missing (update_site ignores it by its valid bit),
            // so that all of them are in flight at once
            const float2 v = gldi2(mine, (uint32_t)(row + h0));
            const float oL = angle_of(gldi(oth, (uint32_t)(row + max(h0 + s - 1, 0))));
            const float oM = angle_of(gldi(oth, (uint32_t)(row + h0 + s)));  // h0 + s <= S - 1
            const float oR = angle_of(gldi(oth, (uint32_t)(row + min(h0 + s + 1, d.S - 1))));
            float2 up = gldi2(oth, (uint32_t)(row + (vU ? -d.S : 0) + h0));
            float2 dn = gldi2(oth, (uint32_t)(row + (vD ? d.S : 0) + h0));
            up.x = angle_of(up.x);
            up.y = angle_of(up.y);
            dn.x = angle_of(dn.x);
            dn.y = angle_of(dn.y);
            const bool fixed0 = is_fixed(v.x), fixed1 = !two || is_fixed(v.y);
            const float a0 = angle_of(v.x), a1 = angle_of(v.y);
            float u0 = 0.5f, r0 = 0.5f, u1 = 0.5f, r1 = 0.5f;
            if (!or_only && (!fixed0 || !fixed1)) {
                const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * h0 + s), sweep, d.chain, d.image_id};
                const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
                u0 = unit24(w.x);
                r0 = unit24(w.y);
                u1 = unit24(w.z);
                r1 = unit24(w.w);
            }
            // site h0: left oL, right oM, up, down; site h0 + 1: left oM, right oR
            const uint32_t val0 = (vL ? 1u : 0u) | (vM ? 2u : 0u) | (vU ? 4u : 0u) | (vD ? 8u : 0u);
            const uint32_t val1 = 1u | (vR ? 2u : 0u) | (vU ? 4u : 0u) | (vD ? 8u : 0u);
            bool n0 = true, n1 = true;
            SiteOut o0 = update_site(a0, oL, oM, up.x, dn.x, val0, u0, r0, inv_T, dscale, or_only != 0, &n0);
            SiteOut o1 = update_site(a1, oM, oR, up.y, dn.y, val1, u1, r1, inv_T, dscale, or_only != 0, &n1);
            // too close to call: left unchanged here, redone in double precision
            n0 = n0 && !fixed0;
            n1 = n1 && !fixed1;
            if (n0) defer_redo(rd, blockIdx.x, 2 * kBlock / 32, 2u * threadIdx.x);
            if (n1) defer_redo(rd, blockIdx.x, 2 * kBlock / 32, 2u * threadIdx.x + 1u);
            const bool w0 = !fixed0 && !n0, w1 = two && !fixed1 && !n1;  // sites written here
            const float out0 = w0 ? o0.phi : v.x;
            const float out1 = w1 ? o1.phi : v.y;
            if (two) {
                v2f w;
                w.x = out0;
                w.y = out1;
                *(gv2f *)gaddr(mine, (uint32_t)(row + h0)) = w;
            } else if (w0) {
                gsti(mine, (uint32_t)(row + h0), out0);
            }
            float *accp = colour ? d.acc[1] : d.acc[0];
            if (phase == PH_EQ && accp) {
                float *m2p = colour ? d.m2[1] : d.m2[0];
                const float ik = stp->inv_k, ikm1 = stp->inv_km1;
                if (w0) accumulate_state_i(accp, m2p, (uint32_t)(row + h0), out0, ik, ikm1);
                if (w1) accumulate_state_i(accp, m2p, (uint32_t)(row + h0 + 1), out1, ik, ikm1);
            }
            acc_thread = (w0 && o0.accepted ? 1u : 0u) + (w1 && o1.accepted ? 1u : 0u);
            // a sampled site's bonds are unchanged by this half-sweep
            if (want_energy)
                e_thread = (fixed0 ? energy_fx(o0.e_before) : (w0 ? energy_fx(o0.e_bonds) : 0u)) +
                           (!two ? 0u : fixed1 ? energy_fx(o1.e_before) : (w1 ? energy_fx(o1.e_bonds) : 0u));
            if (DIAG && flags) {
                const int64_t x0 = 2 * h0 + s;
                if (w0) flags[(int64_t)y * d.nx + x0] = (uint8_t)o0.flags;
                if (w1) flags[(int64_t)y * d.nx + x0 + 2] = (uint8_t)o1.flags;
            }
        }
    }
    if (!want_acc) return;
    // Block sums of the energy (split in 16-bit halves so that 32-bit lane
    // sums cannot overflow) and of the accepted count (packed in the top byte).
    uint32_t lo = (e_thread & 0xFFFFu) | (acc_thread << 24);
    uint32_t hi = e_thread >> 16;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off);
        hi += __shfl_xor(hi, off);
    }
    __shared__ uint32_t red[2][kBlock / 64];
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wid] = lo;
        red[1][wid] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0ull, a = 0ull;
        for (int i = 0; i < kBlock / 64; ++i) {
            e += ((unsigned long long)red[1][i] << 16) + (red[0][i] & 0xFFFFFFu);
            a += red[0][i] >> 24;
        }
        if (e) atomicAdd(&stp->e_fx, e);
        if (a) atomicAdd(&stp->acc, a);
    }
}

template <bool DIAG, int ROWS>
__global__ __launch_bounds__(kBlock) void half_sweep_kernel(const ChainDesc *__restrict__ descs,
                                                            ChainState *__restrict__ states,
                                                            BlockMap bm,
                                                            int colour, SweepConsts sc, int or_only, Redo rd,
                                                            uint8_t *__restrict__ flags)
{
    half_sweep_body<DIAG, ROWS>(descs, states, bm, colour, sc, or_only, rd, flags);
}

// The same sweep for the unconditional e(T, L) runs (a separate symbol so
// that profiles tell the two workloads apart).
template <int ROWS>
__global__ __launch_bounds__(kBlock) void table_half_sweep_kernel(const ChainDesc *__restrict__ descs,
                                                                  ChainState *__restrict__ states,
                                                                  BlockMap bm, int colour, SweepConsts sc, Redo rd)
{
    half_sweep_body<false, ROWS>(descs, states, bm, colour, sc, 0, rd, nullptr);
}

// The same half-sweep with the gap sites compacted onto consecutive lanes
// (q = 1/2 only).  A block covers CR half-rows x (1024 / CR) sites, two
// site pairs per thread.  Pass 1 (one lane per pair) reads the pairs, draws
// the pair's Philox words and lists the block's gap sites in site order in
// LDS (wave ballots + a prefix over the block's waves); pass 2 runs the
// update for the listed sites, 256 at a time, so sampled sites cost no
// update lanes; pass 3 gives sampled sites of colour 1 their bond energies
// when the sweep's energy is wanted.  Every site gets the arithmetic of the
// plain kernel, so the results are bit-identical to it.
template <bool DIAG, int CR>
__device__ __forceinline__ void half_sweep_compact_body(const ChainDesc *__restrict__ descs,
                                                        ChainState *__restrict__ states,
                                                        BlockMap bm,
                                                        int colour, SweepConsts sc, int or_only, Redo rd,
                                                        uint8_t *__restrict__ flags)
{
    constexpr int PPR = kCompactSites / CR / 2;  // site pairs per block row
    constexpr int NW = kBlock / 64;
    // list entry: Philox words for u and r (top 24 bits each) and the site's
    // index in the block (10 bits: low 8 in the u word, high 2 in the r word)
    __shared__ uint2 gap_list[kCompactSites];
    __shared__ uint16_t fixed_list[kCompactSites];
    __shared__ uint32_t wave_count[2][2][NW];  // [list][pair of the thread][wave]
    __shared__ uint32_t red[2][NW];

    int lb;
    const int c = chain_of_block(bm, (int64_t)blockIdx.x, &lb);
    ChainState *stp = states + c;
    const int phase = stp->phase;
    if (phase == PH_DONE) return;
    const ChainDesc d = descs[c];
    const int nbx = ((d.S >> 1) + PPR - 1) / PPR;
    const int by = lb / nbx;
    const int bx = lb - by * nbx;
    const uint32_t sweep = stp->sweep;
    const float inv_T = stp->inv_T, dscale = stp->dscale;
    const bool want_energy = (colour == 1) && (phase != PH_EQ);
    const bool want_acc = phase != PH_EQ;
    float *const mine_base = colour ? d.h[1] : d.h[0];
    const float *const oth_base = colour ? d.h[0] : d.h[1];
    float *const acc_base = (phase == PH_EQ) ? (colour ? d.acc[1] : d.acc[0]) : nullptr;
    float *const m2_base = acc_base ? (colour ? d.m2[1] : d.m2[0]) : nullptr;

    // pass 1: pairs t and t + 256 of the block; both pairs are read before
    // either draws its random numbers, so that the two loads overlap
    bool gap[2][2], fix[2][2];
    uint32_t wu[2][2], wr[2][2];
    float2 pv[2];
    bool in[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pi = (int)threadIdx.x + j * kBlock;
        const int y = by * CR + pi / PPR;
        const int h0 = 2 * (bx * PPR + pi % PPR);
        const int s = (y + colour) & 1;
        in[j] = y < d.ny && h0 < ((d.nx - s + 1) >> 1);
        // rows and pairs outside the grid read pair 0 of row 0 instead
        pv[j] = gldi2(mine_base, in[j] ? (uint32_t)(y * d.S + h0) : 0u);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pi = (int)threadIdx.x + j * kBlock;
        const int y = by * CR + pi / PPR;
        const int h0 = 2 * (bx * PPR + pi % PPR);
        const int s = (y + colour) & 1;
        const bool two = in[j] && (h0 + 1) < ((d.nx - s + 1) >> 1);
        gap[j][0] = in[j] && !is_fixed(pv[j].x);
        gap[j][1] = two && !is_fixed(pv[j].y);
        fix[j][0] = want_energy && in[j] && !gap[j][0];
        fix[j][1] = want_energy && two && !gap[j][1];
        wu[j][0] = wu[j][1] = wr[j][0] = wr[j][1] = 0u;
        if (!or_only && (gap[j][0] || gap[j][1])) {
            const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * h0 + s), sweep, d.chain, d.image_id};
            const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
            wu[j][0] = w.x;
            wr[j][0] = w.y;
            wu[j][1] = w.z;
            wr[j][1] = w.w;
        }
    }
    // positions in the two lists: pair j = 0 of every thread first, then j = 1
    const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // (the list of sampled sites is only wanted for the sweep's energy: the
    // block-uniform test skips its half of the work in the other half-sweeps)
    uint32_t pre[2][2] = {{0u, 0u}, {0u, 0u}};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
        if (L == 1 && !want_energy) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint64_t b0 = __ballot(L ? fix[j][0] : gap[j][0]);
            const uint64_t b1 = __ballot(L ? fix[j][1] : gap[j][1]);
            pre[L][j] = (uint32_t)(__popcll(b0 & below) + __popcll(b1 & below));
            if (lane == 0) wave_count[L][j][wid] = (uint32_t)(__popcll(b0) + __popcll(b1));
        }
    }
    __syncthreads();
    int n_list[2] = {0, 0};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
        if (L == 1 && !want_energy) continue;
        uint32_t base0 = 0u, base1 = 0u, tot0 = 0u, tot1 = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t c0 = wave_count[L][0][w], c1 = wave_count[L][1][w];
            base0 += (w < wid) ? c0 : 0u;
            base1 += (w < wid) ? c1 : 0u;
            tot0 += c0;
            tot1 += c1;
        }
        n_list[L] = (int)(tot0 + tot1);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            uint32_t pos = (j ? tot0 + base1 : base0) + pre[L][j];
            const uint32_t pi = threadIdx.x + (uint32_t)j * kBlock;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t idx = 2u * pi + (uint32_t)k;
                if (L == 0 && gap[j][k]) {
                    gap_list[pos] = make_uint2((wu[j][k] & 0xFFFFFF00u) | (idx & 0xFFu),
                                               (wr[j][k] & 0xFFFFFF00u) | (idx >> 8));
                    ++pos;
                }
                if (L == 1 && fix[j][k]) {
                    fixed_list[pos] = (uint16_t)idx;
                    ++pos;
                }
            }
        }
    }
    __syncthreads();

    // site of a list index: row, half-row position, colour offset, valid neighbours
    auto locate = [&](uint32_t idx, int &y, int &h, int &s, uint32_t &valid) {
        const int pi = (int)(idx >> 1);
        y = by * CR + pi / PPR;
        h = 2 * (bx * PPR + pi % PPR) + (int)(idx & 1u);
        s = (y + colour) & 1;
        const int Wo = (d.nx + s) >> 1;
        valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) | (y > 0 ? 4u : 0u) | (y + 1 < d.ny ? 8u : 0u);
    };
    // all four loads are issued, from clamped positions for missing
    // neighbours (ignored by their valid bits), so that they overlap
    auto neighbours = [&](int y, int h, int s, uint32_t valid, float &nL, float &nR, float &nU, float &nD) {
        const int row = y * d.S;
        nL = angle_of(gldi(oth_base, (uint32_t)(row + max(h + s - 1, 0))));
        nR = angle_of(gldi(oth_base, (uint32_t)(row + min(h + s, d.S - 1))));
        nU = angle_of(gldi(oth_base, (uint32_t)(row + ((valid & 4u) ? -d.S : 0) + h)));
        nD = angle_of(gldi(oth_base, (uint32_t)(row + ((valid & 8u) ? d.S : 0) + h)));
    };

    // a thread sees at most 5 sites (4 gap sites), each below 2^30 in energy units
    uint64_t e_thread = 0u;
    uint32_t acc_thread = 0u;
    // pass 2: the listed gap sites, 256 at a time; the next site's inputs
    // are fetched before the current one is computed (unconditionally, from
    // a clamped list index, so that waiting for the current inputs never
    // waits for these)
    struct Item {
        uint2 e;
        int y, h, s;
        uint32_t valid;
        float a, nL, nR, nU, nD;  // raw words: the sign bit is cleared at use
    };
    auto fetch = [&](int i, Item &it) {
        it.e = gap_list[i];
        locate((it.e.x & 0xFFu) | ((it.e.y & 0xFFu) << 8), it.y, it.h, it.s, it.valid);
        const int row = it.y * d.S;
        it.nL = gldi(oth_base, (uint32_t)(row + max(it.h + it.s - 1, 0)));
        it.nR = gldi(oth_base, (uint32_t)(row + min(it.h + it.s, d.S - 1)));
        it.nU = gldi(oth_base, (uint32_t)(row + ((it.valid & 4u) ? -d.S : 0) + it.h));
        it.nD = gldi(oth_base, (uint32_t)(row + ((it.valid & 8u) ? d.S : 0) + it.h));
        it.a = gldi(mine_base, (uint32_t)(row + it.h));
    };
    const int n_gap = n_list[0];
    Item cur;
    if ((int)threadIdx.x < n_gap) fetch((int)threadIdx.x, cur);
    for (int i = (int)threadIdx.x; i < n_gap; i += kBlock) {
        Item nxt;
        fetch(min(i + kBlock, n_gap - 1), nxt);
        const uint32_t idx = (cur.e.x & 0xFFu) | ((cur.e.y & 0xFFu) << 8);
        const int y = cur.y, h = cur.h, s = cur.s;
        const uint32_t valid = cur.valid;
        const uint32_t site = (uint32_t)(y * d.S + h);
        // the low 8 bits of each word hold the index; unit24 uses the top 24
        const float u = or_only ? 0.5f : unit24(cur.e.x);
        const float r = or_only ? 0.5f : unit24(cur.e.y);
        bool n64 = true;
        const SiteOut o = update_site(angle_of(cur.a), angle_of(cur.nL), angle_of(cur.nR), angle_of(cur.nU),
                                      angle_of(cur.nD), valid, u, r, inv_T, dscale, or_only != 0, &n64);
        cur = nxt;
        if (n64) {  // too close to call: redone in double precision afterwards
            defer_redo(rd, blockIdx.x, kCompactSites / 32, idx);
            continue;
        }
        gsti(mine_base, site, o.phi);
        if (acc_base) accumulate_state_i(acc_base, m2_base, site, o.phi, stp->inv_k, stp->inv_km1);
        acc_thread += o.accepted ? 1u : 0u;
        if (want_energy) e_thread += energy_fx(o.e_bonds);
        if (DIAG && flags) flags[(int64_t)y * d.nx + 2 * h + s] = (uint8_t)o.flags;
    }
    // pass 3: bond energies of the sampled sites of colour 1
    for (int i = (int)threadIdx.x; i < n_list[1]; i += kBlock) {
        int y, h, s;
        uint32_t valid;
        locate((uint32_t)fixed_list[i], y, h, s, valid);
        float nL, nR, nU, nD;
        neighbours(y, h, s, valid, nL, nR, nU, nD);
        const float a = angle_of(gldi(mine_base, (uint32_t)(y * d.S + h)));
        e_thread += energy_fx(bond_energy_half(0.5f * a, nL, nR, nU, nD, valid));
    }
    if (!want_acc) return;
    // wave sums without carries: 64 x 16-bit low parts stay below 2^22, the
    // accepted count (<= 256 per wave) takes bits 22-31, the high parts
    // (< 2^19 per lane) sum in their own word
    uint32_t lo = (uint32_t)(e_thread & 0xFFFFu) | (acc_thread << 22);
    uint32_t hi = (uint32_t)(e_thread >> 16);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off);
        hi += __shfl_xor(hi, off);
    }
    if (lane == 0) {
        red[0][wid] = lo;
        red[1][wid] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0ull, a = 0ull;
        for (int i = 0; i < NW; ++i) {
            e += ((unsigned long long)red[1][i] << 16) + (red[0][i] & 0x3FFFFFu);
            a += red[0][i] >> 22;
        }
        if (e) atomicAdd(&stp->e_fx, e);
        if (a) atomicAdd(&stp->acc, a);
    }
}

template <bool DIAG, int CR>
__global__ __launch_bounds__(kBlock) void half_sweep_compact_kernel(const ChainDesc *__restrict__ descs,
                                                                    ChainState *__restrict__ states,
                                                                    BlockMap bm, int colour, SweepConsts sc,
                                                                    int or_only, Redo rd, uint8_t *__restrict__ flags)
{
    half_sweep_compact_body<DIAG, CR>(descs, states, bm, colour, sc, or_only, rd, flags);
}

__device__ void set_derived(ChainState &st, double q)
{
    st.inv_T = (float)(1.0 / st.T);
    st.dscale = (float)(kTwoPi * q / st.a_cur);
}

// Algorithm 2 steps 5.2-5.5 (relaxation), 6 (equilibrium states) and the
// e(T, L) runs for a chain not done, after both colours of a sweep, on its
// state `st` (in place) with its sums e_fx and acc of that sweep.  The done
// counter (and the work counters) are skipped where null.
__device__ __forceinline__ void control_core(ChainState &st, const ChainDesc &d, const CtlParams &cp,
                                             unsigned int *done_count, unsigned long long *work)
{
    if (work) {
        // work counters: chain-sweeps, gap-site updates, useful bytes
        atomicAdd(&work[0], 1ull);
        atomicAdd(&work[1], (unsigned long long)d.P);
        atomicAdd(&work[2], (unsigned long long)(cp.angle_bytes * ((int64_t)d.nx * d.ny + d.P)));
    }
    const uint32_t t = st.sweep;
    const unsigned long long acc = st.acc, efx = st.e_fx;
    st.acc = 0ull;
    st.e_fx = 0ull;
    // 1 + e = (H + N_GP) / N_GP with H + N_GP = sum over bonds of (1 - cos)
    const double ope = (double)efx * cp.e_unit / (double)d.ngp;
    if (st.phase == PH_RELAX) {
        const double A = (double)acc / (double)d.P;
        if (A < cp.a_targ) st.a_relax = 1.0 + (double)(t + 1u) / cp.k_a;
        st.ring[t % (uint32_t)cp.n_fit] = ope;
        if (t >= (uint32_t)cp.n_fit && t % (uint32_t)cp.n_f == 0u) st.k = ring_slope(st.ring, t, cp.n_fit, cp.w);
        st.A_last = A;
        const uint32_t tn = t + 1u;
        st.sweep = tn;
        bool stop;
        if (cp.fixed_relax >= 0) stop = tn >= (uint32_t)cp.fixed_relax;
        else stop = !(st.k < 0.0 && (int64_t)tn <= (int64_t)cp.i_max);
        st.a_cur = st.a_relax;
        if (stop) {
            st.relax_sweeps = (int32_t)tn;
            st.not_converged = (cp.fixed_relax < 0 && st.k < 0.0) ? 1 : 0;
            st.eq_left = cp.K;
            st.phase = cp.K > 0 ? PH_EQ : PH_DONE;
            st.a_cur = cp.eq_a_mode ? st.a_relax : 1.0;
            st.inv_k = 1.0f;
            st.inv_km1 = 0.0f;
            st.inv_k_d = 1.0;
            st.inv_km1_d = 0.0;
        }
    } else if (st.phase == PH_EQ) {
        st.sweep = t + 1u;
        if (--st.eq_left <= 0) {
            st.phase = PH_DONE;
        } else {
            const int k = cp.K - st.eq_left + 1;  // the next sweep's state number
            st.inv_k = 1.0f / (float)k;
            st.inv_km1 = 1.0f / (float)(k - 1);
            st.inv_k_d = 1.0 / (double)k;
            st.inv_km1_d = 1.0 / (double)(k - 1);
        }
    } else {  // PH_TABLE
        const double A = (double)acc / (double)d.P;
        if (A < cp.a_targ) st.a_relax = 1.0 + (double)(t + 1u) / cp.k_a;
        st.a_cur = st.a_relax;
        if ((int64_t)t >= (int64_t)cp.burn) st.e_sum += ope;
        st.sweep = t + 1u;
        if ((int64_t)t + 1 >= (int64_t)cp.burn + cp.meas) st.phase = PH_DONE;
    }
    set_derived(st, cp.q);
    if (st.phase == PH_DONE && done_count) atomicAdd(done_count, 1u);
}

// The control of chain c of a chain set (control_core on its state in place:
// a copy would put the ring buffer in scratch memory).
__device__ __forceinline__ void control_chain(const ChainDesc *__restrict__ descs, ChainState *__restrict__ states,
                                              int c, const CtlParams &cp, unsigned int *done_count,
                                              unsigned long long *work)
{
    ChainState &st = states[c];
    if (st.phase == PH_DONE) return;
    const ChainDesc d = descs[c];
    control_core(st, d, cp, done_count, work);
}

// The deferred double-precision updates of one half-sweep (block shape
// `rows`, `compact`): each flagged site is redone by update_site_d from the
// inputs the sweep saw (it left the site unchanged), with the same random
// numbers, written back in single precision, and its accepted count and
// bond energy added to its chain.  A wave takes one bitmap word (32 sweep
// blocks) at a time; its lanes split over (flagged block, mask word), 64 /
// words blocks per pass, and a lane redoes the sites of its mask word.  The
// bits are cleared on the way, so the buffers are zero again for the next
// half-sweep.  With `ctl` set (after the colour-1 half-sweep) the last block
// to finish also runs the per-sweep control of all n_all chains, which saves
// the control kernel's launch; it finds out that it is last from the ticket
// counter, which it resets.
struct FusedControl {
    CtlParams cp;
    unsigned int *ticket;  // zero before the first launch; the last block resets it
    unsigned int *done_count;
    unsigned long long *work;
    int32_t n_all;
    int32_t on;
};

template <bool DIAG>
__global__ __launch_bounds__(kBlock) void redo_fp64_kernel(const ChainDesc *__restrict__ descs,
                                                           ChainState *__restrict__ states,
                                                           BlockMap bm,
                                                           int64_t total_blocks, int rows, int compact, int colour,
                                                           SweepConsts sc, int or_only, Redo rd,
                                                           uint8_t *__restrict__ flags, FusedControl ctl)
{
    const int words = compact ? kCompactSites / 32 : 2 * kBlock / 32;  // 32 or 16
    const int per = 64 / words;                                         // blocks per pass
    const int ppr = compact ? kCompactSites / rows / 2 : kBlock / rows;  // site pairs per block row
    const int64_t nw = (total_blocks + 31) >> 5;
    const int lane = (int)(threadIdx.x & 63);
    const int slot = lane / words, k = lane % words;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t wi = wave; wi < nw; wi += n_waves) {
        uint32_t bits = rd.blocks[wi];
        if (!bits) continue;
        if (lane == 0) rd.blocks[wi] = 0u;
        while (bits) {
            // this lane's block: the slot-th lowest set bit of this pass
            uint32_t b = bits;
            for (int i = 0; i < slot; ++i) b &= b - 1u;
            for (int i = 0; i < per; ++i) bits &= bits - 1u;
            if (!b) continue;
            const int64_t gb = (wi << 5) + (__ffs(b) - 1);
            uint32_t m = rd.mask[gb * words + k];
            if (!m) continue;
            rd.mask[gb * words + k] = 0u;
            int lb;
            const int c = chain_of_block(bm, gb, &lb);
            ChainState *stp = states + c;
            const ChainDesc d = descs[c];
            const int nbx = ((d.S >> 1) + ppr - 1) / ppr;
            const int by = lb / nbx;
            const int bx = lb - by * nbx;
            const int phase = stp->phase;
            const bool want_energy = (colour == 1) && (phase != PH_EQ);
            const bool want_acc = phase != PH_EQ;
            float *mine = colour ? d.h[1] : d.h[0];
            const float *oth = colour ? d.h[0] : d.h[1];
            float *accp = (phase == PH_EQ) ? (colour ? d.acc[1] : d.acc[0]) : nullptr;
            float *m2p = accp ? (colour ? d.m2[1] : d.m2[0]) : nullptr;
            while (m) {
                const int bit = __ffs(m) - 1;
                m &= m - 1u;
                const int idx = 32 * k + bit;
                const int pi = idx >> 1, sl = idx & 1;
                const int y = by * rows + pi / ppr;
                const int h = 2 * (bx * ppr + pi % ppr) + sl;
                const int s = (y + colour) & 1;
                const int Wo = (d.nx + s) >> 1;
                const uint32_t valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) |
                                       (y > 0 ? 4u : 0u) | (y + 1 < d.ny ? 8u : 0u);
                const float *orow = oth + (int64_t)y * d.S;
                const float nL = (valid & 1u) ? angle_of(orow[h + s - 1]) : 0.0f;
                const float nR = (valid & 2u) ? angle_of(orow[h + s]) : 0.0f;
                const float nU = (valid & 4u) ? angle_of(orow[h - d.S]) : 0.0f;
                const float nD = (valid & 8u) ? angle_of(orow[h + d.S]) : 0.0f;
                float *mp = mine + (int64_t)y * d.S + h;
                const float a = angle_of(*mp);
                float u = 0.5f, r = 0.5f;
                if (!or_only) {
                    const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * (h & ~1) + s), stp->sweep,
                                    d.chain, d.image_id};
                    const U4 wd = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
                    u = unit24(sl ? wd.z : wd.x);
                    r = unit24(sl ? wd.w : wd.y);
                }
                const SiteOutD o = update_site_d((double)a, (double)nL, (double)nR, (double)nU, (double)nD, valid,
                                                 (double)u, (double)r, stp->a_cur, stp->T, sc.q64,
                                                 or_only != 0);
                const float out = (float)o.phi;
                *mp = out;
                if (accp)
                    accumulate_state(accp + (int64_t)y * d.S + h, m2p ? m2p + (int64_t)y * d.S + h : nullptr, out,
                                     stp->inv_k, stp->inv_km1);
                if (want_acc && o.accepted) atomicAdd(&stp->acc, 1ull);
                if (want_energy) atomicAdd(&stp->e_fx, (unsigned long long)energy_fx((float)o.e_bonds));
                if (DIAG && flags) flags[(int64_t)y * d.nx + 2 * h + s] = (uint8_t)o.flags;
            }
        }
    }
    if (!ctl.on) return;
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ctl.ticket, 1u) == gridDim.x - 1u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // the other blocks' counts and energies are visible
    for (int c = (int)threadIdx.x; c < ctl.n_all; c += (int)blockDim.x)
        control_chain(descs, states, c, ctl.cp, ctl.done_count, ctl.work);
    if (threadIdx.x == 0) *ctl.ticket = 0u;
}

// ================================================================ fused tile sweep
// A whole sweep in one launch.  A block stages one tile of both colours in
// LDS: TH rows x 2 kTileH columns of the grid (kTileH half-columns per
// colour) plus a halo of two rows and columns.  It updates colour 0 on the
// tile and on the ring of sites around it, then colour 1 on the tile, which
// so sees the colour-0 values of its neighbours after their update (the ring
// repeats updates that the neighbouring tiles also make, with the same
// inputs and the same random numbers, so with the same results).  Decisions
// too close to call in single precision are redone in double precision in
// the block after each colour, before anything reads them.  The gap sites
// of the tile are then written to the chain's second half-grids (h2):
// reading h and writing h2 keeps every tile's halo at the state before the
// sweep while other tiles store theirs.  control_kernel then swaps h and h2
// of every chain swept (one thread per chain: no block of the sweep waits
// for the others) before it runs the per-sweep control; a launch of at most
// a few thousand blocks does both in its last block instead.
//
// Within a colour the gap sites are listed in LDS first (wave ballots; each
// wave lists the candidates it read, interleaved with the other waves at 64
// sites, and updates its own list), so that lanes only do gap sites; with
// the sweep's energy wanted, the colour-1 sampled sites of the tile get a
// second list for their bond energies.  Every site gets update_site, the
// arithmetic of the half-sweep kernels, so the results equal theirs bit for
// bit.  `mode` 0 is the full sweep; 1 and 2 update only colour 0 or 1, in
// place (no tile reads a value another tile writes then), for the
// single-colour diagnostics.
constexpr int kTileH = 64;                // half-columns per tile and colour
constexpr int kTileLS = kTileH + 8;       // LDS row: half-columns hx0 - 4 .. hx0 + kTileH + 3
constexpr int kTileNW = kBlock / 64;      // waves per block
// Fused sweeps of at most this many blocks run the control themselves: each
// block then ends with a device-scope fence (a write-back of its XCD's L2)
// and a ticket; measured, that saves the control kernel's node in a 1024^2
// one-chain sweep (344 blocks: 38 -> 34 us per sweep) but costs ~37 us per
// sweep at 2752 blocks (4096^2, one chain).
constexpr int64_t kTileCtlMaxBlocks = 512;

// The double-precision decision of one tile site (colour c, local row r,
// half-column j) from its LDS inputs: the steps of redo_fp64_kernel.  Kept
// out of line, so that the sweep's loops do not hold the double update's
// constants in registers.
__device__ __noinline__ SiteOutD tile_redo_site(const float *a, int rows, int c, int r, int j, int y0, int hx0, int nx,
                                                int ny, uint32_t sweep, uint32_t chain, uint32_t image_id,
                                                SweepConsts sc, int or_only, double a_cur, double T)
{
    const float *own = a + ((size_t)c * rows + r) * kTileLS + j;
    const float *oth = a + ((size_t)(c ^ 1) * rows + r) * kTileLS + j;
    const int s = (r + c) & 1;
    const int y = y0 - 2 + r, h = hx0 - 4 + j;
    const int Wo = (nx + s) >> 1;
    const uint32_t valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) | (y > 0 ? 4u : 0u) |
                           (y + 1 < ny ? 8u : 0u);
    const float nL = (valid & 1u) ? angle_of(oth[s - 1]) : 0.0f;
    const float nR = (valid & 2u) ? angle_of(oth[s]) : 0.0f;
    const float nU = (valid & 4u) ? angle_of(oth[-kTileLS]) : 0.0f;
    const float nD = (valid & 8u) ? angle_of(oth[kTileLS]) : 0.0f;
    float u = 0.5f, rr = 0.5f;
    if (!or_only) {
        const U4 ctr = {(uint32_t)y * (uint32_t)nx + (uint32_t)(2 * (h & ~1) + s), sweep, chain, image_id};
        const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
        const bool second = (h & 1) != 0;
        u = unit24(second ? w.z : w.x);
        rr = unit24(second ? w.w : w.y);
    }
    return update_site_d((double)angle_of(*own), (double)nL, (double)nR, (double)nU, (double)nD, valid, (double)u,
                         (double)rr, a_cur, T, sc.q64, or_only != 0);
}

// The parameters one sweep of a chain reads (written by the control between
// sweeps).
struct SweepState {
    int32_t phase;
    uint32_t sweep;
    float inv_T, dscale, inv_k, inv_km1;
    double T, a_cur;
};

__device__ __forceinline__ SweepState sweep_state_of(const ChainState *stp)
{
    SweepState s;
    s.phase = stp->phase;
    s.sweep = stp->sweep;
    s.inv_T = stp->inv_T;
    s.dscale = stp->dscale;
    s.inv_k = stp->inv_k;
    s.inv_km1 = stp->inv_km1;
    s.T = stp->T;
    s.a_cur = stp->a_cur;
    return s;
}

template <int TH, int NW = kTileNW>
struct TileShared {
    static constexpr int NT = NW * 64;  // threads per block
    // list entries per wave: its rows of the colour-0 pass with the ring
    // (TH + 2 rows of kTileH columns, a row per wave in turn) and its share
    // of the ring's two side columns (at most 64 per wave)
    static constexpr int CAP = (TH + 2 + NW - 1) / NW * 64 + 64;
    static constexpr int RW = ((TH + 4) * kTileLS + 31) / 32;     // redo bitmap words
    alignas(16) float a[2][TH + 4][kTileLS];  // angle words (sign bit: sampled), colour, row, half-column
    // per wave: gap entries from the front, sampled entries from the back;
    // entry = local row << 7 | local half-column
    uint16_t list[NW][CAP];
    uint32_t redo[RW];
    uint32_t red[3][NW];
    int any_redo[2];
};

// Equilibrium sums and squared deviations of a tile's own sites (both
// colours), staged with the angles when the sweep is known to need them.
template <int TH>
struct TilePre {
    alignas(16) float acc[2][TH][kTileH];
    alignas(16) float m2[2][TH][kTileH];
};

// Stages the tile and its halo (both colours, 18 float4 per row and colour;
// the colour loop outside, so that the base pointer of every load is
// uniform) from h into LDS, and with `P` the tile's own equilibrium sums
// (and squared deviations, where kept).  No barrier at the end.
template <int TH, int NW>
__device__ __forceinline__ void tile_stage(TileShared<TH, NW> &L, TilePre<TH> *P, const ChainDesc &d, int y0, int hx0)
{
    constexpr int NT = TileShared<TH, NW>::NT;
    const int tid = (int)threadIdx.x;
    constexpr int NQ = kTileLS / 4;
    constexpr int NLOAD = (TH + 4) * NQ;
    constexpr int IT = (NLOAD + NT - 1) / NT;
    v4f v[2][IT];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        const float *src = cc ? d.h[1] : d.h[0];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int k = tid + it * NT;
            const int r = k / NQ, q = k - r * NQ;
            const int y = y0 - 2 + r, h = hx0 - 4 + 4 * q;
            const bool in = k < NLOAD && y >= 0 && y < d.ny && h >= 0 && h < d.S;
            // outside the grid: zeros, never a candidate (EDGE bounds)
            // nor a valid neighbour
            v[cc][it] = gldi4(src, in ? (uint32_t)(y * d.S + h) : 0u);
            if (!in) v[cc][it] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
    if (P) {
        // the tile's rows y0 .. y0 + TH - 1, half-columns hx0 .. hx0 + kTileH - 1
        constexpr int PQ = kTileH / 4;
        constexpr int PLOAD = TH * PQ;
        constexpr int PIT = (PLOAD + NT - 1) / NT;
        const bool with_m2 = d.m2[0] != nullptr;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const float *ap = cc ? d.acc[1] : d.acc[0];
            const float *mp = cc ? d.m2[1] : d.m2[0];
#pragma unroll
            for (int it = 0; it < PIT; ++it) {
                const int k = tid + it * NT;
                const int r = k / PQ, q = k - r * PQ;
                const int y = y0 + r;
                if (k < PLOAD && y < d.ny) {
                    const uint32_t idx = (uint32_t)(y * d.S + hx0 + 4 * q);
                    *(v4f *)&P->acc[cc][r][4 * q] = gldi4(ap, idx);
                    if (with_m2) *(v4f *)&P->m2[cc][r][4 * q] = gldi4(mp, idx);
                }
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int k = tid + it * NT;
            const int r = k / NQ, q = k - r * NQ;
            if (k < NLOAD) *(v4f *)&L.a[cc][r][4 * q] = v[cc][it];
        }
}

// The sweep (mode 0) or one colour (modes 1, 2) of a staged tile, and the
// write-back of its gap sites and equilibrium sums (those from `P` when
// given: staged by tile_stage for this sweep).
template <bool DIAG, int TH, bool EDGE, int NW>
__device__ __forceinline__ void tile_update(TileShared<TH, NW> &L, const TilePre<TH> *P, const ChainDesc &d,
                                            const SweepState &ss, int y0, int hx0, int mode, const SweepConsts &sc,
                                            int or_only, uint8_t *__restrict__ flags, uint64_t &e_thread,
                                            uint32_t &acc_thread)
{
    constexpr int NT = TileShared<TH, NW>::NT;
    // the wave index through readfirstlane: the compiler then knows it is
    // uniform, and keeps the row loops of the list building and their
    // counters on the scalar unit
    const int tid = (int)threadIdx.x, lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int phase = ss.phase;
    const uint32_t sweep = ss.sweep;
    const float inv_T = ss.inv_T, dscale = ss.dscale;
    const bool eq = phase == PH_EQ;
    float *const dst0 = mode == 0 ? d.h2[0] : d.h[0];
    float *const dst1 = mode == 0 ? d.h2[1] : d.h[1];

    // the tile's gap sites of colour cc to the destination half-grid
    // (16-byte groups holding at least one gap site), and the equilibrium sums
    auto write_back = [&](int cc) {
        constexpr int NQ = kTileH / 4;
        const float ik = ss.inv_k, ikm1 = ss.inv_km1;
        float *const dst = cc ? dst1 : dst0;
        float *const ap = eq ? (cc ? d.acc[1] : d.acc[0]) : nullptr;
        float *const mp = cc ? d.m2[1] : d.m2[0];
        for (int k = tid; k < TH * NQ; k += NT) {
            const int rr = k / NQ, q = k - rr * NQ;
            const int y = y0 + rr;
            if (y >= d.ny) continue;
            const int h = hx0 + 4 * q;
            const v4f v = *(const v4f *)&L.a[cc][rr + 2][4 + 4 * q];
            const bool g0 = !is_fixed(v.x), g1 = !is_fixed(v.y), g2 = !is_fixed(v.z), g3 = !is_fixed(v.w);
            if (!(g0 || g1 || g2 || g3)) continue;
            const uint32_t idx = (uint32_t)(y * d.S + h);
            gsti4(dst, idx, v);
            if (ap) {
                // the group's gap sites into the equilibrium sums (and the
                // squared deviations), the arithmetic of accumulate_state,
                // with 16-byte loads and stores; the other elements keep
                // their values
                const int W = (d.nx - ((y + cc) & 1) + 1) >> 1;
                const bool gg[4] = {g0, g1, g2, g3};
                const v4f s0 = P ? *(const v4f *)&P->acc[cc][rr][4 * q] : gldi4(ap, idx);
                v4f s1 = s0;
                v4f m = mp ? (P ? *(const v4f *)&P->m2[cc][rr][4 * q] : gldi4(mp, idx))
                           : v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (gg[e] && h + e < W) {
                        s1[e] = s0[e] + v[e];
                        m[e] = fmaf(v[e] - s0[e] * ikm1, v[e] - s1[e] * ik, m[e]);
                    }
                gsti4(ap, idx, s1);
                if (mp) gsti4(mp, idx, m);
            }
        }
    };

    const int npass = mode == 0 ? 2 : 1;
    for (int pass = 0; pass < npass; ++pass) {
        const int c = mode == 0 ? pass : mode - 1;
        const bool ring = mode == 0 && c == 0;       // colour 0 of a full sweep: tile and ring
        const bool energy = c == 1 && !eq;           // the sweep's energy comes from colour 1
        const int r_lo = ring ? 1 : 2, r_hi = TH + (ring ? 3 : 2);
        uint16_t *lst = L.list[wid];
        // List the gap sites (and, for the energy, the sampled sites): a
        // wave takes one row at a time, lane l its tile column j = 4 + l;
        // with the ring, then the ring's side columns j = 3 and kTileH + 4,
        // two lanes per row.  A site in the tile is either a gap or a
        // sample, so a lane's rank among the sampled lanes is its rank among
        // the lanes holding a site less its rank among the gap lanes: one
        // ballot per row.  FULL: every lane of the wave holds a site (the
        // interior rows of an interior tile), so that rank among them is the
        // lane index.
        int ng = 0, ns = 0;
        auto add = [&](auto FULL, bool cand, int r, int j) {
            constexpr bool full = decltype(FULL)::value;
            bool in = cand, gap = false;
            if (cand) {
                const float v = L.a[c][r][j];
                if (EDGE) {
                    const int y = y0 - 2 + r, h = hx0 - 4 + j, s = (r + c) & 1;
                    in = y < d.ny && y >= 0 && h >= 0 && h < ((d.nx - s + 1) >> 1);
                }
                gap = in && !is_fixed(v);
            }
            const uint16_t ent = (uint16_t)((r << 7) | j);
            const uint64_t bg = __ballot(gap);
            const int rg = rank_below(bg);
            if (gap) lst[ng + rg] = ent;
            const int cg = __popcll(bg);
            ng += cg;
            if (energy) {
                const uint64_t bi = full ? ~0ull : __ballot(in);
                const int rs = (full ? lane : rank_below(bi)) - rg;
                if (in && !gap) lst[TileShared<TH, NW>::CAP - 1 - (ns + rs)] = ent;
                ns += (full ? 64 : __popcll(bi)) - cg;
            }
        };
        for (int r = r_lo + wid; r < r_hi; r += NW) add(std::integral_constant<bool, !EDGE>{}, true, r, 4 + lane);
        if (ring) {
            const int k = wid * 64 + lane;
            add(std::false_type{}, k < 2 * (TH + 2), 1 + (k >> 1), (k & 1) ? kTileH + 4 : 3);
        }
        __syncthreads();
        // the listed gap sites
        for (int e = lane; e < ng; e += 64) {
            const uint32_t ent = lst[e];
            const int r = (int)(ent >> 7), j = (int)(ent & 127u);
            const int s = (r + c) & 1;  // y0 is even
            const float *oth = &L.a[c ^ 1][r][j];
            const float a0 = L.a[c][r][j];
            const float nL = angle_of(oth[s - 1]), nR = angle_of(oth[s]);
            const float nU = angle_of(oth[-kTileLS]), nD = angle_of(oth[kTileLS]);
            const int y = y0 - 2 + r, h = hx0 - 4 + j;
            uint32_t valid = 15u;
            if (EDGE) {
                const int Wo = (d.nx + s) >> 1;
                valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) | (y > 0 ? 4u : 0u) |
                        (y + 1 < d.ny ? 8u : 0u);
            }
            float u = 0.5f, rr = 0.5f;
            if (!or_only) {
                const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * (h & ~1) + s), sweep, d.chain,
                                d.image_id};
                const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
                const bool second = (h & 1) != 0;
                u = unit24(second ? w.z : w.x);
                rr = unit24(second ? w.w : w.y);
            }
            bool n64 = true;
            const SiteOut o = update_site(a0, nL, nR, nU, nD, valid, u, rr, inv_T, dscale, or_only != 0, &n64);
            if (n64) {  // too close to call: redone in double precision below
                const int wi = r * kTileLS + j;
                atomicOr(&L.redo[wi >> 5], 1u << (wi & 31));
                L.any_redo[pass] = 1;
                continue;
            }
            L.a[c][r][j] = o.phi;
            const bool own = !ring || (r >= 2 && r < TH + 2 && j >= 4 && j < kTileH + 4);
            if (own) {
                acc_thread += o.accepted ? 1u : 0u;
                if (energy) e_thread += energy_fx(o.e_bonds);
                if (DIAG && flags) flags[(int64_t)y * d.nx + 2 * h + s] = (uint8_t)o.flags;
            }
        }
        // bond energies of the tile's sampled colour-1 sites
        for (int e = lane; e < ns; e += 64) {
            const uint32_t ent = lst[TileShared<TH, NW>::CAP - 1 - e];
            const int r = (int)(ent >> 7), j = (int)(ent & 127u);
            const int s = (r + c) & 1;
            const float *oth = &L.a[c ^ 1][r][j];
            const float nL = angle_of(oth[s - 1]), nR = angle_of(oth[s]);
            const float nU = angle_of(oth[-kTileLS]), nD = angle_of(oth[kTileLS]);
            uint32_t valid = 15u;
            if (EDGE) {
                const int y = y0 - 2 + r, h = hx0 - 4 + j;
                const int Wo = (d.nx + s) >> 1;
                valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) | (y > 0 ? 4u : 0u) |
                        (y + 1 < d.ny ? 8u : 0u);
            }
            e_thread += energy_fx(bond_energy_half(0.5f * angle_of(L.a[c][r][j]), nL, nR, nU, nD, valid));
        }
        __syncthreads();
        // the deferred decisions, in double precision from the same inputs
        if (L.any_redo[pass]) {
            for (int wd = tid; wd < TileShared<TH, NW>::RW; wd += NT) {
                uint32_t m = L.redo[wd];
                if (!m) continue;
                L.redo[wd] = 0u;
                while (m) {
                    const int wi = wd * 32 + __ffs(m) - 1;
                    m &= m - 1u;
                    const int r = wi / kTileLS, j = wi - r * kTileLS;
                    const SiteOutD o = tile_redo_site(&L.a[0][0][0], TH + 4, c, r, j, y0, hx0, d.nx, d.ny, sweep, d.chain,
                                                      d.image_id, sc, or_only, ss.a_cur, ss.T);
                    const int y = y0 - 2 + r, h = hx0 - 4 + j, s = (r + c) & 1;
                    L.a[c][r][j] = (float)o.phi;
                    const bool own = !ring || (r >= 2 && r < TH + 2 && j >= 4 && j < kTileH + 4);
                    if (own) {
                        acc_thread += o.accepted ? 1u : 0u;
                        if (energy) e_thread += energy_fx((float)o.e_bonds);
                        if (DIAG && flags) flags[(int64_t)y * d.nx + 2 * h + s] = (uint8_t)o.flags;
                    }
                }
            }
            __syncthreads();
        }
        if (mode == 0 && pass == 0) write_back(0);
    }

    // the colour not written back after its own pass (colour 0 of a full
    // sweep is final once its pass is done: colour 1 only reads it)
    write_back(mode == 1 ? 0 : 1);
}

// Stage, then sweep, the tile of a one-launch-per-sweep kernel.
template <bool DIAG, int TH, bool EDGE>
__device__ __forceinline__ void tile_sweep_body(TileShared<TH> &L, const ChainDesc &d, const SweepState &ss, int y0,
                                                int hx0, int mode, const SweepConsts &sc, int or_only,
                                                uint8_t *__restrict__ flags, uint64_t &e_thread,
                                                uint32_t &acc_thread)
{
    tile_stage<TH, kTileNW>(L, nullptr, d, y0, hx0);
    __syncthreads();
    tile_update<DIAG, TH, EDGE, kTileNW>(L, nullptr, d, ss, y0, hx0, mode, sc, or_only, flags, e_thread, acc_thread);
}

// The block's bond energy and accepted count added to its chain (energy in
// 16-bit halves, so that the 32-bit lane sums cannot carry out).  Called by
// every thread of the block.
template <int TH, int NW>
__device__ __forceinline__ void tile_block_sums(TileShared<TH, NW> &L, uint64_t e_thread, uint32_t acc_thread,
                                                unsigned long long *e_sum, unsigned long long *acc_sum)
{
    const int tid = (int)threadIdx.x;
    uint32_t lo = (uint32_t)(e_thread & 0xFFFFu), hi = (uint32_t)(e_thread >> 16), ac = acc_thread;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off);
        hi += __shfl_xor(hi, off);
        ac += __shfl_xor(ac, off);
    }
    const int wid = tid >> 6;
    if ((tid & 63) == 0) {
        L.red[0][wid] = lo;
        L.red[1][wid] = hi;
        L.red[2][wid] = ac;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long e = 0ull, a = 0ull;
        for (int i = 0; i < NW; ++i) {
            e += ((unsigned long long)L.red[1][i] << 16) + L.red[0][i];
            a += L.red[2][i];
        }
        if (e) atomicAdd(e_sum, e);
        if (a) atomicAdd(acc_sum, a);
    }
}

// The work of the last block of a sweep: h and h2 of every swept chain
// exchanged (the chain's `swapped` flag toggled), then the per-sweep control
// of all chains.  Called by every thread of that block.
__device__ __forceinline__ void swap_and_control(ChainDesc *descs, ChainState *states, const BlockMap &bm,
                                                 const FusedControl &ctl)
{
    const int tid = (int)threadIdx.x;
    for (int k = tid; k < bm.n; k += kBlock) {
        const int c = bm.id[k];
        if (states[c].phase == PH_DONE) continue;
        ChainDesc &dd = descs[c];
        float *t0 = dd.h[0], *t1 = dd.h[1];
        dd.h[0] = dd.h2[0];
        dd.h[1] = dd.h2[1];
        dd.h2[0] = t0;
        dd.h2[1] = t1;
        states[c].swapped ^= 1;
    }
    __syncthreads();
    for (int c = tid; c < ctl.n_all; c += kBlock)
        control_chain(descs, states, c, ctl.cp, ctl.done_count, ctl.work);
}

// With `ctl.on` (launches of a few thousand blocks, where one ticket counter
// costs little) the last block to finish also exchanges h and h2 of the
// swept chains and runs the per-sweep control, which saves the control
// kernel's launch in each sweep of a small fill; it finds out that it is last
// from the ticket counter, which it resets.
template <bool DIAG, int TH>
__global__ __launch_bounds__(kBlock) void sweep_tile_kernel(ChainDesc *__restrict__ descs,
                                                            ChainState *__restrict__ states, BlockMap bm,
                                                            int mode, SweepConsts sc, int or_only,
                                                            uint8_t *__restrict__ flags, FusedControl ctl)
{
    __shared__ TileShared<TH> L;
    const int tid = (int)threadIdx.x;
    for (int w = tid; w < TileShared<TH>::RW; w += kBlock) L.redo[w] = 0u;
    if (tid < 2) L.any_redo[tid] = 0;
    // blocks go round-robin to the 8 XCDs: give each XCD a contiguous run of
    // tiles, so that the halo rows tiles share are read through one L2
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t per = G >> 3, rem = G & 7u, xcd = b & 7u;
    const int64_t lbk = (int64_t)xcd * per + (int64_t)min(xcd, rem) + (int64_t)(b >> 3);
    int lb;
    const int cid = chain_of_block(bm, lbk, &lb);
    ChainState *stp = states + cid;
    uint64_t e_thread = 0u;
    uint32_t acc_thread = 0u;
    const int phase = stp->phase;
    if (phase != PH_DONE) {
        const ChainDesc d = descs[cid];
        const int nbx = d.S / kTileH;
        const int ty = lb / nbx, tx = lb - ty * nbx;
        const int y0 = ty * TH, hx0 = tx * kTileH;
        const bool edge = !(ty >= 1 && y0 + TH + 2 <= d.ny && tx >= 1 && hx0 + kTileH + 2 <= (d.nx >> 1));
        __syncthreads();
        const SweepState ss = sweep_state_of(stp);
        if (edge)
            tile_sweep_body<DIAG, TH, true>(L, d, ss, y0, hx0, mode, sc, or_only, flags, e_thread, acc_thread);
        else
            tile_sweep_body<DIAG, TH, false>(L, d, ss, y0, hx0, mode, sc, or_only, flags, e_thread, acc_thread);
        if (phase != PH_EQ) tile_block_sums(L, e_thread, acc_thread, &stp->e_fx, &stp->acc);
    }
    if (!ctl.on) return;
    __shared__ int last;
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        last = atomicAdd(ctl.ticket, 1u) == gridDim.x - 1u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // the other blocks' sums and stores are visible
    swap_and_control(descs, states, bm, ctl);
    if (tid == 0) *ctl.ticket = 0u;
}

// Persistent fused sweeps, for chain sets whose tiles all fit on the GPU at
// once (small fills: a 1024 x 1024 chain is 256 tiles of 32 rows).  One
// cooperative launch (which guarantees that every block is resident) runs up
// to `count` sweeps of 512-thread blocks, with a grid barrier between two
// sweeps in place of a kernel launch and its gap.  Every block keeps its
// chain's descriptor and state and runs the chain's per-sweep control itself
// (the same inputs give every block of a chain the same result), from the
// sweep's bond energy and accepted count, which the blocks add into one of
// two per-chain slots (alternating sweeps), so that nothing waits for one
// block's control; the chain's first block counts it done and writes its
// state and descriptor back at the end.  The arithmetic is that of
// sweep_tile_kernel, so the results are the same bit for bit.
//
// Barrier: every wave waits for its own stores (they then sit in its XCD's
// L2), one thread per block writes that L2 back (release) and takes a
// ticket; the last ticket-holder clears the slots read in this sweep, resets
// the ticket and publishes the sweep count (bit 31: stop) in `gen`; the
// others poll `gen` and then invalidate their caches (acquire).  A block
// that waits longer than its bound (2 s unless the call sets another) sets
// `abort` and every block leaves at its next barrier; the host then reports
// an error.
struct PersistCtl {
    unsigned int *gen;    // sweeps completed in this launch, | 1 << 31 to stop; zero at launch
    unsigned int *abort;  // nonzero: a block timed out at a barrier
    unsigned long long *slots;  // per chain: [sweep parity][energy, accepted]; zero at launch
    uint64_t wait_ticks;  // the longest wait at a barrier, in ticks of the 100 MHz constant clock
    int32_t count;        // sweeps to run at most
    uint32_t need;        // done-counter value at which every chain has finished
};
constexpr uint64_t kPersistWaitTicks = 200000000ull;  // default wait bound: 2 s
constexpr int kPersistThreads = 512;
constexpr int64_t kPersistMaxChains = 1024;  // chains of a set that can take the persistent shapes
static_assert(kSlotsOffset + 32 * kPersistMaxChains <= kVarOffset, "persistent sweep slots overlap the partials");

__device__ __forceinline__ uint32_t ld_agent(const unsigned int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_agent64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TH>
__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(4))) void sweep_tile_persist_kernel(ChainDesc *descs, ChainState *states,
                                                                             BlockMap bm, SweepConsts sc,
                                                                             FusedControl ctl, PersistCtl pc)
{
    constexpr int NW = kPersistThreads / 64;
    __shared__ TileShared<TH, NW> L;
    __shared__ TilePre<TH> P;
    __shared__ ChainState sst;  // this block's copy of its chain's state
    __shared__ int sh_last, sh_stop;
    const int tid = (int)threadIdx.x;
    for (int w = tid; w < TileShared<TH, NW>::RW; w += kPersistThreads) L.redo[w] = 0u;
    // the tile of this block (the XCD-aware order of sweep_tile_kernel)
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t per = G >> 3, rem = G & 7u, xcd = b & 7u;
    const int64_t lbk = (int64_t)xcd * per + (int64_t)min(xcd, rem) + (int64_t)(b >> 3);
    int lb;
    const int cid = chain_of_block(bm, lbk, &lb);
    const bool lead = lb == 0;  // the chain's first block
    unsigned long long *const slot = pc.slots + 4 * cid;
    // descriptor and state as of the launch (earlier kernels wrote them)
    ChainDesc d = descs[cid];
    {
        const unsigned long long *src = reinterpret_cast<const unsigned long long *>(states + cid);
        unsigned long long *dst = reinterpret_cast<unsigned long long *>(&sst);
        for (int k = tid; k < (int)(sizeof(ChainState) / 8); k += kPersistThreads) dst[k] = src[k];
    }
    const int nbx = d.S / kTileH;
    const int ty = lb / nbx, tx = lb - ty * nbx;
    const int y0 = ty * TH, hx0 = tx * kTileH;
    const bool edge = !(ty >= 1 && y0 + TH + 2 <= d.ny && tx >= 1 && hx0 + kTileH + 2 <= (d.nx >> 1));
    const bool sums = d.acc[0] != nullptr;
    __syncthreads();
    int phase = sst.phase;  // the chain's phase as of the last control
    bool swept = false;     // the previous loop pass swept the chain (its control is due)
    for (int i = 0; i < pc.count; ++i) {
        // the control of the previous sweep: its sums (coherent loads) are
        // read while the tile is staged
        unsigned long long te = 0ull, ta = 0ull;
        const bool due = swept;
        if (tid == 0 && due) {
            te = ld_agent64(slot + 2 * ((i - 1) & 1));
            ta = ld_agent64(slot + 2 * ((i - 1) & 1) + 1);
        }
        // the equilibrium sums are staged too when the last sweep was an
        // equilibrium one (the next is then one as well, or none)
        const bool pre = sums && phase == PH_EQ;
        if (phase != PH_DONE) tile_stage<TH, NW>(L, pre ? &P : nullptr, d, y0, hx0);
        if (tid == 0 && due) {
            sst.e_fx = te;
            sst.acc = ta;
            control_core(sst, d, ctl.cp, lead ? ctl.done_count : nullptr, lead ? ctl.work : nullptr);
        }
        if (tid < 2) L.any_redo[tid] = 0;
        __syncthreads();
        const SweepState ss = sweep_state_of(&sst);
        phase = ss.phase;
        swept = phase != PH_DONE;
        if (swept) {
            uint64_t e_thread = 0u;
            uint32_t acc_thread = 0u;
            const TilePre<TH> *pp = pre ? &P : nullptr;
            if (edge)
                tile_update<false, TH, true, NW>(L, pp, d, ss, y0, hx0, 0, sc, 0, nullptr, e_thread, acc_thread);
            else
                tile_update<false, TH, false, NW>(L, pp, d, ss, y0, hx0, 0, sc, 0, nullptr, e_thread, acc_thread);
            if (ss.phase != PH_EQ) tile_block_sums(L, e_thread, acc_thread, slot + 2 * (i & 1), slot + 2 * (i & 1) + 1);
            // the sweep wrote h2: exchange the buffers (as sweep_tile_kernel's last block does in memory)
            float *t0 = d.h[0], *t1 = d.h[1];
            d.h[0] = d.h2[0];
            d.h[1] = d.h2[1];
            d.h2[0] = t0;
            d.h2[1] = t1;
            if (tid == 0) sst.swapped ^= 1;
        }
        // arrive: this wave's stores are in L2, then one write-back per block
        __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            sh_last = atomicAdd(ctl.ticket, 1u) == G - 1u;
        }
        __syncthreads();
        if (sh_last) {
            // every block has read the sums of the previous sweep: clear
            // their slots for the sweep after next
            for (int k = tid; k < bm.n; k += kPersistThreads) {
                unsigned long long *sk = pc.slots + 4 * bm.id[k] + 2 * ((i + 1) & 1);
                __hip_atomic_store(sk, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(sk + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
            __syncthreads();
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const bool stop = i + 1 >= pc.count || ld_agent(ctl.done_count) >= pc.need || ld_agent(pc.abort) != 0u;
                __hip_atomic_store(ctl.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(pc.gen, (uint32_t)(i + 1) | (stop ? 0x80000000u : 0u), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                sh_stop = stop ? 1 : 0;
            }
        } else if (tid == 0) {
            const uint64_t t0 = wall_clock64();
            int stop = 0;
            for (;;) {
                const uint32_t g = ld_agent(pc.gen);
                if ((g & 0x7FFFFFFFu) >= (uint32_t)(i + 1)) {
                    stop = (g >> 31) ? 1 : 0;
                    break;
                }
                if (ld_agent(pc.abort) != 0u) {
                    stop = 1;
                    break;
                }
                if ((uint64_t)(wall_clock64() - t0) > pc.wait_ticks) {
                    __hip_atomic_store(pc.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            sh_stop = stop;
        }
        __syncthreads();
        if (sh_stop) {
            // the control of the last sweep updated
            if (tid == 0 && swept) {
                sst.e_fx = ld_agent64(slot + 2 * (i & 1));
                sst.acc = ld_agent64(slot + 2 * (i & 1) + 1);
                control_core(sst, d, ctl.cp, lead ? ctl.done_count : nullptr, lead ? ctl.work : nullptr);
            }
            break;
        }
    }
    // the chain's first block writes its state and descriptor back
    __syncthreads();
    if (lead) {
        const unsigned long long *src = reinterpret_cast<const unsigned long long *>(&sst);
        unsigned long long *dst = reinterpret_cast<unsigned long long *>(states + cid);
        for (int k = tid; k < (int)(sizeof(ChainState) / 8); k += kPersistThreads) dst[k] = src[k];
        if (tid == 0) {
            descs[cid].h[0] = d.h[0];
            descs[cid].h[1] = d.h[1];
            descs[cid].h2[0] = d.h2[0];
            descs[cid].h2[1] = d.h2[1];
        }
    }
}

// The double-precision sweep: the layout of half_sweep_body (a thread per
// pair of neighbouring sites of one half-row, one Philox call per pair) on
// half-grids of doubles, each site updated by update_site_d.  Every decision
// is final here, so nothing is deferred.  Bond energies are summed in fixed
// point of 2^-30.
template <bool DIAG, int ROWS>
__global__ __launch_bounds__(kBlock) void half_sweep_fp64_kernel(const ChainDesc *__restrict__ descs,
                                                                 ChainState *__restrict__ states,
                                                                 BlockMap bm,
                                                                 int colour, SweepConsts sc, int or_only,
                                                                 uint8_t *__restrict__ flags)
{
    constexpr int PX = kBlock / ROWS;
    int lb;
    const int c = chain_of_block(bm, (int64_t)blockIdx.x, &lb);
    ChainState *stp = states + c;
    const int phase = stp->phase;
    if (phase == PH_DONE) return;
    const ChainDesc d = descs[c];
    const int nbx = ((d.S >> 1) + PX - 1) / PX;
    const int by = lb / nbx;
    const int bx = lb - by * nbx;
    const int y = by * ROWS + (int)(threadIdx.x / PX);
    const int h0 = 2 * (bx * PX + (int)(threadIdx.x % PX));
    const uint32_t sweep = stp->sweep;
    const double T = stp->T, a = stp->a_cur;
    const bool want_energy = (colour == 1) && (phase != PH_EQ);
    const bool want_acc = phase != PH_EQ;
    unsigned long long e_thread = 0ull;
    uint32_t acc_thread = 0u;

    if (y < d.ny) {
        const int s = (y + colour) & 1;
        const int W = (d.nx - s + 1) >> 1;
        const int Wo = (d.nx + s) >> 1;
        if (h0 < W) {
            const bool two = (h0 + 1) < W;
            double *mine = (double *)(colour ? d.h[1] : d.h[0]) + (int64_t)y * d.S;
            const double *oth = (const double *)(colour ? d.h[0] : d.h[1]) + (int64_t)y * d.S;
            const bool vL = h0 + s - 1 >= 0, vM = h0 + s < Wo, vR = h0 + s + 1 < Wo;
            const bool vU = y > 0, vD = y + 1 < d.ny;
            const double2 v = gldd2(mine + h0);
            const double oL = fabs(gldd(oth + max(h0 + s - 1, 0)));
            const double oM = fabs(gldd(oth + h0 + s));
            const double oR = fabs(gldd(oth + min(h0 + s + 1, d.S - 1)));
            const double2 up = gldd2(oth + (vU ? -(int64_t)d.S : 0) + h0);
            const double2 dn = gldd2(oth + (vD ? (int64_t)d.S : 0) + h0);
            const bool fixed0 = is_fixed_d(v.x), fixed1 = !two || is_fixed_d(v.y);
            double u0 = 0.5, r0 = 0.5, u1 = 0.5, r1 = 0.5;
            if (!or_only && (!fixed0 || !fixed1)) {
                const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * h0 + s), sweep, d.chain, d.image_id};
                const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
                u0 = (double)unit24(w.x);
                r0 = (double)unit24(w.y);
                u1 = (double)unit24(w.z);
                r1 = (double)unit24(w.w);
            }
            const uint32_t val0 = (vL ? 1u : 0u) | (vM ? 2u : 0u) | (vU ? 4u : 0u) | (vD ? 8u : 0u);
            const uint32_t val1 = 1u | (vR ? 2u : 0u) | (vU ? 4u : 0u) | (vD ? 8u : 0u);
            const SiteOutD o0 = update_site_d(fabs(v.x), oL, oM, fabs(up.x), fabs(dn.x), val0, u0, r0, a, T,
                                              sc.q64, or_only != 0);
            const SiteOutD o1 = update_site_d(fabs(v.y), oM, oR, fabs(up.y), fabs(dn.y), val1, u1, r1, a, T,
                                              sc.q64, or_only != 0);
            const bool w0 = !fixed0, w1 = two && !fixed1;
            const double out0 = w0 ? o0.phi : v.x;
            const double out1 = w1 ? o1.phi : v.y;
            if (two) gstd2(mine + h0, make_double2(out0, out1));
            else if (w0) gstd(mine + h0, out0);
            double *accp = (double *)(colour ? d.acc[1] : d.acc[0]);
            if (phase == PH_EQ && accp) {
                double *acc = accp + (int64_t)y * d.S;
                double *m2p = (double *)(colour ? d.m2[1] : d.m2[0]);
                double *m2 = m2p ? m2p + (int64_t)y * d.S : nullptr;
                const double ik = stp->inv_k_d, ikm1 = stp->inv_km1_d;
                if (w0) accumulate_state_d(acc + h0, m2 ? m2 + h0 : nullptr, out0, ik, ikm1);
                if (w1) accumulate_state_d(acc + h0 + 1, m2 ? m2 + h0 + 1 : nullptr, out1, ik, ikm1);
            }
            acc_thread = (w0 && o0.accepted ? 1u : 0u) + (w1 && o1.accepted ? 1u : 0u);
            if (want_energy)
                e_thread = energy_fx_d(fixed0 ? o0.e_before : o0.e_bonds) +
                           (!two ? 0ull : energy_fx_d(fixed1 ? o1.e_before : o1.e_bonds));
            if (DIAG && flags) {
                const int64_t x0 = 2 * h0 + s;
                if (w0) flags[(int64_t)y * d.nx + x0] = (uint8_t)o0.flags;
                if (w1) flags[(int64_t)y * d.nx + x0 + 2] = (uint8_t)o1.flags;
            }
        }
    }
    if (!want_acc) return;
    // block sums: a thread's energy is below 2^34 and its count at most 2,
    // so 64-bit lane sums hold both (count in the top 8 bits)
    unsigned long long sum = e_thread | ((unsigned long long)acc_thread << 56);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    __shared__ unsigned long long red[kBlock / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0ull, n = 0ull;
        for (int i = 0; i < kBlock / 64; ++i) {
            e += red[i] & 0x00FFFFFFFFFFFFFFull;
            n += red[i] >> 56;
        }
        if (e) atomicAdd(&stp->e_fx, e);
        if (n) atomicAdd(&stp->acc, n);
    }
}

// The double-precision sweep with the gap sites compacted onto consecutive
// lanes: the list building of half_sweep_compact_body (1024 sites per block,
// CR half-rows, two site pairs per thread, the pair's Philox words drawn in
// pass 1) on double half-grids, each listed gap site updated by
// update_site_d and each sampled site of colour 1 given its bond energy by
// bond_energy_d when the sweep's energy is wanted.  Per site the arithmetic
// is that of half_sweep_fp64_kernel, so the results are bit-identical to it.
template <bool DIAG, int CR>
__global__ __launch_bounds__(kBlock) void half_sweep_fp64_compact_kernel(const ChainDesc *__restrict__ descs,
                                                                         ChainState *__restrict__ states,
                                                                         BlockMap bm, int colour, SweepConsts sc,
                                                                         int or_only, uint8_t *__restrict__ flags)
{
    constexpr int PPR = kCompactSites / CR / 2;  // site pairs per block row
    constexpr int NW = kBlock / 64;
    __shared__ uint2 gap_list[kCompactSites];  // as in half_sweep_compact_body
    __shared__ uint16_t fixed_list[kCompactSites];
    __shared__ uint32_t wave_count[2][2][NW];
    __shared__ unsigned long long red[NW];

    int lb;
    const int c = chain_of_block(bm, (int64_t)blockIdx.x, &lb);
    ChainState *stp = states + c;
    const int phase = stp->phase;
    if (phase == PH_DONE) return;
    const ChainDesc d = descs[c];
    const int nbx = ((d.S >> 1) + PPR - 1) / PPR;
    const int by = lb / nbx;
    const int bx = lb - by * nbx;
    const uint32_t sweep = stp->sweep;
    const double T = stp->T, a_cur = stp->a_cur;
    const bool want_energy = (colour == 1) && (phase != PH_EQ);
    const bool want_acc = phase != PH_EQ;
    double *const mine = (double *)(colour ? d.h[1] : d.h[0]);
    const double *const oth = (const double *)(colour ? d.h[0] : d.h[1]);
    double *const accp = (phase == PH_EQ) ? (double *)(colour ? d.acc[1] : d.acc[0]) : nullptr;
    double *const m2p = accp ? (double *)(colour ? d.m2[1] : d.m2[0]) : nullptr;

    // pass 1: pairs t and t + 256 of the block, both read first
    bool gap[2][2], fix[2][2];
    uint32_t wu[2][2], wr[2][2];
    double2 pv[2];
    bool in[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pi = (int)threadIdx.x + j * kBlock;
        const int y = by * CR + pi / PPR;
        const int h0 = 2 * (bx * PPR + pi % PPR);
        const int s = (y + colour) & 1;
        in[j] = y < d.ny && h0 < ((d.nx - s + 1) >> 1);
        // rows and pairs outside the grid read pair 0 of row 0 instead
        pv[j] = gldd2(mine + (in[j] ? (int64_t)y * d.S + h0 : 0));
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pi = (int)threadIdx.x + j * kBlock;
        const int y = by * CR + pi / PPR;
        const int h0 = 2 * (bx * PPR + pi % PPR);
        const int s = (y + colour) & 1;
        const bool two = in[j] && (h0 + 1) < ((d.nx - s + 1) >> 1);
        gap[j][0] = in[j] && !is_fixed_d(pv[j].x);
        gap[j][1] = two && !is_fixed_d(pv[j].y);
        fix[j][0] = want_energy && in[j] && !gap[j][0];
        fix[j][1] = want_energy && two && !gap[j][1];
        wu[j][0] = wu[j][1] = wr[j][0] = wr[j][1] = 0u;
        if (!or_only && (gap[j][0] || gap[j][1])) {
            const U4 ctr = {(uint32_t)y * (uint32_t)d.nx + (uint32_t)(2 * h0 + s), sweep, d.chain, d.image_id};
            const U4 w = philox4x32_10(ctr, sc.seed_lo, sc.seed_hi);
            wu[j][0] = w.x;
            wr[j][0] = w.y;
            wu[j][1] = w.z;
            wr[j][1] = w.w;
        }
    }
    const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t pre[2][2] = {{0u, 0u}, {0u, 0u}};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
        if (L == 1 && !want_energy) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint64_t b0 = __ballot(L ? fix[j][0] : gap[j][0]);
            const uint64_t b1 = __ballot(L ? fix[j][1] : gap[j][1]);
            pre[L][j] = (uint32_t)(__popcll(b0 & below) + __popcll(b1 & below));
            if (lane == 0) wave_count[L][j][wid] = (uint32_t)(__popcll(b0) + __popcll(b1));
        }
    }
    __syncthreads();
    int n_list[2] = {0, 0};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
        if (L == 1 && !want_energy) continue;
        uint32_t base0 = 0u, base1 = 0u, tot0 = 0u, tot1 = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t c0 = wave_count[L][0][w], c1 = wave_count[L][1][w];
            base0 += (w < wid) ? c0 : 0u;
            base1 += (w < wid) ? c1 : 0u;
            tot0 += c0;
            tot1 += c1;
        }
        n_list[L] = (int)(tot0 + tot1);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            uint32_t pos = (j ? tot0 + base1 : base0) + pre[L][j];
            const uint32_t pi = threadIdx.x + (uint32_t)j * kBlock;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t idx = 2u * pi + (uint32_t)k;
                if (L == 0 && gap[j][k]) {
                    gap_list[pos] = make_uint2((wu[j][k] & 0xFFFFFF00u) | (idx & 0xFFu),
                                               (wr[j][k] & 0xFFFFFF00u) | (idx >> 8));
                    ++pos;
                }
                if (L == 1 && fix[j][k]) {
                    fixed_list[pos] = (uint16_t)idx;
                    ++pos;
                }
            }
        }
    }
    __syncthreads();

    // a listed site: row, half-row position, colour offset, valid neighbours,
    // and its four neighbours (loaded from clamped positions when missing)
    auto locate = [&](uint32_t idx, int &y, int &h, int &s, uint32_t &valid) {
        const int pi = (int)(idx >> 1);
        y = by * CR + pi / PPR;
        h = 2 * (bx * PPR + pi % PPR) + (int)(idx & 1u);
        s = (y + colour) & 1;
        const int Wo = (d.nx + s) >> 1;
        valid = (h + s - 1 >= 0 ? 1u : 0u) | (h + s < Wo ? 2u : 0u) | (y > 0 ? 4u : 0u) | (y + 1 < d.ny ? 8u : 0u);
    };
    auto neighbours = [&](int y, int h, int s, uint32_t valid, double &nL, double &nR, double &nU, double &nD) {
        const double *orow = oth + (int64_t)y * d.S;
        nL = fabs(gldd(orow + max(h + s - 1, 0)));
        nR = fabs(gldd(orow + min(h + s, d.S - 1)));
        nU = fabs(gldd(orow + ((valid & 4u) ? -(int64_t)d.S : 0) + h));
        nD = fabs(gldd(orow + ((valid & 8u) ? (int64_t)d.S : 0) + h));
    };

    // a thread takes at most 4 gap and 4 sampled sites, each below 2^33 in
    // energy units: the energy stays below 2^44 over a block, the count
    // (at most 1024) rides in the top 12 bits
    unsigned long long e_thread = 0ull;
    uint32_t acc_thread = 0u;
    // pass 2: the listed gap sites.  Unrolled over a thread's at most four
    // entries: in a loop the compiler keeps the double update's constants in
    // registers across iterations (~116 VGPRs, 4 waves per SIMD); unrolled,
    // the kernel takes 50 (8 waves)
#pragma unroll
    for (int k = 0; k < kCompactSites / kBlock; ++k) {
        const int i = (int)threadIdx.x + k * kBlock;
        if (i >= n_list[0]) break;
        const uint2 e = gap_list[i];
        int y, h, s;
        uint32_t valid;
        locate((e.x & 0xFFu) | ((e.y & 0xFFu) << 8), y, h, s, valid);
        double nL, nR, nU, nD;
        neighbours(y, h, s, valid, nL, nR, nU, nD);
        double *sp = mine + (int64_t)y * d.S + h;
        const double a = fabs(gldd(sp));
        // the low 8 bits of each word hold the index; unit24 uses the top 24
        const double u = or_only ? 0.5 : (double)unit24(e.x);
        const double r = or_only ? 0.5 : (double)unit24(e.y);
        const SiteOutD o = update_site_d(a, nL, nR, nU, nD, valid, u, r, a_cur, T, sc.q64, or_only != 0);
        gstd(sp, o.phi);
        if (accp)
            accumulate_state_d(accp + (int64_t)y * d.S + h, m2p ? m2p + (int64_t)y * d.S + h : nullptr, o.phi,
                               stp->inv_k_d, stp->inv_km1_d);
        acc_thread += o.accepted ? 1u : 0u;
        if (want_energy) e_thread += energy_fx_d(o.e_bonds);
        if (DIAG && flags) flags[(int64_t)y * d.nx + 2 * h + s] = (uint8_t)o.flags;
    }
    // pass 3: bond energies of the sampled sites of colour 1
#pragma unroll
    for (int k = 0; k < kCompactSites / kBlock; ++k) {
        const int i = (int)threadIdx.x + k * kBlock;
        if (i >= n_list[1]) break;
        int y, h, s;
        uint32_t valid;
        locate((uint32_t)fixed_list[i], y, h, s, valid);
        double nL, nR, nU, nD;
        neighbours(y, h, s, valid, nL, nR, nU, nD);
        const double a = fabs(gldd(mine + (int64_t)y * d.S + h));
        e_thread += energy_fx_d(bond_energy_d(a, nL, nR, nU, nD, valid, sc.q64));
    }
    if (!want_acc) return;
    unsigned long long sum = e_thread | ((unsigned long long)acc_thread << 52);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (lane == 0) red[wid] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0ull, n = 0ull;
        for (int i = 0; i < NW; ++i) {
            e += red[i] & 0x000FFFFFFFFFFFFFull;
            n += red[i] >> 52;
        }
        if (e) atomicAdd(&stp->e_fx, e);
        if (n) atomicAdd(&stp->acc, n);
    }
}

// control_chain for every chain, one thread per chain.  With `swap` (after
// a fused tile sweep, which read h and wrote h2) it first exchanges h and h2
// of every chain that sweep updated (those not done), toggling the chain's
// `swapped` flag; with `control` 0 it does only that.
__global__ void control_kernel(ChainDesc *__restrict__ descs, ChainState *__restrict__ states, int n,
                               CtlParams cp, unsigned int *done_count, unsigned long long *work, int swap,
                               int control)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (swap && states[c].phase != PH_DONE) {
        ChainDesc &d = descs[c];
        float *t0 = d.h[0], *t1 = d.h[1];
        d.h[0] = d.h2[0];
        d.h[1] = d.h2[1];
        d.h2[0] = t0;
        d.h2[1] = t1;
        states[c].swapped ^= 1;
    }
    if (control) control_chain(descs, states, c, cp, done_count, work);
}

// Zeroes the control words given (null: skipped) and n64 64-bit words at
// `wide`, in one launch of one block: the counters and barrier words a run of
// sweeps starts from (one small kernel in place of a memset per word).
__global__ void clear_words_kernel(unsigned int *w0, unsigned int *w1, unsigned int *w2,
                                   unsigned long long *wide, int n64)
{
    const int t = (int)threadIdx.x;
    if (t == 0) {
        if (w0) *w0 = 0u;
        if (w1) *w1 = 0u;
        if (w2) *w2 = 0u;
    }
    for (int k = t; k < n64; k += (int)blockDim.x) wide[k] = 0ull;
}

// 1 for every chain that is done, else 0 (for rebuilding the launch list).
__global__ void done_flags_kernel(const ChainState *__restrict__ states, int n, uint8_t *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) out[c] = states[c].phase == PH_DONE ? 1 : 0;
}

// phi_sum at every site of image blockIdx.y: sum over its R chains of the
// equilibrium sums (K > 1) or the final states (K == 1).  With phi_m2, also
// the sum over the R K states of the squared deviation from their mean: two
// passes over the R final states (K == 1), or the chains' own sums combined
// with the spread of their means (Chan et al.'s pairwise rule, K > 1).
__global__ void finalize_kernel(const ChainDesc *__restrict__ descs, const ImgDev *__restrict__ imgs, int R,
                                int K, const uint8_t *__restrict__ sampled, float *__restrict__ phi_sum,
                                float *__restrict__ phi_m2)
{
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const ChainDesc *dc = descs + (int64_t)blockIdx.y * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f, q = 0.0f;
        if (!sampled[im.offset + i] && K > 0) {
            const int y = (int)(i / im.nx);
            const int x = (int)(i - (int64_t)y * im.nx);
            const int c = (x + y) & 1;
            const int64_t j = (int64_t)y * dc[0].S + (x >> 1);
            for (int r = 0; r < R; ++r) s += (K > 1) ? dc[r].acc[c][j] : angle_of(dc[r].h[c][j]);
            if (phi_m2) {
                const float mean = s / (float)(R * K);
                for (int r = 0; r < R; ++r) {
                    const float d = ((K > 1) ? dc[r].acc[c][j] / (float)K : angle_of(dc[r].h[c][j])) - mean;
                    q = fmaf((float)K * d, d, q);
                    if (K > 1) q += dc[r].m2[c][j];
                }
            }
        }
        phi_sum[im.offset + i] = s;
        if (phi_m2) phi_m2[im.offset + i] = q;
    }
}

// finalize_kernel for double-precision chains: the same sums taken in
// double and rounded once.
__global__ void finalize_fp64_kernel(const ChainDesc *__restrict__ descs, const ImgDev *__restrict__ imgs, int R,
                                     int K, const uint8_t *__restrict__ sampled, float *__restrict__ phi_sum,
                                     float *__restrict__ phi_m2)
{
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const ChainDesc *dc = descs + (int64_t)blockIdx.y * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0, q = 0.0;
        if (!sampled[im.offset + i] && K > 0) {
            const int y = (int)(i / im.nx);
            const int x = (int)(i - (int64_t)y * im.nx);
            const int c = (x + y) & 1;
            const int64_t j = (int64_t)y * dc[0].S + (x >> 1);
            for (int r = 0; r < R; ++r)
                s += (K > 1) ? ((const double *)dc[r].acc[c])[j] : fabs(((const double *)dc[r].h[c])[j]);
            if (phi_m2) {
                const double mean = s / (double)(R * K);
                for (int r = 0; r < R; ++r) {
                    const double dv = ((K > 1) ? ((const double *)dc[r].acc[c])[j] / (double)K
                                               : fabs(((const double *)dc[r].h[c])[j])) - mean;
                    q = fma((double)K * dv, dv, q);
                    if (K > 1) q += ((const double *)dc[r].m2[c])[j];
                }
            }
        }
        phi_sum[im.offset + i] = (float)s;
        if (phi_m2) phi_m2[im.offset + i] = (float)q;
    }
}

// Records the current states of the listed chains that are in their
// equilibrium phase (after both half-sweeps of an equilibrium sweep, before
// the control kernel counts it): state r K + k of chain r after its k-th
// equilibrium sweep goes to out[(r K + k) n_total + offset + i], row-major
// over the image's sites (samples included).  `segs` blocks per listed chain.
__global__ void record_states_kernel(const ChainDesc *__restrict__ descs, const ChainState *__restrict__ states,
                                     const int64_t *__restrict__ offsets, const int32_t *__restrict__ ids,
                                     int segs, int K, int fp64, int64_t n_total, float *__restrict__ out)
{
    const int c = ids[blockIdx.x / segs];
    const ChainState *stp = states + c;
    if (stp->phase != PH_EQ) return;
    const ChainDesc d = descs[c];
    const int64_t n = (int64_t)d.nx * d.ny;
    const int64_t m = (int64_t)d.chain * K + (K - stp->eq_left);
    float *o = out + m * n_total + offsets[c];
    const int seg = (int)(blockIdx.x % segs);
    for (int64_t i = (int64_t)seg * blockDim.x + threadIdx.x; i < n; i += (int64_t)segs * blockDim.x) {
        const int y = (int)(i / d.nx);
        const int x = (int)(i - (int64_t)y * d.nx);
        const int64_t j = (int64_t)y * d.S + (x >> 1);
        const float *hp = ((x + y) & 1) ? d.h[1] : d.h[0];
        o[i] = fp64 ? (float)fabs(((const double *)hp)[j]) : angle_of(hp[j]);
    }
}

// Quantiles of the M realizations at each gap site of image blockIdx.y: the
// M states (states[m n_total + site]) are sorted in LDS (insertion sort, one
// wave per block, a lane's values 64 apart so that lanes use distinct banks),
// the p-quantile interpolates linearly between the order statistics around
// h = (M - 1) p, and is back-transformed like the mean (double precision,
// rounded once).  Sampled sites get their data value.
constexpr int kQuantileLanes = 64;
constexpr int kMaxQuantileStates = 256;

__global__ __launch_bounds__(kQuantileLanes) void quantile_kernel(const ImgDev *__restrict__ imgs,
                                                                  const double *__restrict__ zmm,
                                                                  const double *__restrict__ probs, int nq,
                                                                  const float *__restrict__ z,
                                                                  const uint8_t *__restrict__ sampled,
                                                                  const float *__restrict__ st, int M,
                                                                  int64_t n_total, float *__restrict__ out)
{
#pragma clang fp contract(off)
    __shared__ float v[kMaxQuantileStates * kQuantileLanes];
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const double lo = zmm[2 * blockIdx.y], hi = zmm[2 * blockIdx.y + 1];
    const int t = threadIdx.x;
    for (int64_t i0 = (int64_t)blockIdx.x * kQuantileLanes; i0 < n; i0 += (int64_t)gridDim.x * kQuantileLanes) {
        const int64_t i = i0 + t;
        if (i >= n) continue;
        const int64_t k = im.offset + i;
        if (sampled[k]) {
            for (int q = 0; q < nq; ++q) out[q * n_total + k] = z[k];
            continue;
        }
        for (int m = 0; m < M; ++m) {
            // insertion of state m into the sorted prefix
            const float x = st[(int64_t)m * n_total + k];
            int j = m - 1;
            while (j >= 0 && v[j * kQuantileLanes + t] > x) {
                v[(j + 1) * kQuantileLanes + t] = v[j * kQuantileLanes + t];
                --j;
            }
            v[(j + 1) * kQuantileLanes + t] = x;
        }
        for (int q = 0; q < nq; ++q) {
            const double h = (double)(M - 1) * probs[q];
            const int a = (int)floor(h);
            double phi_p;
            if (a >= M - 1) {
                phi_p = (double)v[(M - 1) * kQuantileLanes + t];
            } else {
                const double va = (double)v[a * kQuantileLanes + t], vb = (double)v[(a + 1) * kQuantileLanes + t];
                phi_p = va + (h - (double)a) * (vb - va);
            }
            const double tt = phi_p / kTwoPi;
            out[q * n_total + k] = (float)(lo * (1.0 - tt) + hi * tt);
        }
    }
}

// The sampled sites kept for fitting when a fraction `hold` of them is held
// out for validation: a sample is held out when the uniform of its site,
// word 0 of Philox4x32-10 with counter (y nx + x, 0xFFFFFFFE, 0, 0x40000000)
// and the seed as key, is below `hold`.
constexpr uint32_t kHoldoutSweep = 0xFFFFFFFEu;
constexpr uint32_t kHoldoutStream = 0x40000000u;

__global__ void holdout_kernel(int nx, int ny, const uint8_t *__restrict__ sampled, uint32_t seed_lo,
                               uint32_t seed_hi, double hold, uint8_t *__restrict__ fit)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t keep = 0;
        if (sampled[i]) {
            const U4 w = philox4x32_10(U4{(uint32_t)i, kHoldoutSweep, 0u, kHoldoutStream}, seed_lo, seed_hi);
            keep = (double)unit24(w.x) < hold ? 0 : 1;
        }
        fit[i] = keep;
    }
}

// Partial sums of |z - z_hat| and counts over the held-out samples
// (sampled but not kept for fitting), one pair per block.
__global__ void holdout_error_kernel(int64_t n, const float *__restrict__ z, const uint8_t *__restrict__ sampled,
                                     const uint8_t *__restrict__ fit, const float *__restrict__ z_hat,
                                     double *__restrict__ psum, unsigned long long *__restrict__ pcount)
{
    double s = 0.0;
    unsigned long long c = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (sampled[i] && !fit[i]) {
            s += fabs((double)z[i] - (double)z_hat[i]);
            ++c;
        }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        c += __shfl_xor(c, off);
    }
    __shared__ double ss[kBlock / 64];
    __shared__ unsigned long long sc[kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        ss[threadIdx.x >> 6] = s;
        sc[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            ss[0] += ss[i];
            sc[0] += sc[i];
        }
        psum[blockIdx.x] = ss[0];
        pcount[blockIdx.x] = sc[0];
    }
}

// Sorts v[0..N-1] ascending with Batcher's odd-even merge sort, a fixed
// network of compare-exchanges: with N a compile-time constant and every loop
// unrolled, all indices are constants, so v stays in registers.
template <int N>
__device__ __forceinline__ void odd_even_merge_sort(float (&v)[N])
{
#pragma unroll
    for (int p = 1; p < N; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const float a = v[i + j], b = v[i + j + k];
                        v[i + j] = fminf(a, b);
                        v[i + j + k] = fmaxf(a, b);
                    }
}

// quantile_kernel for M <= N states per site with the sort in registers (a
// thread per site; states beyond M are +inf and sort last); the order
// statistics at the runtime positions are picked by unrolled selects.
template <int N>
__global__ __launch_bounds__(kBlock) void quantile_net_kernel(const ImgDev *__restrict__ imgs,
                                                              const double *__restrict__ zmm,
                                                              const double *__restrict__ probs, int nq,
                                                              const float *__restrict__ z,
                                                              const uint8_t *__restrict__ sampled,
                                                              const float *__restrict__ st, int M, int64_t n_total,
                                                              float *__restrict__ out)
{
#pragma clang fp contract(off)
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const double lo = zmm[2 * blockIdx.y], hi = zmm[2 * blockIdx.y + 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = im.offset + i;
        if (sampled[k]) {
            for (int q = 0; q < nq; ++q) out[q * n_total + k] = z[k];
            continue;
        }
        float v[N];
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = m < M ? st[(int64_t)m * n_total + k] : INFINITY;
        odd_even_merge_sort<N>(v);
        for (int q = 0; q < nq; ++q) {
            const double h = (double)(M - 1) * probs[q];
            const int a = (int)floor(h);
            float va = v[0], vb = v[0];
#pragma unroll
            for (int m = 0; m < N; ++m) {
                va = m == a ? v[m] : va;
                vb = m == a + 1 ? v[m] : vb;
            }
            const double phi_p = a >= M - 1 ? (double)va : (double)va + (h - (double)a) * ((double)vb - (double)va);
            const double tt = phi_p / kTwoPi;
            out[q * n_total + k] = (float)(lo * (1.0 - tt) + hi * tt);
        }
    }
}

// Spread of the prediction: the standard deviation over the M realizations
// of z = G^{-1}(phi), which is (z_max - z_min) / (2 pi) times that of phi,
// sqrt(m2 / (M - 1)); zero at sampled sites and for M = 1.
__global__ void spread_kernel(const ImgDev *__restrict__ imgs, const double *__restrict__ zmin_zmax, int M,
                              const uint8_t *__restrict__ sampled, const float *__restrict__ phi_m2,
                              float *__restrict__ z_std)
{
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const double scale = (zmin_zmax[2 * blockIdx.y + 1] - zmin_zmax[2 * blockIdx.y]) / kTwoPi;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = im.offset + i;
        float v = 0.0f;
        if (!sampled[k] && M > 1) v = (float)(scale * sqrt(fmax((double)phi_m2[k], 0.0) / (double)(M - 1)));
        z_std[k] = v;
    }
}

// Half-grids of one double-precision chain back to a full row-major grid.
__global__ void unsplit_fp64_kernel(const ChainDesc *__restrict__ descs, double *__restrict__ phi)
{
    const ChainDesc d = descs[0];
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / d.nx);
        const int x = (int)(i - (int64_t)y * d.nx);
        const double *hp = (const double *)(((x + y) & 1) ? d.h[1] : d.h[0]);
        phi[i] = fabs(hp[(int64_t)y * d.S + (x >> 1)]);
    }
}

// Half-grids of one chain back to a full row-major grid of angles.
__global__ void unsplit_kernel(const ChainDesc *__restrict__ descs, float *__restrict__ phi)
{
    const ChainDesc d = descs[0];
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / d.nx);
        const int x = (int)(i - (int64_t)y * d.nx);
        const float *hp = ((x + y) & 1) ? d.h[1] : d.h[0];
        phi[i] = angle_of(hp[(int64_t)y * d.S + (x >> 1)]);
    }
}

// Energy of a full grid of angles as the sweep accumulates it.
__global__ void grid_energy_kernel(const float *__restrict__ phi, int nx, int ny, float q,
                                   unsigned long long *out)
{
    unsigned long long e = 0ull;
    const int64_t n = (int64_t)nx * ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / nx);
        const int x = (int)(i - (int64_t)y * nx);
        if (((x + y) & 1) != 1) continue;
        float nb[4] = {0.f, 0.f, 0.f, 0.f};
        uint32_t valid = 0u;
        if (x > 0) { nb[0] = phi[i - 1]; valid |= 1u; }
        if (x + 1 < nx) { nb[1] = phi[i + 1]; valid |= 2u; }
        if (y > 0) { nb[2] = phi[i - nx]; valid |= 4u; }
        if (y + 1 < ny) { nb[3] = phi[i + nx]; valid |= 8u; }
        e += energy_fx(site_energy(phi[i], nb, valid, q));
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(out, e);
}

// Per-block min / max / count of the sampled values of image blockIdx.y.
__global__ void map_minmax_kernel(const ImgDev *__restrict__ imgs, const float *__restrict__ z,
                                  const uint8_t *__restrict__ sampled, float *__restrict__ pmin,
                                  float *__restrict__ pmax, unsigned long long *__restrict__ pcount,
                                  unsigned int *__restrict__ pbad)
{
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    float lo = INFINITY, hi = -INFINITY;
    unsigned long long cnt = 0ull;
    unsigned int bad = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!sampled[im.offset + i]) continue;
        const float v = z[im.offset + i];
        if (!isfinite(v)) {
            bad = 1u;
            continue;
        }
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
        ++cnt;
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off));
        hi = fmaxf(hi, __shfl_xor(hi, off));
        cnt += __shfl_xor(cnt, off);
        bad |= __shfl_xor(bad, off);
    }
    __shared__ float slo[kBlock / 64], shi[kBlock / 64];
    __shared__ unsigned long long scnt[kBlock / 64];
    __shared__ unsigned int sbad[kBlock / 64];
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[wid] = lo;
        shi[wid] = hi;
        scnt[wid] = cnt;
        sbad[wid] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            slo[0] = fminf(slo[0], slo[i]);
            shi[0] = fmaxf(shi[0], shi[i]);
            scnt[0] += scnt[i];
            sbad[0] |= sbad[i];
        }
        const int64_t k = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        pmin[k] = slo[0];
        pmax[k] = shi[0];
        pcount[k] = scnt[0];
        pbad[k] = sbad[0];
    }
}

__global__ void map_apply_kernel(const ImgDev *__restrict__ imgs, const double *__restrict__ zmm,
                                 const float *__restrict__ z, const uint8_t *__restrict__ sampled,
                                 float *__restrict__ phi)
{
#pragma clang fp contract(off)
    const ImgDev im = imgs[blockIdx.y];
    const double zmin = zmm[2 * blockIdx.y], zmax = zmm[2 * blockIdx.y + 1];
    const int64_t n = (int64_t)im.nx * im.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = im.offset + i;
        phi[j] = sampled[j] ? (float)(kTwoPi * (((double)z[j] - zmin) / (zmax - zmin))) : 0.0f;
    }
}

__global__ void predict_kernel(const ImgDev *__restrict__ imgs, const double *__restrict__ zmm, int M,
                               const float *__restrict__ z, const uint8_t *__restrict__ sampled,
                               const float *__restrict__ phi_sum, float *__restrict__ z_hat)
{
#pragma clang fp contract(off)
    const ImgDev im = imgs[blockIdx.y];
    const double zmin = zmm[2 * blockIdx.y], zmax = zmm[2 * blockIdx.y + 1];
    const int64_t n = (int64_t)im.nx * im.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = im.offset + i;
        if (sampled[j]) {
            z_hat[j] = z[j];
        } else {
            const double t = ((double)phi_sum[j] / (double)M) / kTwoPi;
            z_hat[j] = (float)(zmin * (1.0 - t) + zmax * t);
        }
    }
}

// Per-block sums of -cos(q (phi_i - phi_j)) over sample-sample bonds.
// Partial-result blocks of an image of n sites: one per 4096 sites, at most
// kMapBlocks.  A function of the image alone, so that an image's e_s (a sum
// of doubles) does not depend on the batch it is in.
__host__ __device__ inline int image_blocks(int64_t n)
{
    const int64_t b = (n + 4095) / 4096;
    return (int)(b < 1 ? 1 : (b > kMapBlocks ? kMapBlocks : b));
}

__global__ void sample_energy_kernel(const ImgDev *__restrict__ imgs, const float *__restrict__ phi,
                                     const uint8_t *__restrict__ sampled, double q, double *__restrict__ psum,
                                     unsigned long long *__restrict__ pcount)
{
    const ImgDev im = imgs[blockIdx.y];
    const int64_t n = (int64_t)im.nx * im.ny;
    const int nbk = image_blocks(n);  // this image's blocks (the grid covers the largest image)
    if ((int)blockIdx.x >= nbk) return;
    double s = 0.0;
    unsigned long long cnt = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)nbk * blockDim.x) {
        const int64_t j = im.offset + i;
        if (!sampled[j]) continue;
        const int y = (int)(i / im.nx);
        const int x = (int)(i - (int64_t)y * im.nx);
        const double a = (double)phi[j];
        if (x + 1 < im.nx && sampled[j + 1]) {
            s -= cos(q * (a - (double)phi[j + 1]));
            ++cnt;
        }
        if (y + 1 < im.ny && sampled[j + im.nx]) {
            s -= cos(q * (a - (double)phi[j + im.nx]));
            ++cnt;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        cnt += __shfl_xor(cnt, off);
    }
    __shared__ double ss[kBlock / 64];
    __shared__ unsigned long long sc[kBlock / 64];
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ss[wid] = s;
        sc[wid] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            ss[0] += ss[i];
            sc[0] += sc[i];
        }
        const int64_t k = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        psum[k] = ss[0];
        pcount[k] = sc[0];
    }
}

__global__ void philox_kernel(const uint32_t *__restrict__ ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    U4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    const U4 w = philox4x32_10(c, k0, k1);
    out[4 * i] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

// Plain copy of n 16-byte words: the calibration probe for HBM byte counters.
__global__ void copy_probe_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void ring_slope_kernel(const double *e, int n, CtlParams cp, double *out)
{
    double ring[kMaxFit];
    for (int j = 0; j < n; ++j) ring[j] = e[j];
    // values e[0..n-1] sit in ring slots 0..n-1, i.e. the newest is at t = n-1
    *out = ring_slope(ring, (uint32_t)(n - 1), n, cp.w);
}

// ====================================================================== host

struct mpr_ctx {
    int device = 0;
    std::string err;
    void *scratch = nullptr;          // small device scratch (partials, counters)
    void *static_ws = nullptr;        // this device's static_workspace (device address)
    // pinned host memory: the first kHostWordsBytes mirror the scratch's
    // control words (done counter, barrier generation, abort word); the
    // rest stages small read-backs (the per-block partials of the map and
    // of the sample energies) in one copy each
    unsigned int *done_host = nullptr;
    // resident blocks of the persistent sweep kernel by tile rows (0: no
    // cooperative launch on this device)
    std::map<int, int64_t> persist_cap;
    // sweeps run on a context-owned stream (captured into HIP graphs),
    // ordered after and before the caller's stream with two events
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    // tuned block shape (tile rows) by batch shape
    std::map<std::tuple<int, int, int, int>, int> tuned_rows;
    // profiling
    bool profile = false;
    double prof_ms = 0.0;
    int64_t prof_launches = 0;
    int32_t last_tile = 0;
    // e(T, L) tables: key -> (1 + e) per temperature
    std::map<std::tuple<int, int, double, int, double, double, int, int, double, double, uint64_t>,
             std::vector<double>>
        tables;
};

// Records an error text on the context (also used by the network kernels' host code).
int mpr_set_error(mpr_ctx *ctx, int code, const char *msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

// Checks the device pointers of a call (name, pointer; null ones are
// skipped, the callers test the required ones first): each must be device
// memory of the context's device, or managed memory.  A host pointer would
// otherwise reach a kernel and fault the GPU.  Returns MPR_OK, or
// MPR_ERR_ARG with an error text naming the argument.
int mpr_check_device(mpr_ctx *ctx, const char *call,
                     std::initializer_list<std::pair<const char *, const void *>> ptrs)
{
    for (const auto &np : ptrs) {
        if (!np.second) continue;
        hipPointerAttribute_t a;
        std::memset(&a, 0, sizeof a);
        const hipError_t e = hipPointerGetAttributes(&a, np.second);
        if (e != hipSuccess) (void)hipGetLastError();  // not an address HIP knows: clear the error
        const bool managed = a.isManaged || a.type == hipMemoryTypeManaged || a.type == hipMemoryTypeUnified;
        if (e != hipSuccess || !(managed || (a.type == hipMemoryTypeDevice && a.device == ctx->device))) {
            char buf[256];
            snprintf(buf, sizeof buf, "%s: %s is not device memory of device %d", call, np.first, ctx->device);
            return mpr_set_error(ctx, MPR_ERR_ARG, buf);
        }
    }
    return MPR_OK;
}

namespace {

int fail(mpr_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, expr)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail((ctx), MPR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int half_stride(int nx) { return (int)round_up((nx + 1) / 2, 64); }

// Bytes of one half-grid of `eb`-byte angles.
int64_t half_grid_bytes(int nx, int ny, int eb = 4) { return (int64_t)ny * half_stride(nx) * eb; }

// Simple bump allocator over the caller's workspace.
// Host memory for a read-back of `bytes`: the context's pinned staging
// area when it fits, else `spill` (pageable), resized.
char *stage_for(mpr_ctx *ctx, int64_t bytes, std::vector<char> &spill)
{
    if (bytes <= kHostStageBytes - kHostWordsBytes) return (char *)ctx->done_host + kHostWordsBytes;
    spill.resize((size_t)bytes);
    return spill.data();
}

struct Carver {
    char *base;
    int64_t cap, used = 0;
    void *take(int64_t bytes)
    {
        used = round_up(used, 256);
        if (used + bytes > cap) return nullptr;
        void *p = base + used;
        used += bytes;
        return p;
    }
};

// Sweep block shapes: half-rows per block, and whether gap sites are
// compacted onto lanes (1024 sites per block) or not (512 sites per block);
// or a fused tile sweep (a whole sweep per launch on tiles of `rows` rows x
// 2 kTileH columns, single precision only).
struct Shape {
    int rows;
    bool compact;
    bool fused;
    bool persist;  // fused sweeps, many per cooperative launch (sweep_tile_persist_kernel)
};
constexpr int kNumShapes = 18;
constexpr int kNumPlainShapes = 4;
constexpr int kNumUnfusedShapes = 7;   // the shapes of double-precision chains
constexpr Shape kShapes[kNumShapes] = {{1, false, false}, {2, false, false}, {4, false, false}, {8, false, false},
                                       {2, true, false},  {4, true, false},  {8, true, false},
                                       {16, false, true}, {24, false, true}, {32, false, true},
                                       {48, false, true}, {8, false, true},  {12, false, true},
                                       {8, false, true, true},  {12, false, true, true}, {16, false, true, true},
                                       {24, false, true, true}, {32, false, true, true}};
constexpr int kDefaultShape = 2;  // plain, 4 half-rows

int tile_code(const Shape &sh)
{
    return sh.rows | (sh.compact ? MPR_TILE_COMPACT : 0) | (sh.fused ? MPR_TILE_FUSED : 0) |
           (sh.persist ? MPR_TILE_PERSIST : 0);
}

// Shape index of a tile_rows value (rows | MPR_TILE_COMPACT, MPR_TILE_FUSED or
// MPR_TILE_FUSED | MPR_TILE_PERSIST), or -1.
int shape_of(int tile)
{
    for (int k = 0; k < kNumShapes; ++k)
        if (tile == tile_code(kShapes[k])) return k;
    return -1;
}

// Sweep blocks of one chain (half-row stride S, ny rows) for block shape k.
int64_t shape_blocks(int S, int ny, int k)
{
    const Shape sh = kShapes[k];
    if (sh.fused) return (int64_t)(S / kTileH) * ((ny + sh.rows - 1) / sh.rows);
    const int px = sh.compact ? kCompactSites / sh.rows / 2 : kBlock / sh.rows;  // site pairs per block row
    return (int64_t)((S / 2 + px - 1) / px) * ((ny + sh.rows - 1) / sh.rows);
}

int64_t chain_blocks(const ChainDesc &d, int k) { return shape_blocks(d.S, d.ny, k); }

// Mask words per sweep block of shape k (one bit per site of the block).
int redo_words(int k) { return kShapes[k].fused ? 0 : (kShapes[k].compact ? kCompactSites : 2 * kBlock) / 32; }

// Workspace bytes of the deferred-redo buffers for `chains` chains of an
// nx x ny grid (an upper bound over every block shape).
int64_t redo_bytes(int nx, int ny, int64_t chains)
{
    int64_t words = 0, blocks = 0;
    for (int k = 0; k < kNumShapes; ++k) {
        const int64_t b = shape_blocks(half_stride(nx), ny, k);
        words = std::max(words, b * redo_words(k));
        blocks = std::max(blocks, b);
    }
    return chains * (words * 4 + blocks / 8 + 8) + 1024;
}

bool valid_params(const mpr_params *p)
{
    // q = 1/2 (the paper's value) runs on either sweep; 0 < q < 1/2 on the
    // double-precision one (the single-precision kernels are written for 1/2)
    return p && (p->q == 0.5 || (p->q > 0.0 && p->q < 0.5 && p->fp64 == 1)) && p->R >= 1 && p->K >= 0 &&
           p->n_f >= 1 && p->n_fit >= 2 &&
           p->n_fit <= kMaxFit && p->sg_degree >= 1 && p->sg_degree <= 4 && p->sg_degree < p->n_fit &&
           p->k_a > 0.0 && p->a_targ >= 0.0 && p->table_nT >= 2 && p->table_meas >= 1 && p->table_burn >= 0 &&
           p->table_T_lo > 0.0 && p->table_T_hi > p->table_T_lo &&
           (p->tile_rows == 0 || shape_of(p->tile_rows) >= 0) &&
           p->sweeps_per_launch >= 0 && p->sweeps_per_launch <= 4096 && (p->spread == 0 || p->spread == 1) &&
           (p->fp64 == 0 || p->fp64 == 1) &&
           (p->table_side_cap == 0 || p->table_side_cap >= 2) && p->warm_min_states >= 0 && p->sweep_limit >= 0 &&
           (p->resume == 0 || p->resume == 1) && p->barrier_timeout_us >= 0;
}

bool valid_images(const mpr_image *imgs, int n)
{
    if (!imgs || n < 1) return false;
    for (int b = 0; b < n; ++b) {
        if (imgs[b].nx < 1 || imgs[b].ny < 1 || imgs[b].offset < 0) return false;
        if ((int64_t)imgs[b].nx * imgs[b].ny > (int64_t)1 << 31) return false;
        // the sweep kernels address a single-precision half-grid with 32-bit byte offsets
        if (half_grid_bytes(imgs[b].nx, imgs[b].ny) >= ((int64_t)1 << 32)) return false;
        if (imgs[b].id >= 0x80000000u) return false;
    }
    return true;
}

// Head of a simulate workspace: what a resumed call checks before it
// continues the run the workspace holds.
struct RunHeader {
    uint64_t magic;     // kRunMagic
    uint64_t key;       // run_key of the images and parameters
    int64_t bytes;      // sim_bytes of the run
    int32_t n_chains;
    int32_t state;      // 1: stopped at sweep_limit with chains running (resumable)
};
constexpr uint64_t kRunMagic = 0x4D50522D52554E31ull;  // "MPR-RUN1"
constexpr int64_t kRunHeaderBytes = 256;

int64_t sim_bytes(const mpr_image *imgs, int n, const mpr_params *p)
{
    int64_t b = kRunHeaderBytes;
    for (int i = 0; i < n; ++i) {
        const int64_t hg = round_up(half_grid_bytes(imgs[i].nx, imgs[i].ny, p->fp64 ? 8 : 4), 256);
        // angles (twice for single precision: the fused sweep's second buffer),
        // equilibrium sums, squared deviations
        b += (int64_t)p->R * 2 * hg * ((p->fp64 ? 1 : 2) + (p->K > 1 ? (p->spread ? 2 : 1) : 0));
    }
    const int64_t chains = (int64_t)n * p->R;
    b += round_up(chains * (int64_t)sizeof(ChainDesc), 256) + round_up(chains * (int64_t)sizeof(ChainState), 256);
    b += round_up(chains * 8, 256) + round_up((int64_t)n * sizeof(ImgDev), 256) + 4096;
    b += round_up(kNumShapes * (chains + 1) * 8, 256) + round_up(chains * 4 + 4, 256);
    for (int i = 0; i < n; ++i) b += redo_bytes(imgs[i].nx, imgs[i].ny, p->R);
    return b;
}

// FNV-1a over the images (size, offset, id), the parameters that shape a
// run's chains (all but sweep_limit, resume, tile_rows and
// sweeps_per_launch, which do not change its results) and the temperatures.
uint64_t run_key(const mpr_image *imgs, int n, const mpr_params *p, const double *T_hat)
{
    uint64_t h = 0xCBF29CE484222325ull;
    auto mix = [&h](const void *v, size_t len) {
        const unsigned char *b = (const unsigned char *)v;
        for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 0x100000001B3ull;
    };
    mix(&n, sizeof n);
    for (int i = 0; i < n; ++i) {
        mix(&imgs[i].nx, 4);
        mix(&imgs[i].ny, 4);
        mix(&imgs[i].offset, 8);
        mix(&imgs[i].id, 4);
    }
    mpr_params q = *p;
    q.sweep_limit = 0;
    q.resume = 0;
    q.tile_rows = 0;
    q.sweeps_per_launch = 0;
    q.barrier_timeout_us = 0;
    mix(&q, sizeof q);
    mix(T_hat, sizeof(double) * (size_t)n);
    return h;
}

// Table chains run in double precision when q != 1/2 (the single-precision
// kernels are written for q = 1/2).
int table_angle_bytes(const mpr_params *p) { return p->q == 0.5 ? 4 : 8; }

// Grid on which the e(T, L) table of an image is built: its own, or each
// side capped at table_side_cap.
struct TableGrid {
    int32_t nx, ny;
};
TableGrid table_grid(const mpr_image &im, const mpr_params *p)
{
    const int32_t c = p->table_side_cap;
    return c > 0 ? TableGrid{std::min(im.nx, c), std::min(im.ny, c)} : TableGrid{im.nx, im.ny};
}

int64_t table_bytes(const mpr_image *imgs, int n, const mpr_params *p)
{
    int64_t best = 0;
    for (int i = 0; i < n; ++i) {
        const TableGrid t = table_grid(imgs[i], p);
        const int64_t hg = round_up(half_grid_bytes(t.nx, t.ny, table_angle_bytes(p)), 256);
        best = std::max(best, (int64_t)p->table_nT * 2 * hg);
    }
    const int64_t chains = p->table_nT;
    best += round_up(chains * (int64_t)sizeof(ChainDesc), 256) + round_up(chains * (int64_t)sizeof(ChainState), 256);
    best += round_up(chains * 8, 256) + round_up((int64_t)n * sizeof(ImgDev), 256) + 4096;
    best += round_up((int64_t)n * kMapBlocks * 16, 256);
    best += round_up(kNumShapes * (chains + 1) * 8, 256) + round_up(chains * 4 + 4, 256);
    int64_t rb = 0;
    for (int i = 0; i < n; ++i) {
        const TableGrid t = table_grid(imgs[i], p);
        rb = std::max(rb, redo_bytes(t.nx, t.ny, chains));
    }
    return best + rb;
}

// Derivative at the newest point of the degree-d least-squares polynomial
// through n equally spaced points, as weights on the values (oldest first):
// w = V (V^T V)^{-1} g with V_jk = s_j^k, s_j = j - (n-1)/2, g_k = k s_end^(k-1).
void sg_weights(int n, int degree, double *w)
{
    const int m = degree + 1;
    std::vector<double> A(m * m, 0.0), G(m, 0.0);
    const double c = 0.5 * (n - 1);
    for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += std::pow(j - c, k + l);
            A[k * m + l] = s;
        }
    const double send = (n - 1) - c;
    for (int k = 1; k < m; ++k) G[k] = k * std::pow(send, k - 1);
    // solve A x = G (A symmetric positive definite) by Gaussian elimination
    std::vector<double> M(A), x(G);
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(M[r * m + col]) > std::fabs(M[piv * m + col])) piv = r;
        if (piv != col) {
            for (int l = 0; l < m; ++l) std::swap(M[col * m + l], M[piv * m + l]);
            std::swap(x[col], x[piv]);
        }
        for (int r = col + 1; r < m; ++r) {
            const double f = M[r * m + col] / M[col * m + col];
            for (int l = col; l < m; ++l) M[r * m + l] -= f * M[col * m + l];
            x[r] -= f * x[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = x[r];
        for (int l = r + 1; l < m; ++l) s -= M[r * m + l] * x[l];
        x[r] = s / M[r * m + r];
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += std::pow(j - c, k) * x[k];
        w[j] = s;
    }
}

CtlParams make_ctl(const mpr_params *p)
{
    CtlParams cp;
    std::memset(&cp, 0, sizeof cp);
    cp.a_targ = p->a_targ;
    cp.k_a = p->k_a;
    cp.q = p->q;
    cp.n_f = p->n_f;
    cp.n_fit = p->n_fit;
    cp.i_max = p->i_max;
    cp.fixed_relax = p->fixed_relax;
    cp.eq_a_mode = p->eq_a_mode;
    cp.K = p->K;
    cp.burn = p->table_burn;
    cp.meas = p->table_meas;
    cp.e_unit = kEnergyUnit;
    cp.angle_bytes = 4;
    sg_weights(p->n_fit, p->sg_degree, cp.w);
    return cp;
}

SweepConsts make_sc(double q, uint64_t seed)
{
    SweepConsts sc;
    sc.q64 = q;
    sc.seed_lo = (uint32_t)seed;
    sc.seed_hi = (uint32_t)(seed >> 32);
    return sc;
}

int blocks_for(int64_t n, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, cap)); }


// A set of chains resident in the workspace.
struct ChainSet {
    std::vector<ChainDesc> desc;
    std::vector<ChainState> state;
    std::vector<int64_t> offset;  // image offset per chain (init)
    ChainDesc *d_desc = nullptr;
    ChainState *d_state = nullptr;
    int64_t *d_offset = nullptr;
    // the chains a sweep launch covers (those not done when the launch list
    // was last built): block prefix sums per shape and chain ids
    int64_t *d_start[kNumShapes] = {};
    int32_t *d_ids = nullptr;
    int n_active = 0;
    int64_t total_blocks[kNumShapes] = {};
    std::vector<int64_t> h_start;  // host copies (kept until their upload is done)
    std::vector<int32_t> h_ids;
    Redo redo = {nullptr, nullptr};      // deferred double-precision updates (zeroed)
    bool fp64 = false;                   // double-precision chains (no deferred redo)
    float *states_out = nullptr;         // recorded equilibrium states (nullable)
    int64_t states_n_total = 0;          // sites of the whole batch (stride of a state)
    int K = 0;
};

BlockMap block_map(const ChainSet &cs, int v) { return BlockMap{cs.d_start[v], cs.d_ids, cs.n_active, 0}; }

template <int ROWS>
void launch_half_rows(hipStream_t st, const ChainSet &cs, int v, bool table, int colour, const SweepConsts &sc)
{
    const dim3 grid((unsigned)cs.total_blocks[v]);
    if (table)
        hipLaunchKernelGGL(table_half_sweep_kernel<ROWS>, grid, dim3(kBlock), 0, st, cs.d_desc, cs.d_state,
                           block_map(cs, v), colour, sc, cs.redo);
    else
        hipLaunchKernelGGL((half_sweep_kernel<false, ROWS>), grid, dim3(kBlock), 0, st, cs.d_desc, cs.d_state,
                           block_map(cs, v), colour, sc, 0, cs.redo, nullptr);
}

template <int CR>
void launch_half_compact(hipStream_t st, const ChainSet &cs, int v, int colour, const SweepConsts &sc)
{
    hipLaunchKernelGGL((half_sweep_compact_kernel<false, CR>), dim3((unsigned)cs.total_blocks[v]), dim3(kBlock), 0,
                       st, cs.d_desc, cs.d_state, block_map(cs, v), colour, sc, 0, cs.redo, nullptr);
}

// The deferred double-precision updates after a half-sweep in shape v.
template <bool DIAG>
void launch_redo(hipStream_t st, const ChainSet &cs, int v, int colour, const SweepConsts &sc, int or_only,
                 uint8_t *flags, const FusedControl *ctl = nullptr)
{
    FusedControl fc;
    if (ctl) fc = *ctl;
    else std::memset(&fc, 0, sizeof fc);
    // a wave per bitmap word, at most 16384 waves
    const int64_t nw = (cs.total_blocks[v] + 31) / 32;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nw + 3) / 4, 4096));
    hipLaunchKernelGGL((redo_fp64_kernel<DIAG>), dim3(grid), dim3(kBlock), 0, st, cs.d_desc, cs.d_state,
                       block_map(cs, v), cs.total_blocks[v], kShapes[v].rows,
                       kShapes[v].compact ? 1 : 0, colour, sc, or_only, cs.redo, flags, fc);
}

template <bool DIAG, int ROWS>
void launch_half_fp64_rows(hipStream_t st, const ChainSet &cs, int v, int colour, const SweepConsts &sc, int or_only,
                           uint8_t *flags)
{
    hipLaunchKernelGGL((half_sweep_fp64_kernel<DIAG, ROWS>), dim3((unsigned)cs.total_blocks[v]), dim3(kBlock), 0, st,
                       cs.d_desc, cs.d_state, block_map(cs, v), colour, sc, or_only, flags);
}

template <bool DIAG, int CR>
void launch_half_fp64_compact(hipStream_t st, const ChainSet &cs, int v, int colour, const SweepConsts &sc,
                              int or_only, uint8_t *flags)
{
    hipLaunchKernelGGL((half_sweep_fp64_compact_kernel<DIAG, CR>), dim3((unsigned)cs.total_blocks[v]), dim3(kBlock),
                       0, st, cs.d_desc, cs.d_state, block_map(cs, v), colour, sc, or_only, flags);
}

// One half-sweep of double-precision chains in shape v.
template <bool DIAG>
void launch_half_fp64(hipStream_t st, const ChainSet &cs, int v, int colour, const SweepConsts &sc, int or_only,
                      uint8_t *flags)
{
    if (kShapes[v].compact) {
        switch (kShapes[v].rows) {
            case 2: launch_half_fp64_compact<DIAG, 2>(st, cs, v, colour, sc, or_only, flags); break;
            case 4: launch_half_fp64_compact<DIAG, 4>(st, cs, v, colour, sc, or_only, flags); break;
            default: launch_half_fp64_compact<DIAG, 8>(st, cs, v, colour, sc, or_only, flags); break;
        }
        return;
    }
    switch (kShapes[v].rows) {
        case 1: launch_half_fp64_rows<DIAG, 1>(st, cs, v, colour, sc, or_only, flags); break;
        case 2: launch_half_fp64_rows<DIAG, 2>(st, cs, v, colour, sc, or_only, flags); break;
        case 4: launch_half_fp64_rows<DIAG, 4>(st, cs, v, colour, sc, or_only, flags); break;
        default: launch_half_fp64_rows<DIAG, 8>(st, cs, v, colour, sc, or_only, flags); break;
    }
}

// One half-sweep of every chain in shape v (the e(T, L) runs use the plain
// shapes only); `ctl` (single precision only) makes the redo kernel run the
// per-sweep control as well.
void launch_half(hipStream_t st, const ChainSet &cs, int v, bool table, int colour, const SweepConsts &sc,
                 const FusedControl *ctl = nullptr)
{
    if (cs.fp64) {
        launch_half_fp64<false>(st, cs, v, colour, sc, 0, nullptr);
        return;
    }
    const Shape sh = kShapes[v];
    if (sh.compact && !table) {
        switch (sh.rows) {
            case 2: launch_half_compact<2>(st, cs, v, colour, sc); break;
            case 4: launch_half_compact<4>(st, cs, v, colour, sc); break;
            default: launch_half_compact<8>(st, cs, v, colour, sc); break;
        }
    } else {
        switch (sh.rows) {
            case 1: launch_half_rows<1>(st, cs, v, table, colour, sc); break;
            case 2: launch_half_rows<2>(st, cs, v, table, colour, sc); break;
            case 4: launch_half_rows<4>(st, cs, v, table, colour, sc); break;
            default: launch_half_rows<8>(st, cs, v, table, colour, sc); break;
        }
    }
    launch_redo<false>(st, cs, v, colour, sc, 0, nullptr, ctl);
}

// One fused sweep of every listed chain in shape v (mode 0), or one colour
// of it in place (mode 1, 2: diagnostics).
template <bool DIAG>
void launch_tile(hipStream_t st, const ChainSet &cs, int v, int mode, const SweepConsts &sc, int or_only,
                 uint8_t *flags, const FusedControl *ctl = nullptr)
{
    FusedControl fc;
    if (ctl) fc = *ctl;
    else std::memset(&fc, 0, sizeof fc);
    const dim3 grid((unsigned)cs.total_blocks[v]), blk(kBlock);
    switch (kShapes[v].rows) {
        case 16:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 16>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
        case 24:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 24>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
        case 48:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 48>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
        case 8:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 8>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
        case 12:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 12>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
        default:
            hipLaunchKernelGGL((sweep_tile_kernel<DIAG, 32>), grid, blk, 0, st, cs.d_desc, cs.d_state,
                               block_map(cs, v), mode, sc, or_only, flags, fc);
            break;
    }
}

template <int TH>
const void *persist_kernel() { return reinterpret_cast<const void *>(&sweep_tile_persist_kernel<TH>); }

const void *persist_kernel_of(int rows)
{
    switch (rows) {
        case 8: return persist_kernel<8>();
        case 12: return persist_kernel<12>();
        case 16: return persist_kernel<16>();
        case 24: return persist_kernel<24>();
        default: return persist_kernel<32>();
    }
}

// Blocks of the persistent sweep kernel (tile rows `rows`) that the device
// holds at once, 0 without cooperative launches; cached on the context.
int64_t persist_capacity(mpr_ctx *ctx, int rows)
{
    auto it = ctx->persist_cap.find(rows);
    if (it != ctx->persist_cap.end()) return it->second;
    int coop = 0, cus = 0, per_cu = 0;
    int64_t cap = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx->device) == hipSuccess && coop &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel_of(rows), kPersistThreads, 0) ==
            hipSuccess)
        cap = (int64_t)per_cu * cus;
    (void)hipGetLastError();
    ctx->persist_cap[rows] = cap;
    return cap;
}

// Up to `count` fused sweeps of every listed chain in persistent shape v,
// in one cooperative launch (the barrier generation cleared first).
hipError_t launch_persist(hipStream_t st, const ChainSet &cs, int v, const SweepConsts &sc, const FusedControl &ctl,
                          unsigned int *gen, unsigned int *abort_word, unsigned long long *slots, int count,
                          uint32_t need, uint64_t wait_ticks)
{
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(kBlock), 0, st, gen, nullptr, nullptr, slots,
                       (int)cs.desc.size() * 4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ChainDesc *descs = cs.d_desc;
    ChainState *states = cs.d_state;
    BlockMap bm = block_map(cs, v);
    SweepConsts scc = sc;
    FusedControl fc = ctl;
    PersistCtl pc;
    pc.gen = gen;
    pc.abort = abort_word;
    pc.slots = slots;
    pc.wait_ticks = wait_ticks;
    pc.count = count;
    pc.need = need;
    void *args[] = {&descs, &states, &bm, &scc, &fc, &pc};
    return hipLaunchCooperativeKernel(persist_kernel_of(kShapes[v].rows), dim3((unsigned)cs.total_blocks[v]),
                                      dim3(kPersistThreads), args, 0, st);
}

// Builds the launch list of a chain set from the chains in `active`: block
// prefix sums for every shape and the chain ids, uploaded on `stream` (and
// waited for, so that the host copies can be reused).
int set_active(mpr_ctx *ctx, ChainSet &cs, const std::vector<int32_t> &active, hipStream_t stream)
{
    const int n = (int)cs.desc.size();
    const int na = (int)active.size();
    cs.h_start.assign((size_t)kNumShapes * (n + 1), 0);
    for (int k = 0; k < kNumShapes; ++k) {
        int64_t *sk = cs.h_start.data() + (size_t)k * (n + 1);
        for (int j = 0; j < na; ++j) sk[j + 1] = sk[j] + chain_blocks(cs.desc[active[j]], k);
        cs.total_blocks[k] = sk[na];
        if (sk[na] >= ((int64_t)1 << 31)) return fail(ctx, MPR_ERR_ARG, "batch too large for one launch");
    }
    cs.h_ids = active;
    cs.n_active = na;
    HIP_TRY(ctx, hipMemcpyAsync(cs.d_start[0], cs.h_start.data(), cs.h_start.size() * 8, hipMemcpyHostToDevice,
                                stream));
    if (na > 0)
        HIP_TRY(ctx, hipMemcpyAsync(cs.d_ids, cs.h_ids.data(), (size_t)na * 4, hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

// Runs sweeps until every chain is done.  Returns 0 or an error code.
// Sweeps run on ctx->gstream: a few direct sweeps per block shape first (to
// tune it, unless fixed or cached), then groups of `spl` sweeps replayed as
// a captured graph (launched directly when `graphs` is false: instantiating
// a graph allocates), checking the done-counter after each group.  At most
// max_sweeps sweeps run; chains still running then are an error, or with
// `stop_ok` the result MPR_INCOMPLETE.
int run_chains(mpr_ctx *ctx, ChainSet &cs, const mpr_params *p, hipStream_t stream, int64_t max_sweeps,
               int poll_every, bool table, bool graphs = true, bool stop_ok = false)
{
    const int n = (int)cs.desc.size();
    unsigned int *d_done = reinterpret_cast<unsigned int *>((char *)ctx->scratch + kDoneOffset);
    unsigned int *d_ticket = reinterpret_cast<unsigned int *>((char *)ctx->scratch + kTicketOffset);
    unsigned long long *d_work = reinterpret_cast<unsigned long long *>((char *)ctx->scratch + kWorkOffset);
    unsigned int *d_gen = reinterpret_cast<unsigned int *>((char *)ctx->scratch + kGenOffset);
    unsigned int *d_abort = reinterpret_cast<unsigned int *>((char *)ctx->scratch + kAbortOffset);
    unsigned long long *d_slots = reinterpret_cast<unsigned long long *>((char *)ctx->scratch + kSlotsOffset);
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(kBlock), 0, stream, d_done, d_abort, d_ticket, nullptr, 0);
    HIP_TRY(ctx, hipGetLastError());
    unsigned int already = 0;
    for (const auto &s : cs.state)
        if (s.phase == PH_DONE) ++already;
    if (already == (unsigned int)n) return MPR_OK;
    CtlParams cp = make_ctl(p);
    if (cs.fp64) {
        cp.e_unit = kEnergyUnit64;
        cp.angle_bytes = 8;
    }
    const SweepConsts sc = make_sc(p->q, p->seed);
    const int cblocks = (n + 63) / 64;
    hipStream_t st = ctx->gstream;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_in, stream));
    HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->ev_in, 0));

    // the control runs at the end of the colour-1 redo kernel unless
    // something must run between them (the state record) or there is no
    // redo kernel (double-precision chains)
    const bool fuse = !cs.fp64 && !cs.states_out;
    FusedControl fc;
    std::memset(&fc, 0, sizeof fc);
    fc.cp = cp;
    fc.ticket = d_ticket;
    fc.done_count = d_done;
    fc.work = d_work;
    fc.n_all = n;
    fc.on = 1;
    auto control = [&](int swap, int ctl) {
        hipLaunchKernelGGL(control_kernel, dim3(cblocks), dim3(64), 0, st, cs.d_desc, cs.d_state, n, cp, d_done,
                           d_work, swap, ctl);
    };
    // A sweep: the fused tile sweep, then control_kernel with the swap of
    // h and h2 (and the control, unless the states are recorded in between);
    // a fused sweep of at most kTileCtlMaxBlocks blocks does the swap and the
    // control in its last block instead (unless states are recorded); or two
    // half-sweeps, the colour-1 redo kernel running the control unless the
    // states are recorded (or the chains are double precision).
    // The persistent shapes: single-precision chains whose tiles the device
    // holds at once, states not recorded (nothing runs between the sweep and
    // the control).
    auto persist_ok = [&](int v) {
        return kShapes[v].persist && fuse && !table && n <= kPersistMaxChains && cs.total_blocks[v] > 0 &&
               cs.total_blocks[v] <= persist_capacity(ctx, kShapes[v].rows);
    };
    const uint32_t need = (uint32_t)(n - (int)already);
    const uint64_t wait_ticks = p->barrier_timeout_us > 0 ? (uint64_t)p->barrier_timeout_us * 100u : kPersistWaitTicks;
    hipError_t perr = hipSuccess;
    auto sweeps = [&](int v, int count) {
        if (kShapes[v].persist) {
            perr = launch_persist(st, cs, v, sc, fc, d_gen, d_abort, d_slots, count, need, wait_ticks);
            return;
        }
        for (int i = 0; i < count; ++i) {
            const bool fused = kShapes[v].fused;
            if (fused && fuse && cs.total_blocks[v] <= kTileCtlMaxBlocks) {
                launch_tile<false>(st, cs, v, 0, sc, 0, nullptr, &fc);  // swap and control in its last block
            } else if (fused) {
                launch_tile<false>(st, cs, v, 0, sc, 0, nullptr);
                control(1, cs.states_out ? 0 : 1);
            } else {
                launch_half(st, cs, v, table, 0, sc);
                launch_half(st, cs, v, table, 1, sc, fuse ? &fc : nullptr);
            }
            if (cs.states_out && cs.n_active > 0)
                hipLaunchKernelGGL(record_states_kernel, dim3((unsigned)(cs.n_active * kRecordSegs)), dim3(kBlock), 0,
                                   st, cs.d_desc, cs.d_state, cs.d_offset, cs.d_ids, kRecordSegs, cs.K,
                                   cs.fp64 ? 1 : 0, cs.states_n_total, cs.states_out);
            if (fused ? cs.states_out != nullptr : !fuse) control(0, 1);
        }
    };
    int64_t done_sweeps = 0;
    bool finished = false;
    // Runs `count` sweeps directly or as graph `ge`, timed; then polls.
    auto block = [&](int v, int count, hipGraphExec_t ge, float *ms_out) -> int {
        HIP_TRY(ctx, hipEventRecord(ctx->ev_t0, st));
        if (ge) HIP_TRY(ctx, hipGraphLaunch(ge, st));
        else sweeps(v, count);
        if (perr != hipSuccess) return fail(ctx, MPR_ERR_HIP, "persistent sweep launch: %s", hipGetErrorString(perr));
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipEventRecord(ctx->ev_t1, st));
        // the done counter; after a persistent launch the words up to the
        // abort word, in one copy (done counter, generation, abort word)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->done_host, d_done,
                                    kShapes[v].persist ? (size_t)(kAbortOffset + 4) : sizeof(unsigned int),
                                    hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        if (kShapes[v].persist) {
            if (ctx->done_host[kAbortOffset / 4] != 0u)
                return fail(ctx, MPR_ERR_HIP, "persistent sweep: a block timed out at the grid barrier");
            // the launch stops early once every chain is done
            count = (int)(ctx->done_host[kGenOffset / 4] & 0x7FFFFFFFu);
        }
        float ms = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        if (ms_out) *ms_out = ms;
        if (ctx->profile) {
            ctx->prof_ms += ms;
            ctx->prof_launches += (kShapes[v].fused ? 1 : 2) * (int64_t)count;
        }
        done_sweeps += count;
        finished = *ctx->done_host + already >= (unsigned int)n;
        return MPR_OK;
    };

    // block shape: fixed, cached, or tuned on the first sweeps (the table
    // chains take the plain shapes, double-precision chains every unfused one)
    const int n_shapes = table ? kNumPlainShapes : (cs.fp64 ? kNumUnfusedShapes : kNumShapes);
    int v = p->tile_rows ? shape_of(p->tile_rows) : -1;
    if (v >= n_shapes) v = kDefaultShape;
    // a persistent shape that does not apply here: its rows, one launch per sweep
    auto usable = [&](int k) { return k < 0 || !kShapes[k].persist || persist_ok(k); };
    if (!usable(v)) v = shape_of(kShapes[v].rows | MPR_TILE_FUSED);
    int maxnx = 0, maxny = 0;
    for (const auto &d : cs.desc) {
        maxnx = std::max(maxnx, d.nx);
        maxny = std::max(maxny, d.ny);
    }
    const auto key = std::make_tuple((table ? 1 : 0) | (cs.fp64 ? 2 : 0), n, maxnx, maxny);
    float sweep_ms = -1.0f;
    if (v < 0) {
        auto it = ctx->tuned_rows.find(key);
        if (it != ctx->tuned_rows.end()) v = usable(it->second) ? it->second
                                                                 : shape_of(kShapes[it->second].rows | MPR_TILE_FUSED);
    }
    if (v < 0) {
        const int ts = std::max(1, std::min(poll_every, 3));
        float best = 0.0f;
        int tried = 0;
        for (int k = 0; k < n_shapes && !finished && done_sweeps + ts <= max_sweeps; ++k, ++tried) {
            if (!usable(k)) continue;
            // time per sweep; a persistent launch over more sweeps, so that
            // its one launch does not weigh on the comparison
            if (kShapes[k].persist) {
                // an untimed first launch (the first of a kernel costs more)
                int rc = block(k, 1, nullptr, nullptr);
                if (rc) return rc;
                if (finished || done_sweeps + ts > max_sweeps) break;
            }
            const int tk = kShapes[k].persist ? (int)std::min<int64_t>(4 * ts, max_sweeps - done_sweeps) : ts;
            float ms = 0.0f;
            const int64_t before = done_sweeps;
            int rc = block(k, tk, nullptr, &ms);
            if (rc) return rc;
            ms /= (float)std::max<int64_t>(1, done_sweeps - before);
            if (v < 0 || ms < best) {
                best = ms;
                v = k;
            }
        }
        if (v < 0) v = kDefaultShape;
        else sweep_ms = best;
        if (tried == n_shapes) ctx->tuned_rows[key] = v;
    }
    if (!table) ctx->last_tile = tile_code(kShapes[v]);
    // sweeps per graph: at least about a millisecond of work per done-check
    int spl = p->sweeps_per_launch > 0 ? p->sweeps_per_launch : poll_every;
    if (p->sweeps_per_launch <= 0 && sweep_ms > 0.0f && (float)spl * sweep_ms < 1.0f)
        spl = std::min(64, poll_every * (int)std::ceil(1.0f / ((float)poll_every * sweep_ms)));
    // a persistent launch ends by itself when every chain is done: a group
    // of 256 sweeps covers a whole small fill in one launch and one poll
    if (p->sweeps_per_launch <= 0 && kShapes[v].persist) spl = 256;
    // the captured sweep group, released on every return path
    struct Captured {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        void release()
        {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
        }
        ~Captured() { release(); }
    } cap;
    hipGraphExec_t &ge = cap.exec;
    auto capture = [&]() {
        cap.release();
        // (a persistent launch runs a whole group itself and is not captured)
        if (graphs && !kShapes[v].persist && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            sweeps(v, spl);
            if (hipStreamEndCapture(st, &cap.graph) != hipSuccess ||
                hipGraphInstantiate(&cap.exec, cap.graph, nullptr, nullptr, 0) != hipSuccess)
                cap.exec = nullptr;
        }
        (void)hipGetLastError();
    };
    if (!finished) capture();
    // Chains stop at different sweeps.  When at least an eighth of the
    // listed chains have finished, the launch list is rebuilt from the
    // chains still running if that drops a fifth or more of the blocks a
    // launch covers (the blocks of finished chains return at once, but
    // still have to be dispatched).
    unsigned int done_listed = already;
    std::vector<uint8_t> done_flag(n);
    uint8_t *d_flags = (uint8_t *)ctx->scratch + kVarOffset;
    const bool can_shrink = (int64_t)n <= (int64_t)kScratchBytes - kVarOffset;
    int rc = MPR_OK;
    while (!finished && done_sweeps < max_sweeps) {
        // the last group may be shorter: exactly max_sweeps sweeps run
        const int cnt = (int)std::min<int64_t>(spl, max_sweeps - done_sweeps);
        rc = block(v, cnt, cnt == spl ? ge : nullptr, nullptr);
        if (rc) break;
        const unsigned int done_now = *ctx->done_host + already;
        if (finished || !can_shrink || done_now - done_listed < std::max(1u, (unsigned int)cs.n_active / 8u))
            continue;
        done_listed = done_now;
        hipLaunchKernelGGL(done_flags_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, cs.d_state, n,
                           d_flags);
        HIP_TRY(ctx, hipMemcpyAsync(done_flag.data(), d_flags, (size_t)n, hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        std::vector<int32_t> active;
        int64_t blocks = 0;
        for (int c = 0; c < n; ++c)
            if (!done_flag[c]) {
                active.push_back(c);
                blocks += chain_blocks(cs.desc[c], v);
            }
        if (active.empty() || 5 * blocks > 4 * cs.total_blocks[v]) continue;
        rc = set_active(ctx, cs, active, st);
        if (rc) break;
        capture();
    }
    cap.release();
    if (rc) return rc;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_out, st));
    HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev_out, 0));
    if (!finished)
        return stop_ok ? MPR_INCOMPLETE
                       : fail(ctx, MPR_ERR_HIP, "chains did not finish within %lld sweeps", (long long)max_sweeps);
    return MPR_OK;
}

// Carves the launch list and the deferred-redo buffers (sized for every
// chain) of a chain set from the workspace and fills the list with the
// chains that are not done.
int upload_starts(mpr_ctx *ctx, ChainSet &cs, Carver &cv, hipStream_t stream)
{
    const int n = (int)cs.desc.size();
    int64_t *d = (int64_t *)cv.take((int64_t)kNumShapes * (n + 1) * 8);
    cs.d_ids = (int32_t *)cv.take((int64_t)n * 4 + 4);
    if (!d || !cs.d_ids) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    for (int k = 0; k < kNumShapes; ++k) cs.d_start[k] = d + (size_t)k * (n + 1);
    int64_t words = 0, blocks = 0;
    for (int k = 0; k < kNumShapes; ++k) {
        int64_t b = 0;
        for (int c = 0; c < n; ++c) b += chain_blocks(cs.desc[c], k);
        words = std::max(words, b * redo_words(k));
        blocks = std::max(blocks, b);
    }
    const int64_t mask_bytes = words * 4, bits_bytes = (blocks + 31) / 32 * 4;
    cs.redo.mask = (uint32_t *)cv.take(mask_bytes);
    cs.redo.blocks = (uint32_t *)cv.take(bits_bytes);
    if (!cs.redo.mask || !cs.redo.blocks) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    HIP_TRY(ctx, hipMemsetAsync(cs.redo.mask, 0, mask_bytes, stream));
    HIP_TRY(ctx, hipMemsetAsync(cs.redo.blocks, 0, bits_bytes, stream));
    std::vector<int32_t> active;
    for (int c = 0; c < n; ++c)
        if (cs.state[c].phase != PH_DONE) active.push_back(c);
    return set_active(ctx, cs, active, stream);
}

ChainState fresh_state(double T, int phase)
{
    ChainState s;
    std::memset(&s, 0, sizeof s);
    s.phase = phase;
    s.sweep = 0;
    s.T = T;
    s.a_cur = 1.0;
    s.a_relax = 1.0;
    s.k = -1.0;
    s.inv_k = 1.0f;
    s.inv_km1 = 0.0f;
    s.inv_k_d = 1.0;
    s.inv_km1_d = 0.0;
    return s;
}

// With `resume` the states are not uploaded but read back from the
// workspace (the run it holds), and each chain whose fused sweeps left h and
// h2 exchanged gets them exchanged in its descriptor too.
int upload_chains(mpr_ctx *ctx, ChainSet &cs, Carver &cv, hipStream_t stream, double q, bool resume = false)
{
    const int n = (int)cs.desc.size();
    cs.d_desc = (ChainDesc *)cv.take(n * (int64_t)sizeof(ChainDesc));
    cs.d_state = (ChainState *)cv.take(n * (int64_t)sizeof(ChainState));
    cs.d_offset = (int64_t *)cv.take(n * 8);
    if (!cs.d_desc || !cs.d_state || !cs.d_offset) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    if (resume) {
        HIP_TRY(ctx, hipMemcpyAsync(cs.state.data(), cs.d_state, n * sizeof(ChainState), hipMemcpyDeviceToHost,
                                    stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        for (int c = 0; c < n; ++c)
            if (cs.state[c].swapped) {
                std::swap(cs.desc[c].h[0], cs.desc[c].h2[0]);
                std::swap(cs.desc[c].h[1], cs.desc[c].h2[1]);
            }
    } else {
        for (auto &s : cs.state) {
            s.inv_T = (float)(1.0 / s.T);
            s.dscale = (float)(kTwoPi * q / s.a_cur);
        }
        HIP_TRY(ctx, hipMemcpyAsync(cs.d_state, cs.state.data(), n * sizeof(ChainState), hipMemcpyHostToDevice,
                                    stream));
    }
    HIP_TRY(ctx, hipMemcpyAsync(cs.d_desc, cs.desc.data(), n * sizeof(ChainDesc), hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(cs.d_offset, cs.offset.data(), n * 8, hipMemcpyHostToDevice, stream));
    return upload_starts(ctx, cs, cv, stream);
}

// Allocates both half-grids (and accumulators) of a chain of `eb`-byte
// angles from the workspace.
bool carve_chain(Carver &cv, ChainDesc &d, int nx, int ny, bool with_acc, bool with_m2 = false, int eb = 4,
                 bool with_h2 = false)
{
    const int64_t hg = half_grid_bytes(nx, ny, eb);
    d.nx = nx;
    d.ny = ny;
    d.S = half_stride(nx);
    for (int c = 0; c < 2; ++c) {
        d.h[c] = (float *)cv.take(hg);
        d.h2[c] = with_h2 ? (float *)cv.take(hg) : nullptr;
        d.acc[c] = with_acc ? (float *)cv.take(hg) : nullptr;
        d.m2[c] = with_acc && with_m2 ? (float *)cv.take(hg) : nullptr;
        if (!d.h[c] || (with_h2 && !d.h2[c]) || (with_acc && !d.acc[c]) || (with_acc && with_m2 && !d.m2[c]))
            return false;
    }
    return true;
}

// Monotone (pool-adjacent-violators) fit of y, then log T interpolated
// linearly in y; y = log(1 + e).
double invert_table(const std::vector<double> &Tg, const std::vector<double> &ope, double e_s, int *clamped)
{
    const int n = (int)Tg.size();
    std::vector<double> val, wt;
    std::vector<int> len;
    for (int k = 0; k < n; ++k) {
        val.push_back(std::log(std::max(ope[k], 1e-300)));
        wt.push_back(1.0);
        len.push_back(1);
        while (val.size() > 1 && val[val.size() - 2] > val.back()) {
            const double w2 = wt[wt.size() - 2] + wt.back();
            const double v2 = (wt[wt.size() - 2] * val[val.size() - 2] + wt.back() * val.back()) / w2;
            const int l2 = len[len.size() - 2] + len.back();
            val.pop_back();
            wt.pop_back();
            len.pop_back();
            val.back() = v2;
            wt.back() = w2;
            len.back() = l2;
        }
    }
    std::vector<double> y;
    for (size_t b = 0; b < val.size(); ++b)
        for (int j = 0; j < len[b]; ++j) y.push_back(val[b]);
    const double ys = std::log(std::max(1.0 + e_s, 1e-300));
    *clamped = 0;
    if (ys <= y[0]) {
        *clamped = 1;
        return Tg[0];
    }
    if (ys >= y[n - 1]) {
        *clamped = 1;
        return Tg[n - 1];
    }
    int k = 0;
    while (!(y[k + 1] >= ys && y[k + 1] > y[k])) ++k;
    const double x0 = std::log(Tg[k]), x1 = std::log(Tg[k + 1]);
    return std::exp(x0 + (ys - y[k]) * (x1 - x0) / (y[k + 1] - y[k]));
}

// Device address of static_workspace on `device` (the current device),
// looked up once per device and kept for the process.
std::mutex g_static_ws_mu;
void *g_static_ws_addr[kMaxDevices] = {};

hipError_t static_ws_addr(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_ws_mu);
    if (!g_static_ws_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(static_workspace));
        if (e != hipSuccess) return e;
        g_static_ws_addr[device] = ptr;
    }
    *out = g_static_ws_addr[device];
    return hipSuccess;
}

std::vector<double> temperature_grid(const mpr_params *p)
{
    std::vector<double> Tg(p->table_nT);
    for (int k = 0; k < p->table_nT; ++k)
        Tg[k] = std::exp(std::log(p->table_T_lo) +
                         (std::log(p->table_T_hi) - std::log(p->table_T_lo)) * (double)k / (double)(p->table_nT - 1));
    return Tg;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

int32_t mpr_create(mpr_ctx **out, int32_t device)
{
    if (!out) return MPR_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MPR_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return MPR_ERR_HIP;
    mpr_ctx *ctx = new mpr_ctx();
    ctx->device = device;
    // without it only mpr_simulate_noalloc is unavailable (it reports so)
    if (static_ws_addr(device, &ctx->static_ws) != hipSuccess) {
        ctx->static_ws = nullptr;
        (void)hipGetLastError();
    }
    if (hipMalloc(&ctx->scratch, kScratchBytes) != hipSuccess ||
        hipHostMalloc((void **)&ctx->done_host, kHostStageBytes, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&ctx->ev_t0) != hipSuccess || hipEventCreate(&ctx->ev_t1) != hipSuccess) {
        mpr_destroy(ctx);
        return MPR_ERR_HIP;
    }
    *out = ctx;
    return MPR_OK;
}

void mpr_destroy(mpr_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->gstream) (void)hipStreamSynchronize(ctx->gstream);
    for (hipEvent_t ev : {ctx->ev_in, ctx->ev_out, ctx->ev_t0, ctx->ev_t1})
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->done_host) (void)hipHostFree(ctx->done_host);
    delete ctx;
}

const char *mpr_last_error(const mpr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void mpr_default_params(mpr_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->q = 0.5;
    p->R = 1;
    p->K = 100;
    p->n_f = 5;
    p->n_fit = 20;
    p->sg_degree = 1;
    p->i_max = 20000;
    p->a_targ = 0.3;
    p->k_a = 3.0;
    p->fixed_relax = -1;
    p->eq_a_mode = 0;
    p->table_nT = 32;
    p->table_burn = 200;
    p->table_meas = 400;
    p->table_T_lo = 1e-5;
    p->table_T_hi = 10.0;
    p->seed = 3000;
    p->tile_rows = 0;
    p->sweeps_per_launch = 0;
    p->spread = 0;
    p->fp64 = 0;
    p->table_side_cap = 0;
    p->warm_min_states = kWarmMinStates;
}

int64_t mpr_workspace_size(const mpr_image *imgs, int32_t n, const mpr_params *p)
{
    if (!valid_images(imgs, n) || !valid_params(p)) return -1;
    return std::max(sim_bytes(imgs, n, p), table_bytes(imgs, n, p));
}

int32_t mpr_map_to_angles(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *z, const uint8_t *sampled,
                          float *phi, double *zmin_zmax, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !z || !sampled || !phi || !zmin_zmax)
        return fail(ctx, MPR_ERR_ARG, "map_to_angles: invalid argument");
    if (int rc = mpr_check_device(ctx, "map_to_angles", {{"z", z}, {"sampled", sampled}, {"phi", phi}})) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int chunk = (int)((kScratchBytes - kVarOffset - 4096) / (kMapBlocks * 24 + 64));
    for (int b0 = 0; b0 < n; b0 += chunk) {
        const int nb = std::min(chunk, n - b0);
        char *sp = (char *)ctx->scratch + kVarOffset;
        ImgDev *d_img = (ImgDev *)sp;
        float *pmin = (float *)(sp + round_up((int64_t)nb * sizeof(ImgDev), 256));
        float *pmax = pmin + (int64_t)nb * kMapBlocks;
        unsigned long long *pcnt = (unsigned long long *)(pmax + (int64_t)nb * kMapBlocks);
        unsigned int *pbad = (unsigned int *)(pcnt + (int64_t)nb * kMapBlocks);
        double *d_zmm = (double *)(pbad + (int64_t)nb * kMapBlocks + 64);
        d_zmm = (double *)round_up((int64_t)d_zmm, 256);
        std::vector<ImgDev> hi(nb);
        for (int b = 0; b < nb; ++b) hi[b] = {imgs[b0 + b].offset, imgs[b0 + b].nx, imgs[b0 + b].ny};
        HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), nb * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
        int mb = 1;  // partial blocks per image: the largest image's count (min, max and counts are exact)
        for (int b = 0; b < nb; ++b) mb = std::max(mb, image_blocks((int64_t)hi[b].nx * hi[b].ny));
        hipLaunchKernelGGL(map_minmax_kernel, dim3(mb, nb), dim3(kBlock), 0, stream, d_img, z, sampled, pmin,
                           pmax, pcnt, pbad);
        HIP_TRY(ctx, hipGetLastError());
        std::vector<float> hmin(nb * mb), hmax(nb * mb);
        std::vector<unsigned long long> hcnt(nb * mb);
        std::vector<unsigned int> hbad(nb * mb);
        // the four partial arrays lie one after the other: one copy
        {
            const char *src = (const char *)pmin;
            const int64_t span = (const char *)(pbad + (int64_t)nb * mb) - src;
            std::vector<char> big;
            char *h = stage_for(ctx, span, big);
            HIP_TRY(ctx, hipMemcpyAsync(h, src, (size_t)span, hipMemcpyDeviceToHost, stream));
            HIP_TRY(ctx, hipStreamSynchronize(stream));
            std::memcpy(hmin.data(), h + ((const char *)pmin - src), hmin.size() * 4);
            std::memcpy(hmax.data(), h + ((const char *)pmax - src), hmax.size() * 4);
            std::memcpy(hcnt.data(), h + ((const char *)pcnt - src), hcnt.size() * 8);
            std::memcpy(hbad.data(), h + ((const char *)pbad - src), hbad.size() * 4);
        }
        std::vector<double> zmm(2 * nb);
        for (int b = 0; b < nb; ++b) {
            float lo = INFINITY, hi2 = -INFINITY;
            unsigned long long cnt = 0;
            unsigned int bad = 0;
            for (int k = 0; k < mb; ++k) {
                lo = std::min(lo, hmin[b * mb + k]);
                hi2 = std::max(hi2, hmax[b * mb + k]);
                cnt += hcnt[b * mb + k];
                bad |= hbad[b * mb + k];
            }
            if (bad) return fail(ctx, MPR_ERR_ARG, "image %d: non-finite sampled value", b0 + b);
            if (cnt < 2 || !(hi2 > lo))
                return fail(ctx, MPR_ERR_DEGENERATE, "image %d: fewer than 2 samples or z_max == z_min", b0 + b);
            zmm[2 * b] = lo;
            zmm[2 * b + 1] = hi2;
            zmin_zmax[2 * (b0 + b)] = lo;
            zmin_zmax[2 * (b0 + b) + 1] = hi2;
        }
        HIP_TRY(ctx, hipMemcpyAsync(d_zmm, zmm.data(), zmm.size() * 8, hipMemcpyHostToDevice, stream));
        int64_t maxn = 0;
        for (int b = 0; b < nb; ++b) maxn = std::max(maxn, (int64_t)hi[b].nx * hi[b].ny);
        hipLaunchKernelGGL(map_apply_kernel, dim3(blocks_for(maxn, 4096), nb), dim3(kBlock), 0, stream, d_img, d_zmm,
                           z, sampled, phi);
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipStreamSynchronize(stream));
    }
    return MPR_OK;
}

int32_t mpr_estimate_temperature(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *phi,
                                 const uint8_t *sampled, const mpr_params *p, void *ws, int64_t ws_bytes,
                                 double *e_s, double *T_hat, int32_t *t_clamped, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !valid_params(p) || !phi || !sampled || !e_s || !T_hat)
        return fail(ctx, MPR_ERR_ARG, "estimate_temperature: invalid argument");
    if (!ws || ws_bytes < table_bytes(imgs, n, p)) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    if (int rc = mpr_check_device(ctx, "estimate_temperature", {{"phi", phi}, {"sampled", sampled}, {"workspace", ws}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    // e_s per image (equation mpr-sse)
    {
        Carver cv{(char *)ws, ws_bytes};
        ImgDev *d_img = (ImgDev *)cv.take(n * (int64_t)sizeof(ImgDev));
        double *psum = (double *)cv.take((int64_t)n * kMapBlocks * 8);
        unsigned long long *pcnt = (unsigned long long *)cv.take((int64_t)n * kMapBlocks * 8);
        if (!d_img || !psum || !pcnt) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
        std::vector<ImgDev> hi(n);
        for (int b = 0; b < n; ++b) hi[b] = {imgs[b].offset, imgs[b].nx, imgs[b].ny};
        HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), n * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
        int mb = 1;  // the grid covers the largest image; each image uses image_blocks of its own size
        for (int b = 0; b < n; ++b) mb = std::max(mb, image_blocks((int64_t)hi[b].nx * hi[b].ny));
        hipLaunchKernelGGL(sample_energy_kernel, dim3(mb, n), dim3(kBlock), 0, stream, d_img, phi, sampled,
                           p->q, psum, pcnt);
        HIP_TRY(ctx, hipGetLastError());
        std::vector<double> hs((size_t)n * mb);
        std::vector<unsigned long long> hc((size_t)n * mb);
        // the sums, then the counts (carved after them): one copy
        {
            const char *src = (const char *)psum;
            const int64_t span = (const char *)(pcnt + (int64_t)n * mb) - src;
            std::vector<char> big;
            char *h = stage_for(ctx, span, big);
            HIP_TRY(ctx, hipMemcpyAsync(h, src, (size_t)span, hipMemcpyDeviceToHost, stream));
            HIP_TRY(ctx, hipStreamSynchronize(stream));
            std::memcpy(hs.data(), h, hs.size() * 8);
            std::memcpy(hc.data(), h + ((const char *)pcnt - src), hc.size() * 8);
        }
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            unsigned long long c = 0;
            const int nbk = image_blocks((int64_t)hi[b].nx * hi[b].ny);
            for (int k = 0; k < nbk; ++k) {
                s += hs[(size_t)b * mb + k];
                c += hc[(size_t)b * mb + k];
            }
            if (c == 0) return fail(ctx, MPR_ERR_DEGENERATE, "image %d: no sample-sample pair", b);
            e_s[b] = s / (double)c;
        }
    }
    // e(T, L) tables per table grid size (equation ene), cached.  The
    // missing ones are built together: the table chains of as many grid
    // sizes as the workspace holds run as one ragged chain set (a table does
    // not depend on the chains run beside it: its random numbers are keyed by
    // temperature index and site).
    const std::vector<double> Tg = temperature_grid(p);
    std::vector<TableGrid> tg(n);
    for (int b = 0; b < n; ++b) tg[b] = table_grid(imgs[b], p);
    auto key_of = [&](int b) {
        return std::make_tuple(tg[b].nx, tg[b].ny, p->q, p->table_nT, p->table_T_lo, p->table_T_hi, p->table_burn,
                               p->table_meas, p->a_targ, p->k_a, p->seed);
    };
    std::vector<int> missing;  // first image of each table grid size without a table
    for (int b = 0; b < n; ++b) {
        if (ctx->tables.count(key_of(b))) continue;
        if ((int64_t)tg[b].nx * tg[b].ny < 2) return fail(ctx, MPR_ERR_DEGENERATE, "image %d: one site", b);
        bool dup = false;
        for (int m : missing) dup = dup || (tg[m].nx == tg[b].nx && tg[m].ny == tg[b].ny);
        if (!dup) missing.push_back(b);
    }
    const int nT = p->table_nT;
    // workspace of one grid size's table chains (grids, descriptors, block
    // offsets and redo buffers), as upload_chains carves them
    const int teb = table_angle_bytes(p);
    auto table_chain_bytes = [&](int b) {
        const int64_t hg = round_up(half_grid_bytes(tg[b].nx, tg[b].ny, teb), 256);
        return nT * 2 * hg + redo_bytes(tg[b].nx, tg[b].ny, nT) +
               nT * (int64_t)(sizeof(ChainDesc) + sizeof(ChainState) + 8 + (kNumShapes + 1) * 8) + 4096;
    };
    for (size_t first = 0; first < missing.size();) {
        // as many grid sizes as fit (at least one: the workspace holds the largest)
        size_t last = first;
        int64_t need = 65536 + table_chain_bytes(missing[first]);
        while (last + 1 < missing.size() && need + table_chain_bytes(missing[last + 1]) <= ws_bytes)
            need += table_chain_bytes(missing[++last]);
        Carver cv{(char *)ws, ws_bytes};
        ChainSet cs;
        cs.fp64 = teb == 8;
        int64_t maxn = 0;
        for (size_t g = first; g <= last; ++g) {
            const int b = missing[g];
            const int64_t tnx = tg[b].nx, tny = tg[b].ny;
            maxn = std::max(maxn, tnx * tny);
            for (int k = 0; k < nT; ++k) {
                ChainDesc d;
                std::memset(&d, 0, sizeof d);
                if (!carve_chain(cv, d, (int)tnx, (int)tny, false, false, teb))
                    return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
                d.image_id = kTableStream;
                d.chain = (uint32_t)k;
                d.P = tnx * tny;
                d.ngp = tnx * (tny - 1) + tny * (tnx - 1);
                cs.desc.push_back(d);
                cs.state.push_back(fresh_state(Tg[k], PH_TABLE));
                cs.offset.push_back(0);
            }
        }
        int rc = upload_chains(ctx, cs, cv, stream, p->q);
        if (rc) return rc;
        hipLaunchKernelGGL(init_chains_kernel, dim3(blocks_for(maxn, 2048), (unsigned)cs.desc.size()), dim3(kBlock),
                           0, stream, cs.d_desc, cs.d_offset, nullptr, nullptr, nullptr, 0u, 0u, 1, cs.fp64 ? 1 : 0);
        HIP_TRY(ctx, hipGetLastError());
        rc = run_chains(ctx, cs, p, stream, (int64_t)p->table_burn + p->table_meas, 50, true);
        if (rc) return rc;
        HIP_TRY(ctx, hipMemcpyAsync(cs.state.data(), cs.d_state, cs.state.size() * sizeof(ChainState),
                                    hipMemcpyDeviceToHost, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        for (size_t g = first; g <= last; ++g) {
            std::vector<double> ope(nT);
            for (int k = 0; k < nT; ++k) ope[k] = cs.state[(g - first) * nT + k].e_sum / (double)p->table_meas;
            ctx->tables.emplace(key_of(missing[g]), ope);
        }
        first = last + 1;
    }
    for (int b = 0; b < n; ++b) {
        int cl = 0;
        T_hat[b] = invert_table(Tg, ctx->tables.at(key_of(b)), e_s[b], &cl);
        if (t_clamped) t_clamped[b] = cl;
    }
    return MPR_OK;
}

// mpr_simulate on the workspace ws (the caller's, checked as device memory,
// or this device's static workspace, `caller_ws` false); `graphs` false
// launches every sweep directly.
static int32_t simulate_call(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *phi,
                             const uint8_t *sampled, const double *T_hat, const mpr_params *p,
                             const float *phi_init, void *ws, int64_t ws_bytes, float *phi_sum, float *phi_m2,
                             float *phi_states, mpr_chain_stats *stats, void *stream_, bool caller_ws, bool graphs)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !valid_params(p) || !phi || !sampled || !T_hat || !phi_sum)
        return fail(ctx, MPR_ERR_ARG, "simulate: invalid argument");
    if (int rc = mpr_check_device(ctx, "simulate",
                                  {{"phi", phi}, {"sampled", sampled}, {"phi_init", phi_init},
                                   {"workspace", caller_ws ? ws : nullptr}, {"phi_sum", phi_sum},
                                   {"phi_m2", phi_m2}, {"phi_states", phi_states}}))
        return rc;
    if (phi_m2 && p->K > 1 && !p->spread)
        return fail(ctx, MPR_ERR_ARG, "simulate: phi_m2 with K > 1 needs params.spread = 1");
    if (phi_init && p->K < p->warm_min_states)
        return fail(ctx, MPR_ERR_ARG,
                    "simulate: a warm start (phi_init) needs K >= warm_min_states = %d equilibrium states per "
                    "chain (K = %d): every chain starts from the same angles",
                    p->warm_min_states, p->K);
    for (int b = 0; b < n; ++b)
        if (!(T_hat[b] > 0.0) || !std::isfinite(T_hat[b])) return fail(ctx, MPR_ERR_ARG, "image %d: bad T_hat", b);
    if (!ws || ws_bytes < sim_bytes(imgs, n, p)) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    // gap counts (host needs them for the acceptance ratio): from the mask
    // via a device reduction would need scratch; count with the e_s-style
    // partials instead, reusing the map kernel's layout.
    Carver cv{(char *)ws, ws_bytes};
    // the run header: checked before a resumed run continues; a fresh run
    // marks the workspace as not resumable until it stops at sweep_limit
    RunHeader *d_hdr = (RunHeader *)cv.take(kRunHeaderBytes);
    const uint64_t key = run_key(imgs, n, p, T_hat);
    const bool resume = p->resume != 0;
    RunHeader hdr{kRunMagic, key, sim_bytes(imgs, n, p), n * p->R, 0};
    if (resume) {
        RunHeader old;
        HIP_TRY(ctx, hipMemcpyAsync(&old, d_hdr, sizeof old, hipMemcpyDeviceToHost, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        if (old.magic != hdr.magic || old.key != hdr.key || old.bytes != hdr.bytes || old.n_chains != hdr.n_chains ||
            old.state != 1)
            return fail(ctx, MPR_ERR_ARG,
                        "simulate: resume needs a workspace holding a run stopped at sweep_limit with the same "
                        "images, parameters and temperatures");
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(d_hdr, &hdr, sizeof hdr, hipMemcpyHostToDevice, stream));
    }
    ImgDev *d_img = (ImgDev *)cv.take(n * (int64_t)sizeof(ImgDev));
    std::vector<ImgDev> hi(n);
    for (int b = 0; b < n; ++b) hi[b] = {imgs[b].offset, imgs[b].nx, imgs[b].ny};
    HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), n * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
    std::vector<int64_t> gaps(n, 0);
    {
        // count gaps with the map reduction on a constant z
        char *sp = (char *)ctx->scratch + kVarOffset;
        float *pmin = (float *)sp;
        int mb = 1;  // partial blocks per image (the counts are exact for any number)
        for (int b = 0; b < n; ++b) mb = std::max(mb, image_blocks((int64_t)hi[b].nx * hi[b].ny));
        mb = (int)std::max<int64_t>(1, std::min<int64_t>(mb, ((int64_t)kScratchBytes - kVarOffset - 512) / (24 * (int64_t)n)));
        float *pmax = pmin + (int64_t)n * mb;
        unsigned long long *pcnt = (unsigned long long *)(pmax + (int64_t)n * mb);
        unsigned int *pbad = (unsigned int *)(pcnt + (int64_t)n * mb);
        if ((int64_t)n * mb * 24 + 512 > (int64_t)kScratchBytes - kVarOffset)
            return fail(ctx, MPR_ERR_ARG, "too many images in one call");
        // map_minmax counts sampled sites of finite value; phi is finite
        hipLaunchKernelGGL(map_minmax_kernel, dim3(mb, n), dim3(kBlock), 0, stream, d_img, phi, sampled, pmin,
                           pmax, pcnt, pbad);
        HIP_TRY(ctx, hipGetLastError());
        std::vector<unsigned long long> hc((size_t)n * mb);
        HIP_TRY(ctx, hipMemcpyAsync(hc.data(), pcnt, hc.size() * 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        for (int b = 0; b < n; ++b) {
            unsigned long long c = 0;
            for (int k = 0; k < mb; ++k) c += hc[(size_t)b * mb + k];
            gaps[b] = (int64_t)imgs[b].nx * imgs[b].ny - (int64_t)c;
        }
    }
    ChainSet cs;
    for (int b = 0; b < n; ++b) {
        const int nx = imgs[b].nx, ny = imgs[b].ny;
        if ((int64_t)nx * ny < 2) return fail(ctx, MPR_ERR_DEGENERATE, "image %d: one site", b);
        for (int r = 0; r < p->R; ++r) {
            ChainDesc d;
            std::memset(&d, 0, sizeof d);
            if (!carve_chain(cv, d, nx, ny, p->K > 1, p->spread != 0, p->fp64 ? 8 : 4, !p->fp64))
                return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
            d.image_id = imgs[b].id;
            d.chain = (uint32_t)r;
            d.P = gaps[b];
            d.ngp = (int64_t)nx * (ny - 1) + (int64_t)ny * (nx - 1);
            cs.desc.push_back(d);
            int phase = PH_RELAX;
            if (d.P == 0) phase = PH_DONE;
            else if (p->fixed_relax == 0) phase = p->K > 0 ? PH_EQ : PH_DONE;
            ChainState st = fresh_state(T_hat[b], phase);
            st.eq_left = p->K;
            if (phase == PH_EQ && !p->eq_a_mode) st.a_cur = 1.0;
            cs.state.push_back(st);
            cs.offset.push_back(imgs[b].offset);
        }
    }
    cs.fp64 = p->fp64 != 0;
    cs.K = p->K;
    if (phi_states && p->K > 0) {
        cs.states_out = phi_states;
        for (int b = 0; b < n; ++b)
            cs.states_n_total = std::max(cs.states_n_total, imgs[b].offset + (int64_t)imgs[b].nx * imgs[b].ny);
    }
    const int eb = cs.fp64 ? 8 : 4;
    int rc = upload_chains(ctx, cs, cv, stream, p->q, resume);
    if (rc) return rc;
    int64_t maxn = 0;
    for (int b = 0; b < n; ++b) maxn = std::max(maxn, (int64_t)imgs[b].nx * imgs[b].ny);
    if (!resume) {
        for (auto &d : cs.desc)
            for (int c = 0; c < 2; ++c) {
                HIP_TRY(ctx, hipMemsetAsync(d.h[c], 0, half_grid_bytes(d.nx, d.ny, eb), stream));
                if (d.h2[c]) HIP_TRY(ctx, hipMemsetAsync(d.h2[c], 0, half_grid_bytes(d.nx, d.ny, eb), stream));
            }
        hipLaunchKernelGGL(init_chains_kernel, dim3(blocks_for(maxn, 2048), (unsigned)cs.desc.size()), dim3(kBlock),
                           0, stream, cs.d_desc, cs.d_offset, phi, sampled, phi_init, (uint32_t)p->seed,
                           (uint32_t)(p->seed >> 32), 0, cs.fp64 ? 1 : 0);
        HIP_TRY(ctx, hipGetLastError());
    }
    // sweeps left to the run's cap (a resumed run has done `swept` of them),
    // and to this call's sweep_limit
    const int64_t relax_cap = p->fixed_relax >= 0 ? p->fixed_relax : (int64_t)p->i_max + 1;
    int64_t swept = 0;
    for (const auto &st : cs.state) swept = std::max<int64_t>(swept, (int64_t)st.sweep);
    int64_t limit = std::max<int64_t>(1, relax_cap + p->K + 1 - swept);
    if (p->sweep_limit > 0) limit = std::min<int64_t>(limit, p->sweep_limit);
    rc = run_chains(ctx, cs, p, stream, limit, p->n_f, false, graphs, p->sweep_limit > 0);
    const bool incomplete = rc == MPR_INCOMPLETE;
    if (rc && !incomplete) return rc;
    if (incomplete || resume) {
        // resumable while chains are running, not once the run is finished
        hdr.state = incomplete ? 1 : 0;
        HIP_TRY(ctx, hipMemcpyAsync(d_hdr, &hdr, sizeof hdr, hipMemcpyHostToDevice, stream));
    }
    if (!incomplete) {  // an incomplete run writes no outputs, only its statistics so far
        if (cs.fp64)
            hipLaunchKernelGGL(finalize_fp64_kernel, dim3(blocks_for(maxn, 4096), n), dim3(kBlock), 0, stream,
                               cs.d_desc, d_img, p->R, p->K, sampled, phi_sum, phi_m2);
        else
            hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(maxn, 4096), n), dim3(kBlock), 0, stream,
                               cs.d_desc, d_img, p->R, p->K, sampled, phi_sum, phi_m2);
        HIP_TRY(ctx, hipGetLastError());
    }
    if (stats) {
        HIP_TRY(ctx, hipMemcpyAsync(cs.state.data(), cs.d_state, cs.state.size() * sizeof(ChainState),
                                    hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    if (stats) {
        for (size_t c = 0; c < cs.state.size(); ++c) {
            const ChainState &s = cs.state[c];
            stats[c].relax_sweeps = s.relax_sweeps;
            stats[c].not_converged = s.not_converged;
            stats[c].a_final = s.a_relax;
            stats[c].A_last = s.A_last;
            stats[c].k_last = s.k;
        }
    }
    return incomplete ? MPR_INCOMPLETE : MPR_OK;
}

int32_t mpr_simulate(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *phi, const uint8_t *sampled,
                     const double *T_hat, const mpr_params *p, const float *phi_init, void *ws, int64_t ws_bytes,
                     float *phi_sum, float *phi_m2, float *phi_states, mpr_chain_stats *stats, void *stream_)
{
    return simulate_call(ctx, imgs, n, phi, sampled, T_hat, p, phi_init, ws, ws_bytes, phi_sum, phi_m2, phi_states,
                         stats, stream_, true, true);
}

int32_t mpr_simulate_noalloc(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *phi,
                             const uint8_t *sampled, const double *T_hat, const mpr_params *p,
                             const float *phi_init, float *phi_sum, float *phi_m2, float *phi_states,
                             mpr_chain_stats *stats, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !valid_params(p))
        return fail(ctx, MPR_ERR_ARG, "simulate_noalloc: invalid argument");
    if (!ctx->static_ws)
        return fail(ctx, MPR_ERR_HIP, "simulate_noalloc: no static workspace on device %d", ctx->device);
    const int64_t need = sim_bytes(imgs, n, p);
    if (need > kStaticWorkspaceBytes)
        return fail(ctx, MPR_ERR_WORKSPACE,
                    "simulate_noalloc: this batch needs %lld workspace bytes, the static workspace holds %lld "
                    "(use mpr_simulate with a workspace of mpr_workspace_size bytes)",
                    (long long)need, (long long)kStaticWorkspaceBytes);
    return simulate_call(ctx, imgs, n, phi, sampled, T_hat, p, phi_init, ctx->static_ws, kStaticWorkspaceBytes,
                         phi_sum, phi_m2, phi_states, stats, stream_, false, false);
}

int64_t mpr_simulate_noalloc_max_bytes(void) { return kStaticWorkspaceBytes; }

int32_t mpr_predict(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *z, const uint8_t *sampled,
                    const float *phi_sum, const double *zmin_zmax, int32_t M, float *z_hat, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !z || !sampled || !phi_sum || !zmin_zmax || !z_hat || M < 1)
        return fail(ctx, MPR_ERR_ARG, "predict: invalid argument");
    if (int rc = mpr_check_device(ctx, "predict",
                                  {{"z", z}, {"sampled", sampled}, {"phi_sum", phi_sum}, {"z_hat", z_hat}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t need = round_up((int64_t)n * sizeof(ImgDev), 256) + (int64_t)n * 16;
    if (need > (int64_t)kScratchBytes - kVarOffset) return fail(ctx, MPR_ERR_ARG, "too many images in one call");
    char *sp = (char *)ctx->scratch + kVarOffset;
    ImgDev *d_img = (ImgDev *)sp;
    double *d_zmm = (double *)(sp + round_up((int64_t)n * sizeof(ImgDev), 256));
    std::vector<ImgDev> hi(n);
    int64_t maxn = 0;
    for (int b = 0; b < n; ++b) {
        hi[b] = {imgs[b].offset, imgs[b].nx, imgs[b].ny};
        maxn = std::max(maxn, (int64_t)imgs[b].nx * imgs[b].ny);
    }
    HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), n * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_zmm, zmin_zmax, n * 16, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(predict_kernel, dim3(blocks_for(maxn, 4096), n), dim3(kBlock), 0, stream, d_img, d_zmm, M, z,
                       sampled, phi_sum, z_hat);
    HIP_TRY(ctx, hipGetLastError());
    // the host arrays above must outlive the copies
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

int32_t mpr_quantiles(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const float *z, const uint8_t *sampled,
                      const float *phi_states, int32_t M, const double *probs, int32_t nq, const double *zmin_zmax,
                      float *z_q, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !z || !sampled || !phi_states || !probs || !zmin_zmax || !z_q || M < 1 ||
        M > kMaxQuantileStates || nq < 1 || nq > 64)
        return fail(ctx, MPR_ERR_ARG, "quantiles: invalid argument (1 <= M <= %d, 1 <= nq <= 64)",
                    kMaxQuantileStates);
    for (int k = 0; k < nq; ++k)
        if (!(probs[k] >= 0.0 && probs[k] <= 1.0)) return fail(ctx, MPR_ERR_ARG, "quantiles: p outside [0, 1]");
    if (int rc = mpr_check_device(ctx, "quantiles",
                                  {{"z", z}, {"sampled", sampled}, {"phi_states", phi_states}, {"z_q", z_q}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t img_bytes = round_up((int64_t)n * sizeof(ImgDev), 256);
    const int64_t need = img_bytes + round_up((int64_t)n * 16, 256) + nq * 8;
    if (need > (int64_t)kScratchBytes - kVarOffset) return fail(ctx, MPR_ERR_ARG, "too many images in one call");
    char *sp = (char *)ctx->scratch + kVarOffset;
    ImgDev *d_img = (ImgDev *)sp;
    double *d_zmm = (double *)(sp + img_bytes);
    double *d_probs = (double *)(sp + img_bytes + round_up((int64_t)n * 16, 256));
    std::vector<ImgDev> hi(n);
    int64_t maxn = 0, n_total = 0;
    for (int b = 0; b < n; ++b) {
        hi[b] = {imgs[b].offset, imgs[b].nx, imgs[b].ny};
        maxn = std::max(maxn, (int64_t)imgs[b].nx * imgs[b].ny);
        n_total = std::max(n_total, imgs[b].offset + (int64_t)imgs[b].nx * imgs[b].ny);
    }
    HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), n * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_zmm, zmin_zmax, n * 16, hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_probs, probs, nq * 8, hipMemcpyHostToDevice, stream));
    if (M <= 128) {
        // sort in registers: a network of the smallest power-of-two size >= M
        const int gb = blocks_for(maxn, 8192);
        if (M <= 16)
            hipLaunchKernelGGL(quantile_net_kernel<16>, dim3(gb, n), dim3(kBlock), 0, stream, d_img, d_zmm, d_probs,
                               nq, z, sampled, phi_states, M, n_total, z_q);
        else if (M <= 32)
            hipLaunchKernelGGL(quantile_net_kernel<32>, dim3(gb, n), dim3(kBlock), 0, stream, d_img, d_zmm, d_probs,
                               nq, z, sampled, phi_states, M, n_total, z_q);
        else if (M <= 64)
            hipLaunchKernelGGL(quantile_net_kernel<64>, dim3(gb, n), dim3(kBlock), 0, stream, d_img, d_zmm, d_probs,
                               nq, z, sampled, phi_states, M, n_total, z_q);
        else
            hipLaunchKernelGGL(quantile_net_kernel<128>, dim3(gb, n), dim3(kBlock), 0, stream, d_img, d_zmm, d_probs,
                               nq, z, sampled, phi_states, M, n_total, z_q);
    } else {
        const int gx =
            (int)std::max<int64_t>(1, std::min<int64_t>((maxn + kQuantileLanes - 1) / kQuantileLanes, 8192));
        hipLaunchKernelGGL(quantile_kernel, dim3(gx, n), dim3(kQuantileLanes), 0, stream, d_img, d_zmm, d_probs, nq,
                           z, sampled, phi_states, M, n_total, z_q);
    }
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

int32_t mpr_spread(mpr_ctx *ctx, const mpr_image *imgs, int32_t n, const uint8_t *sampled, const float *phi_m2,
                   const double *zmin_zmax, int32_t M, float *z_std, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(imgs, n) || !sampled || !phi_m2 || !zmin_zmax || !z_std || M < 1)
        return fail(ctx, MPR_ERR_ARG, "spread: invalid argument");
    if (int rc = mpr_check_device(ctx, "spread", {{"sampled", sampled}, {"phi_m2", phi_m2}, {"z_std", z_std}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t need = round_up((int64_t)n * sizeof(ImgDev), 256) + (int64_t)n * 16;
    if (need > (int64_t)kScratchBytes - kVarOffset) return fail(ctx, MPR_ERR_ARG, "too many images in one call");
    char *sp = (char *)ctx->scratch + kVarOffset;
    ImgDev *d_img = (ImgDev *)sp;
    double *d_zmm = (double *)(sp + round_up((int64_t)n * sizeof(ImgDev), 256));
    std::vector<ImgDev> hi(n);
    int64_t maxn = 0;
    for (int b = 0; b < n; ++b) {
        hi[b] = {imgs[b].offset, imgs[b].nx, imgs[b].ny};
        maxn = std::max(maxn, (int64_t)imgs[b].nx * imgs[b].ny);
    }
    HIP_TRY(ctx, hipMemcpyAsync(d_img, hi.data(), n * sizeof(ImgDev), hipMemcpyHostToDevice, stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_zmm, zmin_zmax, n * 16, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(spread_kernel, dim3(blocks_for(maxn, 4096), n), dim3(kBlock), 0, stream, d_img, d_zmm, M,
                       sampled, phi_m2, z_std);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

// Workspace of mpr_select_q: four per-site buffers of the image and the
// largest simulation/temperature workspace over the candidate q.
int64_t select_q_bytes(const mpr_image *img, const mpr_params *p, const double *q_grid, int nq)
{
    const int64_t n = (int64_t)img->nx * img->ny;
    mpr_image im0 = *img;
    im0.offset = 0;
    int64_t best = 0;
    for (int k = 0; k < nq; ++k) {
        mpr_params pk = *p;
        pk.q = q_grid[k];
        pk.fp64 = q_grid[k] == 0.5 ? p->fp64 : 1;
        if (!valid_params(&pk)) return -1;
        best = std::max(best, std::max(sim_bytes(&im0, 1, &pk), table_bytes(&im0, 1, &pk)));
    }
    return best + round_up(n, 256) + 3 * round_up(4 * n, 256) + 1024;
}

int64_t mpr_select_q_workspace_size(const mpr_image *img, const mpr_params *p, const double *q_grid, int32_t nq)
{
    if (!valid_images(img, 1) || !p || !q_grid || nq < 1) return -1;
    return select_q_bytes(img, p, q_grid, nq);
}

int32_t mpr_select_q(mpr_ctx *ctx, const mpr_image *img, const float *z, const uint8_t *sampled, const mpr_params *p,
                     const double *q_grid, int32_t nq, double holdout, void *ws, int64_t ws_bytes, double *val_mae,
                     double *T_hat, double *q_best, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!valid_images(img, 1) || !z || !sampled || !p || !q_grid || nq < 1 || nq > 64 || !(holdout > 0.0) ||
        !(holdout < 1.0) || !val_mae || !q_best || p->K < 1)
        return fail(ctx, MPR_ERR_ARG, "select_q: invalid argument");
    const int64_t need = select_q_bytes(img, p, q_grid, nq);
    if (need < 0) return fail(ctx, MPR_ERR_ARG, "select_q: a candidate q is outside (0, 1/2]");
    if (!ws || ws_bytes < need) return fail(ctx, MPR_ERR_WORKSPACE, "workspace too small");
    if (int rc = mpr_check_device(ctx, "select_q", {{"z", z}, {"sampled", sampled}, {"workspace", ws}})) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t n = (int64_t)img->nx * img->ny;
    mpr_image im0 = *img;
    im0.offset = 0;
    const float *zi = z + img->offset;
    const uint8_t *si = sampled + img->offset;
    // per-site buffers first, the calls' workspace after them
    const int64_t head = round_up(n, 256) + 3 * round_up(4 * n, 256);
    uint8_t *fit = (uint8_t *)ws;
    float *phi = (float *)((char *)ws + round_up(n, 256));
    float *psum = (float *)((char *)phi + round_up(4 * n, 256));
    float *zhat = (float *)((char *)psum + round_up(4 * n, 256));
    void *iws = (char *)ws + head;
    const int64_t inner = ws_bytes - head;
    hipLaunchKernelGGL(holdout_kernel, dim3(blocks_for(n, 2048)), dim3(kBlock), 0, stream, img->nx, img->ny, si,
                       (uint32_t)p->seed, (uint32_t)(p->seed >> 32), holdout, fit);
    HIP_TRY(ctx, hipGetLastError());
    double zmm[2];
    int rc = mpr_map_to_angles(ctx, &im0, 1, zi, fit, phi, zmm, stream);
    if (rc) return rc;
    double *d_ps = (double *)((char *)ctx->scratch + kVarOffset);
    unsigned long long *d_pc = (unsigned long long *)(d_ps + kHoldoutBlocks);
    int best = -1;
    for (int k = 0; k < nq; ++k) {
        mpr_params pk = *p;
        pk.q = q_grid[k];
        pk.fp64 = q_grid[k] == 0.5 ? p->fp64 : 1;
        double e_s = 0.0, T = 0.0;
        rc = mpr_estimate_temperature(ctx, &im0, 1, phi, fit, &pk, iws, inner, &e_s, &T, nullptr, stream);
        if (rc) return rc;
        rc = mpr_simulate(ctx, &im0, 1, phi, fit, &T, &pk, nullptr, iws, inner, psum, nullptr, nullptr, nullptr,
                          stream);
        if (rc) return rc;
        rc = mpr_predict(ctx, &im0, 1, zi, fit, psum, zmm, pk.R * pk.K, zhat, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(holdout_error_kernel, dim3(kHoldoutBlocks), dim3(kBlock), 0, stream, n, zi, si, fit,
                           zhat, d_ps, d_pc);
        HIP_TRY(ctx, hipGetLastError());
        double hs[kHoldoutBlocks];
        unsigned long long hc[kHoldoutBlocks];
        HIP_TRY(ctx, hipMemcpyAsync(hs, d_ps, sizeof hs, hipMemcpyDeviceToHost, stream));
        HIP_TRY(ctx, hipMemcpyAsync(hc, d_pc, sizeof hc, hipMemcpyDeviceToHost, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        double sum = 0.0;
        unsigned long long cnt = 0;
        for (int b = 0; b < kHoldoutBlocks; ++b) {
            sum += hs[b];
            cnt += hc[b];
        }
        if (cnt == 0) return fail(ctx, MPR_ERR_DEGENERATE, "select_q: no sample held out");
        val_mae[k] = sum / (double)cnt;
        if (T_hat) T_hat[k] = T;
        // smallest error; on a tie the larger q
        if (best < 0 || val_mae[k] < val_mae[best] || (val_mae[k] == val_mae[best] && q_grid[k] > q_grid[best]))
            best = k;
    }
    *q_best = q_grid[best];
    return MPR_OK;
}

int32_t mpr_profile_enable(mpr_ctx *ctx, int32_t on)
{
    if (!ctx) return MPR_ERR_ARG;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->profile = on != 0;
    ctx->prof_ms = 0.0;
    ctx->prof_launches = 0;
    HIP_TRY(ctx, hipMemset((char *)ctx->scratch + kWorkOffset, 0, 3 * sizeof(unsigned long long)));
    return MPR_OK;
}

int32_t mpr_profile_read(mpr_ctx *ctx, mpr_profile *out)
{
    if (!ctx || !out) return MPR_ERR_ARG;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    unsigned long long w[3] = {0, 0, 0};
    HIP_TRY(ctx, hipMemcpy(w, (char *)ctx->scratch + kWorkOffset, sizeof w, hipMemcpyDeviceToHost));
    out->sweep_kernel_ms = ctx->prof_ms;
    out->sweep_launches = ctx->prof_launches;
    out->last_tile = ctx->last_tile;
    out->reserved = 0;
    out->chain_sweeps = (int64_t)w[0];
    out->site_updates = (int64_t)w[1];
    out->useful_bytes = (double)w[2];
    return MPR_OK;
}

// ------------------------------------------------------------ diagnostics

int32_t mpr_diag_philox(mpr_ctx *ctx, const uint32_t *ctr, uint64_t seed, int64_t n, uint32_t *out, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!ctr || !out || n < 0) return fail(ctx, MPR_ERR_ARG, "diag_philox: invalid argument");
    if (int rc = mpr_check_device(ctx, "diag_philox", {{"ctr", ctr}, {"out", out}})) return rc;
    if (n == 0) return MPR_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, ctr,
                       (uint32_t)seed, (uint32_t)(seed >> 32), n, out);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

int32_t mpr_diag_half_sweep(mpr_ctx *ctx, int32_t nx, int32_t ny, float *phi, const uint8_t *sampled, int32_t colour,
                            double T, double a, double q, uint64_t seed, uint32_t sweep, uint32_t chain,
                            uint32_t stream_id, int32_t mode, int32_t tile, uint8_t *flags, int64_t *accepted,
                            double *bond_energy, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    const int v = tile ? shape_of(tile) : kDefaultShape;
    if (nx < 1 || ny < 1 || (int64_t)nx * ny < 2 || half_grid_bytes(nx, ny) >= ((int64_t)1 << 32) || !phi ||
        !sampled || (colour != 0 && colour != 1) || !(T > 0) || !(a > 0) || q != 0.5 || (mode != 0 && mode != 1) ||
        v < 0)
        return fail(ctx, MPR_ERR_ARG, "diag_half_sweep: invalid argument");
    if (int rc = mpr_check_device(ctx, "diag_half_sweep", {{"phi", phi}, {"sampled", sampled}, {"flags", flags}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t hg = half_grid_bytes(nx, ny);
    const int64_t bytes = 2 * round_up(hg, 256) + 8192 + redo_bytes(nx, ny, 1);
    void *buf = nullptr;
    HIP_TRY(ctx, hipMalloc(&buf, bytes));
    Carver cv{(char *)buf, bytes};
    ChainSet cs;
    ChainDesc d;
    std::memset(&d, 0, sizeof d);
    carve_chain(cv, d, nx, ny, false);
    d.image_id = stream_id;
    d.chain = chain;
    d.P = 1;
    d.ngp = (int64_t)nx * (ny - 1) + (int64_t)ny * (nx - 1);
    cs.desc.push_back(d);
    ChainState st = fresh_state(T, PH_RELAX);
    st.sweep = sweep;
    st.a_cur = a;
    cs.state.push_back(st);
    cs.offset.push_back(0);
    int rc = upload_chains(ctx, cs, cv, stream, q);
    if (rc) {
        (void)hipFree(buf);
        return rc;
    }
    (void)hipMemsetAsync(d.h[0], 0, hg, stream);
    (void)hipMemsetAsync(d.h[1], 0, hg, stream);
    const int64_t nsite = (int64_t)nx * ny;
    // the gap values of phi are the starting state
    hipLaunchKernelGGL(init_chains_kernel, dim3(blocks_for(nsite, 2048), 1), dim3(kBlock), 0, stream, cs.d_desc,
                       cs.d_offset, phi, sampled, phi, 0u, 0u, 0, 0);
    if (flags) (void)hipMemsetAsync(flags, 0, nsite, stream);
    const SweepConsts sc = make_sc(q, seed);
    const dim3 grid((unsigned)cs.total_blocks[v]);
    const Shape sh = kShapes[v];
    const Redo rd = cs.redo;
    if (sh.fused) {
        launch_tile<true>(stream, cs, v, colour + 1, sc, mode, flags);
    } else if (sh.compact) {
        if (sh.rows == 2)
            hipLaunchKernelGGL((half_sweep_compact_kernel<true, 2>), grid, dim3(kBlock), 0, stream, cs.d_desc,
                               cs.d_state, block_map(cs, v), colour, sc, mode, rd, flags);
        else if (sh.rows == 4)
            hipLaunchKernelGGL((half_sweep_compact_kernel<true, 4>), grid, dim3(kBlock), 0, stream, cs.d_desc,
                               cs.d_state, block_map(cs, v), colour, sc, mode, rd, flags);
        else
            hipLaunchKernelGGL((half_sweep_compact_kernel<true, 8>), grid, dim3(kBlock), 0, stream, cs.d_desc,
                               cs.d_state, block_map(cs, v), colour, sc, mode, rd, flags);
    } else {
        if (sh.rows == 1)
            hipLaunchKernelGGL((half_sweep_kernel<true, 1>), grid, dim3(kBlock), 0, stream, cs.d_desc, cs.d_state,
                               block_map(cs, v), colour, sc, mode, rd, flags);
        else if (sh.rows == 2)
            hipLaunchKernelGGL((half_sweep_kernel<true, 2>), grid, dim3(kBlock), 0, stream, cs.d_desc, cs.d_state,
                               block_map(cs, v), colour, sc, mode, rd, flags);
        else if (sh.rows == 4)
            hipLaunchKernelGGL((half_sweep_kernel<true, 4>), grid, dim3(kBlock), 0, stream, cs.d_desc, cs.d_state,
                               block_map(cs, v), colour, sc, mode, rd, flags);
        else
            hipLaunchKernelGGL((half_sweep_kernel<true, 8>), grid, dim3(kBlock), 0, stream, cs.d_desc, cs.d_state,
                               block_map(cs, v), colour, sc, mode, rd, flags);
    }
    if (!sh.fused) launch_redo<true>(stream, cs, v, colour, sc, mode, flags);
    hipLaunchKernelGGL(unsplit_kernel, dim3(blocks_for(nsite, 2048)), dim3(kBlock), 0, stream, cs.d_desc, phi);
    ChainState out;
    (void)hipMemcpyAsync(&out, cs.d_state, sizeof out, hipMemcpyDeviceToHost, stream);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(stream);
    (void)hipFree(buf);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(ctx, MPR_ERR_HIP, "diag_half_sweep: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    if (accepted) *accepted = (int64_t)out.acc;
    if (bond_energy) *bond_energy = (double)out.e_fx * kEnergyUnit;
    return MPR_OK;
}

int32_t mpr_diag_half_sweep_fp64(mpr_ctx *ctx, int32_t nx, int32_t ny, double *phi, const uint8_t *sampled,
                                 int32_t colour, double T, double a, double q, uint64_t seed, uint32_t sweep,
                                 uint32_t chain, uint32_t stream_id, int32_t mode, int32_t tile, uint8_t *flags,
                                 int64_t *accepted, double *bond_energy, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    const int v = tile ? shape_of(tile) : kDefaultShape;
    if (nx < 1 || ny < 1 || (int64_t)nx * ny < 2 || half_grid_bytes(nx, ny) >= ((int64_t)1 << 32) || !phi ||
        !sampled || (colour != 0 && colour != 1) || !(T > 0) || !(a > 0) || !(q > 0.0 && q <= 0.5) ||
        (mode != 0 && mode != 1) || v < 0)
        return fail(ctx, MPR_ERR_ARG, "diag_half_sweep_fp64: invalid argument");
    if (int rc = mpr_check_device(ctx, "diag_half_sweep_fp64", {{"phi", phi}, {"sampled", sampled}, {"flags", flags}}))
        return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t hg = half_grid_bytes(nx, ny, 8);
    const int64_t bytes = 2 * round_up(hg, 256) + 8192 + redo_bytes(nx, ny, 1);
    void *buf = nullptr;
    HIP_TRY(ctx, hipMalloc(&buf, bytes));
    Carver cv{(char *)buf, bytes};
    ChainSet cs;
    cs.fp64 = true;
    ChainDesc d;
    std::memset(&d, 0, sizeof d);
    carve_chain(cv, d, nx, ny, false, false, 8);
    d.image_id = stream_id;
    d.chain = chain;
    d.P = 1;
    d.ngp = (int64_t)nx * (ny - 1) + (int64_t)ny * (nx - 1);
    cs.desc.push_back(d);
    ChainState st = fresh_state(T, PH_RELAX);
    st.sweep = sweep;
    st.a_cur = a;
    cs.state.push_back(st);
    cs.offset.push_back(0);
    int rc = upload_chains(ctx, cs, cv, stream, q);
    if (rc) {
        (void)hipFree(buf);
        return rc;
    }
    (void)hipMemsetAsync(d.h[0], 0, hg, stream);
    (void)hipMemsetAsync(d.h[1], 0, hg, stream);
    const int64_t nsite = (int64_t)nx * ny;
    hipLaunchKernelGGL(split_fp64_kernel, dim3(blocks_for(nsite, 2048)), dim3(kBlock), 0, stream, cs.d_desc, phi,
                       sampled);
    if (flags) (void)hipMemsetAsync(flags, 0, nsite, stream);
    launch_half_fp64<true>(stream, cs, v, colour, make_sc(q, seed), mode, flags);
    hipLaunchKernelGGL(unsplit_fp64_kernel, dim3(blocks_for(nsite, 2048)), dim3(kBlock), 0, stream, cs.d_desc, phi);
    ChainState out;
    (void)hipMemcpyAsync(&out, cs.d_state, sizeof out, hipMemcpyDeviceToHost, stream);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(stream);
    (void)hipFree(buf);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(ctx, MPR_ERR_HIP, "diag_half_sweep_fp64: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    if (accepted) *accepted = (int64_t)out.acc;
    if (bond_energy) *bond_energy = (double)out.e_fx * kEnergyUnit64;
    return MPR_OK;
}

int32_t mpr_diag_copy(mpr_ctx *ctx, const void *src, void *dst, int64_t bytes, void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!src || !dst || bytes < 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return fail(ctx, MPR_ERR_ARG, "diag_copy: invalid argument");
    if (int rc = mpr_check_device(ctx, "diag_copy", {{"src", src}, {"dst", dst}})) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t n = bytes / 16;
    if (n > 0)
        hipLaunchKernelGGL(copy_probe_kernel, dim3(blocks_for(n, 8192)), dim3(kBlock), 0, stream,
                           (const float4 *)src, (float4 *)dst, n);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    return MPR_OK;
}

int32_t mpr_diag_energy(mpr_ctx *ctx, int32_t nx, int32_t ny, const float *phi, double q, double *h_plus_ngp,
                        void *stream_)
{
    if (!ctx) return MPR_ERR_ARG;
    if (nx < 1 || ny < 1 || !phi || !h_plus_ngp || !(q > 0 && q <= 0.5))
        return fail(ctx, MPR_ERR_ARG, "diag_energy: invalid argument");
    if (int rc = mpr_check_device(ctx, "diag_energy", {{"phi", phi}})) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t stream = (hipStream_t)stream_;
    unsigned long long *d_e = (unsigned long long *)((char *)ctx->scratch + kEnergyOffset);
    HIP_TRY(ctx, hipMemsetAsync(d_e, 0, 8, stream));
    hipLaunchKernelGGL(grid_energy_kernel, dim3(blocks_for((int64_t)nx * ny, 2048)), dim3(kBlock), 0, stream, phi, nx,
                       ny, (float)q, d_e);
    HIP_TRY(ctx, hipGetLastError());
    unsigned long long e = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&e, d_e, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    *h_plus_ngp = (double)e * kEnergyUnit;
    return MPR_OK;
}

int32_t mpr_diag_sg_slope(mpr_ctx *ctx, const double *e, int32_t n, int32_t degree, double *slope)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!e || !slope || n < 2 || n > kMaxFit || degree < 1 || degree >= n)
        return fail(ctx, MPR_ERR_ARG, "diag_sg_slope: invalid argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    mpr_params p;
    mpr_default_params(&p);
    p.n_fit = n;
    p.sg_degree = degree;
    const CtlParams cp = make_ctl(&p);
    double *d = (double *)((char *)ctx->scratch + kSlopeOffset);
    HIP_TRY(ctx, hipMemcpy(d, e, n * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(ring_slope_kernel, dim3(1), dim3(1), 0, 0, d, n, cp, d + kMaxFit);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpy(slope, d + kMaxFit, 8, hipMemcpyDeviceToHost));
    return MPR_OK;
}

}  // extern "C"
