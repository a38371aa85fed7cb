// Warm-start network for the MPR chains on gfx950: a residual CNN of 3x3
// convolutions with 32 channels, bfloat16 weights and activations, float
// accumulation on the matrix cores (v_mfma_f32_32x32x16_bf16).
//
// Tensors are NHWC bfloat16 with C = 32 channels (64 bytes per pixel).  A
// conv layer's float master weights are W[tap][ci][co] (tap = 3 (dy+1) +
// (dx+1)) followed by b[co]; they are packed to bfloat16 in two layouts:
//   forward  F[tap][co][ci] = W[tap][ci][co]
//   dgrad    D[tap][ci][co] = W[8 - tap][ci][co]   (input gradient = a
//            forward conv of the output gradient with flipped taps and the
//            channel roles swapped)
// so that one kernel serves both; its epilogue adds the bias, an optional
// residual tensor, and applies ReLU or the ReLU derivative (zero where a
// reference activation is <= 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mpr.h"

namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int CH = 32;
constexpr int NBLK = 8;
constexpr int NLAYER = 2 + 2 * NBLK;
constexpr int WSZ = 9 * CH * CH;            // weights per layer
constexpr int LSZ = WSZ + CH;                // weights + bias per layer
constexpr int TH = 8, TW = 32;               // output tile (rows x cols)
constexpr int PIXS = 40;                     // staged pixel stride in bf16 (80 B)
constexpr int IN_T = (TH + 2) * (TW + 2);    // staged input pixels
constexpr int WG_BLOCKS = 256;               // persistent blocks of the weight-gradient kernel
constexpr int WG_PART = WSZ + CH;            // floats per partial

struct ConvArgs {
    const bf16 *in;        // N x H x W x 32
    const bf16 *w;         // packed [9][32 out][32 in]
    const float *bias;     // [32] or null
    const bf16 *add;       // residual, same shape as out, or null
    const bf16 *ref;       // zero the output where ref <= 0, or null
    bf16 *out;
    int N, H, W;
    int relu;
    // the network's own input and output (SIDE bits 2 and 3): encoded from
    // the sample angles while staging, decoded into starting gap angles in
    // the epilogue
    const float *phi;
    const uint8_t *sampled;
    float *phi_out;
};

// Stages the (TH+2) x (TW+2) input pixels around an output tile into LDS,
// zero outside the image.
__device__ __forceinline__ void stage_tile(const bf16 *__restrict__ src, bf16 *tile, int n, int H, int W, int y0,
                                           int x0, const bf16 *__restrict__ ref)
{
    for (int k = threadIdx.x; k < IN_T * 4; k += blockDim.x) {
        const int chunk = k & 3, pix = k >> 2;
        const int r = pix / (TW + 2), c = pix - r * (TW + 2);
        const int gy = y0 - 1 + r, gx = x0 - 1 + c;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const int64_t off = (((int64_t)n * H + gy) * W + gx) * CH + chunk * 8;
            v = *reinterpret_cast<const uint4 *>(src + off);
            (void)ref;
        }
        *reinterpret_cast<uint4 *>(tile + pix * PIXS + chunk * 8) = v;
    }
}

// Forward convolution (and, with the dgrad packing, the input gradient).
// Persistent blocks of 4 waves loop over 16 x 32-pixel output tiles.  The
// layer's packed weights are copied to LDS once per block (rows of 32
// input channels padded to 80 bytes, like the staged pixels, so 16-byte
// reads are conflict-free); a tile's (16+2) x (32+2) input pixels are
// staged in LDS, and the next tile's pixels are loaded into registers while
// the current tile computes.  Wave w computes output rows 4w .. 4w+3 with
// v_mfma_f32_32x32x16_bf16 taking the weights as A (32 output channels x 16
// input channels) and the pixels as B (16 input channels x 32 pixels): per
// column shift and channel half, the three taps' weight operands are read
// once and each staged input row once, feeding the up to three output rows
// it touches.  Each lane ends with 16 channels of one pixel (4 runs of 4),
// so the epilogue moves 8-byte vectors, and the residual input of a tile is
// loaded before its products so that it arrives while they run.
constexpr int CTH = 16, CTW = 32;                 // output tile of the forward conv
constexpr int C_IN_W = CTW + 2;                   // staged input columns
constexpr int C_IN_T = (CTH + 2) * C_IN_W;        // staged input pixels
constexpr int C_CHUNKS = C_IN_T * 4;              // 16-byte chunks per staged tile
constexpr int C_PER_THREAD = (C_CHUNKS + 255) / 256;
constexpr int C_W_ROWS = 9 * CH;                  // packed weight rows (tap, out-channel)

__device__ __forceinline__ void conv_tile_origin(int tile, int tiles_x, int tiles_y, int &n, int &y0, int &x0)
{
    const int tx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int ty = rest % tiles_y;
    n = rest / tiles_y;
    y0 = ty * CTH;
    x0 = tx * CTW;
}

// Loads this thread's chunks of a staged tile.  Every load is issued (a
// chunk outside the image reads a clamped in-image address and its bit in
// `valid` is cleared; conv_store_tile writes zeros for it): a fixed number of
// loads in flight lets later waits for other loads leave these outstanding.
__device__ __forceinline__ void conv_load_tile(const bf16 *__restrict__ src, int n, int H, int W, int y0, int x0,
                                               uint4 (&r)[C_PER_THREAD], uint32_t &valid)
{
    valid = 0u;
#pragma unroll
    for (int j = 0; j < C_PER_THREAD; ++j) {
        const int k = min((int)threadIdx.x + 256 * j, C_CHUNKS - 1);
        const int chunk = k & 3, pix = k >> 2;
        const int rr = pix / C_IN_W, cc = pix - rr * C_IN_W;
        const int gy = y0 - 1 + rr, gx = x0 - 1 + cc;
        const bool ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
        valid |= ok ? (1u << j) : 0u;
        const int gyc = min(max(gy, 0), H - 1), gxc = min(max(gx, 0), W - 1);
        r[j] = *reinterpret_cast<const uint4 *>(src + (((int64_t)n * H + gyc) * W + gxc) * CH + chunk * 8);
    }
}

__device__ __forceinline__ void conv_store_tile(bf16 *tile, const uint4 (&r)[C_PER_THREAD], uint32_t valid)
{
#pragma unroll
    for (int j = 0; j < C_PER_THREAD; ++j) {
        const int k = (int)threadIdx.x + 256 * j;
        if (k < C_CHUNKS)
            *reinterpret_cast<uint4 *>(tile + (k >> 2) * PIXS + (k & 3) * 8) =
                ((valid >> j) & 1u) ? r[j] : make_uint4(0u, 0u, 0u, 0u);
    }
}

// The stem's staging with the network input computed on the way (SIDE bit
// 2): chunk 0 of a sampled pixel inside the image is (cos q phi, sin q phi,
// 1) in bfloat16 with q = 1/2 (encode_kernel's values), every other chunk
// zero.  The loads keep the raw angle and flag; the encoding is done when
// the chunk is stored, after the products that the loads overlap.
__device__ __forceinline__ void enc_load_tile(const float *__restrict__ phi, const uint8_t *__restrict__ sampled,
                                              int n, int H, int W, int y0, int x0, uint4 (&r)[C_PER_THREAD],
                                              uint32_t &valid)
{
    valid = 0u;
#pragma unroll
    for (int j = 0; j < C_PER_THREAD; ++j) {
        const int k = min((int)threadIdx.x + 256 * j, C_CHUNKS - 1);
        const int chunk = k & 3, pix = k >> 2;
        const int rr = pix / C_IN_W, cc = pix - rr * C_IN_W;
        const int gy = y0 - 1 + rr, gx = x0 - 1 + cc;
        const bool ok = chunk == 0 && gy >= 0 && gy < H && gx >= 0 && gx < W;
        valid |= ok ? (1u << j) : 0u;
        const int gyc = min(max(gy, 0), H - 1), gxc = min(max(gx, 0), W - 1);
        const int64_t p = ((int64_t)n * H + gyc) * W + gxc;
        // only chunk 0 carries data: the other three lanes of a pixel load nothing
        r[j] = chunk == 0 ? make_uint4(__float_as_uint(phi[p]), (uint32_t)sampled[p], 0u, 0u)
                          : make_uint4(0u, 0u, 0u, 0u);
    }
}

__device__ __forceinline__ void enc_store_tile(bf16 *tile, const uint4 (&r)[C_PER_THREAD], uint32_t valid)
{
#pragma unroll
    for (int j = 0; j < C_PER_THREAD; ++j) {
        const int k = (int)threadIdx.x + 256 * j;
        if (k >= C_CHUNKS) continue;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (((valid >> j) & 1u) && r[j].y) {
            const float th = 0.5f * fabsf(__uint_as_float(r[j].x));
            bf16 e[8];
            e[0] = (bf16)cosf(th);
            e[1] = (bf16)sinf(th);
            e[2] = (bf16)1.0f;
#pragma unroll
            for (int i = 3; i < 8; ++i) e[i] = (bf16)0.0f;
            v = *reinterpret_cast<const uint4 *>(e);
        }
        *reinterpret_cast<uint4 *>(tile + (k >> 2) * PIXS + (k & 3) * 8) = v;
    }
}

// SIDE: bit 0 = the layer adds a residual input, bit 1 = its output is
// zeroed where a ReLU reference is <= 0 (the residual, else the reference,
// is loaded ahead; with both, the reference is read in the epilogue), bit 2
// = the network's stem (input encoded while staging), bit 3 = its head
// (output channels 0 and 1 decoded into starting gap angles, decode_kernel's
// arithmetic, instead of stored)
template <int SIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void conv3x3_kernel(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) bf16 tile[C_IN_T * PIXS];
    __shared__ __attribute__((aligned(16))) bf16 wl[C_W_ROWS * PIXS];
    __shared__ float bl[CH];
    const int tiles_x = (a.W + CTW - 1) / CTW, tiles_y = (a.H + CTH - 1) / CTH;
    const int n_tiles = tiles_x * tiles_y * a.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, kq = lane >> 5;
    for (int k = threadIdx.x; k < C_W_ROWS * 4; k += blockDim.x)
        *reinterpret_cast<uint4 *>(wl + (k >> 2) * PIXS + (k & 3) * 8) =
            *reinterpret_cast<const uint4 *>(a.w + (k >> 2) * CH + (k & 3) * 8);
    if (threadIdx.x < CH) bl[threadIdx.x] = a.bias ? a.bias[threadIdx.x] : 0.0f;
    uint4 pre[C_PER_THREAD];
    uint32_t pre_valid = 0u;
    int tile_id = blockIdx.x;
    if (tile_id < n_tiles) {
        int n, y0, x0;
        conv_tile_origin(tile_id, tiles_x, tiles_y, n, y0, x0);
        if (SIDE & 4) {
            enc_load_tile(a.phi, a.sampled, n, a.H, a.W, y0, x0, pre, pre_valid);
            enc_store_tile(tile, pre, pre_valid);
        } else {
            conv_load_tile(a.in, n, a.H, a.W, y0, x0, pre, pre_valid);
            conv_store_tile(tile, pre, pre_valid);
        }
    }
    __syncthreads();
    // Per tile: side loads, next tile's loads, products from LDS; barrier;
    // the next tile into LDS (its wait comes before this tile's stores, so
    // it never waits for them); epilogue; barrier.
    for (; tile_id < n_tiles; tile_id += gridDim.x) {
        int n, y0, x0;
        conv_tile_origin(tile_id, tiles_x, tiles_y, n, y0, x0);
        // D: lane holds pixel column m, channels 8 j + 4 kq + (0 .. 3) in acc[4 j .. 4 j + 3]
        const int gx = x0 + m;
        // the residual input (or the ReLU reference of a gradient) of the
        // tile's outputs, loaded ahead of the products
        uint2 addv[4][4];
        const bf16 *side = (SIDE & 1) ? a.add : a.ref;
        if (SIDE) {
            // outputs outside the image are never stored: their loads read a
            // clamped pixel instead of being selected away, so that no wait
            // for these loads (or the prefetch after them) is needed here
            const int gxc = min(gx, a.W - 1);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int gyc = min(y0 + 4 * wave + o, a.H - 1);
                const int64_t pix = ((int64_t)n * a.H + gyc) * a.W + gxc;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    addv[o][j] = *reinterpret_cast<const uint2 *>(side + pix * CH + 8 * j + 4 * kq);
            }
        }
        // the next tile's pixels, issued after the side loads (the wait
        // counter is in order) and unconditionally (a fixed count in flight;
        // a block's last tile re-reads itself)
        {
            const int next = tile_id + (int)gridDim.x < n_tiles ? tile_id + (int)gridDim.x : tile_id;
            int n2, y2, x2;
            conv_tile_origin(next, tiles_x, tiles_y, n2, y2, x2);
            if (SIDE & 4) enc_load_tile(a.phi, a.sampled, n2, a.H, a.W, y2, x2, pre, pre_valid);
            else conv_load_tile(a.in, n2, a.H, a.W, y2, x2, pre, pre_valid);
        }
        // keep the loads above ahead of the products (the scheduler would
        // otherwise sink them to their use and expose their latency)
        __builtin_amdgcn_sched_barrier(0);
        f32x16 acc[4];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[o][i] = 0.0f;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
            // the stem's encoded input has three nonzero channels: input
            // channels 16 .. 31 are zero, and their products (exact zeros
            // added to sums that start at +0) change nothing
#pragma unroll
            for (int kh = 0; kh < ((SIDE & 4) ? 1 : 2); ++kh) {
                // weights of taps (dy, dx - 1), dy = -1, 0, 1: out-channel m, in-channels kh*16 + kq*8 .. +7
                bf16x8 wa[3];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    wa[d] = *reinterpret_cast<const bf16x8 *>(wl + ((d * 3 + dx) * CH + m) * PIXS + kh * 16 + kq * 8);
                // staged row ir is input row 4 wave + ir - 1 of the tile
#pragma unroll
                for (int ir = 0; ir < 6; ++ir) {
                    const bf16x8 pb = *reinterpret_cast<const bf16x8 *>(
                        tile + ((4 * wave + ir) * C_IN_W + m + dx) * PIXS + kh * 16 + kq * 8);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const int o = ir - d;  // output row fed through tap dy = d - 1
                        if (o < 0 || o > 3) continue;
                        acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[d], pb, acc[o], 0, 0, 0);
                    }
                }
            }
        __syncthreads();  // every wave is done reading this tile from LDS
        if (tile_id + (int)gridDim.x < n_tiles) {
            if (SIDE & 4) enc_store_tile(tile, pre, pre_valid);
            else conv_store_tile(tile, pre, pre_valid);
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int gy = y0 + 4 * wave + o;
            if (gy >= a.H || gx >= a.W) continue;
            const int64_t pix = ((int64_t)n * a.H + gy) * a.W + gx;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c0 = 8 * j + 4 * kq;
                const int64_t idx = pix * CH + c0;
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = acc[o][4 * j + r] + bl[c0 + r];
                if (SIDE & 1) {
                    // bf16 -> float by bit position (keeps the loaded words whole until here)
                    const uint2 w2 = addv[o][j];
                    v[0] += __uint_as_float(w2.x << 16);
                    v[1] += __uint_as_float(w2.x & 0xFFFF0000u);
                    v[2] += __uint_as_float(w2.y << 16);
                    v[3] += __uint_as_float(w2.y & 0xFFFF0000u);
                }
                if (a.relu)
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.0f);
                if (SIDE & 2) {
                    // prefetched unless the layer also has a residual input
                    const uint2 rf = (SIDE & 1) ? *reinterpret_cast<const uint2 *>(a.ref + idx) : addv[o][j];
                    const float rv[4] = {__uint_as_float(rf.x << 16), __uint_as_float(rf.x & 0xFFFF0000u),
                                         __uint_as_float(rf.y << 16), __uint_as_float(rf.y & 0xFFFF0000u)};
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (!(rv[r] > 0.0f)) v[r] = 0.0f;
                }
                if (SIDE & 8) {
                    // channels 0 and 1 (lanes of kq = 0, run j = 0): the
                    // starting angle atan2(max(s, 0), c) / q below 2 pi, 0 at
                    // sampled pixels, from the bfloat16-rounded outputs
                    if (j == 0 && kq == 0) {
                        const float c = (float)(bf16)v[0], s = (float)(bf16)v[1];
                        const float th = atan2f(fmaxf(s, 0.0f) + 0.0f, c);
                        a.phi_out[pix] = a.sampled[pix] ? 0.0f : fminf(th / 0.5f, 6.28318501f);
                    }
                    continue;
                }
                uint2 ov;
                bf16 *op = reinterpret_cast<bf16 *>(&ov);
#pragma unroll
                for (int r = 0; r < 4; ++r) op[r] = (bf16)v[r];
                *reinterpret_cast<uint2 *>(a.out + idx) = ov;
            }
        }
        __syncthreads();  // the next tile is in LDS
    }
}

// A residual block of the inference forward pass in one kernel:
//   out = h + conv2(t) + b2,  t = bf16(ReLU(conv1(h) + b1))
// with the inner activation t kept on chip instead of a round trip through
// HBM.  Persistent blocks of 8 waves, one per CU, loop over 14 x 30-pixel
// output tiles; both layers' packed weights stay in LDS for the whole
// kernel.  The (14 + 4) x (30 + 4) input pixels around a tile are staged in
// LDS like conv3x3_kernel's tile (the same 18 x 34 shape), and conv1
// computes t on the 16 x 32 pixels around the output tile, each wave two
// rows (the MFMA scheme of conv3x3_kernel, whose products for one output
// row come in the same order), so two waves per SIMD hide each other's LDS
// latency.  Each lane then keeps the skip inputs of its conv2 outputs in
// registers, and t, rounded to bfloat16 as the layer-by-layer path stores
// it, overwrites the staged tile (zero outside the image, conv2's zero
// padding, and in the tile's last two rows and columns).  conv2 computes
// 16 x 32 outputs of which the first 14 x 30 are the tile's (the rest read
// the zero border); the next tile's pixels are loaded into registers while
// it runs, and its epilogue adds b2 and the skip input.  Every product and
// rounding is that of the two conv3x3_kernel launches, so the output is the
// same bits.  Tiles are ordered so that each XCD takes a contiguous run of
// them: tiles in flight on one XCD are neighbours and share their halo
// pixels in its L2.
constexpr int RTH = CTH - 2, RTW = CTW - 2;             // output tile of the fused block

struct ResArgs {
    const bf16 *in;    // block input h, N x H x W x 32
    const bf16 *w1;    // packed forward weights of the two convs
    const bf16 *w2;
    const float *b1;
    const float *b2;
    bf16 *out;
    int N, H, W;
};

__device__ __forceinline__ void res_tile_origin(int tile, int tiles_x, int tiles_y, int &n, int &y0, int &x0)
{
    const int tx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int ty = rest % tiles_y;
    n = rest / tiles_y;
    y0 = ty * RTH;
    x0 = tx * RTW;
}

constexpr int RES_NT = 512;                                          // threads of a residual-block block
constexpr int RES_PT = (C_CHUNKS + RES_NT - 1) / RES_NT;             // staged chunks per thread
constexpr int W_CHUNKS = C_W_ROWS * 4;                               // 16-byte chunks of one layer's weights

// One layer's packed weights into LDS rows of 80 B.
__device__ __forceinline__ void res_copy_w(const bf16 *__restrict__ w, bf16 *wl)
{
    for (int k = (int)threadIdx.x; k < W_CHUNKS; k += RES_NT)
        *reinterpret_cast<uint4 *>(wl + (k >> 2) * PIXS + (k & 3) * 8) =
            *reinterpret_cast<const uint4 *>(w + (k >> 2) * CH + (k & 3) * 8);
}

// conv_load_tile / conv_store_tile for 512-thread blocks.
__device__ __forceinline__ void res_load_tile(const bf16 *__restrict__ src, int n, int H, int W, int y0, int x0,
                                              uint4 (&r)[RES_PT], uint32_t &valid)
{
    valid = 0u;
#pragma unroll
    for (int j = 0; j < RES_PT; ++j) {
        const int k = min((int)threadIdx.x + RES_NT * j, C_CHUNKS - 1);
        const int chunk = k & 3, pix = k >> 2;
        const int rr = pix / C_IN_W, cc = pix - rr * C_IN_W;
        const int gy = y0 - 1 + rr, gx = x0 - 1 + cc;
        const bool ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
        valid |= ok ? (1u << j) : 0u;
        const int gyc = min(max(gy, 0), H - 1), gxc = min(max(gx, 0), W - 1);
        r[j] = *reinterpret_cast<const uint4 *>(src + (((int64_t)n * H + gyc) * W + gxc) * CH + chunk * 8);
    }
}

__device__ __forceinline__ void res_store_tile(bf16 *tile, const uint4 (&r)[RES_PT], uint32_t valid)
{
#pragma unroll
    for (int j = 0; j < RES_PT; ++j) {
        const int k = (int)threadIdx.x + RES_NT * j;
        if (k < C_CHUNKS)
            *reinterpret_cast<uint4 *>(tile + (k >> 2) * PIXS + (k & 3) * 8) =
                ((valid >> j) & 1u) ? r[j] : make_uint4(0u, 0u, 0u, 0u);
    }
}

// One convolution's products over a staged tile for wave w's output rows
// 2w and 2w + 1 (pixel column m = lane & 31, weights from LDS rows of
// 80 B): per output row the products of conv3x3_kernel in its order (column
// shift dx, channel chunk kh, row tap d).
__device__ __forceinline__ void res_products(const bf16 *tile, const bf16 *wl, int wave, int m, int kq,
                                             f32x16 (&acc)[2])
{
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[o][i] = 0.0f;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            bf16x8 wa[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                wa[d] = *reinterpret_cast<const bf16x8 *>(wl + ((d * 3 + dx) * CH + m) * PIXS + kh * 16 + kq * 8);
#pragma unroll
            for (int ir = 0; ir < 4; ++ir) {
                const bf16x8 pb = *reinterpret_cast<const bf16x8 *>(
                    tile + ((2 * wave + ir) * C_IN_W + m + dx) * PIXS + kh * 16 + kq * 8);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int o = ir - d;
                    if (o < 0 || o > 1) continue;
                    acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[d], pb, acc[o], 0, 0, 0);
                }
            }
        }
}

// res_products with the weight operands in registers: this lane's output
// channel m and input-channel half kq, per column shift dx, channel chunk
// kh and row tap d.
__device__ __forceinline__ void res_products_reg(const bf16 *tile, const bf16x8 (&wr)[3][2][3], int wave, int m,
                                                 int kq, f32x16 (&acc)[2])
{
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[o][i] = 0.0f;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int kh = 0; kh < 2; ++kh)
#pragma unroll
            for (int ir = 0; ir < 4; ++ir) {
                const bf16x8 pb = *reinterpret_cast<const bf16x8 *>(
                    tile + ((2 * wave + ir) * C_IN_W + m + dx) * PIXS + kh * 16 + kq * 8);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int o = ir - d;
                    if (o < 0 || o > 1) continue;
                    acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[dx][kh][d], pb, acc[o], 0, 0, 0);
                }
            }
}

__global__ __launch_bounds__(RES_NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void resblock_kernel(ResArgs a)
{
    __shared__ __attribute__((aligned(16))) bf16 tile[C_IN_T * PIXS];  // staged input, then t: 18 x 34 pixels
    __shared__ __attribute__((aligned(16))) bf16 wl1[C_W_ROWS * PIXS];  // conv1's packed weights
    __shared__ float bl[2 * CH];                                        // b1, b2
    const int tiles_x = (a.W + RTW - 1) / RTW, tiles_y = (a.H + RTH - 1) / RTH;
    const int n_tiles = tiles_x * tiles_y * a.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, kq = lane >> 5;
    if (threadIdx.x < CH) {
        bl[threadIdx.x] = a.b1[threadIdx.x];
        bl[CH + threadIdx.x] = a.b2[threadIdx.x];
    }
    // conv1's weights in LDS, conv2's weight operands in registers, for the whole kernel
    res_copy_w(a.w1, wl1);
    bf16x8 w2r[3][2][3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int kh = 0; kh < 2; ++kh)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                w2r[dx][kh][d] =
                    *reinterpret_cast<const bf16x8 *>(a.w2 + ((d * 3 + dx) * CH + m) * CH + kh * 16 + kq * 8);
    // this block's tiles: the blocks of XCD x = blockIdx % 8 (there are
    // ceil((G - x) / 8) of them) take a contiguous run of the tile sequence
    // in proportion to their number, in turn
    const int G = (int)gridDim.x, xcd = (int)blockIdx.x & 7;
    int before = 0;  // blocks on the XCDs below this one
    for (int x = 0; x < xcd; ++x) before += (G - x + 7) >> 3;
    const int nx8 = (G - xcd + 7) >> 3;  // blocks on this XCD (>= 1: this one)
    const int t_lo = (int)((int64_t)n_tiles * before / G), t_hi = (int)((int64_t)n_tiles * (before + nx8) / G);
    const int step = nx8;
    int tile_id = t_lo + ((int)blockIdx.x >> 3);
    uint4 pre[RES_PT];
    uint32_t pre_valid = 0u;
    if (tile_id < t_hi) {
        int n, y0, x0;
        res_tile_origin(tile_id, tiles_x, tiles_y, n, y0, x0);
        res_load_tile(a.in, n, a.H, a.W, y0 - 1, x0 - 1, pre, pre_valid);
        res_store_tile(tile, pre, pre_valid);
    }
    __syncthreads();
    for (; tile_id < t_hi; tile_id += step) {
        int n, y0, x0;
        res_tile_origin(tile_id, tiles_x, tiles_y, n, y0, x0);
        f32x16 acc[2];
        // conv1: t at rows y0 - 1 + 2 wave + o, columns x0 - 1 + m
        res_products(tile, wl1, wave, m, kq, acc);
        // the skip inputs of this lane's conv2 outputs (staged pixel
        // (2 wave + o + 2, m + 2)), read before t overwrites the tile
        uint2 skip[2][4];
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                skip[o][j] = *reinterpret_cast<const uint2 *>(
                    tile + (min(2 * wave + o + 2, CTH + 1) * C_IN_W + m + 2) * PIXS + 8 * j + 4 * kq);
        __syncthreads();  // every wave is done with the input tile
        {
            const int gx = x0 - 1 + m;
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const int tr = 2 * wave + o, gy = y0 - 1 + tr;
                const bool inside = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c0 = 8 * j + 4 * kq;
                    uint2 tv = make_uint2(0u, 0u);
                    if (inside) {
                        bf16 *tp = reinterpret_cast<bf16 *>(&tv);
#pragma unroll
                        for (int r = 0; r < 4; ++r) tp[r] = (bf16)fmaxf(acc[o][4 * j + r] + bl[c0 + r], 0.0f);
                    }
                    *reinterpret_cast<uint2 *>(tile + (tr * C_IN_W + m) * PIXS + c0) = tv;
                }
            }
            // the tile's last two rows and columns: zero
            for (int k = threadIdx.x; k < (2 * C_IN_W + 2 * CTH) * 4; k += RES_NT) {
                const int q = k >> 2, chunk = k & 3;
                const int pix = q < 2 * C_IN_W ? (CTH + q / C_IN_W) * C_IN_W + q % C_IN_W
                                               : ((q - 2 * C_IN_W) >> 1) * C_IN_W + CTW + ((q - 2 * C_IN_W) & 1);
                *reinterpret_cast<uint4 *>(tile + pix * PIXS + chunk * 8) = make_uint4(0u, 0u, 0u, 0u);
            }
        }
        __syncthreads();  // t is in LDS
        // the next tile's pixels, in flight during conv2 and the epilogue
        const bool more = tile_id + step < t_hi;
        if (more) {
            int n2, y2, x2;
            res_tile_origin(tile_id + step, tiles_x, tiles_y, n2, y2, x2);
            res_load_tile(a.in, n2, a.H, a.W, y2 - 1, x2 - 1, pre, pre_valid);
        }
        // conv2: outputs at rows y0 + 2 wave + o, columns x0 + m
        res_products_reg(tile, w2r, wave, m, kq, acc);
        {
            const int gx = x0 + m;
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const int orow = 2 * wave + o, gy = y0 + orow;
                if (orow >= RTH || m >= RTW || gy >= a.H || gx >= a.W) continue;
                const int64_t pix = ((int64_t)n * a.H + gy) * a.W + gx;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c0 = 8 * j + 4 * kq;
                    const uint2 w2 = skip[o][j];
                    float v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = acc[o][4 * j + r] + bl[CH + c0 + r];
                    v[0] += __uint_as_float(w2.x << 16);
                    v[1] += __uint_as_float(w2.x & 0xFFFF0000u);
                    v[2] += __uint_as_float(w2.y << 16);
                    v[3] += __uint_as_float(w2.y & 0xFFFF0000u);
                    uint2 ov;
                    bf16 *op = reinterpret_cast<bf16 *>(&ov);
#pragma unroll
                    for (int r = 0; r < 4; ++r) op[r] = (bf16)v[r];
                    *reinterpret_cast<uint2 *>(a.out + pix * CH + c0) = ov;
                }
            }
        }
        __syncthreads();  // every wave is done with t
        if (more) res_store_tile(tile, pre, pre_valid);
        __syncthreads();  // the next tile is in LDS
    }
}

struct WgradArgs {
    const bf16 *in;     // layer input, N x H x W x 32
    const bf16 *gout;   // output gradient, N x H x W x 32
    const bf16 *gref;   // multiply gout by (gref > 0), or null
    float *partial;     // [gridDim.x * 4][WG_PART]
    int N, H, W;
};

// Weight and bias gradients of one conv layer: dW[tap][ci][co] = sum over
// pixels of in(p + tap)[ci] * gout(p)[co]; db[co] = sum of gout(p)[co].
// Persistent blocks loop over output tiles; each wave accumulates its own
// partial sums, written out per wave and reduced in a fixed order.
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) bf16 itile[IN_T * PIXS];
    __shared__ __attribute__((aligned(16))) bf16 gtile[TH * TW * PIXS];
    const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + TH - 1) / TH;
    const int n_tiles = tiles_x * tiles_y * a.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, kq = lane >> 5;
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
    float db = 0.0f;
    for (int tile_id = blockIdx.x; tile_id < n_tiles; tile_id += gridDim.x) {
        int b = tile_id;
        const int tx = b % tiles_x;
        b /= tiles_x;
        const int ty = b % tiles_y;
        const int n = b / tiles_y;
        const int y0 = ty * TH, x0 = tx * TW;
        __syncthreads();
        stage_tile(a.in, itile, n, a.H, a.W, y0, x0, nullptr);
        for (int k = threadIdx.x; k < TH * TW * 4; k += blockDim.x) {
            const int chunk = k & 3, pix = k >> 2;
            const int r = pix / TW, c = pix - r * TW;
            const int gy = y0 + r, gx = x0 + c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (gy < a.H && gx < a.W) {
                const int64_t off = (((int64_t)n * a.H + gy) * a.W + gx) * CH + chunk * 8;
                v = *reinterpret_cast<const uint4 *>(a.gout + off);
                if (a.gref) {
                    const uint4 rv = *reinterpret_cast<const uint4 *>(a.gref + off);
                    const bf16 *rp = reinterpret_cast<const bf16 *>(&rv);
                    bf16 *vp = reinterpret_cast<bf16 *>(&v);
                    for (int j = 0; j < 8; ++j)
                        if (!((float)rp[j] > 0.0f)) vp[j] = (bf16)0.0f;
                }
            }
            *reinterpret_cast<uint4 *>(gtile + pix * PIXS + chunk * 8) = v;
        }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const int row = wave * 2 + mt;
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                // B[k = pixel][n = co]: lane holds co = m, pixels kc*16 + kq*8 .. +7 of this row
                bf16x8 bv;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bv[i] = gtile[(row * TW + kc * 16 + kq * 8 + i) * PIXS + m];
                    db += (float)bv[i];
                }
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int dy = t / 3 - 1, dx = t % 3 - 1;
                    // A[m = ci][k = pixel]: lane holds ci = m at the shifted pixels
                    bf16x8 av;
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        av[i] = itile[((row + 1 + dy) * (TW + 2) + kc * 16 + kq * 8 + i + 1 + dx) * PIXS + m];
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[t], 0, 0, 0);
                }
            }
        }
    }
    // D[m = ci][n = co]: lane holds co = m for ci = 8 (i/4) + 4 kq + (i%4)
    float *part = a.partial + (int64_t)(blockIdx.x * 4 + wave) * WG_PART;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int ci = 8 * (i >> 2) + 4 * kq + (i & 3);
            part[(t * CH + ci) * CH + m] = acc[t][i];
        }
    db += __shfl_xor(db, 32);
    if (kq == 0) part[WSZ + m] = db;
}

// grads[j] = sum over partials p of partial[p][j], in order.
__global__ void wgrad_reduce_kernel(const float *__restrict__ partial, int n_parts, float *__restrict__ grads)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= WG_PART) return;
    float s = 0.0f;
    for (int p = 0; p < n_parts; ++p) s += partial[(int64_t)p * WG_PART + j];
    grads[j] = s;
}

// Network input: (cos q phi, sin q phi, 1) at sampled sites, zeros elsewhere.
__global__ void encode_kernel(const float *__restrict__ phi, const uint8_t *__restrict__ sampled, int64_t npix,
                              float q, bf16 *__restrict__ x)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    bf16 v[CH];
    for (int c = 0; c < CH; ++c) v[c] = (bf16)0.0f;
    if (sampled[p]) {
        const float th = q * fabsf(phi[p]);
        v[0] = (bf16)cosf(th);
        v[1] = (bf16)sinf(th);
        v[2] = (bf16)1.0f;
    }
    uint4 *dst = reinterpret_cast<uint4 *>(x + p * CH);
    const uint4 *s = reinterpret_cast<const uint4 *>(v);
    for (int k = 0; k < 4; ++k) dst[k] = s[k];
}

// Head output -> starting gap angle: atan2(max(s, 0), c) / q, below 2 pi.
__global__ void decode_kernel(const bf16 *__restrict__ y, const uint8_t *__restrict__ sampled, int64_t npix, float q,
                              float *__restrict__ phi)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    if (sampled[p]) {
        phi[p] = 0.0f;
        return;
    }
    const float c = (float)y[p * CH], s = (float)y[p * CH + 1];
    // + 0.0f turns a -0.0 (which fmaxf may return) into +0.0: atan2(-0, c < 0)
    // would be -pi
    const float th = atan2f(fmaxf(s, 0.0f) + 0.0f, c);
    phi[p] = fminf(th / q, 6.28318501f);
}

// Masked squared error on channels 0, 1 and its gradient (bf16, all channels).
__global__ void loss_kernel(const bf16 *__restrict__ y, const float *__restrict__ target,
                            const uint8_t *__restrict__ sampled, int64_t npix, float inv_n, bf16 *__restrict__ dy,
                            double *__restrict__ partial)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (p < npix) {
        bf16 g[CH];
        for (int c = 0; c < CH; ++c) g[c] = (bf16)0.0f;
        if (!sampled[p]) {
            const float d0 = (float)y[p * CH] - target[2 * p];
            const float d1 = (float)y[p * CH + 1] - target[2 * p + 1];
            l = (double)d0 * d0 + (double)d1 * d1;
            g[0] = (bf16)(2.0f * d0 * inv_n);
            g[1] = (bf16)(2.0f * d1 * inv_n);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(dy + p * CH);
        const uint4 *s = reinterpret_cast<const uint4 *>(g);
        for (int k = 0; k < 4; ++k) dst[k] = s[k];
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// bfloat16 packs of every layer: forward [tap][co][ci] and dgrad [tap][ci][co] (flipped taps).
__global__ void pack_kernel(const float *__restrict__ params, bf16 *__restrict__ packed)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NLAYER * WSZ) return;
    const int layer = j / WSZ, r = j - layer * WSZ;
    const int t = r / (CH * CH), rem = r - t * CH * CH;
    const int o = rem / CH, i = rem - o * CH;
    const float *W = params + (int64_t)layer * LSZ;
    bf16 *F = packed + (int64_t)layer * 2 * WSZ;
    bf16 *D = F + WSZ;
    F[(t * CH + o) * CH + i] = (bf16)W[(t * CH + i) * CH + o];        // F[t][o][i] = W[t][i][o]
    D[(t * CH + o) * CH + i] = (bf16)W[((8 - t) * CH + o) * CH + i];  // D[t][ci=o][co=i] = W[8-t][o][i]
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ mo,
                            float *__restrict__ ve, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * mo[j] + (1.0f - b1) * gj;
    const float vj = b2 * ve[j] + (1.0f - b2) * gj * gj;
    mo[j] = mj;
    ve[j] = vj;
    p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

}  // namespace

// ===================================================================== host

int mpr_set_error(mpr_ctx *ctx, int code, const char *msg);  // defined with the context
// MPR_ERR_ARG unless every non-null pointer is device memory of the context's device
int mpr_check_device(mpr_ctx *ctx, const char *call,
                     std::initializer_list<std::pair<const char *, const void *>> ptrs);

namespace {

int cfail(mpr_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return mpr_set_error(ctx, code, buf);
}

#define CHIP(ctx, expr)                                                                                  \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return cfail((ctx), MPR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t act_bytes(int n, int h, int w) { return ((int64_t)n * h * w * CH * 2 + 255) / 256 * 256; }

bool shape_ok(int n, int h, int w) { return n >= 1 && h >= 1 && w >= 1 && (int64_t)n * h * w <= ((int64_t)1 << 31); }

int64_t conv_blocks(int n, int h, int w) { return (int64_t)n * ((h + TH - 1) / TH) * ((w + TW - 1) / TW); }

void launch_conv(hipStream_t st, const bf16 *in, const bf16 *wpack, const float *bias, const bf16 *add,
                 const bf16 *ref, int relu, bf16 *out, int n, int h, int w)
{
    ConvArgs a;
    a.in = in;
    a.w = wpack;
    a.bias = bias;
    a.add = add;
    a.ref = ref;
    a.out = out;
    a.N = n;
    a.H = h;
    a.W = w;
    a.relu = relu;
    // persistent: two blocks per compute unit (256 CUs), or one per tile if fewer
    const int64_t tiles = (int64_t)n * ((h + CTH - 1) / CTH) * ((w + CTW - 1) / CTW);
    const dim3 grid((unsigned)std::min<int64_t>(tiles, 512));
    switch ((add ? 1 : 0) | (ref ? 2 : 0)) {
        case 0: hipLaunchKernelGGL(conv3x3_kernel<0>, grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL(conv3x3_kernel<1>, grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL(conv3x3_kernel<2>, grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL(conv3x3_kernel<3>, grid, dim3(256), 0, st, a); break;
    }
}

// The network's stem with its input encoded from the sample angles while
// staging (SIDE 4), or its head with the output decoded into starting gap
// angles (SIDE 8).
void launch_conv_io(hipStream_t st, bool stem, const bf16 *in, const bf16 *wpack, const float *bias, bf16 *out,
                    const float *phi, const uint8_t *sampled, float *phi_out, int n, int h, int w)
{
    ConvArgs a;
    std::memset(&a, 0, sizeof a);
    a.in = in;
    a.w = wpack;
    a.bias = bias;
    a.out = out;
    a.N = n;
    a.H = h;
    a.W = w;
    a.relu = stem ? 1 : 0;
    a.phi = phi;
    a.sampled = sampled;
    a.phi_out = phi_out;
    const int64_t tiles = (int64_t)n * ((h + CTH - 1) / CTH) * ((w + CTW - 1) / CTW);
    const dim3 grid((unsigned)std::min<int64_t>(tiles, 512));
    if (stem) hipLaunchKernelGGL(conv3x3_kernel<4>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(conv3x3_kernel<8>, grid, dim3(256), 0, st, a);
}

void launch_resblock(hipStream_t st, const bf16 *in, const bf16 *w1, const float *b1, const bf16 *w2,
                     const float *b2, bf16 *out, int n, int h, int w)
{
    ResArgs a;
    a.in = in;
    a.w1 = w1;
    a.w2 = w2;
    a.b1 = b1;
    a.b2 = b2;
    a.out = out;
    a.N = n;
    a.H = h;
    a.W = w;
    // persistent: one 512-thread block per compute unit (95 KB of LDS)
    const int64_t tiles = (int64_t)n * ((h + RTH - 1) / RTH) * ((w + RTW - 1) / RTW);
    hipLaunchKernelGGL(resblock_kernel, dim3((unsigned)std::min<int64_t>(tiles, 256)), dim3(RES_NT), 0, st, a);
}

void launch_wgrad(hipStream_t st, const bf16 *in, const bf16 *gout, const bf16 *gref, float *partial, float *grads,
                  int n, int h, int w)
{
    WgradArgs a;
    a.in = in;
    a.gout = gout;
    a.gref = gref;
    a.partial = partial;
    a.N = n;
    a.H = h;
    a.W = w;
    const int blocks = (int)std::min<int64_t>(WG_BLOCKS, conv_blocks(n, h, w));
    hipLaunchKernelGGL(conv3x3_wgrad_kernel, dim3(blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((WG_PART + 255) / 256), dim3(256), 0, st, partial, blocks * 4,
                       grads);
}

// Activation buffers of a training forward pass inside the workspace.
struct Acts {
    bf16 *h[NBLK + 1];  // h[0] stem output, h[b+1] block b output
    bf16 *t[NBLK];      // block b inner activation
    bf16 *g0, *g1;      // backward scratch
    float *partial;
};

bool carve_acts(void *ws, int64_t ws_bytes, int n, int h, int w, bool training, Acts &A)
{
    char *p = (char *)ws;
    const int64_t ab = act_bytes(n, h, w);
    int64_t used = 0;
    auto take = [&](int64_t b) -> char * {
        if (used + b > ws_bytes) return nullptr;
        char *r = p + used;
        used += (b + 255) / 256 * 256;
        return r;
    };
    if (training) {
        for (int k = 0; k <= NBLK; ++k)
            if (!(A.h[k] = (bf16 *)take(ab))) return false;
        for (int k = 0; k < NBLK; ++k)
            if (!(A.t[k] = (bf16 *)take(ab))) return false;
        if (!(A.g0 = (bf16 *)take(ab)) || !(A.g1 = (bf16 *)take(ab))) return false;
        if (!(A.partial = (float *)take((int64_t)WG_BLOCKS * 4 * WG_PART * 4))) return false;
    } else {
        // inference: ping-pong h and one t
        bf16 *b0 = (bf16 *)take(ab), *b1 = (bf16 *)take(ab), *b2 = (bf16 *)take(ab);
        if (!b0 || !b1 || !b2) return false;
        for (int k = 0; k <= NBLK; ++k) A.h[k] = (k & 1) ? b1 : b0;
        for (int k = 0; k < NBLK; ++k) A.t[k] = b2;
        A.g0 = A.g1 = nullptr;
        A.partial = nullptr;
    }
    return true;
}

const bf16 *fwd_pack(const void *packed, int layer) { return (const bf16 *)packed + (int64_t)layer * 2 * WSZ; }
const bf16 *dgrad_pack(const void *packed, int layer) { return fwd_pack(packed, layer) + WSZ; }
const float *bias_of(const float *params, int layer) { return params + (int64_t)layer * LSZ + WSZ; }

}  // namespace

extern "C" {

int64_t mpr_cnn_param_count(void) { return (int64_t)NLAYER * LSZ; }

int64_t mpr_cnn_packed_bytes(void) { return (int64_t)NLAYER * 2 * WSZ * 2; }

int64_t mpr_cnn_workspace_size(int32_t n, int32_t h, int32_t w, int32_t training)
{
    if (!shape_ok(n, h, w)) return -1;
    const int64_t ab = act_bytes(n, h, w);
    if (training) return (2 * NBLK + 3) * ab + (int64_t)WG_BLOCKS * 4 * WG_PART * 4 + 4096;
    return 3 * ab + 4096;
}

int32_t mpr_cnn_pack(mpr_ctx *ctx, const float *params, void *packed, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!params || !packed) return cfail(ctx, MPR_ERR_ARG, "cnn_pack: null pointer");
    if (int rc = mpr_check_device(ctx, "cnn_pack", {{"params", params}, {"packed", packed}})) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(pack_kernel, dim3((NLAYER * WSZ + 255) / 256), dim3(256), 0, st, params, (bf16 *)packed);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_encode(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *phi, const uint8_t *sampled,
                       void *x, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !phi || !sampled || !x) return cfail(ctx, MPR_ERR_ARG, "cnn_encode: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_encode", {{"phi", phi}, {"sampled", sampled}, {"x", x}})) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = (int64_t)n * h * w;
    hipLaunchKernelGGL(encode_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, phi, sampled, np, 0.5f,
                       (bf16 *)x);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_forward(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params, const void *packed,
                        const void *x, void *ws, int64_t ws_bytes, int32_t training, void *y, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !params || !packed || !x || !ws || !y)
        return cfail(ctx, MPR_ERR_ARG, "cnn_forward: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_forward",
                                  {{"params", params}, {"packed", packed}, {"x", x}, {"workspace", ws}, {"y", y}}))
        return rc;
    if (ws_bytes < mpr_cnn_workspace_size(n, h, w, training))
        return cfail(ctx, MPR_ERR_WORKSPACE, "cnn_forward: workspace too small");
    Acts A;
    if (!carve_acts(ws, ws_bytes, n, h, w, training != 0, A)) return cfail(ctx, MPR_ERR_WORKSPACE, "workspace");
    hipStream_t st = (hipStream_t)stream;
    launch_conv(st, (const bf16 *)x, fwd_pack(packed, 0), bias_of(params, 0), nullptr, nullptr, 1, A.h[0], n, h, w);
    for (int b = 0; b < NBLK; ++b) {
        if (training) {  // the inner activations are kept for the backward pass
            launch_conv(st, A.h[b], fwd_pack(packed, 1 + 2 * b), bias_of(params, 1 + 2 * b), nullptr, nullptr, 1,
                        A.t[b], n, h, w);
            launch_conv(st, A.t[b], fwd_pack(packed, 2 + 2 * b), bias_of(params, 2 + 2 * b), A.h[b], nullptr, 0,
                        A.h[b + 1], n, h, w);
        } else {  // the same bits with the inner activation in LDS
            launch_resblock(st, A.h[b], fwd_pack(packed, 1 + 2 * b), bias_of(params, 1 + 2 * b),
                            fwd_pack(packed, 2 + 2 * b), bias_of(params, 2 + 2 * b), A.h[b + 1], n, h, w);
        }
    }
    launch_conv(st, A.h[NBLK], fwd_pack(packed, NLAYER - 1), bias_of(params, NLAYER - 1), nullptr, nullptr, 0,
                (bf16 *)y, n, h, w);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_infer(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params, const void *packed,
                      const float *phi, const uint8_t *sampled, void *ws, int64_t ws_bytes, float *phi_init,
                      void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !params || !packed || !phi || !sampled || !ws || !phi_init)
        return cfail(ctx, MPR_ERR_ARG, "cnn_infer: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_infer",
                                  {{"params", params}, {"packed", packed}, {"phi", phi}, {"sampled", sampled},
                                   {"workspace", ws}, {"phi_init", phi_init}}))
        return rc;
    if (ws_bytes < mpr_cnn_workspace_size(n, h, w, 0))
        return cfail(ctx, MPR_ERR_WORKSPACE, "cnn_infer: workspace too small");
    Acts A;
    if (!carve_acts(ws, ws_bytes, n, h, w, false, A)) return cfail(ctx, MPR_ERR_WORKSPACE, "workspace");
    hipStream_t st = (hipStream_t)stream;
    launch_conv_io(st, true, nullptr, fwd_pack(packed, 0), bias_of(params, 0), A.h[0], phi, sampled, nullptr, n, h,
                   w);
    for (int b = 0; b < NBLK; ++b)
        launch_resblock(st, A.h[b], fwd_pack(packed, 1 + 2 * b), bias_of(params, 1 + 2 * b),
                        fwd_pack(packed, 2 + 2 * b), bias_of(params, 2 + 2 * b), A.h[b + 1], n, h, w);
    launch_conv_io(st, false, A.h[NBLK], fwd_pack(packed, NLAYER - 1), bias_of(params, NLAYER - 1), nullptr,
                   nullptr, sampled, phi_init, n, h, w);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_loss(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *y, const float *target,
                     const uint8_t *sampled, int64_t n_gaps, void *dy, void *ws, int64_t ws_bytes, double *loss,
                     void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !y || !target || !sampled || !dy || !loss || !ws || n_gaps < 0)
        return cfail(ctx, MPR_ERR_ARG, "cnn_loss: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_loss",
                                  {{"y", y}, {"target", target}, {"sampled", sampled}, {"dy", dy}, {"workspace", ws}}))
        return rc;
    const int64_t np = (int64_t)n * h * w;
    const unsigned blocks = (unsigned)((np + 255) / 256);
    if (ws_bytes < (int64_t)blocks * 8) return cfail(ctx, MPR_ERR_WORKSPACE, "cnn_loss: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    double *partial = (double *)ws;
    hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, st, (const bf16 *)y, target, sampled, np,
                       n_gaps > 0 ? 1.0f / (float)n_gaps : 0.0f, (bf16 *)dy, partial);
    CHIP(ctx, hipGetLastError());
    std::vector<double> hp(blocks);
    CHIP(ctx, hipMemcpyAsync(hp.data(), partial, blocks * sizeof(double), hipMemcpyDeviceToHost, st));
    CHIP(ctx, hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : hp) s += v;
    *loss = n_gaps > 0 ? s / (double)n_gaps : 0.0;
    return MPR_OK;
}

int32_t mpr_cnn_backward(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *params, const void *packed,
                         const void *x, const void *dy, void *ws, int64_t ws_bytes, float *grads, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !params || !packed || !x || !dy || !ws || !grads)
        return cfail(ctx, MPR_ERR_ARG, "cnn_backward: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_backward",
                                  {{"params", params}, {"packed", packed}, {"x", x}, {"dy", dy}, {"workspace", ws},
                                   {"grads", grads}}))
        return rc;
    if (ws_bytes < mpr_cnn_workspace_size(n, h, w, 1))
        return cfail(ctx, MPR_ERR_WORKSPACE, "cnn_backward: workspace too small");
    Acts A;
    if (!carve_acts(ws, ws_bytes, n, h, w, true, A)) return cfail(ctx, MPR_ERR_WORKSPACE, "workspace");
    hipStream_t st = (hipStream_t)stream;
    const bf16 *g = (const bf16 *)dy;
    float *G = grads;
    // head
    launch_wgrad(st, A.h[NBLK], g, nullptr, A.partial, G + (int64_t)(NLAYER - 1) * LSZ, n, h, w);
    bf16 *dh = A.g0, *dt = A.g1;
    launch_conv(st, g, dgrad_pack(packed, NLAYER - 1), nullptr, nullptr, nullptr, 0, dh, n, h, w);
    for (int b = NBLK - 1; b >= 0; --b) {
        const int l2 = 2 + 2 * b, l1 = 1 + 2 * b;
        launch_wgrad(st, A.t[b], dh, nullptr, A.partial, G + (int64_t)l2 * LSZ, n, h, w);
        launch_conv(st, dh, dgrad_pack(packed, l2), nullptr, nullptr, A.t[b], 0, dt, n, h, w);
        launch_wgrad(st, A.h[b], dt, nullptr, A.partial, G + (int64_t)l1 * LSZ, n, h, w);
        // dh <- dh + dgrad(dt) (in place: each output reads only its own dh entry)
        launch_conv(st, dt, dgrad_pack(packed, l1), nullptr, dh, nullptr, 0, dh, n, h, w);
    }
    // stem: gradient through its ReLU applied while staging
    launch_wgrad(st, (const bf16 *)x, dh, A.h[0], A.partial, G, n, h, w);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_opt_step(mpr_ctx *ctx, float *params, const float *grads, float *m, float *v, int64_t step,
                         double lr, double beta1, double beta2, double eps, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!params || !grads || !m || !v || step < 1) return cfail(ctx, MPR_ERR_ARG, "cnn_opt_step: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_opt_step", {{"params", params}, {"grads", grads}, {"m", m}, {"v", v}}))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = mpr_cnn_param_count();
    const float c1 = (float)(1.0 - std::pow(beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow(beta2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, grads, m, v, n,
                       (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_decode(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *y, const uint8_t *sampled,
                       float *phi_init, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !y || !sampled || !phi_init) return cfail(ctx, MPR_ERR_ARG, "cnn_decode: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_decode", {{"y", y}, {"sampled", sampled}, {"phi_init", phi_init}}))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = (int64_t)n * h * w;
    hipLaunchKernelGGL(decode_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, (const bf16 *)y, sampled,
                       np, 0.5f, phi_init);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_diag_conv(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *in, const void *wpack,
                          const float *bias, const void *add, const void *ref, int32_t relu, void *out, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !in || !wpack || !out) return cfail(ctx, MPR_ERR_ARG, "cnn_diag_conv: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_diag_conv",
                                  {{"in", in}, {"wpack", wpack}, {"bias", bias}, {"add", add}, {"ref", ref}, {"out", out}}))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    launch_conv(st, (const bf16 *)in, (const bf16 *)wpack, bias, (const bf16 *)add, (const bf16 *)ref, relu,
                (bf16 *)out, n, h, w);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

int32_t mpr_cnn_diag_wgrad(mpr_ctx *ctx, int32_t n, int32_t h, int32_t w, const void *in, const void *gout,
                           const void *gref, float *grads, void *ws, int64_t ws_bytes, void *stream)
{
    if (!ctx) return MPR_ERR_ARG;
    if (!shape_ok(n, h, w) || !in || !gout || !grads || !ws) return cfail(ctx, MPR_ERR_ARG, "cnn_diag_wgrad: invalid argument");
    if (int rc = mpr_check_device(ctx, "cnn_diag_wgrad",
                                  {{"in", in}, {"gout", gout}, {"gref", gref}, {"grads", grads}, {"workspace", ws}}))
        return rc;
    if (ws_bytes < (int64_t)WG_BLOCKS * 4 * WG_PART * 4) return cfail(ctx, MPR_ERR_WORKSPACE, "cnn_diag_wgrad: workspace");
    hipStream_t st = (hipStream_t)stream;
    launch_wgrad(st, (const bf16 *)in, (const bf16 *)gout, (const bf16 *)gref, (float *)ws, grads, n, h, w);
    CHIP(ctx, hipGetLastError());
    CHIP(ctx, hipStreamSynchronize(st));
    return MPR_OK;
}

}  // extern "C"
