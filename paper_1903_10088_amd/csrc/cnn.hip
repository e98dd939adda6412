// Learned warm start: residual CNN inference and training kernels for gfx950.
//
// Layout: hidden activations and backward signals are bfloat16, channels last
// ([batch][row][col][32], 64 bytes per pixel), so one 16-byte load holds 8
// channels of a pixel.  The 32 -> 32 convolutions (forward, and the input
// gradient "dgrad", which is the same convolution with flipped taps and
// transposed channel blocks) run on the matrix cores as implicit GEMMs:
//   D[out channel][pixel] += W_tap[out][in] x A_shifted[in][pixel]
// with v_mfma_f32_16x16x32_bf16 (M = 16 output channels, N = 16 pixels of a
// tile row, K = the 32 input channels of one tap).  A 16x16-pixel output tile
// and its one-pixel halo are staged in LDS (80-byte pixel stride: the 16-byte
// reads of 16 lanes hit distinct banks); each wave keeps all 9 x 2 weight
// fragments in registers and computes 4 output rows, so each staged input
// fragment feeds up to 3 output rows.
//
// The weight gradient of a 32 -> 32 layer is a GEMM over pixels:
//   dW_tap[out][in] = sum_p G[out][p] x A[in][p + tap]
// also on the matrix cores, with K = 32 pixels per instruction.  Its operands
// must hold 8 consecutive pixels of one channel per lane: the tiles stay
// channels-last in LDS and the LDS transpose read (ds_read_b64_tr_b16) hands
// each lane its channel of 4 pixels.  Blocks loop over a fixed set of tiles
// and write partial sums; a second kernel adds the partials in a fixed order,
// so gradients are bitwise deterministic.
//
// The 1 -> 32 and 32 -> 1 layers (0.6% of the work) run in float32 on the
// vector ALUs.  None of the path uses atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gather.h"
#include "internal.h"
#include "recon_cnn.h"

using namespace recon;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int C = 32;           // hidden channels
constexpr int T = 16;           // output tile edge
constexpr int HALO = T + 2;     // staged tile edge
constexpr int LDS_PIX = 40;     // bf16 per staged pixel (32 + 8 pad)
constexpr int NHID = 6;         // 32 -> 32 layers (layers 2..7)
constexpr int W32 = 9 * C * C;  // weights of one 32 -> 32 layer
constexpr int P32 = W32 + C;    // weights + bias of one 32 -> 32 layer
// offsets of the parameter vector
constexpr int OFF_W1 = 0, OFF_B1 = 288;
constexpr int OFF_HID = 320;  // layer 2 starts here; layer l (2..7) at OFF_HID + (l - 2) * P32
constexpr int OFF_W8 = OFF_HID + NHID * P32, OFF_B8 = OFF_W8 + 288;
constexpr int NPARAM = OFF_B8 + 1;
static_assert(NPARAM == 56097, "parameter count");
constexpr int WG_BLOCKS = 512;  // blocks of the weight-gradient kernels (fixed: fixes the summation order)
constexpr int P_IN = 320;       // partial row of the first layer (288 weights + 32 biases)
constexpr int P_OUT = 289;      // partial row of the last layer

// Adam constants; 1 - beta is given directly (1.0f - 0.999f is 4.7e-5 off in float32)
constexpr float kB1 = 0.9f, kB2 = 0.999f, kOneMinusB1 = 0.1f, kOneMinusB2 = 0.001f, kEps = 1e-8f;

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

__device__ __forceinline__ uint32_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ bf16x8 as_bf8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
// Makes the compiler wait here for the load that produced v: an empty asm that reads it.  Called
// on a persistent kernel's weights before its tile loop, so that no wait for them is left inside
// the loop (where the in-order load/store counter would also wait for the tile prefetches).
template <class V>
__device__ __forceinline__ void settle(const V& v)
{
    asm volatile("" ::"v"(v));
}
// two floats -> packed bf16 pair (lo, hi), rounded to nearest even by the conversion instruction
__device__ __forceinline__ uint32_t pack_bf2(float lo, float hi)
{
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}
// max(x, 0) of both halves of a bf16 pair: a bf16 is negative exactly when it is negative as an
// int16, so one packed integer max does it (negative values and -0 become +0)
__device__ __forceinline__ uint32_t relu_bf2(uint32_t v)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{0, 0}));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Block index -> tile, XCD-aware: the dispatcher sends block b to XCD b mod 8;
// tile order is remapped so every XCD works on one contiguous run of tiles
// (neighbouring tiles share halos in that XCD's L2).
struct Tile {
    int b, i0, j0;  // image, first row, first column
};
__device__ __forceinline__ Tile tile_of(int bid, int nblocks, int tiles_x, int tiles_per_img)
{
    const int x = bid & 7, k = bid >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    const int t = x * q + min(x, r) + k;
    const int b = t / tiles_per_img;
    const int rem = t - b * tiles_per_img;
    const int ty = rem / tiles_x;
    return Tile{b, ty * T, (rem - ty * tiles_x) * T};
}
__device__ __forceinline__ Tile tile_plain(int t, int tiles_x, int tiles_per_img)
{
    const int b = t / tiles_per_img;
    const int rem = t - b * tiles_per_img;
    const int ty = rem / tiles_x;
    return Tile{b, ty * T, (rem - ty * tiles_x) * T};
}

__device__ __forceinline__ size_t pix(int b, int i, int j, int n) { return ((size_t)b * n + i) * n + j; }

// Stages the (T+2)^2 halo tile of a channels-last bf16 tensor into LDS (zeros
// outside the image); called by all NT threads of a block.  halo_issue starts
// a thread's loads (pixels outside the image load the tensor's first element
// and keep a cleared bit in `in`), halo_store waits for them and writes LDS,
// so a caller can keep the loads in flight while it works on another tile.
//
// Chunk slot e (thread e mod NT, step e / NT) holds 16-byte part (e / 16) mod 4
// of staged pixel 16 (e / 64) + e mod 16: the 16 lanes of a quarter-wave take
// one part of 16 consecutive pixels, the pattern of the matrix-operand reads
// (fewer LDS bank conflicts at the 80-byte pixel stride than four parts of four
// pixels), while each wave instruction still covers 16 whole pixels of global
// memory.
constexpr int HALO_GROUPS = (HALO * HALO + 15) / 16;  // 16-pixel groups of the halo tile
template <int NT>
struct HaloRegs {
    static constexpr int PER = (HALO_GROUPS * 64 + NT - 1) / NT;  // chunks per thread
    u32x4 v[PER];
    uint32_t in;  // bit k: chunk k lies in the image
};
template <int NT>
__device__ __forceinline__ int halo_pixel(int tid, int k)
{
    const int e = tid + NT * k;
    return 16 * (e >> 6) + (e & 15);
}
template <int NT>
__device__ __forceinline__ void halo_issue(HaloRegs<NT>& h, const uint16_t* __restrict__ act, Tile t, int n)
{
    // the chunk coordinates are recomputed on every call (an empty asm hides that the thread
    // index is loop-invariant): kept live across a persistent kernel's tile loop they would
    // take a dozen registers
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    h.in = 0u;
#pragma unroll
    for (int k = 0; k < HaloRegs<NT>::PER; ++k) {
        const int p = halo_pixel<NT>(tid, k), q = (tid >> 4) & 3;
        const int ly = p / HALO, lx = p - ly * HALO;
        const int gi = t.i0 + ly - 1, gj = t.j0 + lx - 1;
        const bool in = p < HALO * HALO && gi >= 0 && gi < n && gj >= 0 && gj < n;
        h.in |= in ? 1u << k : 0u;
        const size_t off = in ? pix(t.b, gi, gj, n) * C + q * 8 : 0;
        h.v[k] = *(const u32x4*)(act + off);
    }
}
template <int NT>
__device__ __forceinline__ void halo_store(uint16_t (*s)[HALO][LDS_PIX], const HaloRegs<NT>& h)
{
    // slots past the last pixel store into the unused padding of pixel (0, 0) instead of branching,
    // which lets the compiler wait for each prefetched chunk exactly
    const int tid = (int)threadIdx.x;
    uint16_t* base = &s[0][0][0] + halo_pixel<NT>(tid, 0) * LDS_PIX + ((tid >> 4) & 3) * 8;
#pragma unroll
    for (int k = 0; k < HaloRegs<NT>::PER; ++k) {
        // every slot of step k is a real pixel when the step's last group ends inside the tile
        const bool real = 16 * ((NT * (k + 1) - 1) >> 6) + 15 < HALO * HALO || halo_pixel<NT>(tid, k) < HALO * HALO;
        uint16_t* dst = real ? base + 16 * (NT / 64) * k * LDS_PIX : &s[0][0][C];
        *(u32x4*)dst = (h.in >> k) & 1u ? h.v[k] : u32x4{0u, 0u, 0u, 0u};
    }
}
static_assert(LDS_PIX >= C + 8, "the halo store's spare slot lies in a staged pixel's padding");

// Writes the 64-byte channel rows of the block's 256 consecutive pixels (pixel
// first + threadIdx.x holds words w) so that every store instruction of a wave
// covers 1 KB of contiguous memory: the rows pass through LDS (80-byte stride)
// and wave v then writes pixels v*64 + q*16 .. +15, lane l taking 16-byte part
// l / 16 of pixel l mod 16 (the halo tile's lane pattern).
// Called by all 256 threads; pixels at or beyond `total` are not written.
constexpr int ROW_STAGE_WORDS = 256 * 5;
__device__ __forceinline__ void store_pixel_rows(u32x4* __restrict__ stage, const u32x4 (&w)[4],
                                                 uint16_t* __restrict__ dst, long first, long total)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) stage[threadIdx.x * 5 + q] = w[q];
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int px = wv * 64 + q * 16 + (l & 15), part = l >> 4;
        if (first + px < total) ((u32x4*)dst)[(first + px) * 4 + part] = stage[px * 5 + part];
    }
}

// ----------------------------------------------------------------------------
// Weight preparation: float32 master -> bfloat16 copies in kernel layouts
// ----------------------------------------------------------------------------

// wf[l][tap][o][c] = bf(W[o][c][tap]); wt[l][tap][c][o] = bf(W[o][c][8 - tap])
// (the dgrad convolution); w8r[c][tap] = bf(W8) as float;
// w1a[o][k] = bf(W1[o][tap k]) for k < 9, 0 for k = 9..31 (the first layer's
// matrix-core operand: K = the 9 taps, padded);
// w8a[m][c] = bf(W8[c][tap m]) for m < 9, 0 for m = 9..15 (the last layer's
// matrix-core operand: 16 rows, 9 of them taps).
constexpr int PREP_W8R = NHID * W32, PREP_W1A = PREP_W8R + 288, PREP_W8A = PREP_W1A + C * C,
              PREP_END = PREP_W8A + 16 * C;
__global__ __launch_bounds__(256) void prep_weights_kernel(const float* __restrict__ th, uint16_t* __restrict__ wf,
                                                           uint16_t* __restrict__ wt, float* __restrict__ w8r,
                                                           uint16_t* __restrict__ w1a, uint16_t* __restrict__ w8a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < PREP_W8R) {
        const int l = k / W32, r = k - l * W32;
        const int tap = r / (C * C), oc = r - tap * C * C;
        const int a = oc / C, bq = oc - a * C;  // wf: a = o, bq = c; wt: a = c, bq = o
        const float* W = th + OFF_HID + l * P32;
        wf[k] = (uint16_t)f2bf(W[(a * C + bq) * 9 + tap]);
        wt[k] = (uint16_t)f2bf(W[(bq * C + a) * 9 + (8 - tap)]);
    } else if (k < PREP_W1A) {
        const int r = k - PREP_W8R;  // c * 9 + tap
        w8r[r] = bfround(th[OFF_W8 + r]);
    } else if (k < PREP_W8A) {
        const int r = k - PREP_W1A;  // o * 32 + k
        const int o = r / C, q = r - o * C;
        w1a[r] = q < 9 ? (uint16_t)f2bf(th[OFF_W1 + o * 9 + q]) : (uint16_t)0;
    } else if (k < PREP_END) {
        const int r = k - PREP_W8A;  // m * 32 + c
        const int m = r / C, c = r - m * C;
        w8a[r] = m < 9 ? (uint16_t)f2bf(th[OFF_W8 + c * 9 + m]) : (uint16_t)0;
    }
}

// ----------------------------------------------------------------------------
// Forward
// ----------------------------------------------------------------------------

// Layer 1 (1 -> 32): a0 = bf(mu / scale), a1 = bf(relu(b1 + sum_tap w1 a0)) on
// the matrix cores: per 16 pixels of a tile row and 16 output channels, one
// 16 x 16 x 32 product with K = the 9 taps (padded with zeros), A = the weights
// (w1a), B = lane (m, g) holding taps 8g .. 8g+7 of pixel m, formed from the
// tile's a0 halo staged in LDS; accumulators start at the bias.  The outputs
// are staged in LDS and written one contiguous 1 KB row per store instruction.
// Persistent over the XCD-aware tile order; the next tile's mu halo is loaded
// while the current tile is computed.
constexpr int IN_GRID = 256 * 4;  // blocks resident at once, a multiple of 8
struct InHalo {
    float v[2];   // mu at halo pixels threadIdx.x and threadIdx.x + 256
    uint32_t in;  // bit k: halo pixel k lies in the image (else it counts as 0)
};
__device__ __forceinline__ void in_issue(InHalo& h, const float* __restrict__ mu, Tile t, int n)
{
    h.in = 0u;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        const int ly = e / HALO, lx = e - ly * HALO;
        const int gi = t.i0 + ly - 1, gj = t.j0 + lx - 1;
        const bool in = e < HALO * HALO && gi >= 0 && gi < n && gj >= 0 && gj < n;
        h.in |= in ? 1u << k : 0u;
        h.v[k] = mu[in ? pix(t.b, gi, gj, n) : 0];  // (masked where it is stored, so the load stays in flight)
    }
}
__global__ __launch_bounds__(256) void conv_in_kernel(const float* __restrict__ mu, float inv_scale,
                                                      const uint16_t* __restrict__ w1a, const float* __restrict__ b1,
                                                      uint16_t* __restrict__ a0, uint16_t* __restrict__ a1, int n,
                                                      int tiles_x, int tiles_per_img, int nblocks)
{
    __shared__ float xs[HALO][HALO + 1];                                 // bf(mu / scale) as float
    __shared__ __attribute__((aligned(16))) uint16_t o[T * T * LDS_PIX];  // staged outputs, 80-byte pixel stride
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    // A operands: lane (m, g) holds W1[hh*16 + m][taps 8g .. 8g+7]
    bf16x8 A[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) A[hh] = as_bf8(*(const u32x4*)(w1a + (hh * 16 + m) * C + g * 8));
    f32x4 bias[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[hh][i] = b1[hh * 16 + 4 * g + i];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        settle(A[hh]);
        settle(bias[hh]);
    }
    InHalo h;
    if ((int)blockIdx.x < nblocks) in_issue(h, mu, tile_of(blockIdx.x, nblocks, tiles_x, tiles_per_img), n);
    for (int v = blockIdx.x; v < nblocks; v += gridDim.x) {
        const Tile tl = tile_of(v, nblocks, tiles_x, tiles_per_img);
        if (v != (int)blockIdx.x) __syncthreads();  // the previous tile's reads of xs and o are done
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = (int)threadIdx.x + 256 * k;
            // lanes past the halo store into the spare column of row 0 instead of branching
            float* dst = e < HALO * HALO ? &xs[e / HALO][e % HALO] : &xs[0][HALO];
            *dst = (h.in >> k) & 1u ? bfround(h.v[k] * inv_scale) : 0.0f;
        }
        __syncthreads();
        if (v + (int)gridDim.x < nblocks) in_issue(h, mu, tile_of(v + gridDim.x, nblocks, tiles_x, tiles_per_img), n);
        {
            // a0: this thread's pixel of the tile (the halo centre)
            const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
            const int i = tl.i0 + ty, j = tl.j0 + tx;
            if (i < n && j < n) a0[pix(tl.b, i, j, n)] = (uint16_t)f2bf(xs[ty + 1][tx + 1]);
        }
        // tile rows r = wave, wave + 4, ...: B operand of pixel (r, m)
#pragma unroll
        for (int k = 0; k < T / 4; ++k) {
            const int r = wave + 4 * k;
            uint32_t bw[4] = {0u, 0u, 0u, 0u};
            if (g == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t0 = 2 * q, t1 = 2 * q + 1;
                    bw[q] = pack_bf2(xs[r + t0 / 3][m + t0 % 3], xs[r + t1 / 3][m + t1 % 3]);
                }
            } else if (g == 1) {
                bw[0] = pack_bf2(xs[r + 2][m + 2], 0.0f);
            }
            const bf16x8 B = as_bf8(u32x4{bw[0], bw[1], bw[2], bw[3]});
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const f32x4 d = mfma(A[hh], B, bias[hh]);
                // D[4g + i][m]: channel hh*16 + 4g + i of pixel (r, m)
                *(u32x2*)(o + (r * T + m) * LDS_PIX + hh * 16 + 4 * g) =
                    u32x2{relu_bf2(pack_bf2(d[0], d[1])), relu_bf2(pack_bf2(d[2], d[3]))};
            }
        }
        __syncthreads();
        // out: wave w writes rows 4w .. 4w+3, one contiguous 1 KB row per instruction
        const int px = lane & 15, c4 = lane >> 4;  // the halo tile's lane pattern
        const int gj = tl.j0 + px;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = wave * 4 + k, gi = tl.i0 + r;
            if (gi < n && gj < n)
                *(u32x4*)(a1 + pix(tl.b, gi, gj, n) * C + c4 * 8) = *(const u32x4*)(o + (r * T + px) * LDS_PIX + c4 * 8);
        }
    }
}

// Matrix products of one 16x16 output tile of the 32 -> 32 convolution from its
// halo staged in LDS.  Wave w computes output channels hh*16 .. hh*16+15 (hh =
// w mod 2) of the 8 output rows r0 .. r0+7 (r0 = 8 (w / 2)), reading staged rows
// r0 .. r0+9; each staged fragment feeds up to 3 output rows.  Every output sums
// its taps in the order (ky, kx) = (0,0), (0,1), ..., (2,2).
__device__ __forceinline__ void conv32_mma(const uint16_t (*s)[HALO][LDS_PIX], const bf16x8 (&A)[9],
                                           f32x4 (&acc)[8], int wave, int m, int g)
{
    const int r0 = (wave >> 1) * 8;
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int R = 0; R < 10; ++R)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            // B operand: lane (m, g) holds channels 8g .. 8g+7 of staged pixel (r0 + R, m + kx)
            const bf16x8 Bf = as_bf8(*(const u32x4*)(&s[r0 + R][m + kx][g * 8]));
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
                const int ky = R - rr;
                if (ky >= 0 && ky < 3) acc[rr] = mfma(A[ky * 3 + kx], Bf, acc[rr]);
            }
        }
}

// The tile's outputs as bf16 into the LDS tile o (pixel (r, c) at (r T + c)
// LDS_PIX): the forward adds the bias and applies the ReLU, dgrad stores the
// unmasked sums (its mask is applied on the way out).  D[4g + i][m] of row rr
// is output channel hh*16 + 4g + i of pixel column m.
template <int MODE>
__device__ __forceinline__ void conv32_stage(uint16_t* __restrict__ o, const f32x4 (&acc)[8],
                                             const float* __restrict__ bias, int wave, int m, int g)
{
    const int hh = wave & 1, r0 = (wave >> 1) * 8;
    const int o0 = hh * 16 + g * 4;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        u32x2 w;
        if constexpr (MODE == 0) {
            w = u32x2{relu_bf2(pack_bf2(acc[rr][0] + bias[o0], acc[rr][1] + bias[o0 + 1])),
                      relu_bf2(pack_bf2(acc[rr][2] + bias[o0 + 2], acc[rr][3] + bias[o0 + 3]))};
        } else {
            w = u32x2{pack_bf2(acc[rr][0], acc[rr][1]), pack_bf2(acc[rr][2], acc[rr][3])};
        }
        *(u32x2*)(o + ((r0 + rr) * T + m) * LDS_PIX + o0) = w;
    }
}

// Keeps each bf16 half of v where the same half of mk is positive (a bf16 is
// positive exactly when it is positive as an int16), zero elsewhere.
__device__ __forceinline__ uint32_t mask_bf2(uint32_t v, uint32_t mk)
{
    const uint32_t keep = ((int16_t)(mk & 0xffffu) > 0 ? 0x0000ffffu : 0u) | ((int16_t)(mk >> 16) > 0 ? 0xffff0000u : 0u);
    return v & keep;
}

// Copies the staged tile to the output: wave w writes rows 4w .. 4w+3, one
// contiguous 1 KB row (16 pixels x 64 bytes) per instruction; dgrad zeroes the
// channels whose forward activation (mask) is not positive, reading the mask
// the same way.
template <int MODE>
__device__ __forceinline__ void conv32_copy_out(const uint16_t* __restrict__ o, const uint16_t* __restrict__ mask,
                                                uint16_t* __restrict__ out, int n, Tile tl, int wave, int lane)
{
    const int px = lane & 15, c4 = lane >> 4;  // the halo tile's lane pattern
    const int gj = tl.j0 + px;
    u32x4 mk[4];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int gi = tl.i0 + wave * 4 + k;
            const size_t off = (gi < n && gj < n) ? pix(tl.b, gi, gj, n) * C + c4 * 8 : 0;
            mk[k] = *(const u32x4*)(mask + off);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = wave * 4 + k, gi = tl.i0 + r;
        if (gi >= n || gj >= n) continue;
        u32x4 v = *(const u32x4*)(o + (r * T + px) * LDS_PIX + c4 * 8);
        if constexpr (MODE == 1)
            v = u32x4{mask_bf2(v.x, mk[k].x), mask_bf2(v.y, mk[k].y), mask_bf2(v.z, mk[k].z), mask_bf2(v.w, mk[k].w)};
        *(u32x4*)(out + pix(tl.b, gi, gj, n) * C + c4 * 8) = v;
    }
}

// 32 -> 32 convolution on the matrix cores.  MODE 0 (forward): out =
// bf(relu(conv(in, W) + bias)).  MODE 1 (dgrad): out = bf(conv(in, Wt) *
// [mask > 0]) with Wt the flipped, transposed taps.  wts: [9][32 out][32 in]
// bfloat16.  Persistent: each wave loads the weights of its output-channel half
// into registers once, then the block takes tiles blockIdx.x, blockIdx.x +
// gridDim.x, ... of the XCD-aware order (gridDim.x a multiple of 8 or equal to
// the tile count, so a block's tiles stay on its own XCD).  Per tile: the halo
// goes from registers into LDS, the next tile's halo loads are issued (they stay
// in flight through this tile's work), the matrix products read the halo, the
// outputs are staged in the same LDS and written out row by row.
template <int MODE>
__device__ __forceinline__ void conv32_body(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wts,
                                            const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                            uint16_t* __restrict__ out, int n, int tiles_x, int tiles_per_img,
                                            int nblocks)
{
    __shared__ __attribute__((aligned(16))) uint16_t s[HALO][HALO][LDS_PIX];
    __shared__ __attribute__((aligned(16))) float sbias[C];
    static_assert(T * T <= HALO * HALO, "the output tile fits the halo buffer");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int hh = wave & 1;
    if (MODE == 0 && threadIdx.x < C) sbias[threadIdx.x] = bias[threadIdx.x];  // read after the first barrier
    // A operands: lane (m, g) holds W_tap[hh*16 + m][8g .. 8g+7]
    bf16x8 A[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) A[tap] = as_bf8(*(const u32x4*)(wts + ((tap * C) + hh * 16 + m) * C + g * 8));
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) settle(A[tap]);
    HaloRegs<256> h;
    if ((int)blockIdx.x < nblocks) halo_issue<256>(h, in, tile_of(blockIdx.x, nblocks, tiles_x, tiles_per_img), n);
    for (int v = blockIdx.x; v < nblocks; v += gridDim.x) {
        const Tile tl = tile_of(v, nblocks, tiles_x, tiles_per_img);
        if (v != (int)blockIdx.x) __syncthreads();  // the previous tile's reads of s are done
        halo_store<256>(s, h);
        __syncthreads();
        if (v + (int)gridDim.x < nblocks)
            halo_issue<256>(h, in, tile_of(v + gridDim.x, nblocks, tiles_x, tiles_per_img), n);
        f32x4 acc[8];
        conv32_mma(s, A, acc, wave, m, g);
        __syncthreads();  // every wave's reads of the halo are done
        conv32_stage<MODE>(&s[0][0][0], acc, sbias, wave, m, g);
        __syncthreads();
        conv32_copy_out<MODE>(&s[0][0][0], mask, out, n, tl, wave, lane);
    }
}

// Held to 4 waves per SIMD (each wave keeps only its output-channel half of
// the weights, 36 registers, so this fits without spills).
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void conv32_kernel(
    const uint16_t* __restrict__ in, const uint16_t* __restrict__ wts, const float* __restrict__ bias,
    const uint16_t* __restrict__ mask, uint16_t* __restrict__ out, int n, int tiles_x, int tiles_per_img, int nblocks)
{
    conv32_body<MODE>(in, wts, bias, mask, out, n, tiles_x, tiles_per_img, nblocks);
}

// Layer 8 (32 -> 1): z = b8 + sum_tap sum_c w8 a7, y = x + z with x = mu / scale
// (float32).  mu_out (optional) = mu + scale * z, projected onto the
// constraints when asked.  On the matrix cores: for every pixel p of a tile's
// 18x18 halo, D[tap][p] = sum_c W8[c][tap] a7[p][c] (a 16 x 16 x 32 product per
// 16 halo pixels, rows = the 9 taps and 7 zero rows, operands straight from
// memory: lane (m, g) loads channels 8g .. 8g+7 of halo pixel m), the 9 x 324
// tap sums go to LDS, and each output pixel adds its 9 neighbours' sums in tap
// order (0,0), (0,1), ..., (2,2).  Persistent over the XCD-aware tile order, the
// next tile's operand loads in flight while the current tile is finished.
constexpr int OUT_THREADS = 256;
constexpr int OUT_GRID = 256 * 4;                             // blocks resident at once, a multiple of 8
constexpr int OUT_GROUPS = (HALO * HALO + 15) / 16;           // 16-pixel groups of the halo (21)
constexpr int OUT_PER_WAVE = (OUT_GROUPS + 3) / 4;            // groups per wave (6)
__device__ __forceinline__ void out_issue(u32x4 (&b)[OUT_PER_WAVE], const uint16_t* __restrict__ a7, Tile t, int n,
                                          int wave, int m, int g)
{
#pragma unroll
    for (int k = 0; k < OUT_PER_WAVE; ++k) {
        const int p = 16 * (wave + 4 * k) + m;  // halo pixel of this lane in group wave + 4k
        const int ly = p / HALO, lx = p - ly * HALO;
        const int gi = t.i0 + ly - 1, gj = t.j0 + lx - 1;
        const bool in = p < HALO * HALO && gi >= 0 && gi < n && gj >= 0 && gj < n;
        const u32x4 v = *(const u32x4*)(a7 + (in ? pix(t.b, gi, gj, n) * C + g * 8 : 0));
        b[k] = in ? v : u32x4{0u, 0u, 0u, 0u};
    }
}
__global__ __launch_bounds__(OUT_THREADS) void conv_out_kernel(const uint16_t* __restrict__ a7,
                                                               const uint16_t* __restrict__ w8a,
                                                               const float* __restrict__ b8,
                                                               const float* __restrict__ mu, float inv_scale,
                                                               float scale, float* __restrict__ y,
                                                               float* __restrict__ mu_out, int project, int n,
                                                               int tiles_x, int tiles_per_img, int nblocks)
{
    __shared__ float dt[HALO * HALO][9];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    // A operand: lane (m, g) holds W8[8g .. 8g+7][tap m] (zero rows past tap 8)
    const bf16x8 A = as_bf8(*(const u32x4*)(w8a + m * C + g * 8));
    const float bias = b8[0];
    settle(A);
    settle(bias);
    u32x4 bq[OUT_PER_WAVE];
    if ((int)blockIdx.x < nblocks) out_issue(bq, a7, tile_of(blockIdx.x, nblocks, tiles_x, tiles_per_img), n, wave, m, g);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int v = blockIdx.x; v < nblocks; v += gridDim.x) {
        const Tile tl = tile_of(v, nblocks, tiles_x, tiles_per_img);
        f32x4 d[OUT_PER_WAVE];
#pragma unroll
        for (int k = 0; k < OUT_PER_WAVE; ++k) d[k] = mfma(A, as_bf8(bq[k]), f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        if (v != (int)blockIdx.x) __syncthreads();  // the previous tile's reads of dt are done
        // D[4g + i][m]: tap 4g + i of halo pixel 16 (wave + 4k) + m
#pragma unroll
        for (int k = 0; k < OUT_PER_WAVE; ++k) {
            const int p = 16 * (wave + 4 * k) + m;
            if (p < HALO * HALO && g < 3) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * g + i < 9) dt[p][4 * g + i] = d[k][i];
            }
        }
        __syncthreads();
        if (v + (int)gridDim.x < nblocks)
            out_issue(bq, a7, tile_of(v + gridDim.x, nblocks, tiles_x, tiles_per_img), n, wave, m, g);
        const int i = tl.i0 + ty, j = tl.j0 + tx;
        if (i < n && j < n) {
            float z = bias;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) z += dt[(ty + tap / 3) * HALO + tx + tap % 3][tap];
            const size_t p = pix(tl.b, i, j, n);
            const float xin = mu[p];
            if (y) y[p] = fmaf(xin, inv_scale, z);
            if (mu_out) {
                // mu + scale * z = scale * y, formed so that z = 0 returns mu exactly
                const float mo = fmaf(scale, z, xin);
                mu_out[p] = project ? (in_disc(j, i, n) ? fmaxf(mo, 0.0f) : 0.0f) : mo;
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Loss and backward
// ----------------------------------------------------------------------------

// g8 = 2 (y - t) [p in disc] / count; per-block sums of (y - t)^2 over the disc
// (FP64, fixed tree).
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y, const float* __restrict__ target,
                                                   float inv_scale, float two_over_count, float* __restrict__ g8,
                                                   double* __restrict__ part, int n, long total)
{
    __shared__ double red[256];
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (idx < total) {
        const int j = (int)(idx % n);
        const int i = (int)((idx / n) % n);
        const float d = in_disc(j, i, n) ? y[idx] - target[idx] * inv_scale : 0.0f;
        g8[idx] = d * two_over_count;
        sq = (double)d * (double)d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = (sum of part[0..nparts)) / count, one block, fixed order.
__global__ __launch_bounds__(256) void loss_final_kernel(const double* __restrict__ part, int nparts, double count,
                                                         double* __restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / count;
}

// Layer 8 dgrad: g7[p][c] = bf([a7 > 0] sum_tap w8[c][tap] g8[p - tap]).
__global__ __launch_bounds__(256) void dgrad_out_kernel(const float* __restrict__ g8, const float* __restrict__ w8r,
                                                        const uint16_t* __restrict__ a7, uint16_t* __restrict__ g7,
                                                        int n, long total)
{
    __shared__ u32x4 stage[ROW_STAGE_WORDS];
    const long first = (long)blockIdx.x * blockDim.x;
    const long idx = first + threadIdx.x;
    u32x4 rows[4] = {};
    if (idx < total) {
        const int j = (int)(idx % n);
        const long bi = idx / n;
        const int i = (int)(bi % n);
        const int b = (int)(bi / n);
        float gn[9];  // g8 at (i - dy, j - dx) for tap (dy + 1, dx + 1)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int gi = i - (ky - 1), gj = j - (kx - 1);
                gn[ky * 3 + kx] = (gi >= 0 && gi < n && gj >= 0 && gj < n) ? g8[pix(b, gi, gj, n)] : 0.0f;
            }
        const u32x4* msk = (const u32x4*)(a7 + (size_t)idx * C);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4 mv = msk[q];
            const uint32_t mw[4] = {mv.x, mv.y, mv.z, mv.w};
            uint32_t pk[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = q * 8 + e * 2;
                float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    d0 = fmaf(w8r[c * 9 + t], gn[t], d0);
                    d1 = fmaf(w8r[(c + 1) * 9 + t], gn[t], d1);
                }
                d0 = bf_lo(mw[e]) > 0.0f ? d0 : 0.0f;
                d1 = bf_hi(mw[e]) > 0.0f ? d1 : 0.0f;
                pk[e] = f2bf(d0) | (f2bf(d1) << 16);
            }
            rows[q] = u32x4{pk[0], pk[1], pk[2], pk[3]};
        }
    }
    store_pixel_rows(stage, rows, g7, first, total);
}

// Weight gradient of a 32 -> 32 layer on the matrix cores:
//   dW[o][c][tap] = sum_p g[p][o] a[p + tap][c],  db[o] = sum_p g[p][o].
// Block k handles tiles k, k + gridDim.x, ... in turn and writes its partial
// sums (parameter layout, 9216 weights then 32 biases) to part[k].
//
// The g tile and the activation halo stay channels-last in LDS, as loaded
// (16-byte stores).  The operands of v_mfma_f32_16x16x32_bf16 need 8
// consecutive pixels of one channel per lane; ds_read_b64_tr_b16 provides
// them: within each 16-lane group, lane r points at 4 consecutive channels
// (4 (r mod 4) ...) of pixel r / 4, and lane i receives channel i of those 4
// pixels.  Each lane gives its own address, so the tap's pixel shift is an
// address offset (no shifted copies).
constexpr int WG_PSTR = 32;  // bf16 per staged pixel

typedef short s16x4 __attribute__((ext_vector_type(4)));

// 4 consecutive pixels (pixel0 + 0..3, channels-last rows of WG_PSTR bf16,
// row stride `pstride` bf16 between them) of channel `c16 + lane mod 16`.
__device__ __forceinline__ u32x2 tr_read(const uint16_t* lds_row0, int pstride, int c16)
{
    const int r = threadIdx.x & 15;
    const uint16_t* p = lds_row0 + (r >> 2) * pstride + c16 + 4 * (r & 3);
    const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)p);
    return __builtin_bit_cast(u32x2, v);
}

__device__ __forceinline__ bf16x8 cat(u32x2 lo, u32x2 hi) { return as_bf8(u32x4{lo.x, lo.y, hi.x, hi.y}); }

__global__ __launch_bounds__(256) void wgrad32_kernel(const uint16_t* __restrict__ g, const uint16_t* __restrict__ a,
                                                      float* __restrict__ part, int n, int tiles_x, int tiles_per_img,
                                                      int ntiles)
{
    // the g tile, then the activation halo; reused for the cross-wave sum at the end
    __shared__ __attribute__((aligned(16))) uint16_t lds[(T * T + HALO * HALO) * WG_PSTR];
    __shared__ float bpart[256];
    uint16_t* gS = lds;
    uint16_t* aS = lds + T * T * WG_PSTR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, g4 = lane >> 4;
    // wave w: input channels 16 h2 ... 16 h2 + 15 (h2 = w mod 2), pixel blocks 4 (w / 2) ... + 3
    const int h2 = wave & 1, kb0 = 4 * (wave >> 1);
    f32x4 acc[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // bias partial of channel tid mod 32 over pixels 32 (tid / 32) ... + 31 of every tile
    float bacc = 0.0f;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tile_plain(t, tiles_x, tiles_per_img);
        __syncthreads();  // the previous tile's reads are done
        {
            const int li = tid >> 4, lj = tid & 15;
            const int gi = tl.i0 + li, gj = tl.j0 + lj;
            u32x4 v[4] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
            if (gi < n && gj < n) {
                const u32x4* src = (const u32x4*)(g + pix(tl.b, gi, gj, n) * C);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = src[q];
            }
            u32x4* dst = (u32x4*)(gS + tid * WG_PSTR);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = v[q];
        }
        for (int e = tid; e < HALO * HALO; e += 256) {
            // activation halo: aS[row][col] = a[i0 + row - 1][j0 + col - 1], zero outside the image
            const int ly = e / HALO, lx = e - ly * HALO;
            const int gi = tl.i0 + ly - 1, gj = tl.j0 + lx - 1;
            u32x4 v[4] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
            if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
                const u32x4* src = (const u32x4*)(a + pix(tl.b, gi, gj, n) * C);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = src[q];
            }
            u32x4* dst = (u32x4*)(aS + e * WG_PSTR);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = v[q];
        }
        __syncthreads();
        {
            const int c = tid & 31, p0 = 32 * (tid >> 5);
            float s = 0.0f;
            for (int p = p0; p < p0 + 32; ++p) s += bf2f(gS[p * WG_PSTR + c]);
            bacc += s;
        }
        // pixel block kb = 32 pixels = tile rows 2 kb, 2 kb + 1; lane group g4 holds pixels
        // 8 g4 ... 8 g4 + 7 of the block: row R, columns c0 ... c0 + 7
        for (int kb = kb0; kb < kb0 + 4; ++kb) {
            const int R = 2 * kb + (g4 >> 1), c0 = 8 * (g4 & 1);
            const uint16_t* grow = gS + (R * T + c0) * WG_PSTR;
            bf16x8 Af[2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
                Af[h] = cat(tr_read(grow, WG_PSTR, 16 * h), tr_read(grow + 4 * WG_PSTR, WG_PSTR, 16 * h));
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const uint16_t* arow = aS + ((R + ky) * HALO + c0 + kx) * WG_PSTR;
                    const bf16x8 Bf =
                        cat(tr_read(arow, WG_PSTR, 16 * h2), tr_read(arow + 4 * WG_PSTR, WG_PSTR, 16 * h2));
                    acc[ky * 3 + kx][0] = mfma(Af[0], Bf, acc[ky * 3 + kx][0]);
                    acc[ky * 3 + kx][1] = mfma(Af[1], Bf, acc[ky * 3 + kx][1]);
                }
        }
    }
    // add the pixel halves' sums (waves h2 and h2 + 2, in that order), in LDS (reusing the tiles)
    __syncthreads();
    float* red = (float*)lds;
    static_assert(W32 <= (T * T + HALO * HALO) * WG_PSTR / 2, "reduction fits the tile buffer");
    for (int w = 0; w < 4; w += 2) {
        if ((wave >> 1) == (w >> 1)) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = h * 16 + g4 * 4 + i, c = h2 * 16 + m;
                        const int idx = (o * C + c) * 9 + tap;
                        red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[tap][h][i];
                    }
        }
        __syncthreads();
    }
    bpart[tid] = bacc;
    __syncthreads();
    float* dst = part + (size_t)blockIdx.x * P32;
    for (int k = tid; k < W32; k += 256) dst[k] = red[k];
    if (tid < C) {
        // the 8 pixel groups' partials of channel tid, in group order
        float b = 0.0f;
        for (int q = 0; q < 8; ++q) b += bpart[32 * q + tid];
        dst[W32 + tid] = b;
    }
}

// Weight gradients of the first layer (g1 x a0; 288 weights + 32 biases) and
// of the last (g8 x a7; 288 weights + 1 bias), float32 on the vector ALUs.
// Thread t owns a channel pair cp = t mod 16 and a tile row r = t / 16: for
// each pixel of its row it loads the pair once and each of the 9 neighbours
// once and adds into 9 x 2 register accumulators.  At the end the 16 rows'
// sums are added in row order through LDS.  The loads of a block's next tile
// are issued before the current tile's sums, so they are in flight meanwhile.
struct WgradInRegs {
    uint32_t g[T];   // the thread's channel pair of g1 at the 16 pixels of its tile row
    uint16_t a[2];   // a0 at halo pixels tid and tid + 256
};
__device__ __forceinline__ void wgrad_in_issue(WgradInRegs& q, const uint16_t* __restrict__ g1,
                                               const uint16_t* __restrict__ a0, Tile tl, int n, int r, int cp)
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        const int ly = e / HALO, lx = e - ly * HALO;
        const int gi = tl.i0 + ly - 1, gj = tl.j0 + lx - 1;
        const bool in = e < HALO * HALO && gi >= 0 && gi < n && gj >= 0 && gj < n;
        q.a[k] = in ? a0[pix(tl.b, gi, gj, n)] : (uint16_t)0;
    }
    const int gi = tl.i0 + r;
#pragma unroll
    for (int x = 0; x < T; ++x) {
        const int gj = tl.j0 + x;
        q.g[x] = (gi < n && gj < n) ? *(const uint32_t*)(g1 + pix(tl.b, gi, gj, n) * C + 2 * cp) : 0u;
    }
}

__global__ __launch_bounds__(256) void wgrad_in_kernel(const uint16_t* __restrict__ g1, const uint16_t* __restrict__ a0,
                                                       float* __restrict__ part, int n, int tiles_x,
                                                       int tiles_per_img, int ntiles)
{
    __shared__ float as[HALO][HALO + 1];
    __shared__ float red[T][T][19];
    const int tid = threadIdx.x, cp = tid & 15, r = tid >> 4;
    float acc[9][2], bacc[2] = {0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = 0.0f;
    WgradInRegs q;
    if ((int)blockIdx.x < ntiles) wgrad_in_issue(q, g1, a0, tile_plain(blockIdx.x, tiles_x, tiles_per_img), n, r, cp);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tile_plain(t, tiles_x, tiles_per_img);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = tid + 256 * k;
            if (e < HALO * HALO) as[e / HALO][e % HALO] = bf2f(q.a[k]);
        }
        uint32_t gw[T];
#pragma unroll
        for (int x = 0; x < T; ++x) gw[x] = q.g[x];
        __syncthreads();
        if (t + (int)gridDim.x < ntiles)
            wgrad_in_issue(q, g1, a0, tile_plain(t + gridDim.x, tiles_x, tiles_per_img), n, r, cp);
        const int gi = tl.i0 + r;
        if (gi < n) {
#pragma unroll
            for (int x = 0; x < T; ++x) {
                const int gj = tl.j0 + x;
                if (gj >= n) break;
                const float g0 = bf_lo(gw[x]), gq = bf_hi(gw[x]);
                bacc[0] += g0;
                bacc[1] += gq;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    const float av = as[r + tap / 3][x + tap % 3];
                    acc[tap][0] = fmaf(g0, av, acc[tap][0]);
                    acc[tap][1] = fmaf(gq, av, acc[tap][1]);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        red[r][cp][tap] = acc[tap][0];
        red[r][cp][9 + tap] = acc[tap][1];
    }
    red[r][cp][18] = 0.0f;
    __syncthreads();
    // part row: W1[o][tap] at o * 9 + tap, then b1[o] at 288 + o
    for (int k = tid; k < P_IN; k += 256) {
        float sum = 0.0f;
        if (k < 288) {
            const int o = k / 9, tap = k - o * 9;
            for (int rr = 0; rr < T; ++rr) sum += red[rr][o >> 1][(o & 1) * 9 + tap];
        }
        part[(size_t)blockIdx.x * P_IN + k] = sum;
    }
    __syncthreads();
    red[r][cp][0] = bacc[0];
    red[r][cp][1] = bacc[1];
    __syncthreads();
    if (tid < C) {
        float sum = 0.0f;
        for (int rr = 0; rr < T; ++rr) sum += red[rr][tid >> 1][tid & 1];
        part[(size_t)blockIdx.x * P_IN + 288 + tid] = sum;
    }
}

__global__ __launch_bounds__(256) void wgrad_out_kernel(const float* __restrict__ g8, const uint16_t* __restrict__ a7,
                                                        float* __restrict__ part, int n, int tiles_x,
                                                        int tiles_per_img, int ntiles)
{
    __shared__ __attribute__((aligned(16))) uint16_t s[HALO][HALO][LDS_PIX];
    __shared__ float gs[T][T];
    __shared__ float red[T][T][19];
    const int tid = threadIdx.x, cp = tid & 15, r = tid >> 4;
    float acc[9][2], bacc = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = 0.0f;
    HaloRegs<256> h;
    float gnext = 0.0f;  // g8 at pixel (r, cp) of the next tile
    auto issue = [&](Tile tl) {
        halo_issue<256>(h, a7, tl, n);
        const int gi = tl.i0 + r, gj = tl.j0 + cp;
        gnext = (gi < n && gj < n) ? g8[pix(tl.b, gi, gj, n)] : 0.0f;
    };
    if ((int)blockIdx.x < ntiles) issue(tile_plain(blockIdx.x, tiles_x, tiles_per_img));
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();
        halo_store<256>(s, h);
        gs[r][cp] = gnext;
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) issue(tile_plain(t + gridDim.x, tiles_x, tiles_per_img));
        for (int x = 0; x < T; ++x) {
            const float g = gs[r][x];
            bacc += g;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const uint32_t w = *(const uint32_t*)(&s[r + tap / 3][x + tap % 3][2 * cp]);
                acc[tap][0] = fmaf(g, bf_lo(w), acc[tap][0]);
                acc[tap][1] = fmaf(g, bf_hi(w), acc[tap][1]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        red[r][cp][tap] = acc[tap][0];
        red[r][cp][9 + tap] = acc[tap][1];
    }
    red[r][cp][18] = bacc;
    __syncthreads();
    // part row: W8[0][c][tap] at c * 9 + tap, then b8 at 288
    for (int k = tid; k < P_OUT; k += 256) {
        float sum = 0.0f;
        if (k < 288) {
            const int c = k / 9, tap = k - c * 9;
            for (int rr = 0; rr < T; ++rr) sum += red[rr][c >> 1][(c & 1) * 9 + tap];
        } else {
            for (int rr = 0; rr < T; ++rr) sum += red[rr][0][18];
        }
        part[(size_t)blockIdx.x * P_OUT + k] = sum;
    }
}

// Partial rows are added in two fixed-order stages: groups of RG consecutive
// block rows, then the groups (the single-stage sum was one long dependent
// chain of loads per output).
constexpr int RG = 32;

__global__ __launch_bounds__(256) void reduce_group_kernel(const float* __restrict__ part, int nblocks, int row,
                                                           float* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= row) return;
    const int b0 = blockIdx.y * RG, b1 = min(b0 + RG, nblocks);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[(size_t)b * row + k];
    out[(size_t)blockIdx.y * row + k] = s;
}

// out[k] = sum over blocks b = 0, 1, ... of part[b][k] (fixed order).
__global__ __launch_bounds__(256) void reduce_part_kernel(const float* __restrict__ part, int nblocks, int row,
                                                          float* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= row) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * row + k];
    out[k] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ th, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, int np, float lr,
                                                   float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float gk = g[k];
    const float mk = kB1 * m[k] + kOneMinusB1 * gk;
    const float vk = kB2 * v[k] + kOneMinusB2 * gk * gk;
    m[k] = mk;
    v[k] = vk;
    th[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + kEps);
}

}  // namespace

// ----------------------------------------------------------------------------
// Handle
// ----------------------------------------------------------------------------

struct recon_cnn {
    int max_batch = 0, max_n = 0;
    float mu_scale = 1.0f;
    int step = 0;
    float* d_theta = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_grad = nullptr;
    uint16_t* d_wf = nullptr;  // [6][9][32][32]
    uint16_t* d_wt = nullptr;  // [6][9][32][32]
    uint16_t* d_w1a = nullptr;  // [32][32] bf16: the first layer's matrix-core operand
    float* d_w8r = nullptr;     // [32][9]
    uint16_t* d_w8a = nullptr;  // [16][32] bf16: the last layer's matrix-core operand
    uint16_t* d_a0 = nullptr;  // [B][n][n]
    uint16_t* d_act[8] = {};   // 1..7: [B][n][n][32]
    uint16_t* d_g[8] = {};     // 1..7: [B][n][n][32]
    float* d_y = nullptr;      // [B][n][n]
    float* d_g8 = nullptr;     // [B][n][n]
    float* d_part = nullptr;   // [WG_BLOCKS][P32]
    float* d_part2 = nullptr;  // [WG_BLOCKS / RG][P32], first stage of the fixed-order reduction
    double* d_loss_part = nullptr;
    int last_batch = 0, last_n = 0;  // shape of the tensors held
};

namespace {

struct Shape {
    int batch, n, tiles_x, tiles_per_img, ntiles;
    long pixels;
};
Shape shape_of(int batch, int n)
{
    Shape s;
    s.batch = batch;
    s.n = n;
    s.tiles_x = (n + T - 1) / T;
    s.tiles_per_img = s.tiles_x * s.tiles_x;
    s.ntiles = s.tiles_per_img * batch;
    s.pixels = (long)batch * n * n;
    return s;
}

void free_cnn(recon_cnn* c)
{
    if (!c) return;
    void* ptrs[] = {c->d_theta, c->d_m, c->d_v, c->d_grad, c->d_wf, c->d_wt, c->d_w1a, c->d_w8r, c->d_w8a,
                    c->d_a0, c->d_y, c->d_g8, c->d_part, c->d_part2, c->d_loss_part};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < 8; ++l) {
        if (c->d_act[l]) (void)hipFree(c->d_act[l]);
        if (c->d_g[l]) (void)hipFree(c->d_g[l]);
    }
    delete c;
}

hipError_t launch_prep(recon_cnn* c, hipStream_t s)
{
    prep_weights_kernel<<<cdiv(PREP_END, 256), 256, 0, s>>>(c->d_theta, c->d_wf, c->d_wt, c->d_w8r, c->d_w1a,
                                                           c->d_w8a);
    return hipGetLastError();
}

// Blocks of the persistent 32 -> 32 convolution: as many as are resident at
// once (256 CUs x 4), a multiple of 8.
constexpr int CONV_GRID = 256 * 4;

hipError_t launch_conv32(int mode, const uint16_t* in, const uint16_t* w, const float* bias, const uint16_t* mask,
                         uint16_t* out, const Shape& S, hipStream_t s)
{
    const int grid = std::min(S.ntiles, CONV_GRID);
    if (mode == 0)
        conv32_kernel<0><<<grid, 256, 0, s>>>(in, w, bias, mask, out, S.n, S.tiles_x, S.tiles_per_img, S.ntiles);
    else
        conv32_kernel<1><<<grid, 256, 0, s>>>(in, w, bias, mask, out, S.n, S.tiles_x, S.tiles_per_img, S.ntiles);
    return hipGetLastError();
}

// Forward pass of `batch` images (batch <= max_batch) from mu; y and mu_out optional.
hipError_t enqueue_forward(recon_cnn* c, const float* mu, float* mu_out, int project, const Shape& S, hipStream_t s)
{
    const float inv = 1.0f / c->mu_scale;
    conv_in_kernel<<<std::min(S.ntiles, IN_GRID), 256, 0, s>>>(mu, inv, c->d_w1a, c->d_theta + OFF_B1, c->d_a0,
                                                               c->d_act[1], S.n, S.tiles_x, S.tiles_per_img, S.ntiles);
    hipError_t e = hipGetLastError();
    for (int l = 2; l <= 7 && e == hipSuccess; ++l)
        e = launch_conv32(0, c->d_act[l - 1], c->d_wf + (size_t)(l - 2) * W32,
                          c->d_theta + OFF_HID + (l - 2) * P32 + W32, nullptr, c->d_act[l], S, s);
    if (e != hipSuccess) return e;
    conv_out_kernel<<<std::min(S.ntiles, OUT_GRID), OUT_THREADS, 0, s>>>(
        c->d_act[7], c->d_w8a, c->d_theta + OFF_B8, mu, inv, c->mu_scale, c->d_y, mu_out, project, S.n, S.tiles_x,
        S.tiles_per_img, S.ntiles);
    return hipGetLastError();
}

int wg_blocks(const Shape& S) { return S.ntiles < WG_BLOCKS ? S.ntiles : WG_BLOCKS; }

// out[k] = sum of part[b][k] over the nb partial rows: groups of RG rows, then the groups.
hipError_t enqueue_reduce(recon_cnn* c, int nb, int row, float* out, hipStream_t s)
{
    const int groups = (nb + RG - 1) / RG;
    reduce_group_kernel<<<dim3(cdiv(row, 256), groups), 256, 0, s>>>(c->d_part, nb, row, c->d_part2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_part_kernel<<<cdiv(row, 256), 256, 0, s>>>(c->d_part2, groups, row, out);
    return hipGetLastError();
}

hipError_t enqueue_wgrad32(recon_cnn* c, int l, const Shape& S, hipStream_t s)
{
    const int nb = wg_blocks(S);
    wgrad32_kernel<<<nb, 256, 0, s>>>(c->d_g[l], c->d_act[l - 1], c->d_part, S.n, S.tiles_x, S.tiles_per_img,
                                      S.ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return enqueue_reduce(c, nb, P32, c->d_grad + OFF_HID + (l - 2) * P32, s);
}

// Loss and gradient (into d_grad) for a batch held in the workspace.
hipError_t enqueue_loss_grad(recon_cnn* c, const float* mu, const float* target, double* d_loss, const Shape& S,
                             hipStream_t s)
{
    hipError_t e = enqueue_forward(c, mu, nullptr, 0, S, s);
    if (e != hipSuccess) return e;
    long disc = 0;
    for (int i = 0; i < S.n; ++i)
        for (int j = 0; j < S.n; ++j) disc += in_disc(j, i, S.n) ? 1 : 0;
    const double count = (double)disc * S.batch;
    const unsigned nlb = cdiv(S.pixels, 256);
    loss_kernel<<<nlb, 256, 0, s>>>(c->d_y, target, 1.0f / c->mu_scale, (float)(2.0 / count), c->d_g8,
                                    c->d_loss_part, S.n, S.pixels);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (d_loss) {
        loss_final_kernel<<<1, 256, 0, s>>>(c->d_loss_part, (int)nlb, count, d_loss);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // layer 8: weights from g8 x a7, then g7
    const int nb = wg_blocks(S);
    wgrad_out_kernel<<<nb, 256, 0, s>>>(c->d_g8, c->d_act[7], c->d_part, S.n, S.tiles_x, S.tiles_per_img, S.ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = enqueue_reduce(c, nb, P_OUT, c->d_grad + OFF_W8, s)) != hipSuccess) return e;
    dgrad_out_kernel<<<cdiv(S.pixels, 256), 256, 0, s>>>(c->d_g8, c->d_w8r, c->d_act[7], c->d_g[7], S.n, S.pixels);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // layers 7 .. 2
    for (int l = 7; l >= 2; --l) {
        if ((e = enqueue_wgrad32(c, l, S, s)) != hipSuccess) return e;
        if ((e = launch_conv32(1, c->d_g[l], c->d_wt + (size_t)(l - 2) * W32, nullptr, c->d_act[l - 1],
                               c->d_g[l - 1], S, s)) != hipSuccess)
            return e;
    }
    // layer 1
    wgrad_in_kernel<<<nb, 256, 0, s>>>(c->d_g[1], c->d_a0, c->d_part, S.n, S.tiles_x, S.tiles_per_img, S.ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return enqueue_reduce(c, nb, P_IN, c->d_grad + OFF_W1, s);
}

recon_status check_batch(recon_cnn* net, int batch, int n, bool training)
{
    if (!net) return fail(RECON_INVALID_ARG, "NULL network");
    if (n < 1 || n > net->max_n) return fail(RECON_INVALID_ARG, "n must be in [1, max_n]");
    if (batch < 1 || (training && batch > net->max_batch))
        return fail(RECON_INVALID_ARG, training ? "batch must be in [1, max_batch]" : "batch must be >= 1");
    return RECON_OK;
}

}  // namespace

extern "C" {

int64_t recon_cnn_param_count(void) { return NPARAM; }

recon_status recon_cnn_create(const float* h_params, int32_t max_batch, int32_t max_n, float mu_scale,
                              recon_cnn** out)
{
    if (!out) return fail(RECON_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_n < 1 || max_n > 16384) return fail(RECON_INVALID_ARG, "bad max_batch or max_n");
    if (!(mu_scale > 0) || !std::isfinite(mu_scale)) return fail(RECON_INVALID_ARG, "mu_scale must be > 0");
    if ((double)max_batch * max_n * max_n * C * 2 > 64.0 * (1ull << 30))
        return fail(RECON_INVALID_ARG, "workspace above 64 GiB per tensor");
    recon_cnn* c = new (std::nothrow) recon_cnn();
    if (!c) return fail(RECON_OOM, "host allocation failed");
    c->max_batch = max_batch;
    c->max_n = max_n;
    c->mu_scale = mu_scale;
    auto bail = [&](hipError_t e, const char* what) {
        free_cnn(c);
        return fail(e == hipErrorOutOfMemory ? RECON_OOM : RECON_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    const size_t px = (size_t)max_batch * max_n * max_n;
    hipError_t e = hipSuccess;
#define C_TRY(expr)                          \
    do {                                     \
        e = (expr);                          \
        if (e != hipSuccess) return bail(e, #expr); \
    } while (0)
    C_TRY(hipMalloc(&c->d_theta, NPARAM * sizeof(float)));
    C_TRY(hipMalloc(&c->d_m, NPARAM * sizeof(float)));
    C_TRY(hipMalloc(&c->d_v, NPARAM * sizeof(float)));
    C_TRY(hipMalloc(&c->d_grad, NPARAM * sizeof(float)));
    C_TRY(hipMalloc(&c->d_wf, NHID * W32 * sizeof(uint16_t)));
    C_TRY(hipMalloc(&c->d_wt, NHID * W32 * sizeof(uint16_t)));
    C_TRY(hipMalloc(&c->d_w1a, C * C * sizeof(uint16_t)));
    C_TRY(hipMalloc(&c->d_w8r, 288 * sizeof(float)));
    C_TRY(hipMalloc(&c->d_w8a, 16 * C * sizeof(uint16_t)));
    C_TRY(hipMalloc(&c->d_a0, px * sizeof(uint16_t)));
    for (int l = 1; l <= 7; ++l) {
        C_TRY(hipMalloc(&c->d_act[l], px * C * sizeof(uint16_t)));
        C_TRY(hipMalloc(&c->d_g[l], px * C * sizeof(uint16_t)));
    }
    C_TRY(hipMalloc(&c->d_y, px * sizeof(float)));
    C_TRY(hipMalloc(&c->d_g8, px * sizeof(float)));
    C_TRY(hipMalloc(&c->d_part, (size_t)WG_BLOCKS * P32 * sizeof(float)));
    C_TRY(hipMalloc(&c->d_part2, (size_t)(WG_BLOCKS / RG) * P32 * sizeof(float)));
    C_TRY(hipMalloc(&c->d_loss_part, cdiv((long)px, 256) * sizeof(double)));
    if (h_params)
        C_TRY(hipMemcpy(c->d_theta, h_params, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    else
        C_TRY(hipMemset(c->d_theta, 0, NPARAM * sizeof(float)));
    C_TRY(hipMemset(c->d_m, 0, NPARAM * sizeof(float)));
    C_TRY(hipMemset(c->d_v, 0, NPARAM * sizeof(float)));
    C_TRY(hipMemset(c->d_grad, 0, NPARAM * sizeof(float)));
    C_TRY(launch_prep(c, nullptr));
    C_TRY(hipDeviceSynchronize());
#undef C_TRY
    *out = c;
    return RECON_OK;
}

recon_status recon_cnn_destroy(recon_cnn* net)
{
    if (!net) return RECON_OK;
    (void)hipDeviceSynchronize();
    free_cnn(net);
    return RECON_OK;
}

recon_status recon_cnn_get_state(recon_cnn* net, float* h_params, float* h_m, float* h_v, int32_t* h_step)
{
    if (!net) return fail(RECON_INVALID_ARG, "NULL network");
    RECON_HIP_TRY(hipDeviceSynchronize());
    if (h_params) RECON_HIP_TRY(hipMemcpy(h_params, net->d_theta, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    if (h_m) RECON_HIP_TRY(hipMemcpy(h_m, net->d_m, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    if (h_v) RECON_HIP_TRY(hipMemcpy(h_v, net->d_v, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    if (h_step) *h_step = net->step;
    return RECON_OK;
}

recon_status recon_cnn_set_state(recon_cnn* net, const float* h_params, const float* h_m, const float* h_v,
                                 int32_t step)
{
    if (!net) return fail(RECON_INVALID_ARG, "NULL network");
    if (step < 0) return fail(RECON_INVALID_ARG, "step must be >= 0");
    RECON_HIP_TRY(hipDeviceSynchronize());
    if (h_params) RECON_HIP_TRY(hipMemcpy(net->d_theta, h_params, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    if (h_m) RECON_HIP_TRY(hipMemcpy(net->d_m, h_m, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    if (h_v) RECON_HIP_TRY(hipMemcpy(net->d_v, h_v, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    net->step = step;
    RECON_HIP_TRY(launch_prep(net, nullptr));
    RECON_HIP_TRY(hipDeviceSynchronize());
    return RECON_OK;
}

recon_status recon_cnn_save(recon_cnn* net, const char* path)
{
    if (!net || !path) return fail(RECON_INVALID_ARG, "NULL argument");
    std::vector<float> buf(3 * (size_t)NPARAM);
    int32_t step = 0;
    recon_status st = recon_cnn_get_state(net, buf.data(), buf.data() + NPARAM, buf.data() + 2 * NPARAM, &step);
    if (st != RECON_OK) return st;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(RECON_INVALID_ARG, std::string("cannot open ") + path);
    const int64_t np = NPARAM;
    const int32_t zero = 0;
    bool ok = std::fwrite("RCNNv001", 1, 8, f) == 8 && std::fwrite(&np, 8, 1, f) == 1 &&
              std::fwrite(&step, 4, 1, f) == 1 && std::fwrite(&zero, 4, 1, f) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? RECON_OK : fail(RECON_INVALID_ARG, std::string("write failed: ") + path);
}

recon_status recon_cnn_load(recon_cnn* net, const char* path)
{
    if (!net || !path) return fail(RECON_INVALID_ARG, "NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(RECON_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    int64_t np = 0;
    int32_t step = 0, zero = 0;
    std::vector<float> buf(3 * (size_t)NPARAM);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RCNNv001", 8) == 0 &&
              std::fread(&np, 8, 1, f) == 1 && np == NPARAM && std::fread(&step, 4, 1, f) == 1 &&
              std::fread(&zero, 4, 1, f) == 1 && step >= 0 &&
              std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(RECON_INVALID_ARG, std::string("not a network file of this version: ") + path);
    return recon_cnn_set_state(net, buf.data(), buf.data() + NPARAM, buf.data() + 2 * NPARAM, step);
}

recon_status recon_cnn_forward(recon_cnn* net, const float* d_mu, float* d_mu_out, int32_t batch, int32_t n,
                               int32_t project, void* stream)
{
    recon_status st = check_batch(net, batch, n, false);
    if (st != RECON_OK) return st;
    if (!d_mu || !d_mu_out) return fail(RECON_INVALID_ARG, "NULL image");
    hipStream_t s = as_stream(stream);
    const size_t img = (size_t)n * n;
    for (int b0 = 0; b0 < batch; b0 += net->max_batch) {
        const int nb = batch - b0 < net->max_batch ? batch - b0 : net->max_batch;
        const Shape S = shape_of(nb, n);
        RECON_HIP_TRY(enqueue_forward(net, d_mu + b0 * img, d_mu_out + b0 * img, project ? 1 : 0, S, s));
        net->last_batch = nb;
        net->last_n = n;
    }
    return RECON_OK;
}

recon_status recon_cnn_loss_grad(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch, int32_t n,
                                 float* d_grad, double* d_loss, void* stream)
{
    recon_status st = check_batch(net, batch, n, true);
    if (st != RECON_OK) return st;
    if (!d_mu || !d_target) return fail(RECON_INVALID_ARG, "NULL image");
    hipStream_t s = as_stream(stream);
    const Shape S = shape_of(batch, n);
    RECON_HIP_TRY(enqueue_loss_grad(net, d_mu, d_target, d_loss, S, s));
    net->last_batch = batch;
    net->last_n = n;
    if (d_grad)
        RECON_HIP_TRY(hipMemcpyAsync(d_grad, net->d_grad, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, s));
    return RECON_OK;
}

recon_status recon_cnn_adam_step(recon_cnn* net, float lr, void* stream)
{
    if (!net) return fail(RECON_INVALID_ARG, "NULL network");
    if (!(lr >= 0) || !std::isfinite(lr)) return fail(RECON_INVALID_ARG, "lr must be finite and >= 0");
    hipStream_t s = as_stream(stream);
    const int t = net->step + 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
    adam_kernel<<<cdiv(NPARAM, 256), 256, 0, s>>>(net->d_theta, net->d_m, net->d_v, net->d_grad, NPARAM, lr, c1, c2);
    RECON_HIP_TRY(hipGetLastError());
    RECON_HIP_TRY(launch_prep(net, s));
    net->step = t;
    return RECON_OK;
}

recon_status recon_cnn_train_step(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch, int32_t n,
                                  float lr, double* d_loss, void* stream)
{
    recon_status st = recon_cnn_loss_grad(net, d_mu, d_target, batch, n, nullptr, d_loss, stream);
    if (st != RECON_OK) return st;
    return recon_cnn_adam_step(net, lr, stream);
}

recon_status recon_cnn_tensor(recon_cnn* net, int32_t kind, int32_t layer, void* d_dst, int64_t bytes, void* stream)
{
    if (!net || !d_dst) return fail(RECON_INVALID_ARG, "NULL argument");
    if (net->last_batch == 0) return fail(RECON_INVALID_ARG, "no forward pass has run");
    const size_t px = (size_t)net->last_batch * net->last_n * net->last_n;
    const void* src = nullptr;
    size_t size = 0;
    if (kind == 0 && layer == 0) {
        src = net->d_a0;
        size = px * 2;
    } else if (kind == 0 && layer >= 1 && layer <= 7) {
        src = net->d_act[layer];
        size = px * C * 2;
    } else if (kind == 1 && layer >= 1 && layer <= 7) {
        src = net->d_g[layer];
        size = px * C * 2;
    } else if (kind == 2) {
        src = net->d_y;
        size = px * 4;
    } else if (kind == 3) {
        src = net->d_g8;
        size = px * 4;
    } else {
        return fail(RECON_INVALID_ARG, "bad tensor kind or layer");
    }
    if (bytes < (int64_t)size) return fail(RECON_INVALID_ARG, "destination too small");
    RECON_HIP_TRY(hipMemcpyAsync(d_dst, src, size, hipMemcpyDeviceToDevice, as_stream(stream)));
    return RECON_OK;
}

recon_status recon_cnn_time_kernels(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch, int32_t n,
                                    int32_t reps, double* ms_out, void* stream)
{
    recon_status st = check_batch(net, batch, n, true);
    if (st != RECON_OK) return st;
    if (!d_mu || !d_target || !ms_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (reps < 1 || reps > 10000) return fail(RECON_INVALID_ARG, "reps must be in [1, 10000]");
    hipStream_t s = as_stream(stream);
    const Shape S = shape_of(batch, n);
    RECON_HIP_TRY(enqueue_loss_grad(net, d_mu, d_target, nullptr, S, s));
    net->last_batch = batch;
    net->last_n = n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RECON_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RECON_DEVICE, "hipEventCreate failed");
    }
    hipError_t err = hipSuccess;
    auto timed = [&](auto&& launch, double* out) {
        if (err != hipSuccess) return;
        err = launch();
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        *out = (double)ms / reps;
    };
    // layer 4 stands for every 32 -> 32 layer (same shapes)
    timed([&] { return launch_conv32(0, net->d_act[3], net->d_wf + 2 * W32, net->d_theta + OFF_HID + 2 * P32 + W32,
                                     nullptr, net->d_act[4], S, s); },
          &ms_out[0]);
    timed([&] { return launch_conv32(1, net->d_g[4], net->d_wt + 2 * W32, nullptr, net->d_act[3], net->d_g[3], S, s); },
          &ms_out[1]);
    timed([&] {
        const int nb = wg_blocks(S);
        wgrad32_kernel<<<nb, 256, 0, s>>>(net->d_g[4], net->d_act[3], net->d_part, S.n, S.tiles_x, S.tiles_per_img,
                                          S.ntiles);
        return hipGetLastError();
    }, &ms_out[2]);
    timed([&] { return enqueue_forward(net, d_mu, nullptr, 0, S, s); }, &ms_out[3]);
    timed([&] { return enqueue_loss_grad(net, d_mu, d_target, nullptr, S, s); }, &ms_out[4]);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(RECON_DEVICE, std::string("timing run: ") + hipGetErrorString(err));
    return RECON_OK;
}

}  // extern "C"
