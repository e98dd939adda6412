// HIP kernels of the ordered-subset TV reconstruction for gfx950.
//
// Per sub-iteration of one slice the path is two launches:
//   fp_kernel<OS>     Joseph forward projection of the subset (section 4.C
//                     "reprojection") fused with the likelihood epilogue:
//                     t = exp(-l), weighted residual w = (t - y/I0) * path,
//                     squared difference e = (l - p)^2 (section 3.C.2);
//                     (e summed in fixed groups of rays);
//   bp_update_kernel  (bp.hip) gather backprojection of w (the exact
//                     transpose of the projector, no atomics), then in every
//                     block the fixed-order FP64 mean of e and the step rule
//                     of Eqs. 4-5, the TV gradient from an LDS tile with a
//                     one-pixel halo, and the update of Eq. 3.
// (Batches take the step rule once per slice in a launch of its own.)
// None of these is a dense contraction: they are gather / stencil kernels
// bound by the memory hierarchy and VALU, so no MFMA is used.
#include <hip/hip_runtime.h>

#include "gather.h"
#include "internal.h"

namespace recon {

namespace {

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ----------------------------------------------------------------------------
// Layout kernels
// ----------------------------------------------------------------------------

// [n][n] image -> padded row-major and padded transposed copies (32x32 tiles
// transposed through LDS so both writes are coalesced); tile (bx, by).
__device__ __forceinline__ void pad_tile(const float* __restrict__ src, float* __restrict__ dst,
                                         float* __restrict__ dstT, int n, int P, bool mask_disc, int bx, int by,
                                         float (&tile)[32][33])
{
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int j = by + r, i = bx + tx;
        float v = 0.0f;
        if (j < n && i < n) {
            v = (mask_disc && !in_disc(i, j, n)) ? 0.0f : src[(size_t)j * n + i];
            dst[(size_t)j * P + i + PAD] = v;
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + r, j = by + tx;
        if (i < n && j < n) dstT[(size_t)i * P + j + PAD] = tile[tx][r];
    }
}

// Counts in natural view order -> y / I0 and p = ln(I0 / max(y, 1)) in subset order; ray r.
__device__ __forceinline__ void prep_count(const float* __restrict__ counts, const ViewRec* __restrict__ views,
                                           int nch, float i0, float* __restrict__ yt, float* __restrict__ p, long r)
{
    const int q = (int)(r / nch), k = (int)(r - (long)q * nch);
    const float y = counts[(size_t)views[q].nat_view * nch + k];
    yt[r] = y / i0;
    p[r] = (float)log((double)i0 / (double)fmaxf(y, 1.0f));
}

__device__ __forceinline__ float initial_value(long idx, int n, float mu0)
{
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    return in_disc(i, j, n) ? mu0 : 0.0f;
}

__device__ __forceinline__ float unpadded_value(const float* __restrict__ src, long idx, int n, int P)
{
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    return src[(size_t)j * P + i + PAD];
}

__global__ __launch_bounds__(256) void pad_image_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                        float* __restrict__ dstT, int n, int P, int mask_disc)
{
    __shared__ float tile[32][33];
    pad_tile(src, dst, dstT, n, P, mask_disc != 0, blockIdx.x * 32, blockIdx.y * 32, tile);
}

__global__ __launch_bounds__(256) void unpad_image_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                          int n, int P)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    dst[idx] = unpadded_value(src, idx, n, P);
}

__global__ __launch_bounds__(256) void initial_image_kernel(float* __restrict__ dst, int n, float mu0)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    dst[idx] = initial_value(idx, n, mu0);
}

__global__ __launch_bounds__(256) void prep_counts_kernel(const float* __restrict__ counts,
                                                          const ViewRec* __restrict__ views, int nv, int nch,
                                                          float i0, float* __restrict__ yt, float* __restrict__ p)
{
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (long)nv * nch) return;
    prep_count(counts, views, nch, i0, yt, p, r);
}

// Batched forms over a group of slices: blockIdx.y is the slice within the
// group, blocks beyond a smaller slice's extent return at once.  Each element
// is computed by the same device function as in the single-slice kernels.

// Start of a run of every slice in the group: blocks [0, count_blocks) prepare
// the counts (block 0 also writes the fresh step-rule state), the rest pad the
// start image (masked to the disc) in 32x32 tiles.
// count_blocks = 1 with counts = false: the slices' y/I0 and p are already
// prepared from these counts (only the state and the images are reset).
__global__ __launch_bounds__(256) void prepare_batch_kernel(const SliceDesc* __restrict__ slices, BatchRunArgs a,
                                                            DevState fresh, int count_blocks, int counts)
{
    __shared__ float tile[32][33];
    const int y = blockIdx.y;
    const SliceDesc* __restrict__ D = slices + a.first + y;
    const Geo G = D->geo;
    if ((int)blockIdx.x < count_blocks) {
        const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
        if (counts && r < (long)G.nv * G.nch) prep_count(a.counts[y], D->views, G.nch, a.i0[y], D->yt, D->p, r);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            fresh.trace = a.trace[y];
            fresh.it = 0;
            D->state[0] = fresh;
        }
        return;
    }
    const int t = (int)blockIdx.x - count_blocks, tiles = (G.n + 31) / 32;
    if (t >= tiles * tiles) return;
    pad_tile(a.img[y], D->img[0], D->imgT[0], G.n, G.P, true, (t % tiles) * 32, (t / tiles) * 32, tile);
}

__global__ __launch_bounds__(256) void unpad_batch_kernel(const SliceDesc* __restrict__ slices, BatchRunArgs a, int in)
{
    const int y = blockIdx.y;
    const SliceDesc* __restrict__ D = slices + a.first + y;
    const int n = D->geo.n;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    a.img[y][idx] = unpadded_value(D->img[in], idx, n, D->geo.P);
}

__global__ __launch_bounds__(256) void initial_batch_kernel(const SliceDesc* __restrict__ slices, BatchRunArgs a)
{
    const int y = blockIdx.y;
    const int n = slices[a.first + y].geo.n;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    a.img[y][idx] = initial_value(idx, n, a.mu0[y]);
}

__global__ __launch_bounds__(256) void copy_batch_kernel(BatchCopyArgs a, long len)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < len) a.dst[blockIdx.y][idx] = a.src[blockIdx.y][idx];
}

// Sinogram rows (natural or subset order) -> path-weighted values in subset order,
// the input form of the gather backprojector.
__global__ __launch_bounds__(256) void scale_sino_kernel(const float* __restrict__ sino,
                                                         const RayMeta* __restrict__ meta,
                                                         const ViewRec* __restrict__ views, int q0, int ray0,
                                                         int nrays, int nch, int natural_rows, float* __restrict__ w)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    const int q = r / nch, k = r - q * nch;
    const int row = natural_rows ? views[q0 + q].nat_view : q;
    w[ray0 + r] = sino[(size_t)row * nch + k] * meta[ray0 + r].scale;
}

// ----------------------------------------------------------------------------
// Forward projection
// ----------------------------------------------------------------------------

struct FpArgs {
    const float* img;   // padded row-major (sampled by y-major rays along rows), followed by
                        // the padded transposed copy (sampled by x-major rays along columns)
    const RayGeo* rg;
    const RayMeta* rm;
    const ViewRec* views;
    int ray0, nrays, n, P, nch, q0, natural_rows;
    float* out;  // plain mode: line integrals
    const float* yt;
    const float* p;
    float* w;
    double* part;  // squared-difference sums of groups of SQ_GROUP consecutive rays
};

// Joseph samples of one ray on sample lines [t0, t1), summed in line order.
// u(t) = lattice + residual; lattice - floor(u) is exact, so the interpolation
// fraction keeps the residual's precision.  The loads of the next four lines
// are issued before the previous four lines are added.  The index clamp to [-PAD, n] keeps every read inside the
// padded row, where out-of-image entries are zero.  img is the buffer's base
// (wave-uniform) and off0 the 32-bit element offset of column 0 of line 0 of
// the copy this ray samples, so addresses are 32-bit offsets from one base.
// two neighbouring floats at any 4-byte-aligned address
typedef float f32x2u __attribute__((ext_vector_type(2), aligned(4)));

__device__ __forceinline__ f32x2u pair_at(const float* __restrict__ img, uint32_t idx)
{
    // 32-bit byte offset from a wave-uniform base
    return *(const f32x2u*)((const char*)img + (idx << 2));
}

__device__ __forceinline__ float chunk_sum(const float* __restrict__ img, uint32_t off0, int P, int n,
                                           const RayGeo& g, int t0, int t1)
{
    const float fn = (float)n;
    // interpolation fraction and the pair of pixels of sample line t (the lattice part minus its
    // floor is exact, so the fraction keeps the residual's precision)
    auto sample = [&](float ft, uint32_t row, float& f, f32x2u& v) {
        const float lat = fmaf(ft, g.s_hi, g.a_int);
        const float res = fmaf(ft, g.s_lo, g.a_frac);
        const float fl = floorf(lat + res);
        f = (lat - fl) + res;
        // clamp in float (fl is integral, so this equals clamping the integer)
        const int j0 = (int)__builtin_amdgcn_fmed3f(fl, (float)-PAD, fn);
        v = pair_at(img, row + (uint32_t)j0);
    };
    float acc = 0.0f;
    int t = t0;
    float ft = (float)t0;  // exact: t < 2^24
    uint32_t row = off0 + (uint32_t)(t0 * P);
    if (t + 3 < t1) {
        // software pipelined by 4 lines: the next 4 lines' loads are in flight while the
        // previous 4 are added (in line order)
        float f[4];
        f32x2u v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sample(ft + (float)u, row + (uint32_t)(u * P), f[u], v[u]);
        t += 4;
        ft += 4.0f;
        row += (uint32_t)(4 * P);
        for (; t + 3 < t1; t += 4) {
            float fn4[4];
            f32x2u vn4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) sample(ft + (float)u, row + (uint32_t)(u * P), fn4[u], vn4[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc += fmaf(f[u], v[u].y - v[u].x, v[u].x);
                f[u] = fn4[u];
                v[u] = vn4[u];
            }
            ft += 4.0f;
            row += (uint32_t)(4 * P);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += fmaf(f[u], v[u].y - v[u].x, v[u].x);
    }
    for (; t < t1; ++t) {
        float f;
        f32x2u v;
        sample(ft, row, f, v);
        acc += fmaf(f, v.y - v.x, v.x);
        ft += 1.0f;
        row += (uint32_t)P;
    }
    return acc;
}

// SEG threads share a ray, each taking a fixed run of whole chunks of sample
// lines, so the 64 lanes of a wave (64 neighbouring rays of one view, same
// chunk) walk the same sample line together and read neighbouring elements of
// one row of the (transposed) image.
//
// OS mode: the epilogue writes the weighted residual of every ray and, for
// every group of SQ_GROUP consecutive rays, the sum of their squared
// differences (in ray order, FP64); blocks hold whole groups, so the sums do
// not depend on SEG.  The step rule itself runs in the update kernel.
// (Finishing it in the projector's last block instead would need
// every block to write back its XCD's L2 before taking a ticket, which costs
// more than it saves.)
// rblock: first ray (within A's ray range) of this block's 256 / SEG rays.
template <int SEG, bool OS>
__device__ __forceinline__ void fp_body(const FpArgs& A, int rblock)
{
    constexpr int RPB = 256 / SEG;
    const int tid = threadIdx.x;
    const int seg = tid / RPB;
    const int lr = tid - seg * RPB;
    const int r = rblock + lr;
    // The line integral is summed in chunks of `ch` sample lines, each chunk in
    // line order, and the chunk sums are added in chunk order.  Segments cover
    // whole chunks, so the result does not depend on SEG.
    const int ch = 32 * ((A.n + 511) / 512);
    const int nchunk = (A.n + ch - 1) / ch;  // <= 16
    const int cps = (nchunk + SEG - 1) / SEG;  // chunks per segment
    float total = 0.0f;
    // SEG > 1: chunk sums go straight to their LDS slots (chunk, ray)
    __shared__ float red[(SEG == 1) ? 1 : 16][RPB];
    float scale = 0.0f;
    if (r < A.nrays) {
        const int gr = A.ray0 + r;
        const RayMeta m = A.rm[gr];
        const RayGeo g = A.rg[gr];
        scale = m.scale;
        const int lo = (int)(m.packed & 0x7fffu);
        const int hi = (int)((m.packed >> 15) & 0x7fffu);
        const int major = (int)(m.packed >> 30);
        // y-major rays sample rows of the row-major copy, x-major rays rows of
        // the transposed copy (n P floats after it)
        const uint32_t off0 = (major ? 0u : (uint32_t)(A.n * A.P)) + (uint32_t)PAD;
        const int c_begin = seg * cps, c_end = min(nchunk, c_begin + cps);
        for (int c = c_begin; c < c_end; ++c) {
            const int t0 = max(lo, c * ch);
            const int t1 = min(min(hi + 1, (c + 1) * ch), A.n);
            const float acc = chunk_sum(A.img, off0, A.P, A.n, g, t0, t1);
            if constexpr (SEG == 1) {
                total += acc;
            } else {
                red[c][lr] = acc;
            }
        }
    }
    if constexpr (SEG > 1) {
        __syncthreads();
        if (seg == 0) {
            for (int c = 0; c < nchunk; ++c) total += red[c][lr];
        }
    }
    const bool owner = (seg == 0) && (r < A.nrays);
    const int gr = A.ray0 + r;
    const float ell = total * scale;
    if constexpr (!OS) {
        if (owner) {
            const int q = r / A.nch, k = r - q * A.nch;
            const int row = A.natural_rows ? A.views[A.q0 + q].nat_view : q;
            A.out[(size_t)row * A.nch + k] = ell;
        }
    } else {
        __shared__ double sq[RPB];
        if (owner) {
            const float t = expf(-ell);
            A.w[gr] = (t - A.yt[gr]) * scale;
            const float d = ell - A.p[gr];
            sq[lr] = (double)(d * d);
        }
        __syncthreads();
        if (owner && (lr % SQ_GROUP) == 0) {
            double s = 0.0;
            const int nv = min(SQ_GROUP, A.nrays - r);
            for (int u = 0; u < nv; ++u) s += sq[lr + u];
            A.part[r / SQ_GROUP] = s;
        }
    }
}

template <int SEG, bool OS>
__global__ __launch_bounds__(256) void fp_kernel(FpArgs A)
{
    fp_body<SEG, OS>(A, blockIdx.x * (256 / SEG));
}

// A batch of slices: block b projects the rays work[b].r0 ... of slice
// work[b].slice's subset s (OS mode) from image buffer `in`.
template <int SEG>
__global__ __launch_bounds__(256) void fp_batch_kernel(const SliceDesc* __restrict__ slices,
                                                       const FpWork* __restrict__ work, int s, int in)
{
    const FpWork wk = work[blockIdx.x];
    if (wk.slice < 0) return;
    const SliceDesc* __restrict__ D = slices + wk.slice;
    const int2 sq = s >= 0 ? D->subs[s] : make_int2(0, D->geo.nv);
    FpArgs A{};
    A.img = as_global(D->img[in]);
    A.rg = as_global(D->rg);
    A.rm = as_global(D->rm);
    A.ray0 = sq.x * D->geo.nch;
    A.nrays = sq.y * D->geo.nch;
    A.n = D->geo.n;
    A.P = D->geo.P;
    A.nch = D->geo.nch;
    A.yt = as_global(D->yt);
    A.p = as_global(D->p);
    A.w = as_global(D->w);
    A.part = as_global(s >= 0 ? D->part : D->part_all);
    fp_body<SEG, true>(A, wk.r0);
}

template <bool OS>
hipError_t launch_fp(int segments, const FpArgs& a, hipStream_t s)
{
    if (a.nrays <= 0) return hipSuccess;
    switch (segments) {
    case 1: fp_kernel<1, OS><<<cdiv(a.nrays, 256), 256, 0, s>>>(a); break;
    case 2: fp_kernel<2, OS><<<cdiv(a.nrays, 128), 256, 0, s>>>(a); break;
    case 4: fp_kernel<4, OS><<<cdiv(a.nrays, 64), 256, 0, s>>>(a); break;
    case 8: fp_kernel<8, OS><<<cdiv(a.nrays, 32), 256, 0, s>>>(a); break;
    case 16: fp_kernel<16, OS><<<cdiv(a.nrays, 16), 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Iteration state
// ----------------------------------------------------------------------------

__global__ void set_state_kernel(DevState* st, DevState v)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    v.it = 0;
    *st = v;
}

__global__ void flush_hist_kernel(const DevState* st, int M)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const DevState v = *st;
    if (v.fhist && v.n_global >= 1) v.fhist[(v.n_global - 1) % M] = v.f_prev;
}

// Full-data residual: block b of a slice reduces its share of the ray groups
// and of the rays (range b of RES_BLOCKS equal ranges), thread-strided and
// then by a fixed tree over the 256 threads; a second kernel adds the
// RES_BLOCKS range sums in range order.  The order is fixed, so a slice gets
// the same bits alone or in a batch.
__device__ __forceinline__ void residual_range(const double* __restrict__ part, int ngroups,
                                               const float* __restrict__ y, long nrays, int b,
                                               double* __restrict__ dst)
{
    __shared__ double r0[256], r1[256];
    const long k0 = nrays * b / RES_BLOCKS, k1 = nrays * (b + 1) / RES_BLOCKS;
    const int g0 = (int)((long)ngroups * b / RES_BLOCKS), g1 = (int)((long)ngroups * (b + 1) / RES_BLOCKS);
    double s0 = 0.0, s1 = 0.0;
    for (int k = g0 + (int)threadIdx.x; k < g1; k += 256) s0 += part[k];
    for (long k = k0 + threadIdx.x; k < k1; k += 256) s1 += 1.0 / (double)fmaxf(y[k], 1.0f);
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dst[0] = r0[0];
        dst[1] = r1[0];
    }
}

__device__ __forceinline__ void residual_combine(const double* __restrict__ res_part, long nrays,
                                                 double* __restrict__ out)
{
    double s0 = 0.0, s1 = 0.0;
    for (int b = 0; b < RES_BLOCKS; ++b) {
        s0 += res_part[2 * b];
        s1 += res_part[2 * b + 1];
    }
    out[0] = s0 / (double)nrays;
    out[1] = s1 / (double)nrays;
}

__global__ __launch_bounds__(256) void residual_range_kernel(const double* __restrict__ part, int ngroups,
                                                             const float* __restrict__ counts, long nrays,
                                                             double* __restrict__ res_part)
{
    residual_range(part, ngroups, counts, nrays, blockIdx.x, res_part + 2 * blockIdx.x);
}

__global__ void residual_combine_kernel(const double* __restrict__ res_part, long nrays, double* __restrict__ out)
{
    if (threadIdx.x == 0) residual_combine(res_part, nrays, out);
}

// Batched: block (b, i) reduces range b of slice i; then thread i adds slice i's ranges.
__global__ __launch_bounds__(256) void residual_range_batch_kernel(const SliceDesc* __restrict__ slices,
                                                                   const float* const* __restrict__ counts)
{
    const SliceDesc* __restrict__ D = slices + blockIdx.y;
    const long nrays = (long)D->geo.nv * D->geo.nch;
    const int ngroups = (int)((nrays + SQ_GROUP - 1) / SQ_GROUP);
    residual_range(D->part_all, ngroups, counts[blockIdx.y], nrays, blockIdx.x, D->res_part + 2 * blockIdx.x);
}

__global__ void residual_combine_batch_kernel(const SliceDesc* __restrict__ slices, int n_slices,
                                              double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_slices) return;
    const SliceDesc* __restrict__ D = slices + i;
    residual_combine(D->res_part, (long)D->geo.nv * D->geo.nch, out + 2 * i);
}

// Residual over every stride-th subset (subsets 0, stride, 2 stride, ...): the
// projector leaves each chosen subset's squared-difference group sums in the
// slice's subset buffer, one block adds them (thread-strided, then a fixed tree)
// into res_part[2 j] (j = the subset's rank among the chosen ones); the noise
// level sums 1 / max(y, 1) over the chosen views' rows of the counts in
// RES_BLOCKS row ranges into res_part[2 b + 1]; the combine adds both in index
// order.  Alone and in a batch the same functions run in the same order, so a
// slice gets the same bits either way.
__device__ __forceinline__ double block_tree_sum(double s, double* red)
{
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__device__ __forceinline__ void residual_subset_sum(const double* __restrict__ part, int ngroups, double* dst)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < ngroups; k += 256) s += part[k];
    const double t = block_tree_sum(s, red);
    if (threadIdx.x == 0) *dst = t;
}

__device__ __forceinline__ void residual_noise_rows(const float* __restrict__ y, int nv, int nch, int M, int stride,
                                                    int b, double* dst)
{
    __shared__ double red[256];
    const int v0 = (int)((long)nv * b / RES_BLOCKS), v1 = (int)((long)nv * (b + 1) / RES_BLOCKS);
    double s = 0.0;
    for (int v = v0; v < v1; ++v) {
        if ((v % M) % stride != 0) continue;
        for (int k = threadIdx.x; k < nch; k += 256) s += 1.0 / (double)fmaxf(y[(size_t)v * nch + k], 1.0f);
    }
    const double t = block_tree_sum(s, red);
    if (threadIdx.x == 0) *dst = t;
}

__device__ __forceinline__ void residual_strided_combine(const double* __restrict__ res_part, int nchosen, long nrays,
                                                         double* __restrict__ out)
{
    double s0 = 0.0, s1 = 0.0;
    for (int j = 0; j < nchosen; ++j) s0 += res_part[2 * j];
    for (int b = 0; b < RES_BLOCKS; ++b) s1 += res_part[2 * b + 1];
    out[0] = s0 / (double)nrays;
    out[1] = s1 / (double)nrays;
}

__global__ __launch_bounds__(256) void residual_subset_kernel(const double* __restrict__ part, int ngroups,
                                                              double* __restrict__ dst)
{
    residual_subset_sum(part, ngroups, dst);
}

__global__ __launch_bounds__(256) void residual_noise_kernel(const float* __restrict__ y, int nv, int nch, int M,
                                                             int stride, double* __restrict__ res_part)
{
    residual_noise_rows(y, nv, nch, M, stride, blockIdx.x, res_part + 2 * blockIdx.x + 1);
}

__global__ void residual_strided_combine_kernel(const double* __restrict__ res_part, int nchosen, long nrays,
                                                double* __restrict__ out)
{
    if (threadIdx.x == 0) residual_strided_combine(res_part, nchosen, nrays, out);
}

// Batched forms: block i -> slice i (subset s, rank j); block (b, i) -> row range b of slice i.
__global__ __launch_bounds__(256) void residual_subset_batch_kernel(const SliceDesc* __restrict__ slices, int s, int j)
{
    const SliceDesc* __restrict__ D = slices + blockIdx.x;
    const int nrays = D->subs[s].y * D->geo.nch;
    residual_subset_sum(D->part, (nrays + SQ_GROUP - 1) / SQ_GROUP, D->res_part + 2 * j);
}

__global__ __launch_bounds__(256) void residual_noise_batch_kernel(const SliceDesc* __restrict__ slices,
                                                                   const float* const* __restrict__ counts, int M,
                                                                   int stride)
{
    const SliceDesc* __restrict__ D = slices + blockIdx.y;
    residual_noise_rows(counts[blockIdx.y], D->geo.nv, D->geo.nch, M, stride, blockIdx.x,
                        D->res_part + 2 * blockIdx.x + 1);
}

__global__ void residual_strided_combine_batch_kernel(const SliceDesc* __restrict__ slices, int n_slices, int M,
                                                      int stride, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_slices) return;
    const SliceDesc* __restrict__ D = slices + i;
    long nrays = 0;
    int nchosen = 0;
    for (int s = 0; s < M; s += stride, ++nchosen) nrays += (long)D->subs[s].y * D->geo.nch;
    residual_strided_combine(D->res_part, nchosen, nrays, out + 2 * i);
}

// Measurement probe of the read bandwidth the caches deliver to gather kernels:
// every block reads the whole buffer (n16 16-byte words, a power of two) once,
// from a block-dependent start, four independent loads in flight per thread;
// each thread writes its sum so that no load can be dropped.
__global__ __launch_bounds__(256) void read_probe_kernel(const float4* __restrict__ buf, uint32_t n16,
                                                         float* __restrict__ out)
{
    const uint32_t mask = n16 - 1;
    const uint32_t start = (blockIdx.x * 4099u * 256u) & mask;
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (uint32_t e = threadIdx.x; e < n16; e += 4 * 256) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = buf[(start + e + u * 256) & mask];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
}

// Measurement probe of the vector ALU's issue rate for one instruction: every
// thread runs VALU_CHAINS independent chains of VALU_ITERS instructions, each
// written as inline assembly so that the compiler can neither fold nor replace
// it; one value per thread is written so that nothing is dropped.
constexpr int VALU_ITERS = 1024, VALU_CHAINS = 16;
typedef __bf16 probe_bf16x2 __attribute__((ext_vector_type(2)));
template <int OP>
__global__ __launch_bounds__(256) void valu_probe_kernel(const uint32_t* __restrict__ seed, float* __restrict__ out)
{
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    const uint32_t b = seed[t & 255], c = seed[(t + 97) & 255];
    const float bf = __uint_as_float((b & 0x007fffffu) | 0x3f000000u), cf = __uint_as_float((c & 0x007fffffu) | 0x3f000000u);
    const uint64_t b64 = ((uint64_t)b << 32) | c;
    float f[VALU_CHAINS];
    uint32_t u[VALU_CHAINS];
    uint64_t w[VALU_CHAINS];
#pragma unroll
    for (int k = 0; k < VALU_CHAINS; ++k) {
        f[k] = (float)k;
        u[k] = t + k;
        w[k] = (uint64_t)(t + k);
    }
    for (int it = 0; it < VALU_ITERS; ++it) {
#pragma unroll
        for (int k = 0; k < VALU_CHAINS; ++k) {
            if constexpr (OP == 0) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[k]) : "v"(bf), "v"(cf));
            if constexpr (OP == 1) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f[k]) : "v"(bf));
            if constexpr (OP == 2) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[k]) : "v"(b));
            if constexpr (OP == 3) asm volatile("v_cvt_f32_i32 %0, %0" : "+v"(f[k]));
            if constexpr (OP == 4) asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(w[k]) : "v"(b64));
            if constexpr (OP == 5) asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(f[k]) : "v"(b), "v"(c));
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < VALU_CHAINS; ++k) r += f[k] + (float)u[k] + (float)(uint32_t)w[k];
    out[t] = r;
}

}  // namespace

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------

hipError_t launch_valu_probe(int op, const uint32_t* seed, int blocks, float* out, long* instructions, hipStream_t s)
{
    switch (op) {
    case 0: valu_probe_kernel<0><<<blocks, 256, 0, s>>>(seed, out); break;
    case 1: valu_probe_kernel<1><<<blocks, 256, 0, s>>>(seed, out); break;
    case 2: valu_probe_kernel<2><<<blocks, 256, 0, s>>>(seed, out); break;
    case 3: valu_probe_kernel<3><<<blocks, 256, 0, s>>>(seed, out); break;
    case 4: valu_probe_kernel<4><<<blocks, 256, 0, s>>>(seed, out); break;
    case 5: valu_probe_kernel<5><<<blocks, 256, 0, s>>>(seed, out); break;
    default: return hipErrorInvalidValue;
    }
    *instructions = (long)blocks * 4 * VALU_ITERS * VALU_CHAINS;  // wave64 instructions of the probed kind
    return hipGetLastError();
}

hipError_t launch_read_probe(const float* buf, uint32_t n16, int blocks, float* out, hipStream_t s)
{
    if ((n16 & (n16 - 1)) != 0 || n16 < 1024) return hipErrorInvalidValue;
    read_probe_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<const float4*>(buf), n16, out);
    return hipGetLastError();
}

hipError_t launch_pad_image(const float* src, float* dst, float* dstT, int n, int P, hipStream_t s, bool mask_disc)
{
    dim3 grid(cdiv(n, 32), cdiv(n, 32));
    pad_image_kernel<<<grid, 256, 0, s>>>(src, dst, dstT, n, P, mask_disc ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_unpad_image(const float* src, float* dst, int n, int P, hipStream_t s)
{
    unpad_image_kernel<<<cdiv((long)n * n, 256), 256, 0, s>>>(src, dst, n, P);
    return hipGetLastError();
}

hipError_t launch_initial_image(float* dst, int n, float mu0, hipStream_t s)
{
    initial_image_kernel<<<cdiv((long)n * n, 256), 256, 0, s>>>(dst, n, mu0);
    return hipGetLastError();
}

hipError_t launch_prep_counts(const float* counts, const ViewRec* views, int nv, int nch, float i0, float* yt,
                              float* p, hipStream_t s)
{
    prep_counts_kernel<<<cdiv((long)nv * nch, 256), 256, 0, s>>>(counts, views, nv, nch, i0, yt, p);
    return hipGetLastError();
}

hipError_t launch_prepare_batch(const SliceDesc* slices, const BatchRunArgs& a, const DevState& fresh, bool counts,
                                hipStream_t s)
{
    if (a.count < 1 || a.count > BATCH_ARGS) return hipErrorInvalidValue;
    const unsigned count_blocks = counts ? cdiv(a.max_rays, 256) : 1, tiles = cdiv(a.max_n, 32);
    prepare_batch_kernel<<<dim3(count_blocks + tiles * tiles, a.count), 256, 0, s>>>(slices, a, fresh,
                                                                                     (int)count_blocks, counts ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_unpad_batch(const SliceDesc* slices, const BatchRunArgs& a, int in, hipStream_t s)
{
    if (a.count < 1 || a.count > BATCH_ARGS) return hipErrorInvalidValue;
    unpad_batch_kernel<<<dim3(cdiv((long)a.max_n * a.max_n, 256), a.count), 256, 0, s>>>(slices, a, in);
    return hipGetLastError();
}

hipError_t launch_initial_batch(const SliceDesc* slices, const BatchRunArgs& a, hipStream_t s)
{
    if (a.count < 1 || a.count > BATCH_ARGS) return hipErrorInvalidValue;
    initial_batch_kernel<<<dim3(cdiv((long)a.max_n * a.max_n, 256), a.count), 256, 0, s>>>(slices, a);
    return hipGetLastError();
}

hipError_t launch_copy_batch(const BatchCopyArgs& a, long len, hipStream_t s)
{
    if (a.count < 1 || a.count > BATCH_ARGS) return hipErrorInvalidValue;
    if (len <= 0) return hipSuccess;
    copy_batch_kernel<<<dim3(cdiv(len, 256), a.count), 256, 0, s>>>(a, len);
    return hipGetLastError();
}

hipError_t launch_scale_sino(const float* sino, const RayMeta* meta, int ray0, int nrays, int nch,
                             const ViewRec* views, int q0, int natural_rows, float* w, hipStream_t s)
{
    if (nrays <= 0) return hipSuccess;
    scale_sino_kernel<<<cdiv(nrays, 256), 256, 0, s>>>(sino, meta, views, q0, ray0, nrays, nch, natural_rows, w);
    return hipGetLastError();
}

hipError_t launch_fp_plain(const Geo& geo, int segments, const float* img, const float* imgT, const RayGeo* rg,
                           const RayMeta* rm, const ViewRec* views, int q0, int nq, int natural_rows, float* out,
                           hipStream_t s)
{
    FpArgs a{};
    a.img = img;  // imgT is img + n P (one allocation)
    a.rg = rg;
    a.rm = rm;
    a.views = views;
    a.ray0 = q0 * geo.nch;
    a.nrays = nq * geo.nch;
    a.n = geo.n;
    a.P = geo.P;
    a.nch = geo.nch;
    a.q0 = q0;
    a.natural_rows = natural_rows;
    a.out = out;
    return launch_fp<false>(segments, a, s);
}

hipError_t launch_fp_os(const Geo& geo, int segments, const float* img, const float* imgT, const RayGeo* rg,
                        const RayMeta* rm, int ray0, int nrays, const float* yt, const float* p, float* w,
                        double* part, hipStream_t s)
{
    FpArgs a{};
    a.img = img;  // imgT is img + n P (one allocation)
    a.rg = rg;
    a.rm = rm;
    a.ray0 = ray0;
    a.nrays = nrays;
    a.n = geo.n;
    a.P = geo.P;
    a.nch = geo.nch;
    a.yt = yt;
    a.p = p;
    a.w = w;
    a.part = part;
    return launch_fp<true>(segments, a, s);
}

int fp_rays_per_block(int segments) { return 256 / segments; }

hipError_t launch_fp_batch(int segments, const SliceDesc* slices, const FpWork* work, int nblocks, int sub, int in,
                           hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    switch (segments) {
    case 1: fp_batch_kernel<1><<<nblocks, 256, 0, s>>>(slices, work, sub, in); break;
    case 2: fp_batch_kernel<2><<<nblocks, 256, 0, s>>>(slices, work, sub, in); break;
    case 4: fp_batch_kernel<4><<<nblocks, 256, 0, s>>>(slices, work, sub, in); break;
    case 8: fp_batch_kernel<8><<<nblocks, 256, 0, s>>>(slices, work, sub, in); break;
    case 16: fp_batch_kernel<16><<<nblocks, 256, 0, s>>>(slices, work, sub, in); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s)
{
    set_state_kernel<<<1, 64, 0, s>>>(st, v);
    return hipGetLastError();
}

DevState fresh_state(double lambda0)
{
    DevState v{};
    v.lambda = lambda0;
    v.best_f = INFINITY;
    return v;
}

hipError_t launch_flush_hist(const DevState* st, int M, hipStream_t s)
{
    flush_hist_kernel<<<1, 64, 0, s>>>(st, M);
    return hipGetLastError();
}

hipError_t launch_residual_final(const double* part, int ngroups, const float* counts, long nrays, double* res_part,
                                 double* out, hipStream_t s)
{
    residual_range_kernel<<<RES_BLOCKS, 256, 0, s>>>(part, ngroups, counts, nrays, res_part);
    residual_combine_kernel<<<1, 64, 0, s>>>(res_part, nrays, out);
    return hipGetLastError();
}

hipError_t launch_residual_subset(const double* part, int ngroups, double* res_part, int j, hipStream_t s)
{
    residual_subset_kernel<<<1, 256, 0, s>>>(part, ngroups, res_part + 2 * j);
    return hipGetLastError();
}

hipError_t launch_residual_strided_final(const float* counts, int nv, int nch, int M, int stride, int nchosen,
                                         long nrays, double* res_part, double* out, hipStream_t s)
{
    residual_noise_kernel<<<RES_BLOCKS, 256, 0, s>>>(counts, nv, nch, M, stride, res_part);
    residual_strided_combine_kernel<<<1, 64, 0, s>>>(res_part, nchosen, nrays, out);
    return hipGetLastError();
}

hipError_t launch_residual_subset_batch(const SliceDesc* slices, int n_slices, int sub, int j, hipStream_t s)
{
    residual_subset_batch_kernel<<<n_slices, 256, 0, s>>>(slices, sub, j);
    return hipGetLastError();
}

hipError_t launch_residual_strided_final_batch(const SliceDesc* slices, const float* const* counts, int n_slices,
                                               int M, int stride, double* out, hipStream_t s)
{
    residual_noise_batch_kernel<<<dim3(RES_BLOCKS, n_slices), 256, 0, s>>>(slices, counts, M, stride);
    residual_strided_combine_batch_kernel<<<cdiv(n_slices, 64), 64, 0, s>>>(slices, n_slices, M, stride, out);
    return hipGetLastError();
}

hipError_t launch_residual_final_batch(const SliceDesc* slices, const float* const* counts, int n_slices,
                                       double* out, hipStream_t s)
{
    residual_range_batch_kernel<<<dim3(RES_BLOCKS, n_slices), 256, 0, s>>>(slices, counts);
    residual_combine_batch_kernel<<<cdiv(n_slices, 64), 64, 0, s>>>(slices, n_slices, out);
    return hipGetLastError();
}

}  // namespace recon
