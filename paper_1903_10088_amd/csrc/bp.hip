// Gather backprojection, TV gradient and the fused update of Eq. 3 (gfx950).
//
// The backprojector is pixel-driven: every thread owns one pixel and, for each
// view of the subset, enumerates the window of channels whose rays cross the
// pixel's sampling line within one pixel of its centre, adding hat weight x
// path-weighted residual.  It reproduces the projector's weights exactly (same
// lattice/residual arithmetic), so it is the projector's transpose, and it has
// no atomics: each pixel's sum runs in a fixed order (views in turn, channels
// in increasing order) and the result is bitwise deterministic.  Rays in a
// window whose weight is zero add exactly zero, so the window's width (any
// margin) does not change the bits.
//
// Two variants of the candidate reads:
//   STAGE = false  each candidate's ray record and residual come from global
//                  memory (L1/L2 resident);
//   STAGE = true   a 16x16 tile first stages, for a chunk of views, the
//                  channels its pixels can touch into LDS, so the candidate
//                  loop reads LDS; a pixel whose window leaves the staged range
//                  (or a view whose range does not fit) reads global memory.
// Both give identical bits.
#include <hip/hip_runtime.h>

#include "gather.h"
#include "internal.h"

namespace recon {

namespace {

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

constexpr int TILE = 16;
constexpr int STAGE_VIEWS = 8;   // views per LDS chunk
constexpr int UNROLL = 4;        // candidates evaluated without a loop (one pixel per thread)
constexpr int QUAD_UNROLL = 5;   // the same for 2x2 pixels per thread
constexpr int STAGE_GAP = QUAD_UNROLL - 1;  // zero-weight slots after each major-axis part of a staged row
constexpr int STAGE_ROW = STAGE_SLOTS + 2 * STAGE_GAP;
static_assert(STAGE_GAP >= UNROLL - 1, "the padded rows must cover every unrolled candidate");

// Summation order of a pixel's backprojection, shared by every variant: view q
// of the subset belongs to group (q - q0) mod VIEW_GROUPS, each group sums its
// views in increasing order (in a view, the x-major channels and then the
// y-major ones, channels in increasing order), and the groups are added as
// (g0 + g1) + (g2 + g3).  Launch shapes that split the views differently
// therefore give the same bits.  Chunks of staged views start at multiples of
// 4 within the subset, so within a chunk the group of view cq is cq mod 4.
constexpr int VIEW_GROUPS = 4;
static_assert(STAGE_VIEWS % VIEW_GROUPS == 0, "chunks must start at a group boundary");

__device__ __forceinline__ float combine_groups(float a0, float a1, float a2, float a3) { return (a0 + a1) + (a2 + a3); }

// Adds the contributions of channels [lo, hi] (lo <= hi) of one view to acc,
// in increasing channel order.  `t` is the pixel's coordinate along the rays'
// major axis, `c` its coordinate across.  The first UNROLL candidates are
// evaluated unconditionally and masked (their reads must be in bounds:
// read(k) is only called with lo <= k <= lo + UNROLL - 1 or k <= hi); further
// candidates run in a loop.
template <class Read>
__device__ __forceinline__ float add_window(float acc, int lo, int hi, float t, float c, Read read)
{
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        float wk;
        const RayGeo g = read(lo + u, wk);
        const float h = hat(ray_offset(g, t, c));
        acc = (lo + u <= hi) ? fmaf(h, wk, acc) : acc;
    }
    for (int k = lo + UNROLL; k <= hi; ++k) {
        float wk;
        const RayGeo g = read(k, wk);
        acc = fmaf(hat(ray_offset(g, t, c)), wk, acc);
    }
    return acc;
}

// Reads channel k of one view from global memory, clamped into [lo, hi] so the
// masked reads of add_window stay inside the view.
struct GlobalRead {
    const RayGeo* gv;
    const float* wv;
    int hi;
    __device__ __forceinline__ RayGeo operator()(int k, float& wk) const
    {
        const int kk = min(k, hi);
        wk = wv[kk];
        return gv[kk];
    }
};

// Adds channels [lo, hi] (lo <= hi) of one view from its staged LDS row with
// no masking: the first UNROLL candidates are always evaluated.  A candidate
// past hi is either a ray of the same major axis outside the pixel's window,
// whose weight is exactly zero (the window holds every ray with nonzero
// weight), or one of the zero-weight slots that follow each major-axis part of
// the row; either adds exactly zero, so the sum has the bits of the masked
// form.
template <class Read>
__device__ __forceinline__ float add_window_padded(float acc, int lo, int hi, float t, float c, Read read)
{
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        float wk;
        const RayGeo g = read(lo + u, wk);
        acc = fmaf(hat(ray_offset(g, t, c)), wk, acc);
    }
    for (int k = lo + UNROLL; k <= hi; ++k) {
        float wk;
        const RayGeo g = read(k, wk);
        acc = fmaf(hat(ray_offset(g, t, c)), wk, acc);
    }
    return acc;
}

// Reads channel k of one view from its LDS row (slot k - k0).
struct LdsRead {
    const float4* sg;
    const float* sw;
    int k0;
    __device__ __forceinline__ RayGeo operator()(int k, float& wk) const
    {
        const int e = k - k0;
        wk = sw[e];
        const float4 f = sg[e];
        return RayGeo{f.x, f.y, f.z, f.w};
    }
};

// g_L at pixel (i, j) from global memory.
__device__ __forceinline__ float gather_global(const Geo& G, const ViewRec* __restrict__ V,
                                               const RayGeo* __restrict__ rg, const float* __restrict__ w, int q0,
                                               int nq, int i, int j)
{
    const float X = (float)i - G.c, Y = (float)j - G.c;
    const float fi = (float)i, fj = (float)j;
    auto one_view = [&](int q, float acc) {
        const ViewRec v = V[q];
        const PixelView pv = pixel_view(G, v, X, Y);
        int x0, x1, y0, y1;
        major_intervals(v, G.nch, x0, x1, y0, y1);
        if (x0 < x1) {
            int lo, hi;
            candidate_range(pv.kp, pv.hwx, x0, x1, lo, hi);
            if (lo <= hi) acc = add_window(acc, lo, hi, fi, fj, GlobalRead{rg + v.ray0, w + v.ray0, hi});
        }
        if (y0 < y1) {
            int lo, hi;
            candidate_range(pv.kp, pv.hwy, y0, y1, lo, hi);
            if (lo <= hi) acc = add_window(acc, lo, hi, fj, fi, GlobalRead{rg + v.ray0, w + v.ray0, hi});
        }
        return acc;
    };
    float acc[VIEW_GROUPS] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int q = q0; q < q0 + nq; q += VIEW_GROUPS) {
#pragma unroll
        for (int g = 0; g < VIEW_GROUPS; ++g)
            if (q + g < q0 + nq) acc[g] = one_view(q + g, acc[g]);
    }
    return combine_groups(acc[0], acc[1], acc[2], acc[3]);
}

// A staged row holds channels [k0, k0 + cnt) in order, with STAGE_GAP
// zero-weight slots inserted before channel k_split when the range straddles
// it (the boundary between the two major axes) and STAGE_GAP more after the
// last channel: channel k sits in slot k - k0 below k_split and k - kb from it
// on (kb = k0 - STAGE_GAP when there is a gap, else k0).  Rows are double
// buffered: chunk c is read from buffer c & 1 while chunk c + 1's rays are in
// flight from L2.
constexpr int STAGE_TABLE = 64;  // views whose tile models are formed together, one per thread
constexpr int STAGE_LOADS = STAGE_VIEWS * STAGE_SLOTS / 256;  // staged slots per thread and chunk

// Per view, what every pixel reads, packed into three 16-byte records:
// va = (kpc, gx, gy, hwx), vb = (hwy, x-part first and last channel, y-part
// first channel), vc = (y-part last channel, staged count, x-part and y-part
// slot bases); channels as floats for the window clamps.
template <int NB>
struct StageLdsT {
    float4 geo[NB][STAGE_VIEWS][STAGE_ROW];
    float w[NB][STAGE_VIEWS][STAGE_ROW];
    float4 va[STAGE_TABLE];
    float4 vb[STAGE_TABLE];
    int4 vc[STAGE_TABLE];
    int k0[STAGE_TABLE];
    int kb[STAGE_TABLE];
    int cnt[STAGE_TABLE];  // staged channels, 0 = view not staged
    int ray0[STAGE_TABLE];
    int ks[STAGE_TABLE];
};
typedef StageLdsT<2> StageLds;   // double-buffered rows (block-wide staging)
typedef StageLdsT<1> StageLdsQ;  // single-buffered rows (per-wave staging)

// One thread's share of a chunk's staged rays, held in registers between the
// load and the LDS store.
struct StagePrefetch {
    float4 g[STAGE_LOADS];
    float w[STAGE_LOADS];
    int slot[STAGE_LOADS];  // row slot, -1 = nothing to store
};

// Loads this thread's slots of the chunk of views [t0, t0 + cv) of the table.
__device__ __forceinline__ void stage_load(const StageLds& S, const RayGeo* __restrict__ rg,
                                           const float* __restrict__ w, int t0, int cv, StagePrefetch& P)
{
#pragma unroll
    for (int r = 0; r < STAGE_LOADS; ++r) {
        const int sl = threadIdx.x + 256 * r;
        const int cq = sl / STAGE_SLOTS, e = sl - cq * STAGE_SLOTS;
        P.slot[r] = -1;
        if (cq < cv) {
            const int t = t0 + cq;
            if (e < S.cnt[t]) {
                const int k = S.k0[t] + e;
                const RayGeo g = rg[S.ray0[t] + k];
                P.g[r] = make_float4(g.a_int, g.a_frac, g.s_hi, g.s_lo);
                P.w[r] = w[S.ray0[t] + k];
                P.slot[r] = cq * STAGE_ROW + (k < S.ks[t] ? e : k - S.kb[t]);
            }
        }
    }
}

// Stores the prefetched slots into buffer b and writes the zero-weight slots.
__device__ __forceinline__ void stage_store(StageLds& S, int b, int t0, int cv, const StagePrefetch& P)
{
    float4* geo = &S.geo[b][0][0];
    float* wr = &S.w[b][0][0];
#pragma unroll
    for (int r = 0; r < STAGE_LOADS; ++r)
        if (P.slot[r] >= 0) {
            geo[P.slot[r]] = P.g[r];
            wr[P.slot[r]] = P.w[r];
        }
    const int tid = threadIdx.x;
    if (tid < cv * 2 * STAGE_GAP) {
        const int cq = tid / (2 * STAGE_GAP), m = tid - cq * (2 * STAGE_GAP);
        const int t = t0 + cq;
        const int k0 = S.k0[t], kb = S.kb[t], cnt = S.cnt[t];
        int pos = -1;
        if (cnt > 0) {
            if (m < STAGE_GAP)
                pos = cnt + (k0 - kb) + m;
            else if (kb != k0)
                pos = S.ks[t] - k0 + (m - STAGE_GAP);
        }
        if (pos >= 0) {
            S.geo[b][cq][pos] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            S.w[b][cq][pos] = 0.0f;
        }
    }
}

// Per-wave staging for a reader that is one wave per view group: wave g reads
// only views cq = g and g + VIEW_GROUPS of a chunk, so it stages exactly those
// rows itself (lane l holds slot l of each: STAGE_SLOTS = 64) and no other wave
// touches them.  Between its store and its reads the wave needs no block
// barrier: LDS operations of one wave are performed in order, and wave_sync
// keeps the compiler from moving the reads above the stores.
static_assert(STAGE_SLOTS == 64 && STAGE_VIEWS == 2 * VIEW_GROUPS, "per-wave staging: one slot per lane, two views");
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class SL>
__device__ __forceinline__ void stage_load_wave(const SL& S, const RayGeo* __restrict__ rg,
                                                const float* __restrict__ w, int t0, int cv, int grp,
                                                StagePrefetch& P)
{
    const int e = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int cq = grp + VIEW_GROUPS * r;
        P.slot[r] = -1;
        if (cq < cv) {
            const int t = t0 + cq;
            if (e < S.cnt[t]) {
                const int k = S.k0[t] + e;
                const RayGeo g = rg[S.ray0[t] + k];
                P.g[r] = make_float4(g.a_int, g.a_frac, g.s_hi, g.s_lo);
                P.w[r] = w[S.ray0[t] + k];
                P.slot[r] = cq * STAGE_ROW + (k < S.ks[t] ? e : k - S.kb[t]);
            }
        }
    }
}

template <class SL>
__device__ __forceinline__ void stage_store_wave(SL& S, int b, int t0, int cv, int grp, const StagePrefetch& P)
{
    float4* geo = &S.geo[b][0][0];
    float* wr = &S.w[b][0][0];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (P.slot[r] >= 0) {
            geo[P.slot[r]] = P.g[r];
            wr[P.slot[r]] = P.w[r];
        }
    const int lane = threadIdx.x & 63;
    if (lane < 2 * 2 * STAGE_GAP) {
        const int cq = grp + VIEW_GROUPS * (lane / (2 * STAGE_GAP)), m = lane % (2 * STAGE_GAP);
        if (cq < cv) {
            const int t = t0 + cq;
            const int k0 = S.k0[t], kb = S.kb[t], cnt = S.cnt[t];
            int pos = -1;
            if (cnt > 0) {
                if (m < STAGE_GAP)
                    pos = cnt + (k0 - kb) + m;
                else if (kb != k0)
                    pos = S.ks[t] - k0 + (m - STAGE_GAP);
            }
            if (pos >= 0) {
                S.geo[b][cq][pos] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                S.w[b][cq][pos] = 0.0f;
            }
        }
    }
}

// Table of views [s0, s0 + sn) for the tile centred at (Xc, Yc), one view per
// thread: each view's linear channel model over the tile, the channel range
// that holds every pixel's window, and the window half-widths, widened by the
// model's spread over a PX x PY block of pixels when a thread owns such a
// block.  The slot bases put the part from k_split on behind the gap.
template <class SL>
__device__ __forceinline__ void stage_table(SL& S, const Geo& G, const ViewRec* __restrict__ V, int s0, int sn,
                                            float Xc, float Yc, int PX, int PY)
{
    const int tid = threadIdx.x;
    if (tid < sn) {
        const ViewRec v = V[s0 + tid];
        const TileView tv = tile_view(G, v, Xc, Yc);
        int k0, cnt;
        stage_range(tv, G.nch, STAGE_SLOTS, k0, cnt);
        const bool gap = k0 < v.k_split && v.k_split < k0 + cnt;
        const int kb = gap ? k0 - STAGE_GAP : k0;
        int x0, x1, y0, y1;
        major_intervals(v, G.nch, x0, x1, y0, y1);
        float hwx = tv.hwx, hwy = tv.hwy;
        if (PX * PY > 1) {
            const float spread = block_spread(tv, PX, PY);
            hwx = tv.hwx + spread;
            hwy = tv.hwy + spread;
        }
        S.va[tid] = make_float4(tv.kpc, tv.gx, tv.gy, hwx);
        S.vb[tid] = make_float4(hwy, (float)x0, (float)(x1 - 1), (float)y0);
        S.vc[tid] = make_int4(__float_as_int((float)(y1 - 1)), cnt, x0 == v.k_split ? kb : k0,
                              y0 == v.k_split ? kb : k0);
        S.k0[tid] = k0;
        S.kb[tid] = kb;
        S.cnt[tid] = cnt;
        S.ray0[tid] = v.ray0;
        S.ks[tid] = v.k_split;
    }
}

// g_L at pixel (i, j) of a 16x16 tile with LDS staging.  Must be called by all
// 256 threads of the block (it has barriers); `inside` marks real pixels.
__device__ __forceinline__ float gather_staged(StageLds& S, const Geo& G, const ViewRec* __restrict__ V,
                                               const RayGeo* __restrict__ rg, const float* __restrict__ w, int q0,
                                               int nq, int i, int j, bool inside, int ti0, int tj0)
{
    const float fi = (float)i, fj = (float)j;
    // offsets from the tile centre (exact in float32)
    const float dX = (float)(i - ti0) - 7.5f, dY = (float)(j - tj0) - 7.5f;
    const float Xc = (float)ti0 + 7.5f - G.c, Yc = (float)tj0 + 7.5f - G.c;
    float acc[VIEW_GROUPS] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int s0 = q0; s0 < q0 + nq; s0 += STAGE_TABLE) {
        const int sn = min(STAGE_TABLE, q0 + nq - s0);
        stage_table(S, G, V, s0, sn, Xc, Yc, 1, 1);
        __syncthreads();
        StagePrefetch P;
        stage_load(S, rg, w, 0, min(STAGE_VIEWS, sn), P);
        for (int t0 = 0, b = 0; t0 < sn; t0 += STAGE_VIEWS, b ^= 1) {
            const int cv = min(STAGE_VIEWS, sn - t0);
            // buffer b was last read by chunk t0 - 2, before the previous barrier
            stage_store(S, b, t0, cv, P);
            __syncthreads();
            if (t0 + STAGE_VIEWS < sn) stage_load(S, rg, w, t0 + STAGE_VIEWS, min(STAGE_VIEWS, sn - t0 - STAGE_VIEWS), P);
            // one view of the chunk (a full chunk is unrolled, so the table
            // reads of later views can be issued ahead of earlier views' work)
            auto view = [&](int cq, float& acc) {
                const int t = t0 + cq;
                const ViewRec v = V[s0 + t];
                const float4 va = S.va[t], vb = S.vb[t];
                const int4 vc = S.vc[t];
                const int cnt = vc.y;
                const float kp = fmaf(va.y, dX, fmaf(va.z, dY, va.x));
                int x0, x1, y0, y1;
                major_intervals(v, G.nch, x0, x1, y0, y1);
                const int bx = vc.z, by = vc.w;
                if (x0 < x1) {
                    int lo, hi;
                    candidate_range_f(kp, va.w, vb.y, vb.z, lo, hi);
                    if (lo <= hi) {
                        if (cnt > 0)  // every window lies in the staged range (stage_range)
                            acc = add_window_padded(acc, lo, hi, fi, fj, LdsRead{S.geo[b][cq], S.w[b][cq], bx});
                        else
                            acc = add_window(acc, lo, hi, fi, fj, GlobalRead{rg + v.ray0, w + v.ray0, hi});
                    }
                }
                if (y0 < y1) {
                    int lo, hi;
                    candidate_range_f(kp, vb.x, vb.w, __int_as_float(vc.x), lo, hi);
                    if (lo <= hi) {
                        if (cnt > 0)
                            acc = add_window_padded(acc, lo, hi, fj, fi, LdsRead{S.geo[b][cq], S.w[b][cq], by});
                        else
                            acc = add_window(acc, lo, hi, fj, fi, GlobalRead{rg + v.ray0, w + v.ray0, hi});
                    }
                }
            };
            if (inside) {
                if (cv == STAGE_VIEWS) {
#pragma unroll
                    for (int cq = 0; cq < STAGE_VIEWS; ++cq) view(cq, acc[cq % VIEW_GROUPS]);
                } else {
#pragma unroll
                    for (int cq = 0; cq < STAGE_VIEWS; ++cq)
                        if (cq < cv) view(cq, acc[cq % VIEW_GROUPS]);
                }
            }
        }
        __syncthreads();  // the table and both buffers are rewritten by the next group of views
    }
    return combine_groups(acc[0], acc[1], acc[2], acc[3]);
}

// ----------------------------------------------------------------------------
// Blocked gather: each thread owns PX x PY pixels of a 16x16 tile
// ----------------------------------------------------------------------------

// One window of channels serves the whole pixel block: the tile's linear
// channel model at the block's centre, widened by the model's spread over the
// block.  For every candidate the lattice and residual parts of the crossing
// are formed once per sampling line of the block and each pixel gets
// hat(...) x w exactly as in the one-pixel gather, so every pixel's sum has
// the same terms in the same order (rays of the window that miss a pixel add
// exactly zero).  The rows are staged once per chunk (no double buffer: a
// tile's LDS is shared by fewer waves here) with BLK_GAP zero-weight slots
// after each major-axis part, so the unrolled candidates need no mask.
constexpr int BLK_UNROLL = 6;
constexpr int BLK_GAP = BLK_UNROLL - 1;
constexpr int BLK_ROW = STAGE_SLOTS + 2 * BLK_GAP;

struct StageLdsBlk {
    float4 geo[STAGE_VIEWS][BLK_ROW];
    float w[STAGE_VIEWS][BLK_ROW];
    TileView tv[STAGE_TABLE];
    int k0[STAGE_TABLE];
    int kb[STAGE_TABLE];
    int cnt[STAGE_TABLE];
    int ray0[STAGE_TABLE];
    int ks[STAGE_TABLE];
};

// Adds channels [lo, hi] (lo <= hi) of one view to the block's accumulators.
// MAJ_X: rays sampled per column (t = column, centre = row) or per row.
// MASK: candidates past hi get w = 0 (global reads, clamped into [lo, hi]);
// without it they must be zero-weight rays or slots (the padded LDS rows).
template <int PX, int PY, bool MAJ_X, bool MASK, int NU = BLK_UNROLL, class Read>
__device__ __forceinline__ void add_window_blk(float (&acc)[PY][PX], int lo, int hi, int i0, int j0, Read read)
{
    constexpr int NT = MAJ_X ? PX : PY;  // sampling lines in the block
    constexpr int NC = MAJ_X ? PY : PX;  // pixels per sampling line
    auto body = [&](int k, bool valid) {
        float wk;
        const RayGeo g = read(k, wk);
        if constexpr (MASK) wk = valid ? wk : 0.0f;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const float t = (float)((MAJ_X ? i0 : j0) + a);
            const float lat = fmaf(t, g.s_hi, g.a_int);
            const float res = fmaf(t, g.s_lo, g.a_frac);
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const float c = (float)((MAJ_X ? j0 : i0) + b);
                const float h = hat((lat - c) + res);
                float& A = MAJ_X ? acc[b][a] : acc[a][b];
                A = fmaf(h, wk, A);
            }
        }
    };
#pragma unroll
    for (int u = 0; u < NU; ++u) body(lo + u, lo + u <= hi);
    for (int k = lo + NU; k <= hi; ++k) body(k, true);
}

// Global reads for the blocked gather, clamped into [lo, hi].
struct GlobalReadBlk {
    const RayGeo* gv;
    const float* wv;
    int hi;
    __device__ __forceinline__ RayGeo operator()(int k, float& wk) const
    {
        const int kk = min(k, hi);
        wk = wv[kk];
        return gv[kk];
    }
};

template <int PX, int PY>
__device__ __forceinline__ void gather_block(StageLdsBlk& S, const Geo& G, const ViewRec* __restrict__ V,
                                             const RayGeo* __restrict__ rg, const float* __restrict__ w, int q0,
                                             int nq, int i0, int j0, bool active,
                                             float (&acc)[VIEW_GROUPS][PY][PX], int ti0, int tj0)
{
    const int tid = threadIdx.x;
    constexpr int NTH = 256 / (PX * PY);
    static_assert(NTH >= STAGE_TABLE, "one thread per table view");
    // the block centre's offsets from the tile centre, and the model's half-spread over the block
    const float dXb = (float)(i0 - ti0) + 0.5f * (PX - 1) - 7.5f;
    const float dYb = (float)(j0 - tj0) + 0.5f * (PY - 1) - 7.5f;
    const float Xc = (float)ti0 + 7.5f - G.c, Yc = (float)tj0 + 7.5f - G.c;
    for (int s0 = q0; s0 < q0 + nq; s0 += STAGE_TABLE) {
        const int sn = min(STAGE_TABLE, q0 + nq - s0);
        if (tid < sn) {
            const ViewRec v = V[s0 + tid];
            const TileView tv = tile_view(G, v, Xc, Yc);
            int k0, cnt;
            stage_range(tv, G.nch, STAGE_SLOTS, k0, cnt);
            const bool gap = k0 < v.k_split && v.k_split < k0 + cnt;
            S.tv[tid] = tv;
            S.k0[tid] = k0;
            S.kb[tid] = gap ? k0 - BLK_GAP : k0;
            S.cnt[tid] = cnt;
            S.ray0[tid] = v.ray0;
            S.ks[tid] = v.k_split;
        }
        __syncthreads();
        for (int t0 = 0; t0 < sn; t0 += STAGE_VIEWS) {
            const int cv = min(STAGE_VIEWS, sn - t0);
            for (int sl = tid; sl < cv * STAGE_SLOTS; sl += NTH) {
                const int cq = sl / STAGE_SLOTS, e = sl - cq * STAGE_SLOTS;
                const int t = t0 + cq;
                if (e < S.cnt[t]) {
                    const int k = S.k0[t] + e;
                    const RayGeo g = rg[S.ray0[t] + k];
                    const int pos = k < S.ks[t] ? e : k - S.kb[t];
                    S.geo[cq][pos] = make_float4(g.a_int, g.a_frac, g.s_hi, g.s_lo);
                    S.w[cq][pos] = w[S.ray0[t] + k];
                }
            }
            for (int z = tid; z < cv * 2 * BLK_GAP; z += NTH) {
                const int cq = z / (2 * BLK_GAP), m = z - cq * (2 * BLK_GAP);
                const int t = t0 + cq;
                const int k0 = S.k0[t], kb = S.kb[t], cnt = S.cnt[t];
                int pos = -1;
                if (cnt > 0) {
                    if (m < BLK_GAP)
                        pos = cnt + (k0 - kb) + m;
                    else if (kb != k0)
                        pos = S.ks[t] - k0 + (m - BLK_GAP);
                }
                if (pos >= 0) {
                    S.geo[cq][pos] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    S.w[cq][pos] = 0.0f;
                }
            }
            __syncthreads();
            // views of the chunk in groups of VIEW_GROUPS, each into its group's accumulators
            auto view = [&](int cq, float (&a)[PY][PX]) {
                    const int t = t0 + cq;
                    const ViewRec v = V[s0 + t];
                    const int cnt = S.cnt[t];
                    const TileView tv = S.tv[t];
                    const float kp = fmaf(tv.gx, dXb, fmaf(tv.gy, dYb, tv.kpc));
                    const float spread = block_spread(tv, PX, PY);
                    int x0, x1, y0, y1;
                    major_intervals(v, G.nch, x0, x1, y0, y1);
                    const int bx = x0 == v.k_split ? S.kb[t] : S.k0[t];
                    const int by = y0 == v.k_split ? S.kb[t] : S.k0[t];
                    if (x0 < x1) {
                        int lo, hi;
                        candidate_range(kp, tv.hwx + spread, x0, x1, lo, hi);
                        if (lo <= hi) {
                            if (cnt > 0)  // every window lies in the staged range (stage_range)
                                add_window_blk<PX, PY, true, false>(a, lo, hi, i0, j0,
                                                                    LdsRead{S.geo[cq], S.w[cq], bx});
                            else
                                add_window_blk<PX, PY, true, true>(a, lo, hi, i0, j0,
                                                                   GlobalReadBlk{rg + v.ray0, w + v.ray0, hi});
                        }
                    }
                    if (y0 < y1) {
                        int lo, hi;
                        candidate_range(kp, tv.hwy + spread, y0, y1, lo, hi);
                        if (lo <= hi) {
                            if (cnt > 0)
                                add_window_blk<PX, PY, false, false>(a, lo, hi, i0, j0,
                                                                     LdsRead{S.geo[cq], S.w[cq], by});
                            else
                                add_window_blk<PX, PY, false, true>(a, lo, hi, i0, j0,
                                                                    GlobalReadBlk{rg + v.ray0, w + v.ray0, hi});
                        }
                    }
            };
            if (active) {
                for (int c0 = 0; c0 < cv; c0 += VIEW_GROUPS) {
#pragma unroll
                    for (int g = 0; g < VIEW_GROUPS; ++g)
                        if (c0 + g < cv) view(c0 + g, acc[g]);
                }
            }
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------
// 2x2 pixels per lane, one view group per wave
// ----------------------------------------------------------------------------

// The four waves of a block share a 16x16 tile and its staged rows; lane l
// owns the 2x2 block of pixels at (2 (l mod 8), 2 (l / 8)) of the tile and wave
// g sums the views of group g (views g and g + 4 of every chunk).  Per view and
// major axis one window of channels serves the lane's four pixels (the tile
// model at the block centre, widened by its spread over the block), and per
// candidate the lattice and residual parts of the crossing are formed once per
// sampling line of the block: a quarter of the window set-ups and half of the
// crossing arithmetic of one pixel per thread, with as many waves per tile.
// acc[b][a] receives group g's sum for pixel (2 (l mod 8) + a, 2 (l / 8) + b).
// Each wave stages its own rows in one buffer: a chunk's rows are overwritten
// only after the wave has read them (its LDS operations are performed in order).
// Returns after a block barrier, so S is free for other use afterwards.
__device__ __forceinline__ void gather_quad(StageLdsQ& S, const Geo& G, const ViewRec* __restrict__ V,
                                            const RayGeo* __restrict__ rg, const float* __restrict__ w, int q0,
                                            int nq, int ti0, int tj0, float (&acc)[2][2])
{
    // the wave's group, read into a scalar register: views, their records and the
    // branches on them are then wave-uniform to the compiler too
    const int lane = threadIdx.x & 63, grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bxl = 2 * (lane & 7), byl = 2 * (lane >> 3);
    const int i0 = ti0 + bxl, j0 = tj0 + byl;
    const bool active = i0 < G.n && j0 < G.n;
    // the block centre's offsets from the tile centre (exact in float32)
    const float dXb = (float)bxl + 0.5f - 7.5f, dYb = (float)byl + 0.5f - 7.5f;
    const float Xc = (float)ti0 + 7.5f - G.c, Yc = (float)tj0 + 7.5f - G.c;
    for (int s0 = q0; s0 < q0 + nq; s0 += STAGE_TABLE) {
        const int sn = min(STAGE_TABLE, q0 + nq - s0);
        stage_table(S, G, V, s0, sn, Xc, Yc, 2, 2);
        __syncthreads();
        StagePrefetch P;
        stage_load_wave(S, rg, w, 0, min(STAGE_VIEWS, sn), grp, P);
        for (int t0 = 0; t0 < sn; t0 += STAGE_VIEWS) {
            const int cv = min(STAGE_VIEWS, sn - t0);
            constexpr int b = 0;
            // this wave's rows were last read by its own previous chunk
            stage_store_wave(S, b, t0, cv, grp, P);
            wave_sync();
            if (t0 + STAGE_VIEWS < sn)
                stage_load_wave(S, rg, w, t0 + STAGE_VIEWS, min(STAGE_VIEWS, sn - t0 - STAGE_VIEWS), grp, P);
            // view cq of the chunk (wave-uniform)
            auto view = [&](int cq) {
                const int t = t0 + cq;
                const ViewRec v = V[s0 + t];
                const float4 va = S.va[t], vb = S.vb[t];
                const int4 vc = S.vc[t];
                const int cnt = vc.y;
                const float kp = fmaf(va.y, dXb, fmaf(va.z, dYb, va.x));
                int x0, x1, y0, y1;
                major_intervals(v, G.nch, x0, x1, y0, y1);
                if (x0 < x1) {
                    int lo, hi;
                    // (integer clamps of candidate_range: the same window for finite kp)
                    lo = max((int)ceilf(kp - va.w), x0);
                    hi = min((int)floorf(kp + va.w), x1 - 1);
                    if (lo <= hi) {
                        if (cnt > 0)  // every window lies in the staged range (stage_range)
                            add_window_blk<2, 2, true, false, QUAD_UNROLL>(acc, lo, hi, i0, j0,
                                                                           LdsRead{S.geo[b][cq], S.w[b][cq], vc.z});
                        else
                            add_window_blk<2, 2, true, true, QUAD_UNROLL>(acc, lo, hi, i0, j0,
                                                                          GlobalReadBlk{rg + v.ray0, w + v.ray0, hi});
                    }
                }
                if (y0 < y1) {
                    int lo, hi;
                    lo = max((int)ceilf(kp - vb.x), y0);
                    hi = min((int)floorf(kp + vb.x), y1 - 1);
                    if (lo <= hi) {
                        if (cnt > 0)
                            add_window_blk<2, 2, false, false, QUAD_UNROLL>(acc, lo, hi, i0, j0,
                                                                            LdsRead{S.geo[b][cq], S.w[b][cq], vc.w});
                        else
                            add_window_blk<2, 2, false, true, QUAD_UNROLL>(acc, lo, hi, i0, j0,
                                                                           GlobalReadBlk{rg + v.ray0, w + v.ray0, hi});
                    }
                }
            };
            if (active) {
                if (grp < cv) view(grp);
                if (grp + VIEW_GROUPS < cv) view(grp + VIEW_GROUPS);
            }
            wave_sync();  // this chunk's reads of the rows come before the next chunk's stores
        }
        __syncthreads();  // the table and both buffers are rewritten by the next group of views
    }
}

__global__ __launch_bounds__(256) void bp_plain_kernel(Geo G, const ViewRec* __restrict__ V,
                                                       const RayGeo* __restrict__ rg, const float* __restrict__ w,
                                                       int q0, int nq, float* __restrict__ out)
{
    const int i = blockIdx.x * TILE + (threadIdx.x & 15);
    const int j = blockIdx.y * TILE + (threadIdx.x >> 4);
    if (i >= G.n || j >= G.n) return;
    out[(size_t)j * G.n + i] = gather_global(G, V, rg, w, q0, nq, i, j);
}

// -dTV/dmu at pixel (i, j) from a tile s holding mu with a one-pixel halo
// (local position (lx, ly)).  Differences past the last column / row are zero.
template <int W>
__device__ __forceinline__ float tv_neg_grad(const float (*s)[W], int lx, int ly, int i, int j, int n, float eps)
{
    const float e2 = eps * eps;
    const float c = s[ly][lx];
    const bool has_r = i + 1 < n, has_d = j + 1 < n;
    const float dx = has_r ? s[ly][lx + 1] - c : 0.0f;
    const float dy = has_d ? s[ly + 1][lx] - c : 0.0f;
    float d = -(dx + dy) / sqrtf(fmaf(dx, dx, fmaf(dy, dy, e2)));
    if (i > 0) {
        const float l = s[ly][lx - 1];
        const float dxl = c - l;
        const float dyl = has_d ? s[ly + 1][lx - 1] - l : 0.0f;
        d += dxl / sqrtf(fmaf(dxl, dxl, fmaf(dyl, dyl, e2)));
    }
    if (j > 0) {
        const float u = s[ly - 1][lx];
        const float dyu = c - u;
        const float dxu = has_r ? s[ly - 1][lx + 1] - u : 0.0f;
        d += dyu / sqrtf(fmaf(dxu, dxu, fmaf(dyu, dyu, e2)));
    }
    return -d;
}

__global__ __launch_bounds__(256) void tv_grad_kernel(const float* __restrict__ img, float* __restrict__ grad, int n,
                                                      float eps)
{
    __shared__ float s[TILE + 2][TILE + 3];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.x * TILE + tx, j = blockIdx.y * TILE + ty;
    for (int e = threadIdx.x; e < (TILE + 2) * (TILE + 2); e += 256) {
        const int ly = e / (TILE + 2), lx = e - ly * (TILE + 2);
        const int gj = blockIdx.y * TILE + ly - 1, gi = blockIdx.x * TILE + lx - 1;
        s[ly][lx] = (gj >= 0 && gj < n && gi >= 0 && gi < n) ? img[(size_t)gj * n + gi] : 0.0f;
    }
    __syncthreads();
    if (i >= n || j >= n) return;
    grad[(size_t)j * n + i] = tv_neg_grad<TILE + 3>(s, tx + 1, ty + 1, i, j, n, eps);
}

// Sum of part[0..n) in a fixed order defined on 256 virtual lanes: lane v adds
// part[v], part[v + 256], ... in turn; each group of 64 lanes combines its sums
// by an xor butterfly (addition commutes, so every lane holds the same bits);
// the four group sums are added as (g0 + g1) + (g2 + g3).  A block of NTH
// threads plays 256 / NTH virtual lanes per thread, so every block size gives
// the same bits.
template <int NTH>
__device__ double block_sum(const double* __restrict__ part, int n, double* red)
{
    constexpr int NV = 256 / NTH;
    const int tid = threadIdx.x;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
        int r = tid + v * NTH;
        for (; r + 3 * 256 < n; r += 4 * 256) {
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = part[r + u * 256];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += x[u];
        }
        for (; r < n; r += 256) acc += part[r];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
        s[v] = acc;
    }
    if ((tid & 63) == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) red[(tid + v * NTH) >> 6] = s[v];
    }
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Step rule of Eqs. 4-5 with the floor: lambda_0 at n = 0, else +inc when
// f_n < f_ref (strictly), -dec otherwise; a replay schedule overrides it.
// f_ref is the previous sub-iteration's f, or with `compare` (from the second
// epoch on) the same subset's f one epoch earlier (fhist; with M = 1 that is
// the previous sub-iteration again).  keep: this sub-iteration ends an epoch
// whose summed f is below every earlier epoch's (section 4.B), and a kept
// image is wanted.
struct StepDecision {
    double lam;
    bool keep;
};

__device__ __forceinline__ StepDecision step_rule(const DevState& in, const StepRule& R, double f)
{
    StepDecision d;
    if (in.n_global == 0) {
        d.lam = R.lambda0;
    } else {
        const bool same_subset = R.compare && R.M > 1 && in.n_global >= R.M;
        const double f_ref = same_subset ? in.fhist[in.n_global % R.M] : in.f_prev;
        d.lam = (f < f_ref) ? in.lambda + R.inc : in.lambda - R.dec;
        if (d.lam < R.lmin) d.lam = R.lmin;
    }
    if (in.schedule) d.lam = in.schedule[in.it];
    d.keep = in.best != nullptr && (in.n_global + 1) % R.M == 0 && in.epoch_sum + f < in.best_f;
    return d;
}

// The next state after sub-iteration in.n_global (written by one thread):
// trace row, the one-late history entry, the epoch sum and the least one.
__device__ __forceinline__ void record_state(const DevState& in, const StepRule& R, double f, double lam,
                                             DevState* st_out)
{
    DevState out = in;
    if (!isfinite(f)) out.flags |= 1;
    if (in.trace) {
        in.trace[2 * in.it] = f;
        in.trace[2 * in.it + 1] = lam;
    }
    // slot (n - 1) mod M differs from the slot n mod M that step_rule reads when M > 1
    if (in.fhist && in.n_global >= 1) in.fhist[(in.n_global - 1) % R.M] = in.f_prev;
    if ((in.n_global + 1) % R.M == 0) {
        const double e = in.epoch_sum + f;
        if (e < in.best_f) {
            out.best_f = e;
            out.best_n = in.n_global + 1;
        }
        out.epoch_sum = 0.0;
    } else {
        out.epoch_sum = in.epoch_sum + f;
    }
    out.lambda = lam;
    out.f_prev = f;
    out.n_global = in.n_global + 1;
    out.it = in.it + 1;
    *st_out = out;
}

struct UpdateScalars {
    int q0, nq, nrays;
    StepRule rule;
    UpdateConst uc;
};

// Fused step rule + backprojection + TV + update (Eq. 3):
//   f_n = mean squared difference of the subset, lambda_n from the step rule,
//   mu' = mask * max(0, mu + lambda_n (c_l g_L + c_r g_R)), all terms at mu^(n);
// writes both the row-major and the transposed padded copies of mu'.  Every
// block evaluates the step rule from the same inputs in the same order, so all
// use the same lambda_n; the block of the first tile records it in the output
// state.  (ti0, tj0) is the tile's first pixel.
template <bool STAGE>
__device__ __forceinline__ void bp_update_tile(Geo G, const ViewRec* __restrict__ V, const RayGeo* __restrict__ rg,
                                               const float* __restrict__ w, const double* __restrict__ part,
                                               const DevState* __restrict__ st_in, DevState* __restrict__ st_out,
                                               const float* __restrict__ img, float* __restrict__ img_out,
                                               float* __restrict__ imgT_out, UpdateScalars sc, int ti0, int tj0,
                                               const DevState* __restrict__ st_pre)
{
    __shared__ float s[TILE + 2][TILE + 3];
    __shared__ float t[TILE][TILE + 1];
    __shared__ double red[4];
    // each wave takes an 8x8 quadrant of the tile, whose pixels span fewer
    // channels of a view than a 16x4 strip
    const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
    const int tx = (lane & 7) + 8 * (wq & 1), ty = (lane >> 3) + 8 * (wq >> 1);
    const int i = ti0 + tx, j = tj0 + ty;

    for (int e = threadIdx.x; e < (TILE + 2) * (TILE + 2); e += 256) {
        const int ly = e / (TILE + 2), lx = e - ly * (TILE + 2);
        const int gj = tj0 + ly - 1, gi = ti0 + lx - 1;
        // columns -1 and n sit in the zero padding; rows -1 and n are outside the buffer
        s[ly][lx] = (gj >= 0 && gj < G.n && gi < G.n + PAD) ? img[(size_t)gj * G.P + gi + PAD] : 0.0f;
    }
    const bool inside = i < G.n && j < G.n;
    float gl = 0.0f;
    if constexpr (STAGE) {
        __shared__ StageLds S;
        gl = gather_staged(S, G, V, rg, w, sc.q0, sc.nq, i, j, inside, ti0, tj0);  // contains barriers
    } else {
        __syncthreads();
        if (inside) gl = gather_global(G, V, rg, w, sc.q0, sc.nq, i, j);
    }

    // step rule (needed only for the update, so its loads overlap other waves' gathers),
    // unless a step kernel has already taken it (st_pre: the new state)
    StepDecision dec{0.0, false};
    DevState in{};
    if (st_pre) {
        dec.lam = st_pre->lambda;
    } else {
        const double f = block_sum<256>(part, (sc.nrays + SQ_GROUP - 1) / SQ_GROUP, red) / (double)sc.nrays;
        in = *st_in;
        dec = step_rule(in, sc.rule, f);
        if (ti0 == 0 && tj0 == 0 && threadIdx.x == 0) record_state(in, sc.rule, f, dec.lam, st_out);
    }
    const float lam = (float)dec.lam;

    float mu_new = 0.0f;
    if (inside) {
        const float gr = tv_neg_grad<TILE + 3>(s, tx + 1, ty + 1, i, j, G.n, sc.uc.eps);
        const float v = s[ty + 1][tx + 1] + lam * fmaf(sc.uc.c_l, gl, sc.uc.c_r * gr);
        mu_new = in_disc(i, j, G.n) ? fmaxf(v, 0.0f) : 0.0f;
        img_out[(size_t)j * G.P + i + PAD] = mu_new;
        if (dec.keep) in.best[(size_t)j * G.n + i] = mu_new;
    }
    t[ty][tx] = mu_new;
    __syncthreads();
    const int ii = ti0 + ty, jj = tj0 + tx;
    if (ii < G.n && jj < G.n) imgT_out[(size_t)ii * G.P + jj + PAD] = t[tx][ty];
}

// Blocked form of bp_update_tile: 256 / (PX PY) threads per 16x16 tile, each
// owning PX x PY pixels.  Same arithmetic per pixel, same bits.
template <int PX, int PY>
__device__ __forceinline__ void bp_update_tile_blk(Geo G, const ViewRec* __restrict__ V,
                                                   const RayGeo* __restrict__ rg, const float* __restrict__ w,
                                                   const double* __restrict__ part,
                                                   const DevState* __restrict__ st_in, DevState* __restrict__ st_out,
                                                   const float* __restrict__ img, float* __restrict__ img_out,
                                                   float* __restrict__ imgT_out, UpdateScalars sc, int ti0, int tj0,
                                                   const DevState* __restrict__ st_pre)
{
    constexpr int NTH = 256 / (PX * PY);
    constexpr int BW = TILE / PX;  // pixel blocks per tile row
    __shared__ float s[TILE + 2][TILE + 3];
    __shared__ float t[TILE][TILE + 1];
    __shared__ double red[4];
    __shared__ StageLdsBlk S;
    const int tid = threadIdx.x;
    const int bxl = (tid % BW) * PX, byl = (tid / BW) * PY;  // block origin in the tile
    const int i0 = ti0 + bxl, j0 = tj0 + byl;

    for (int e = tid; e < (TILE + 2) * (TILE + 2); e += NTH) {
        const int ly = e / (TILE + 2), lx = e - ly * (TILE + 2);
        const int gj = tj0 + ly - 1, gi = ti0 + lx - 1;
        s[ly][lx] = (gj >= 0 && gj < G.n && gi < G.n + PAD) ? img[(size_t)gj * G.P + gi + PAD] : 0.0f;
    }
    float accg[VIEW_GROUPS][PY][PX];
#pragma unroll
    for (int g = 0; g < VIEW_GROUPS; ++g)
#pragma unroll
        for (int b = 0; b < PY; ++b)
#pragma unroll
            for (int a = 0; a < PX; ++a) accg[g][b][a] = 0.0f;
    gather_block<PX, PY>(S, G, V, rg, w, sc.q0, sc.nq, i0, j0, i0 < G.n && j0 < G.n, accg, ti0,
                         tj0);  // has barriers
    float acc[PY][PX];
#pragma unroll
    for (int b = 0; b < PY; ++b)
#pragma unroll
        for (int a = 0; a < PX; ++a) acc[b][a] = combine_groups(accg[0][b][a], accg[1][b][a], accg[2][b][a], accg[3][b][a]);

    StepDecision dec{0.0, false};
    DevState in{};
    if (st_pre) {
        dec.lam = st_pre->lambda;
    } else {
        const double f = block_sum<NTH>(part, (sc.nrays + SQ_GROUP - 1) / SQ_GROUP, red) / (double)sc.nrays;
        in = *st_in;
        dec = step_rule(in, sc.rule, f);
        if (ti0 == 0 && tj0 == 0 && tid == 0) record_state(in, sc.rule, f, dec.lam, st_out);
    }
    const float lam = (float)dec.lam;

#pragma unroll
    for (int b = 0; b < PY; ++b)
#pragma unroll
        for (int a = 0; a < PX; ++a) {
            const int i = i0 + a, j = j0 + b;
            float mu_new = 0.0f;
            if (i < G.n && j < G.n) {
                const float gr = tv_neg_grad<TILE + 3>(s, bxl + a + 1, byl + b + 1, i, j, G.n, sc.uc.eps);
                const float v = s[byl + b + 1][bxl + a + 1] + lam * fmaf(sc.uc.c_l, acc[b][a], sc.uc.c_r * gr);
                mu_new = in_disc(i, j, G.n) ? fmaxf(v, 0.0f) : 0.0f;
                img_out[(size_t)j * G.P + i + PAD] = mu_new;
                if (dec.keep) in.best[(size_t)j * G.n + i] = mu_new;
            }
            t[byl + b][bxl + a] = mu_new;
        }
    __syncthreads();
    for (int e = tid; e < TILE * TILE; e += NTH) {
        const int ly = e / TILE, lx = e - ly * TILE;  // transposed: row ii, column jj
        const int ii = ti0 + ly, jj = tj0 + lx;
        if (ii < G.n && jj < G.n) imgT_out[(size_t)ii * G.P + jj + PAD] = t[lx][ly];
    }
}

// 2x2-pixel, view-group form of bp_update_tile (256 threads per 16x16 tile):
// the four groups' sums meet in LDS and each thread then finishes one pixel.
// Same arithmetic per pixel, same bits.
__device__ __forceinline__ void bp_update_tile_quad(Geo G, const ViewRec* __restrict__ V,
                                                    const RayGeo* __restrict__ rg, const float* __restrict__ w,
                                                    const double* __restrict__ part,
                                                    const DevState* __restrict__ st_in, DevState* __restrict__ st_out,
                                                    const float* __restrict__ img, float* __restrict__ img_out,
                                                    float* __restrict__ imgT_out, UpdateScalars sc, int ti0, int tj0,
                                                    const DevState* __restrict__ st_pre)
{
    __shared__ float s[TILE + 2][TILE + 3];
    __shared__ float t[TILE][TILE + 1];
    __shared__ double red[4];
    // the staging area, and after the gather (which ends at a block barrier) the four groups' sums
    constexpr size_t STAGE_BYTES = sizeof(StageLdsQ) > sizeof(float) * VIEW_GROUPS * TILE * TILE
                                       ? sizeof(StageLdsQ)
                                       : sizeof(float) * VIEW_GROUPS * TILE * TILE;
    __shared__ __attribute__((aligned(16))) unsigned char stage_raw[STAGE_BYTES];
    StageLdsQ& S = *reinterpret_cast<StageLdsQ*>(stage_raw);
    float (*gsum)[TILE * TILE] = reinterpret_cast<float (*)[TILE * TILE]>(stage_raw);
    const int tid = threadIdx.x;
    for (int e = tid; e < (TILE + 2) * (TILE + 2); e += 256) {
        const int ly = e / (TILE + 2), lx = e - ly * (TILE + 2);
        const int gj = tj0 + ly - 1, gi = ti0 + lx - 1;
        s[ly][lx] = (gj >= 0 && gj < G.n && gi < G.n + PAD) ? img[(size_t)gj * G.P + gi + PAD] : 0.0f;
    }
    float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
    gather_quad(S, G, V, rg, w, sc.q0, sc.nq, ti0, tj0, acc);  // has barriers
    {
        const int lane = tid & 63, grp = tid >> 6;
        const int bxl = 2 * (lane & 7), byl = 2 * (lane >> 3);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) gsum[grp][(byl + b) * TILE + bxl + a] = acc[b][a];
    }

    StepDecision dec{0.0, false};
    DevState in{};
    if (st_pre) {
        dec.lam = st_pre->lambda;
    } else {
        const double f = block_sum<256>(part, (sc.nrays + SQ_GROUP - 1) / SQ_GROUP, red) / (double)sc.nrays;
        in = *st_in;
        dec = step_rule(in, sc.rule, f);
        if (ti0 == 0 && tj0 == 0 && tid == 0) record_state(in, sc.rule, f, dec.lam, st_out);
    }
    __syncthreads();  // (block_sum has one too; this covers st_pre) the group sums are in LDS
    const float lam = (float)dec.lam;
    const int tx = tid & 15, ty = tid >> 4;
    const int i = ti0 + tx, j = tj0 + ty;
    float mu_new = 0.0f;
    if (i < G.n && j < G.n) {
        const float gl = combine_groups(gsum[0][tid], gsum[1][tid], gsum[2][tid], gsum[3][tid]);
        const float gr = tv_neg_grad<TILE + 3>(s, tx + 1, ty + 1, i, j, G.n, sc.uc.eps);
        const float v = s[ty + 1][tx + 1] + lam * fmaf(sc.uc.c_l, gl, sc.uc.c_r * gr);
        mu_new = in_disc(i, j, G.n) ? fmaxf(v, 0.0f) : 0.0f;
        img_out[(size_t)j * G.P + i + PAD] = mu_new;
        if (dec.keep) in.best[(size_t)j * G.n + i] = mu_new;
    }
    t[ty][tx] = mu_new;
    __syncthreads();
    const int ii = ti0 + ty, jj = tj0 + tx;
    if (ii < G.n && jj < G.n) imgT_out[(size_t)ii * G.P + jj + PAD] = t[tx][ty];
}

// Update body for variant VAR (0 global, 1 LDS-staged, 2 1x2, 3 2x1, 4 2x2, 5 2x2 per
// lane with one view group per wave).
template <int VAR>
__device__ __forceinline__ void bp_update_any(Geo G, const ViewRec* __restrict__ V, const RayGeo* __restrict__ rg,
                                              const float* __restrict__ w, const double* __restrict__ part,
                                              const DevState* __restrict__ st_in, DevState* __restrict__ st_out,
                                              const float* __restrict__ img, float* __restrict__ img_out,
                                              float* __restrict__ imgT_out, UpdateScalars sc, int ti0, int tj0,
                                              const DevState* __restrict__ st_pre)
{
#define BP_TILE_ARGS G, V, rg, w, part, st_in, st_out, img, img_out, imgT_out, sc, ti0, tj0, st_pre
    if constexpr (VAR == 0) bp_update_tile<false>(BP_TILE_ARGS);
    if constexpr (VAR == 1) bp_update_tile<true>(BP_TILE_ARGS);
    if constexpr (VAR == 2) bp_update_tile_blk<1, 2>(BP_TILE_ARGS);
    if constexpr (VAR == 3) bp_update_tile_blk<2, 1>(BP_TILE_ARGS);
    if constexpr (VAR == 4) bp_update_tile_blk<2, 2>(BP_TILE_ARGS);
    if constexpr (VAR == 5) bp_update_tile_quad(BP_TILE_ARGS);
#undef BP_TILE_ARGS
}

constexpr int bp_threads(int var) { return var == 4 ? 64 : (var == 2 || var == 3 ? 128 : 256); }

// One slice: the grid covers its tiles.
template <int VAR>
__global__ __launch_bounds__(bp_threads(VAR)) void bp_update_kernel(
    Geo G, const ViewRec* __restrict__ V, const RayGeo* __restrict__ rg, const float* __restrict__ w,
    const double* __restrict__ part, const DevState* __restrict__ st_in, DevState* __restrict__ st_out,
    const float* __restrict__ img, float* __restrict__ img_out, float* __restrict__ imgT_out, UpdateScalars sc)
{
    bp_update_any<VAR>(G, V, rg, w, part, st_in, st_out, img, img_out, imgT_out, sc, blockIdx.x * TILE,
                       blockIdx.y * TILE, nullptr);
}

// The step rule of every slice of a batch, once per slice (block i: slice i):
// the same fixed-order sum and rule as the update kernel's own, so the same
// bits; writes the slice's state 1 - in, whose lambda the batched update reads.
__global__ __launch_bounds__(256) void step_batch_kernel(const SliceDesc* __restrict__ slices, int s, int in,
                                                         StepRule rule)
{
    __shared__ double red[4];
    const SliceDesc* __restrict__ D = slices + blockIdx.x;
    const int nrays = D->subs[s].y * D->geo.nch;
    const double f = block_sum<256>(as_global(D->part), (nrays + SQ_GROUP - 1) / SQ_GROUP, red) / (double)nrays;
    const DevState st = D->state[in];
    const StepDecision dec = step_rule(st, rule, f);
    if (threadIdx.x == 0) record_state(st, rule, f, dec.lam, D->state + (1 - in));
}

// A batch of slices: block b updates tile work[b] of slice work[b].slice with
// that slice's subset s and the step size step_batch_kernel left in state
// 1 - in, reading image buffer `in` and writing 1 - in.
// the 2x2 view-group variant (18 KB of LDS) is held to 6 waves per SIMD (80 VGPRs) for batches
constexpr int bp_batch_waves(int var) { return var == 5 ? 6 : 1; }
template <int VAR>
__global__ __launch_bounds__(bp_threads(VAR)) __attribute__((amdgpu_waves_per_eu(bp_batch_waves(VAR))))
void bp_update_batch_kernel(const SliceDesc* __restrict__ slices, const BpWork* __restrict__ work, int s, int in,
                            StepRule rule)
{
    const BpWork wk = work[blockIdx.x];
    if (wk.slice < 0) return;
    const SliceDesc* __restrict__ D = slices + wk.slice;
    const int2 sq = D->subs[s];
    const UpdateScalars sc{sq.x, sq.y, sq.y * D->geo.nch, rule, D->uc};
    bp_update_any<VAR>(D->geo, as_global(D->views), as_global(D->rg), as_global(D->w), as_global(D->part),
                       as_global(D->state + in), as_global(D->state + (1 - in)), as_global(D->img[in]),
                       as_global(D->img[1 - in]), as_global(D->imgT[1 - in]), sc, wk.ti0, wk.tj0,
                       as_global(D->state + (1 - in)));
}

}  // namespace

hipError_t launch_bp_plain(const Geo& geo, const ViewRec* views, const RayGeo* rg, const float* w, int q0, int nq,
                           float* out, hipStream_t s)
{
    dim3 grid(cdiv(geo.n, TILE), cdiv(geo.n, TILE));
    bp_plain_kernel<<<grid, 256, 0, s>>>(geo, views, rg, w, q0, nq, out);
    return hipGetLastError();
}

hipError_t launch_bp_update(const Geo& geo, int variant, const UpdateArgs& a, hipStream_t s)
{
    dim3 grid(cdiv(geo.n, TILE), cdiv(geo.n, TILE));
    const UpdateScalars sc{a.q0, a.nq, a.nrays, a.rule, a.uc};
#define BP_ARGS geo, a.views, a.rg, a.w, a.part, a.st_in, a.st_out, a.img, a.img_out, a.imgT_out, sc
    switch (variant) {
    case 0: bp_update_kernel<0><<<grid, bp_threads(0), 0, s>>>(BP_ARGS); break;
    case 1: bp_update_kernel<1><<<grid, bp_threads(1), 0, s>>>(BP_ARGS); break;
    case 2: bp_update_kernel<2><<<grid, bp_threads(2), 0, s>>>(BP_ARGS); break;
    case 3: bp_update_kernel<3><<<grid, bp_threads(3), 0, s>>>(BP_ARGS); break;
    case 4: bp_update_kernel<4><<<grid, bp_threads(4), 0, s>>>(BP_ARGS); break;
    case 5: bp_update_kernel<5><<<grid, bp_threads(5), 0, s>>>(BP_ARGS); break;
    default: return hipErrorInvalidValue;
    }
#undef BP_ARGS
    return hipGetLastError();
}

hipError_t launch_bp_update_batch(int variant, const SliceDesc* slices, const BpWork* work, int nblocks, int sub,
                                  int in, StepRule rule, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    switch (variant) {
    case 0: bp_update_batch_kernel<0><<<nblocks, bp_threads(0), 0, s>>>(slices, work, sub, in, rule); break;
    case 1: bp_update_batch_kernel<1><<<nblocks, bp_threads(1), 0, s>>>(slices, work, sub, in, rule); break;
    case 2: bp_update_batch_kernel<2><<<nblocks, bp_threads(2), 0, s>>>(slices, work, sub, in, rule); break;
    case 3: bp_update_batch_kernel<3><<<nblocks, bp_threads(3), 0, s>>>(slices, work, sub, in, rule); break;
    case 4: bp_update_batch_kernel<4><<<nblocks, bp_threads(4), 0, s>>>(slices, work, sub, in, rule); break;
    case 5: bp_update_batch_kernel<5><<<nblocks, bp_threads(5), 0, s>>>(slices, work, sub, in, rule); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_batch(const SliceDesc* slices, int n_slices, int sub, int in, StepRule rule, hipStream_t s)
{
    if (n_slices <= 0) return hipSuccess;
    step_batch_kernel<<<n_slices, 256, 0, s>>>(slices, sub, in, rule);
    return hipGetLastError();
}

hipError_t launch_tv_grad(const float* img, float* grad, int n, float eps, hipStream_t s)
{
    dim3 grid(cdiv(n, TILE), cdiv(n, TILE));
    tv_grad_kernel<<<grid, 256, 0, s>>>(img, grad, n, eps);
    return hipGetLastError();
}

}  // namespace recon
