// Geometry helpers shared by the projector, the gather backprojector and the
// host-side table check.  Everything here is __host__ __device__ so that the
// host can verify, without a GPU, that the gather enumerates every ray with a
// nonzero weight on every pixel.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace recon {

// atan on |t| <= 0.45 by its odd Taylor series through t^11 (error below
// |t|^13 / 13 < 2.5e-6 rad); only used to place the candidate window, whose
// margin includes this error.
__host__ __device__ __forceinline__ float atan_small(float t)
{
    const float t2 = t * t;
    float p = -1.0f / 11.0f;
    p = fmaf(p, t2, 1.0f / 9.0f);
    p = fmaf(p, t2, -1.0f / 7.0f);
    p = fmaf(p, t2, 1.0f / 5.0f);
    p = fmaf(p, t2, -1.0f / 3.0f);
    p = fmaf(p, t2, 1.0f);
    return t * p;
}

// Continuous channel coordinate of the ray through pixel offset (X, Y) (pixel
// units from the grid centre) in view v, and the half-widths, in channels, of
// the windows of rays that cross the column through the pixel within one
// pixel of its centre (x-major rays) or the row through it (y-major rays).
struct PixelView {
    float kp, hwx, hwy;
    float ax, ay;  // channels per pixel of offset along y (|px| s) and along x (|py| s)
};

__host__ __device__ __forceinline__ float approx_rcp(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);  // 1 ulp
#else
    return 1.0f / x;
#endif
}

__host__ __device__ __forceinline__ PixelView pixel_view(const Geo& G, const ViewRec& v, float X, float Y)
{
    // with the source at dist * (cb, sb): distance along the central ray (> 0)
    // and offset towards increasing fan angle, both affine in (X, Y)
    const float along = fmaf(-X, v.cb, fmaf(-Y, v.sb, v.dist));
    const float perp = fmaf(X, v.sb, -(Y * v.cb));
    const float px = X - v.sx, py = Y - v.sy;
    const float ra = approx_rcp(along);
    const float tg = perp * ra;
#ifdef __HIP_DEVICE_COMPILE__
    const float gam = G.use_poly ? atan_small(tg) : atanf(tg);
#else
    const float gam = G.use_poly ? atan_small(tg) : std::atan(tg);
#endif
    // d(angle)/d(offset across the sampling line) = |px| / r^2 (x-major) or
    // |py| / r^2 (y-major); 1/along^2 >= 1/r^2 bounds it from above
    const float s = ra * ra * G.dg_inv;
    PixelView o;
    o.kp = fmaf(gam, G.dg_inv, G.kc);
    o.ax = fabsf(px) * s;
    o.ay = fabsf(py) * s;
    o.hwx = o.ax + G.margin;
    o.hwy = o.ay + G.margin;
    return o;
}

// Per (view, 16x16 tile) linear model of the channel coordinate, for the
// LDS-staged gather: for a pixel at offset (dX, dY) from the tile centre
// (Xc, Yc), kp ~ kpc + gx dX + gy dY.  The polar angle seen from the source has
// a Hessian of norm 1/r^2, so over the tile (|d|^2 <= 2 * 7.5^2) the linear
// model is within 56.25 / r_min^2 radians of the angle, r_min >= along - 10.61
// (the tile's half-diagonal); that error, in channels, and the tile's largest
// window half-width (|offset from the source| <= |centre offset| + 7.5) are
// folded into hwx / hwy together with G.margin.  Every ray with a nonzero
// weight on a pixel of the tile therefore lies in [kp - hw, kp + hw].
struct TileView {
    float kpc, gx, gy, hwx, hwy;
};

__host__ __device__ __forceinline__ TileView tile_view(const Geo& G, const ViewRec& v, float Xc, float Yc)
{
    const float along = fmaf(-Xc, v.cb, fmaf(-Yc, v.sb, v.dist));
    const float perp = fmaf(Xc, v.sb, -(Yc * v.cb));
    const float ra = approx_rcp(along);
    const float tg = perp * ra;
#ifdef __HIP_DEVICE_COMPILE__
    const float gam = G.use_poly ? atan_small(tg) : atanf(tg);
#else
    const float gam = G.use_poly ? atan_small(tg) : std::atan(tg);
#endif
    const float r2 = fmaf(along, along, perp * perp);
    const float ir2 = G.dg_inv / r2;
    // (a tile within 10.61 px of the source, possible only for very wide fans,
    // gets a window spanning the whole interval)
    const float rmin = fmaxf(along - 10.61f, 1e-3f);
    const float irmin2 = G.dg_inv / (rmin * rmin);
    const float lin_err = 56.25f * irmin2;
    TileView t;
    t.kpc = fmaf(gam, G.dg_inv, G.kc);
    t.gx = fmaf(along, v.sb, perp * v.cb) * ir2;
    t.gy = fmaf(perp, v.sb, -(along * v.cb)) * ir2;
    t.hwx = (fabsf(Xc - v.sx) + 7.5f) * irmin2 + G.margin + lin_err;
    t.hwy = (fabsf(Yc - v.sy) + 7.5f) * irmin2 + G.margin + lin_err;
    return t;
}

// Channel intervals [x0, x1) of x-major and [y0, y1) of y-major rays in a view.
__host__ __device__ __forceinline__ void major_intervals(const ViewRec& v, int nch, int& x0, int& x1, int& y0,
                                                         int& y1)
{
    if (v.first_major == 0) {
        x0 = 0;
        x1 = v.k_split;
        y0 = v.k_split;
        y1 = nch;
    } else {
        y0 = 0;
        y1 = v.k_split;
        x0 = v.k_split;
        x1 = nch;
    }
}

__host__ __device__ __forceinline__ void candidate_range(float kp, float hw, int a, int b, int& lo, int& hi)
{
    float flo = ceilf(kp - hw), fhi = floorf(kp + hw);
    flo = fmaxf(flo, (float)a);
    fhi = fminf(fhi, (float)(b - 1));
    lo = (int)flo;
    hi = (int)fhi;
}

// candidate_range with the channel interval given as floats [fa, fb] (a and
// b - 1, exact for channel counts below 2^24): the same result.
__host__ __device__ __forceinline__ void candidate_range_f(float kp, float hw, float fa, float fb, int& lo, int& hi)
{
    lo = (int)fmaxf(ceilf(kp - hw), fa);
    hi = (int)fminf(floorf(kp + hw), fb);
}

// A pointer read from device memory is generic to the compiler (flat loads);
// passing it through the global address space lets the loads be global ones.
template <class T>
__device__ __forceinline__ T* as_global(T* p)
{
    const unsigned long long a = (unsigned long long)p;
    return (T*)((__attribute__((address_space(1))) T*)a);
}

// Reconstruction disc x^2 + y^2 <= (n * pixel / 2)^2, in exact integer
// arithmetic on doubled offsets from the grid centre.
__host__ __device__ __forceinline__ bool in_disc(int i, int j, int n)
{
    const long a = 2L * i - n + 1, b = 2L * j - n + 1;
    return a * a + b * b <= (long)n * n;
}

// u(t) - centre for an integer centre: the lattice part minus the centre is
// exact, so only the final addition of the residual rounds.
__host__ __device__ __forceinline__ float ray_offset(const RayGeo& g, float t, float centre)
{
    return (fmaf(t, g.s_hi, g.a_int) - centre) + fmaf(t, g.s_lo, g.a_frac);
}

// Joseph weight of a ray on a pixel: the hat function of the distance d, along
// the ray's minor axis, between the ray's crossing of the pixel's sampling
// line and the pixel centre.  max(0, 1 - |d|) written as a clamp to [0, 1]
// (1 - |d| never exceeds 1), which the device does in the subtraction itself.
__host__ __device__ __forceinline__ float hat(float d) { return fminf(fmaxf(1.0f - fabsf(d), 0.0f), 1.0f); }

// Widening of the per-tile window for a PX x PY block of pixels whose centre
// is the model's point: the model's spread over the block, plus 1/64 channel
// and two ulps of the centre channel so that the block's window, rounded
// differently from its pixels' own, still holds every one of them.
__host__ __device__ __forceinline__ float block_spread(const TileView& tv, int PX, int PY)
{
    return fabsf(tv.gx) * (0.5f * (PX - 1)) + fabsf(tv.gy) * (0.5f * (PY - 1)) + 0.015625f +
           fabsf(tv.kpc) * 2.4e-7f;
}

// Channels per view that the LDS-staged gather can stage for one tile.
constexpr int STAGE_SLOTS = 64;

// Channels of one view that the LDS-staged gather stages for a 16x16 tile:
// [k0, k0 + cnt) covers the window of every pixel of the tile.  The windows
// [ceil(kp - hw), floor(kp + hw)] have |kp - kpc| <= 7.5 (|gx| + |gy|) up to
// the rounding of kp (below 1e-3 channel for any channel count under 2^16),
// and hw <= max(hwx, hwy), so one channel of margin on each side contains
// them.  cnt = 0 when the range exceeds `slots` (the view is then not staged).
__host__ __device__ __forceinline__ void stage_range(const TileView& tv, int nch, int slots, int& k0, int& cnt)
{
    const float spread = (fabsf(tv.gx) + fabsf(tv.gy)) * 7.5f + fmaxf(tv.hwx, tv.hwy);
    k0 = max(0, (int)floorf(tv.kpc - spread) - 1);
    const int k1 = min(nch - 1, (int)ceilf(tv.kpc + spread) + 1);
    cnt = k1 - k0 + 1;
    if (cnt <= 0 || cnt > slots) cnt = 0;
}

}  // namespace recon
