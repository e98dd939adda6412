// Geometry helpers shared by the projector, the gather backprojector and the
// host-side table check.  Everything here is __host__ __device__ so that the
// host can verify, without a GPU, that the gather enumerates every ray with a
// nonzero weight on every pixel.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace recon {

// atan on |t| <= 0.5 by its odd Taylor series through t^19 (error < 3e-8 rad);
// only used to place the candidate window, whose margin absorbs the error.
__host__ __device__ __forceinline__ float atan_small(float t)
{
    const float t2 = t * t;
    float p = -1.0f / 19.0f;
    p = fmaf(p, t2, 1.0f / 17.0f);
    p = fmaf(p, t2, -1.0f / 15.0f);
    p = fmaf(p, t2, 1.0f / 13.0f);
    p = fmaf(p, t2, -1.0f / 11.0f);
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
};

__host__ __device__ __forceinline__ PixelView pixel_view(const Geo& G, const ViewRec& v, float X, float Y)
{
    const float px = X - v.sx, py = Y - v.sy;
    const float along = -(px * v.cb + py * v.sb);  // distance along the central ray (> 0)
    const float perp = px * v.sb - py * v.cb;      // offset towards increasing fan angle
    const float tg = perp / along;
#ifdef __HIP_DEVICE_COMPILE__
    const float gam = G.use_poly ? atan_small(tg) : atanf(tg);
#else
    const float gam = G.use_poly ? atan_small(tg) : std::atan(tg);
#endif
    const float inv_r2 = 1.0f / fmaf(px, px, py * py);
    PixelView o;
    o.kp = fmaf(gam, G.dg_inv, G.kc);
    o.hwx = fmaf(fabsf(px) * inv_r2, G.dg_inv, G.margin);
    o.hwy = fmaf(fabsf(py) * inv_r2, G.dg_inv, G.margin);
    return o;
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

// u(t) - centre for an integer centre: the lattice part minus the centre is
// exact, so only the final addition of the residual rounds.
__host__ __device__ __forceinline__ float ray_offset(const RayGeo& g, float t, float centre)
{
    return (fmaf(t, g.s_hi, g.a_int) - centre) + fmaf(t, g.s_lo, g.a_frac);
}

// Joseph weight of a ray on a pixel: the hat function of the distance d, along
// the ray's minor axis, between the ray's crossing of the pixel's sampling
// line and the pixel centre.
__host__ __device__ __forceinline__ float hat(float d) { return fmaxf(0.0f, 1.0f - fabsf(d)); }

}  // namespace recon
