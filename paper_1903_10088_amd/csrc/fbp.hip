// Fan-beam filtered backprojection (gfx950): the baseline the paper compares
// the iterative method with (sections 1 and 4).  The paper does not describe
// it; this is the textbook equiangular algorithm over the full turn:
//   R'(v, k) = p(v, k) D cos(gamma_k)
//   Q(v, n)  = sum_k R'(v, k) dgamma h(n - k),  h(0) = 1 / (8 dgamma^2),
//              h(m) = 0 (m even), -1 / (2 pi^2 sin^2(m dgamma)) (m odd)
//   f(x, y)  = dbeta sum_v Q(v, gamma') / L^2
// with gamma' the fan angle and L the source distance of (x, y) in view v,
// and Q linearly interpolated in gamma (zero outside the channels).
//
// Two kernels: the filter (one block per view and 256 output channels; the
// weighted projection in LDS, the taps of odd offset and then the centre one
// in channel order) and a pixel-driven backprojection (one thread per pixel,
// views in the handle's fixed order, no atomics), so the image is bitwise
// deterministic.  Lengths are in pixel units; the last step converts to 1/mm.
// The geometry of the backprojection (view angles, fan angle of each pixel)
// is in double precision, the filtered values and sums in float.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace recon {

std::vector<float> fbp_tables(const recon_geometry* g)
{
    const int nch = g->n_channels;
    const double half = 0.5 * g->n * g->pixel_mm;
    const double gmax = g->fan_half_angle_rad > 0 ? g->fan_half_angle_rad : std::asin(half / g->sad_mm);
    const double dg = 2.0 * gmax / nch;
    const double D = g->sad_mm / g->pixel_mm;
    const double pi = 3.14159265358979323846;
    std::vector<float> t((size_t)nch + 2 * (size_t)nch - 1);
    for (int k = 0; k < nch; ++k) t[k] = (float)(D * std::cos((k - 0.5 * (nch - 1)) * dg));
    for (int m = -(nch - 1); m <= nch - 1; ++m) {
        double h = 0.0;
        if (m == 0) {
            h = 1.0 / (8.0 * dg * dg);
        } else if (m % 2 != 0) {
            const double s = std::sin(m * dg);
            h = -1.0 / (2.0 * pi * pi * s * s);
        }
        t[(size_t)nch + (size_t)(m + nch - 1)] = (float)(dg * h);
    }
    return t;
}

namespace {

constexpr int FBP_MAX_CH = 16384;  // the filter holds one view's channels in LDS

// Q(q, n) for view q (subset order) = sum_k p(q, k) wcos(k) ramp(n - k): the
// channels k at odd distance from n in increasing order, then k = n.
__global__ __launch_bounds__(256) void fbp_filter_kernel(const float* __restrict__ p, const float* __restrict__ wcos,
                                                         const float* __restrict__ ramp, int nch,
                                                         float* __restrict__ q_out)
{
    extern __shared__ float r[];
    const int q = blockIdx.x;
    const float* pv = p + (size_t)q * nch;
    for (int k = threadIdx.x; k < nch; k += 256) r[k] = pv[k] * wcos[k];
    __syncthreads();
    const int n = blockIdx.y * 256 + threadIdx.x;
    if (n >= nch) return;
    const float* h = ramp + (nch - 1) + n;  // h[-k] = dgamma h(n - k)
    float acc = 0.0f;
    for (int k = (n + 1) & 1; k < nch; k += 2) acc = fmaf(r[k], h[-k], acc);
    acc = fmaf(r[n], h[-n], acc);
    q_out[(size_t)q * nch + n] = acc;
}

// The fan angle of a pixel, and so its channel position, is formed in double
// precision from double view angles: in float a channel index near 370 resolves
// only 3e-5 channel, and filtered projections of noisy data change by up to
// their own size from one channel to the next.  Interpolation and sums are in
// float.
__global__ __launch_bounds__(256) void fbp_bp_kernel(Geo G, const double* __restrict__ cs, double dist, double dg_inv,
                                                     const float* __restrict__ Q, int nv, float scale,
                                                     float* __restrict__ img)
{
    const int i = blockIdx.x * 16 + (threadIdx.x & 15), j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= G.n || j >= G.n) return;
    const double X = (double)i - 0.5 * (G.n - 1), Y = (double)j - 0.5 * (G.n - 1);
    const double kc = 0.5 * (G.nch - 1);
    float acc = 0.0f;
    for (int q = 0; q < nv; ++q) {
        const double cb = cs[2 * q], sb = cs[2 * q + 1];
        // distance along the central ray (> 0: the source is outside the grid's circumcircle)
        // and offset towards increasing fan angle, in pixels
        const double along = fma(-X, cb, fma(-Y, sb, dist));
        const double perp = fma(X, sb, -(Y * cb));
        const double kf = fma(atan(perp / along), dg_inv, kc);
        const double fl = floor(kf);
        const int k0 = (int)fl;
        const float f = (float)(kf - fl);
        const float* qv = Q + (size_t)q * G.nch;
        const float a = (k0 >= 0 && k0 < G.nch) ? qv[k0] : 0.0f;
        const float b = (k0 + 1 >= 0 && k0 + 1 < G.nch) ? qv[k0 + 1] : 0.0f;
        acc = fmaf(fmaf(f, b - a, a), (float)(1.0 / fma(along, along, perp * perp)), acc);
    }
    img[(size_t)j * G.n + i] = acc * scale;
}

}  // namespace
}  // namespace recon

using namespace recon;

extern "C" recon_status recon_fbp(recon_handle* h, const float* d_counts, float i0, float* d_img, void* stream)
{
    if (!h || !d_counts || !d_img) return fail(RECON_INVALID_ARG, "NULL argument");
    if (!(i0 > 0) || !std::isfinite(i0)) return fail(RECON_INVALID_ARG, "i0 must be finite and > 0");
    const Geo& G = h->geo;
    if (G.nch > FBP_MAX_CH) return fail(RECON_INVALID_ARG, "recon_fbp supports up to 16384 channels");
    if (!full_turn(&h->g)) return fail(RECON_INVALID_ARG, "recon_fbp needs views over a full turn");
    hipStream_t s = as_stream(stream);
    RECON_HIP_TRY(launch_prep_counts(d_counts, h->d_views, G.nv, G.nch, i0, h->d_yt, h->d_p, s));
    const float* wcos = h->d_fbp;
    const float* ramp = h->d_fbp + G.nch;
    fbp_filter_kernel<<<dim3(G.nv, (G.nch + 255) / 256), 256, (size_t)G.nch * sizeof(float), s>>>(h->d_p, wcos, ramp,
                                                                                                   G.nch, h->d_w);
    RECON_HIP_TRY(hipGetLastError());
    const float scale = (float)(2.0 * 3.14159265358979323846 / G.nv / h->g.pixel_mm);
    const double half = 0.5 * h->g.n * h->g.pixel_mm;
    const double gmax = h->g.fan_half_angle_rad > 0 ? h->g.fan_half_angle_rad : std::asin(half / h->g.sad_mm);
    const double dg_inv = G.nch / (2.0 * gmax);
    fbp_bp_kernel<<<dim3((G.n + 15) / 16, (G.n + 15) / 16), 256, 0, s>>>(
        G, h->d_fbp_cs, h->g.sad_mm / h->g.pixel_mm, dg_inv, h->d_w, G.nv, scale, d_img);
    RECON_HIP_TRY(hipGetLastError());
    return RECON_OK;
}
