// HIP kernels of the ordered-subset TV reconstruction for gfx950.
//
// Per sub-iteration the path is three launches:
//   fp_kernel<OS>     Joseph forward projection of the subset (section 4.C
//                     "reprojection") fused with the likelihood epilogue:
//                     t = exp(-l), weighted residual w = (t - y/I0) * path,
//                     squared difference e = (l - p)^2 (section 3.C.2);
//   lambda_kernel     fixed-order FP64 mean of e and the step rule of Eqs. 4-5;
//   bp_update_kernel  gather backprojection of w (the exact transpose of the
//                     projector, no atomics), TV gradient from an LDS tile with
//                     a one-pixel halo, and the update of Eq. 3.
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
// transposed through LDS so both writes are coalesced).
__global__ __launch_bounds__(256) void pad_image_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                        float* __restrict__ dstT, int n, int P)
{
    __shared__ float tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int j = by + r, i = bx + tx;
        float v = 0.0f;
        if (j < n && i < n) {
            v = src[(size_t)j * n + i];
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

__global__ __launch_bounds__(256) void unpad_image_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                          int n, int P)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    dst[idx] = src[(size_t)j * P + i + PAD];
}

__device__ __forceinline__ bool in_disc(int i, int j, int n)
{
    // x^2 + y^2 <= (n * pixel / 2)^2 in exact integer arithmetic (doubled offsets)
    const long a = 2L * i - n + 1, b = 2L * j - n + 1;
    return a * a + b * b <= (long)n * n;
}

__global__ __launch_bounds__(256) void initial_image_kernel(float* __restrict__ dst, int n, float mu0)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int j = (int)(idx / n), i = (int)(idx - (long)j * n);
    dst[idx] = in_disc(i, j, n) ? mu0 : 0.0f;
}

// Counts in natural view order -> y / I0 and p = ln(I0 / max(y, 1)) in subset order.
__global__ __launch_bounds__(256) void prep_counts_kernel(const float* __restrict__ counts,
                                                          const ViewRec* __restrict__ views, int nv, int nch,
                                                          float i0, float* __restrict__ yt, float* __restrict__ p)
{
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (long)nv * nch) return;
    const int q = (int)(r / nch), k = (int)(r - (long)q * nch);
    const float y = counts[(size_t)views[q].nat_view * nch + k];
    yt[r] = y / i0;
    p[r] = (float)log((double)i0 / (double)fmaxf(y, 1.0f));
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
    const float* img;   // padded row-major: sampled by y-major rays along rows
    const float* imgT;  // padded transposed: sampled by x-major rays along columns
    const RayGeo* rg;
    const RayMeta* rm;
    const ViewRec* views;
    int ray0, nrays, n, P, nch, q0, natural_rows;
    float* out;  // plain mode: line integrals
    const float* yt;
    const float* p;
    float* w;
    float* e;
};

// SEG threads share a ray, each taking a fixed window of n/SEG sample lines, so
// the 64 lanes of a wave (64 neighbouring rays of one view, same window) walk
// the same sample line together and read neighbouring elements of one row of
// the (transposed) image.  Partial sums are added in window order.
template <int SEG, bool OS>
__global__ __launch_bounds__(256) void fp_kernel(FpArgs A)
{
    constexpr int RPB = 256 / SEG;
    const int tid = threadIdx.x;
    const int seg = tid / RPB;
    const int lr = tid - seg * RPB;
    const int r = blockIdx.x * RPB + lr;
    float acc = 0.0f;
    float scale = 0.0f;
    if (r < A.nrays) {
        const int gr = A.ray0 + r;
        const RayMeta m = A.rm[gr];
        const RayGeo g = A.rg[gr];
        scale = m.scale;
        const int lo = (int)(m.packed & 0x7fffu);
        const int hi = (int)((m.packed >> 15) & 0x7fffu);
        const int major = (int)(m.packed >> 30);
        const int win = (A.n + SEG - 1) / SEG;
        const int t0 = max(lo, seg * win);
        const int t1 = min(min(hi + 1, (seg + 1) * win), A.n);
        const float* base = (major ? A.img : A.imgT) + PAD;
        for (int t = t0; t < t1; ++t) {
            const float ft = (float)t;
            const float lat = fmaf(ft, g.s_hi, g.a_int);  // exact lattice part of u
            const float res = fmaf(ft, g.s_lo, g.a_frac);  // small residual
            const float fl = floorf(lat + res);
            const float f = (lat - fl) + res;               // lat - fl is exact
            const int j0 = min(max((int)fl, -PAD), A.n);
            const float* row = base + (size_t)t * A.P + j0;
            const float v0 = row[0];
            const float v1 = row[1];
            acc += fmaf(f, v1 - v0, v0);
        }
    }
    if constexpr (SEG > 1) {
        __shared__ float red[SEG][RPB];
        red[seg][lr] = acc;
        __syncthreads();
        if (seg != 0) return;
        acc = red[0][lr];
#pragma unroll
        for (int s = 1; s < SEG; ++s) acc += red[s][lr];
    }
    if (r >= A.nrays) return;
    const int gr = A.ray0 + r;
    const float ell = acc * scale;
    if constexpr (!OS) {
        const int q = r / A.nch, k = r - q * A.nch;
        const int row = A.natural_rows ? A.views[A.q0 + q].nat_view : q;
        A.out[(size_t)row * A.nch + k] = ell;
    } else {
        const float t = expf(-ell);
        A.w[gr] = (t - A.yt[gr]) * scale;
        const float d = ell - A.p[gr];
        A.e[gr] = d * d;
    }
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
// Step rule
// ----------------------------------------------------------------------------

// f_n = mean of e over the subset, summed in a fixed order that does not depend
// on how the projector was launched; then Eqs. 4-5 with the floor.
__global__ __launch_bounds__(1024) void lambda_kernel(const float* __restrict__ e, int ray0, int nrays,
                                                      DevState* __restrict__ st, StepRule R)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    // thread tid adds e[tid], e[tid + 1024], ... in that order; the loads of
    // eight terms are issued before their additions
    double s = 0.0;
    int r = tid;
    for (; r + 7 * 1024 < nrays; r += 8 * 1024) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = e[ray0 + r + u * 1024];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; r < nrays; r += 1024) s += (double)e[ray0 + r];
    red[tid] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid != 0) return;
    const double f = red[0] / (double)nrays;
    const int n = st->n_global;
    const int it = st->it;
    double lam;
    if (n == 0) {
        lam = R.lambda0;
    } else {
        lam = (f < st->f_prev) ? st->lambda + R.inc : st->lambda - R.dec;
        if (lam < R.lmin) lam = R.lmin;
    }
    if (st->schedule) lam = st->schedule[it];
    if (!isfinite(f)) st->flags |= 1;
    if (st->trace) {
        st->trace[2 * it] = f;
        st->trace[2 * it + 1] = lam;
    }
    st->lambda = lam;
    st->f_prev = f;
    st->n_global = n + 1;
    st->it = it + 1;
}

__global__ void set_state_kernel(DevState* st, double lambda, double f_prev, int n_global, int flags, double* trace,
                                 const double* schedule)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->lambda = lambda;
    st->f_prev = f_prev;
    st->n_global = n_global;
    st->it = 0;
    st->flags = flags;
    st->pad = 0;
    st->trace = trace;
    st->schedule = schedule;
}

// ----------------------------------------------------------------------------
// Gather backprojection
// ----------------------------------------------------------------------------

// g_L at pixel (i, j): the sum over the views [q0, q0+nq) and over the rays
// whose Joseph samples touch the pixel of hat weight x w, with w already
// multiplied by the ray's path length per sample line.  The candidate rays of a
// view form a window of channels around the ray through the pixel centre.
__device__ __forceinline__ float gather_pixel(const Geo& G, const ViewRec* __restrict__ V,
                                              const RayGeo* __restrict__ rg, const float* __restrict__ w, int q0,
                                              int nq, int i, int j)
{
    const float X = (float)i - G.c, Y = (float)j - G.c;
    const float fi = (float)i, fj = (float)j;
    float acc = 0.0f;
    for (int q = q0; q < q0 + nq; ++q) {
        const ViewRec v = V[q];
        const PixelView pv = pixel_view(G, v, X, Y);
        const float* wv = w + v.ray0;
        const RayGeo* gv = rg + v.ray0;
        int x0, x1, y0, y1;
        major_intervals(v, G.nch, x0, x1, y0, y1);
        if (x0 < x1) {
            int lo, hi;
            candidate_range(pv.kp, pv.hwx, x0, x1, lo, hi);
            for (int k = lo; k <= hi; ++k) {
                acc = fmaf(hat(ray_offset(gv[k], fi, fj)), wv[k], acc);
            }
        }
        if (y0 < y1) {
            int lo, hi;
            candidate_range(pv.kp, pv.hwy, y0, y1, lo, hi);
            for (int k = lo; k <= hi; ++k) {
                acc = fmaf(hat(ray_offset(gv[k], fj, fi)), wv[k], acc);
            }
        }
    }
    return acc;
}

__global__ __launch_bounds__(256) void bp_plain_kernel(Geo G, const ViewRec* __restrict__ V,
                                                       const RayGeo* __restrict__ rg, const float* __restrict__ w,
                                                       int q0, int nq, float* __restrict__ out)
{
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= G.n || j >= G.n) return;
    out[(size_t)j * G.n + i] = gather_pixel(G, V, rg, w, q0, nq, i, j);
}

// ----------------------------------------------------------------------------
// TV gradient
// ----------------------------------------------------------------------------

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
    __shared__ float s[18][19];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + tx, j = blockIdx.y * 16 + ty;
    for (int e = threadIdx.x; e < 18 * 18; e += 256) {
        const int ly = e / 18, lx = e - ly * 18;
        const int gj = blockIdx.y * 16 + ly - 1, gi = blockIdx.x * 16 + lx - 1;
        s[ly][lx] = (gj >= 0 && gj < n && gi >= 0 && gi < n) ? img[(size_t)gj * n + gi] : 0.0f;
    }
    __syncthreads();
    if (i >= n || j >= n) return;
    grad[(size_t)j * n + i] = tv_neg_grad<19>(s, tx + 1, ty + 1, i, j, n, eps);
}

// ----------------------------------------------------------------------------
// Fused backprojection + TV + update (Eq. 3)
// ----------------------------------------------------------------------------

// mu' = mask * max(0, mu + lambda (c_l g_L + c_r g_R)), all terms at mu^(n);
// writes both the row-major and the transposed padded copies of mu'.
__global__ __launch_bounds__(256) void bp_update_kernel(Geo G, const ViewRec* __restrict__ V,
                                                        const RayGeo* __restrict__ rg, const float* __restrict__ w,
                                                        int q0, int nq, const float* __restrict__ img,
                                                        float* __restrict__ img_out, float* __restrict__ imgT_out,
                                                        const DevState* __restrict__ st, UpdateConst uc)
{
    __shared__ float s[18][19];
    __shared__ float t[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + tx, j = blockIdx.y * 16 + ty;
    for (int e = threadIdx.x; e < 18 * 18; e += 256) {
        const int ly = e / 18, lx = e - ly * 18;
        const int gj = blockIdx.y * 16 + ly - 1, gi = blockIdx.x * 16 + lx - 1;
        // columns -1 and n sit in the zero padding; rows -1 and n are outside the buffer
        s[ly][lx] = (gj >= 0 && gj < G.n && gi < G.n + PAD) ? img[(size_t)gj * G.P + gi + PAD] : 0.0f;
    }
    __syncthreads();
    float mu_new = 0.0f;
    if (i < G.n && j < G.n) {
        const float gl = gather_pixel(G, V, rg, w, q0, nq, i, j);
        const float gr = tv_neg_grad<19>(s, tx + 1, ty + 1, i, j, G.n, uc.eps);
        const float lam = (float)st->lambda;
        const float v = s[ty + 1][tx + 1] + lam * fmaf(uc.c_l, gl, uc.c_r * gr);
        mu_new = in_disc(i, j, G.n) ? fmaxf(v, 0.0f) : 0.0f;
        img_out[(size_t)j * G.P + i + PAD] = mu_new;
    }
    t[ty][tx] = mu_new;
    __syncthreads();
    const int ii = blockIdx.x * 16 + ty, jj = blockIdx.y * 16 + tx;
    if (ii < G.n && jj < G.n) imgT_out[(size_t)ii * G.P + jj + PAD] = t[tx][ty];
}

}  // namespace

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------

hipError_t launch_pad_image(const float* src, float* dst, float* dstT, int n, int P, hipStream_t s)
{
    dim3 grid(cdiv(n, 32), cdiv(n, 32));
    pad_image_kernel<<<grid, 256, 0, s>>>(src, dst, dstT, n, P);
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
    a.img = img;
    a.imgT = imgT;
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
                        const RayMeta* rm, int ray0, int nrays, const float* yt, const float* p, float* w, float* e,
                        hipStream_t s)
{
    FpArgs a{};
    a.img = img;
    a.imgT = imgT;
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
    a.e = e;
    return launch_fp<true>(segments, a, s);
}

hipError_t launch_lambda(const float* e, int ray0, int nrays, DevState* st, StepRule rule, hipStream_t s)
{
    lambda_kernel<<<1, 1024, 0, s>>>(e, ray0, nrays, st, rule);
    return hipGetLastError();
}

hipError_t launch_set_state(DevState* st, double lambda, double f_prev, int n_global, int flags, double* trace,
                            const double* schedule, hipStream_t s)
{
    set_state_kernel<<<1, 64, 0, s>>>(st, lambda, f_prev, n_global, flags, trace, schedule);
    return hipGetLastError();
}

hipError_t launch_bp_plain(const Geo& geo, const ViewRec* views, const RayGeo* rg, const float* w, int q0, int nq,
                           float* out, hipStream_t s)
{
    dim3 grid(cdiv(geo.n, 16), cdiv(geo.n, 16));
    bp_plain_kernel<<<grid, 256, 0, s>>>(geo, views, rg, w, q0, nq, out);
    return hipGetLastError();
}

hipError_t launch_bp_update(const Geo& geo, const ViewRec* views, const RayGeo* rg, const float* w, int q0, int nq,
                            const float* img, float* img_out, float* imgT_out, const DevState* st, UpdateConst uc,
                            hipStream_t s)
{
    dim3 grid(cdiv(geo.n, 16), cdiv(geo.n, 16));
    bp_update_kernel<<<grid, 256, 0, s>>>(geo, views, rg, w, q0, nq, img, img_out, imgT_out, st, uc);
    return hipGetLastError();
}

hipError_t launch_tv_grad(const float* img, float* grad, int n, float eps, hipStream_t s)
{
    dim3 grid(cdiv(n, 16), cdiv(n, 16));
    tv_grad_kernel<<<grid, 256, 0, s>>>(img, grad, n, eps);
    return hipGetLastError();
}

}  // namespace recon
