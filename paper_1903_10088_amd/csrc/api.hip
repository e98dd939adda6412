// C ABI of the reconstruction library: handle creation (ray tables built on the
// host in double precision), the single-operator entry points, and the
// ordered-subset driver that replays each subset epoch from a HIP graph.
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
#include "recon.h"

using namespace recon;

namespace recon {

thread_local std::string g_last_error;

recon_status fail(recon_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

}  // namespace recon

namespace {

#define HIP_TRY RECON_HIP_TRY

constexpr double kPi = 3.14159265358979323846;

struct Tables {
    std::vector<ViewRec> views;
    std::vector<RayGeo> rg;
    std::vector<RayMeta> rm;
    std::vector<int> perm, start, count;
    Geo geo;
};

recon_status check_geometry(const recon_geometry* g, int M)
{
    if (!g) return fail(RECON_INVALID_ARG, "geometry is NULL");
    if (g->n < 2 || g->n > 16384) return fail(RECON_INVALID_ARG, "n must be in [2, 16384]");
    if (!(g->pixel_mm > 0)) return fail(RECON_INVALID_ARG, "pixel_mm must be > 0");
    if (g->n_views < 1) return fail(RECON_INVALID_ARG, "n_views must be >= 1");
    if (g->n_channels < 1 || g->n_channels > 65535) return fail(RECON_INVALID_ARG, "n_channels out of range");
    if ((long)g->n_views * g->n_channels > (1L << 30)) return fail(RECON_INVALID_ARG, "too many rays");
    const double half = 0.5 * g->n * g->pixel_mm;
    if (!(g->sad_mm > std::sqrt(2.0) * half))
        return fail(RECON_INVALID_ARG, "sad_mm must exceed the half-diagonal of the pixel grid");
    const double gmax = g->fan_half_angle_rad > 0 ? g->fan_half_angle_rad : std::asin(half / g->sad_mm);
    if (!(gmax < kPi / 4)) return fail(RECON_INVALID_ARG, "full fan angle must be below 90 degrees");
    if (!(g->scan_arc_rad >= 0.0) || g->scan_arc_rad > 2.0 * kPi)
        return fail(RECON_INVALID_ARG, "scan_arc_rad must be in [0, 2 pi] (0: a full turn)");
    if (M < 1 || M > g->n_views) return fail(RECON_INVALID_ARG, "subsets must be in [1, n_views]");
    return RECON_OK;
}

// Ray tables in subset order, computed in double precision and stored in float.
recon_status build_tables(const recon_geometry* g, int M, Tables& T)
{
    const int N = g->n, nv = g->n_views, nch = g->n_channels;
    const double dpx = g->pixel_mm;
    const double c = 0.5 * (N - 1);
    const double half = 0.5 * N * dpx;
    const double gmax = g->fan_half_angle_rad > 0 ? g->fan_half_angle_rad : std::asin(half / g->sad_mm);
    const double dg = 2.0 * gmax / nch;

    T.perm.clear();
    T.start.assign(M, 0);
    T.count.assign(M, 0);
    for (int s = 0; s < M; ++s) {
        T.start[s] = (int)T.perm.size();
        for (int v = s; v < nv; v += M) T.perm.push_back(v);
        T.count[s] = (int)T.perm.size() - T.start[s];
    }
    T.views.assign(nv, ViewRec{});
    T.rg.assign((size_t)nv * nch, RayGeo{});
    T.rm.assign((size_t)nv * nch, RayMeta{});
    std::vector<int> major(nch);
    std::vector<double> a_tab((size_t)nv * nch), s_tab((size_t)nv * nch);
    for (int q = 0; q < nv; ++q) {
        const int v = T.perm[q];
        const double beta = view_angle(g, v);
        const double sx = g->sad_mm * std::cos(beta) / dpx, sy = g->sad_mm * std::sin(beta) / dpx;
        for (int k = 0; k < nch; ++k) {
            const double gam = ((double)k - 0.5 * (double)(nch - 1)) * dg;
            const double dx = std::cos(beta + kPi + gam), dy = std::sin(beta + kPi + gam);
            const int mj = std::fabs(dx) >= std::fabs(dy) ? 0 : 1;
            major[k] = mj;
            double slope, a, scale;
            if (mj == 0) {  // crossing row u at column t: u = sy + (t - c - sx) * dy/dx + c
                slope = dy / dx;
                a = sy + (-c - sx) * slope + c;
                scale = dpx / std::fabs(dx);
            } else {        // crossing column u at row t
                slope = dx / dy;
                a = sx + (-c - sy) * slope + c;
                scale = dpx / std::fabs(dy);
            }
            // sample lines t in [0, N-1] where -1 < u(t) < N (some in-image pixel has weight),
            // widened by one line on each side
            long lo = 1, hi = 0;
            if (std::fabs(slope) < 1e-300) {
                if (a > -1.0 && a < N) { lo = 0; hi = N - 1; }
            } else {
                double ta = (-1.0 - a) / slope, tb = ((double)N - a) / slope;
                double tmin = std::max(std::min(ta, tb), -4.0), tmax = std::min(std::max(ta, tb), (double)N + 4);
                lo = std::max(0L, (long)std::floor(tmin) - 1);
                hi = std::min((long)N - 1, (long)std::ceil(tmax) + 1);
            }
            if (lo > hi) { lo = 1; hi = 0; }
            const size_t r = (size_t)q * nch + k;
            a_tab[r] = a;
            s_tab[r] = slope;
            T.rm[r] = RayMeta{(float)scale, (uint32_t)lo | ((uint32_t)hi << 15) | ((uint32_t)mj << 30)};
        }
        int flips = 0, k_split = nch;
        for (int k = 1; k < nch; ++k)
            if (major[k] != major[k - 1]) {
                if (flips == 0) k_split = k;
                ++flips;
            }
        if (flips > 1) return fail(RECON_INVALID_ARG, "a view's rays change major axis more than once");
        ViewRec& V = T.views[q];
        V.sx = (float)sx;
        V.sy = (float)sy;
        V.cb = (float)std::cos(beta);
        V.sb = (float)std::sin(beta);
        V.ray0 = q * nch;
        V.k_split = k_split;
        V.first_major = major[0];
        V.nat_view = v;
        V.dist = (float)(g->sad_mm / dpx);
    }
    // Split u(t) = a + t slope into (a_int + t s_hi) + (a_frac + t s_lo): with
    // |a| + N < 2^B, s_hi a multiple of 2^-q and q = 23 - B, every lattice value
    // a_int + t s_hi (t < N) and its difference with an integer is an exact
    // float32, and t s_hi itself is exact because t < 2^B and s_hi has at most
    // q + 1 significant bits.
    double max_u = 0.0;
    for (size_t r = 0; r < a_tab.size(); ++r) max_u = std::max(max_u, std::fabs(a_tab[r]) + N);
    const int B = (int)std::ceil(std::log2(max_u + 2.0));
    const int qbits = 23 - B;
    if (qbits < 4) return fail(RECON_INVALID_ARG, "geometry too large for the float32 ray tables");
    const double quantum = std::ldexp(1.0, -qbits);
    for (size_t r = 0; r < a_tab.size(); ++r) {
        const double a_int = std::floor(a_tab[r]);
        const double s_hi = std::nearbyint(s_tab[r] / quantum) * quantum;
        T.rg[r] = RayGeo{(float)a_int, (float)(a_tab[r] - a_int), (float)s_hi, (float)(s_tab[r] - s_hi)};
    }
    Geo& G = T.geo;
    G.n = N;
    G.P = N + 2 * PAD;
    G.nv = nv;
    G.nch = nch;
    G.c = (float)c;
    G.dg_inv = (float)(1.0 / dg);
    G.kc = (float)(0.5 * (nch - 1));
    // the candidate window is linear in the pixel offset; its curvature error is
    // at most 1 / (2 r^2 dgamma) channels at source distance r (pixels)
    const double rmin = (g->sad_mm - std::sqrt(2.0) * half) / dpx;
    const double max_sin = std::min(1.0, std::sqrt(2.0) * half / g->sad_mm);
    const double max_tan = max_sin / std::sqrt(std::max(1e-12, 1.0 - max_sin * max_sin));
    G.use_poly = max_tan <= 0.45 ? 1 : 0;
    // atan series error bound (in channels) when the polynomial is used
    const double poly_err = G.use_poly ? std::pow(max_tan, 13) / 13.0 / dg : 0.0;
    // (the curvature term covers offsets up to 1.5 px across and 0.5 px along the
    // sampling line, as used by the gather over 2x2 pixel blocks)
    G.margin = (float)(0.05 + 2.5 / (rmin * rmin * dg) + poly_err);
    return RECON_OK;
}

void drop_graphs(recon_handle* h)
{
    for (auto& gexec : h->graph)
        if (gexec) {
            (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
        }
}

}  // namespace

namespace recon {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

recon_status validate_create(const recon_geometry* geom, int subsets, double beta, const recon_params* params)
{
    recon_status st = check_geometry(geom, subsets);
    if (st != RECON_OK) return st;
    if (!(beta >= 0) || !std::isfinite(beta)) return fail(RECON_INVALID_ARG, "beta must be finite and >= 0");
    if (params && (!(params->tv_eps_per_mm > 0) || !(params->lambda_min >= 0) || !(params->lambda0 > 0)))
        return fail(RECON_INVALID_ARG, "bad step-rule or TV parameters");
    if (params && (params->lambda_compare < 0 || params->lambda_compare > 1 || params->keep_best < 0 ||
                   params->keep_best > 1))
        return fail(RECON_INVALID_ARG, "lambda_compare and keep_best must be 0 or 1");
    return RECON_OK;
}

StepRule rule_of(const recon_handle* h)
{
    return StepRule{h->p.lambda0, h->p.lambda_inc, h->p.lambda_dec, h->p.lambda_min, h->M, h->p.lambda_compare};
}

UpdateConst update_const(const recon_handle* h)
{
    UpdateConst uc;
    // The step of Eq. 3 is taken in cm and 1/cm: mu_cm = 10 mu_mm and the
    // likelihood gradient per cm is a tenth of the per-mm one, so in mm units
    // mu' = mu + lambda (g_L,mm / 100 + (beta / M) g_R / 10).
    uc.c_l = 0.01f;
    uc.c_r = (float)(h->beta / (10.0 * h->M));
    uc.eps = (float)h->p.tv_eps_per_mm;
    uc.pad = 0.0f;
    return uc;
}

}  // namespace recon

namespace {

UpdateArgs update_args(recon_handle* h, int s, int in)
{
    UpdateArgs a;
    a.views = h->d_views;
    a.rg = h->d_raygeo;
    a.w = h->d_w;
    a.q0 = h->subset_start[s];
    a.nq = h->subset_count[s];
    a.part = h->d_part;
    a.nrays = a.nq * h->geo.nch;
    a.st_in = h->d_state + in;
    a.st_out = h->d_state + (1 - in);
    a.rule = rule_of(h);
    a.img = h->d_img[in];
    a.img_out = h->d_img[1 - in];
    a.imgT_out = h->d_imgT[1 - in];
    a.uc = update_const(h);
    return a;
}

hipError_t enqueue_fp(recon_handle* h, int s, int in, hipStream_t st)
{
    const Geo& G = h->geo;
    const int ray0 = h->subset_start[s] * G.nch, nrays = h->subset_count[s] * G.nch;
    return launch_fp_os(G, h->fp_segments, h->d_img[in], h->d_imgT[in], h->d_raygeo, h->d_raymeta, ray0, nrays,
                        h->d_yt, h->d_p, h->d_w, h->d_part, st);
}

// One sub-iteration on subset s reading image and state buffers `in`, writing
// 1 - in: the projector with its residual epilogue, then the fused step rule,
// backprojection, TV gradient and update.
hipError_t enqueue_subiter(recon_handle* h, int s, int in, hipStream_t st)
{
    hipError_t e = enqueue_fp(h, s, in, st);
    if (e != hipSuccess) return e;
    return launch_bp_update(h->geo, h->bp_variant, update_args(h, s, in), st);
}

// Graph of one full epoch (subsets 0..M-1) starting from buffer `parity`.
recon_status get_graph(recon_handle* h, int parity, hipGraphExec_t* out)
{
    if (h->graph[parity]) {
        *out = h->graph[parity];
        return RECON_OK;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    int in = parity;
    for (int s = 0; s < h->M && err == hipSuccess; ++s) {
        err = enqueue_subiter(h, s, in, h->cap_stream);
        in = 1 - in;
    }
    hipError_t end = hipStreamEndCapture(h->cap_stream, &graph);
    if (err != hipSuccess || end != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(RECON_DEVICE, std::string("graph capture failed: ") +
                                      hipGetErrorString(err != hipSuccess ? err : end));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(RECON_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    h->graph[parity] = exec;
    *out = exec;
    return RECON_OK;
}

void free_handle(recon_handle* h)
{
    if (!h) return;
    drop_graphs(h);
    void* ptrs[] = {h->d_views, h->d_raygeo, h->d_raymeta, h->d_img[0], h->d_img[1],
                    h->d_yt,    h->d_p,      h->d_w,       h->d_part,   h->d_state,  h->d_part_all,
                    h->d_fhist, h->d_fbp,     h->d_fbp_cs, h->d_res_part};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->h_state) (void)hipHostFree(h->h_state);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

}  // namespace

// ABI layout of the public structs (mirrored by the Python binding)
static_assert(sizeof(recon_geometry) == 64 && offsetof(recon_geometry, scan_arc_rad) == 56, "recon_geometry layout");
static_assert(sizeof(recon_params) == 56 && offsetof(recon_params, keep_best) == 52, "recon_params layout");
static_assert(sizeof(recon_state) == 48 && offsetof(recon_state, best_n) == 40, "recon_state layout");

extern "C" {

void recon_default_params(recon_params* out)
{
    if (!out) return;
    out->lambda0 = 0.01;
    out->lambda_inc = 1e-4;
    out->lambda_dec = 2e-4;
    out->lambda_min = 1e-4;
    out->mu0_per_mm = 0.005;
    out->tv_eps_per_mm = 1e-5;
    out->lambda_compare = 0;
    out->keep_best = 0;
}

const char* recon_status_string(recon_status s)
{
    switch (s) {
    case RECON_OK: return "ok";
    case RECON_INVALID_ARG: return "invalid argument";
    case RECON_DEVICE: return "device error";
    case RECON_NUMERIC: return "non-finite value";
    case RECON_OOM: return "out of memory";
    }
    return "unknown status";
}

const char* recon_last_error(void) { return g_last_error.c_str(); }

recon_status recon_create(const recon_geometry* geom, int32_t subsets, double beta, const recon_params* params,
                          recon_handle** out)
{
    if (!out) return fail(RECON_INVALID_ARG, "out is NULL");
    *out = nullptr;
    recon_status st = validate_create(geom, subsets, beta, params);
    if (st != RECON_OK) return st;
    recon_params p;
    recon_default_params(&p);
    if (params) p = *params;

    Tables T;
    st = build_tables(geom, subsets, T);
    if (st != RECON_OK) return st;

    recon_handle* h = new (std::nothrow) recon_handle();
    if (!h) return fail(RECON_OOM, "host allocation failed");
    h->g = *geom;
    h->p = p;
    h->M = subsets;
    h->beta = beta;
    h->geo = T.geo;
    h->perm = T.perm;
    h->subset_start = T.start;
    h->subset_count = T.count;
    h->max_subset_views = *std::max_element(T.count.begin(), T.count.end());
    // launch-shape defaults from the sweep on 512^2 x 800 views (more threads per
    // ray pay off on large images; results are identical for every choice)
    h->fp_segments = geom->n >= 384 ? 16 : (geom->n >= 192 ? 8 : 4);
    h->h_raygeo = T.rg;
    h->h_raymeta = T.rm;

    auto bail = [&](recon_status s) {
        free_handle(h);
        return s;
    };
#define H_TRY(expr)                                                                                       \
    do {                                                                                                  \
        hipError_t _e = (expr);                                                                           \
        if (_e != hipSuccess)                                                                             \
            return bail(fail(_e == hipErrorOutOfMemory ? RECON_OOM : RECON_DEVICE,                        \
                             std::string(#expr) + ": " + hipGetErrorString(_e)));                         \
    } while (0)

    H_TRY(hipGetDevice(&h->device));
    const size_t nrays = (size_t)geom->n_views * geom->n_channels;
    const size_t pimg = (size_t)geom->n * h->geo.P * sizeof(float);
    H_TRY(hipMalloc(&h->d_views, T.views.size() * sizeof(ViewRec)));
    H_TRY(hipMalloc(&h->d_raygeo, nrays * sizeof(RayGeo)));
    H_TRY(hipMalloc(&h->d_raymeta, nrays * sizeof(RayMeta)));
    for (int b = 0; b < 2; ++b) {
        // one allocation per buffer: the row-major copy, then the transposed one
        H_TRY(hipMalloc(&h->d_img[b], 2 * pimg));
        H_TRY(hipMemset(h->d_img[b], 0, 2 * pimg));
        h->d_imgT[b] = h->d_img[b] + (size_t)geom->n * h->geo.P;
    }
    H_TRY(hipMalloc(&h->d_yt, nrays * sizeof(float)));
    H_TRY(hipMalloc(&h->d_p, nrays * sizeof(float)));
    H_TRY(hipMalloc(&h->d_w, nrays * sizeof(float)));
    const size_t ngroups = ((size_t)h->max_subset_views * geom->n_channels + SQ_GROUP - 1) / SQ_GROUP;
    H_TRY(hipMalloc(&h->d_part, ngroups * sizeof(double)));
    H_TRY(hipMalloc(&h->d_part_all, (nrays + SQ_GROUP - 1) / SQ_GROUP * sizeof(double)));
    H_TRY(hipMalloc(&h->d_state, 2 * sizeof(DevState)));
    H_TRY(hipMalloc(&h->d_res_part, 2 * RES_BLOCKS * sizeof(double)));
    H_TRY(hipMalloc(&h->d_fhist, (size_t)subsets * sizeof(double)));
    // filtered-backprojection tables: D cos(gamma_k) (pixel units) and dgamma x the ramp taps
    const std::vector<float> fbp_tab = fbp_tables(geom);
    H_TRY(hipMalloc(&h->d_fbp, fbp_tab.size() * sizeof(float)));
    H_TRY(hipMemcpy(h->d_fbp, fbp_tab.data(), fbp_tab.size() * sizeof(float), hipMemcpyHostToDevice));
    // and cos / sin of every view's source angle in double, subset order
    {
        std::vector<double> cs(2 * (size_t)geom->n_views);
        for (int q = 0; q < geom->n_views; ++q) {
            const double beta = view_angle(geom, T.perm[q]);
            cs[2 * (size_t)q] = std::cos(beta);
            cs[2 * (size_t)q + 1] = std::sin(beta);
        }
        H_TRY(hipMalloc(&h->d_fbp_cs, cs.size() * sizeof(double)));
        H_TRY(hipMemcpy(h->d_fbp_cs, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    H_TRY(hipHostMalloc(&h->h_state, sizeof(DevState), hipHostMallocDefault));
    H_TRY(hipMemcpy(h->d_views, T.views.data(), T.views.size() * sizeof(ViewRec), hipMemcpyHostToDevice));
    H_TRY(hipMemcpy(h->d_raygeo, T.rg.data(), nrays * sizeof(RayGeo), hipMemcpyHostToDevice));
    H_TRY(hipMemcpy(h->d_raymeta, T.rm.data(), nrays * sizeof(RayMeta), hipMemcpyHostToDevice));
    H_TRY(hipMemset(h->d_w, 0, nrays * sizeof(float)));
    H_TRY(hipMemset(h->d_part, 0, ngroups * sizeof(double)));
    H_TRY(hipMemset(h->d_state, 0, 2 * sizeof(DevState)));
    H_TRY(hipMemset(h->d_fhist, 0, (size_t)subsets * sizeof(double)));
    H_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    H_TRY(hipDeviceSynchronize());
#undef H_TRY
    *out = h;
    return RECON_OK;
}

recon_status recon_destroy(recon_handle* h)
{
    if (!h) return RECON_OK;
    (void)hipDeviceSynchronize();
    free_handle(h);
    return RECON_OK;
}

recon_status recon_subset_size(recon_handle* h, int32_t subset, int32_t* n_views_out)
{
    if (!h || !n_views_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (subset == -1) {
        *n_views_out = h->g.n_views;
        return RECON_OK;
    }
    if (subset < 0 || subset >= h->M) return fail(RECON_INVALID_ARG, "subset out of range");
    *n_views_out = h->subset_count[subset];
    return RECON_OK;
}

recon_status recon_set_launch(recon_handle* h, int32_t fp_segments, int32_t bp_variant)
{
    if (!h) return fail(RECON_INVALID_ARG, "NULL handle");
    if (fp_segments != 0) {
        if (fp_segments != 1 && fp_segments != 2 && fp_segments != 4 && fp_segments != 8 && fp_segments != 16)
            return fail(RECON_INVALID_ARG, "fp_segments must be 1, 2, 4, 8 or 16");
        h->fp_segments = fp_segments;
    }
    if (bp_variant != 0) {
        if (bp_variant < 1 || bp_variant > 6) return fail(RECON_INVALID_ARG, "bp_variant must be in [0, 6]");
        h->bp_variant = bp_variant - 1;
    }
    drop_graphs(h);
    return RECON_OK;
}

recon_status recon_initial_image(recon_handle* h, float* d_img, void* stream)
{
    if (!h || !d_img) return fail(RECON_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_initial_image(d_img, h->g.n, (float)h->p.mu0_per_mm, as_stream(stream)));
    return RECON_OK;
}

recon_status recon_project(recon_handle* h, const float* d_img, float* d_sino, int32_t subset, void* stream)
{
    if (!h || !d_img || !d_sino) return fail(RECON_INVALID_ARG, "NULL argument");
    if (subset < -1 || subset >= h->M) return fail(RECON_INVALID_ARG, "subset out of range");
    hipStream_t s = as_stream(stream);
    const Geo& G = h->geo;
    HIP_TRY(launch_pad_image(d_img, h->d_img[0], h->d_imgT[0], G.n, G.P, s));
    const int q0 = subset < 0 ? 0 : h->subset_start[subset];
    const int nq = subset < 0 ? G.nv : h->subset_count[subset];
    HIP_TRY(launch_fp_plain(G, h->fp_segments, h->d_img[0], h->d_imgT[0], h->d_raygeo, h->d_raymeta, h->d_views, q0,
                            nq, subset < 0 ? 1 : 0, d_sino, s));
    return RECON_OK;
}

recon_status recon_backproject(recon_handle* h, const float* d_sino, float* d_img, int32_t subset, void* stream)
{
    if (!h || !d_img || !d_sino) return fail(RECON_INVALID_ARG, "NULL argument");
    if (subset < -1 || subset >= h->M) return fail(RECON_INVALID_ARG, "subset out of range");
    hipStream_t s = as_stream(stream);
    const Geo& G = h->geo;
    const int q0 = subset < 0 ? 0 : h->subset_start[subset];
    const int nq = subset < 0 ? G.nv : h->subset_count[subset];
    HIP_TRY(launch_scale_sino(d_sino, h->d_raymeta, q0 * G.nch, nq * G.nch, G.nch, h->d_views, q0,
                              subset < 0 ? 1 : 0, h->d_w, s));
    HIP_TRY(launch_bp_plain(G, h->d_views, h->d_raygeo, h->d_w, q0, nq, d_img, s));
    return RECON_OK;
}

recon_status recon_tv_grad(recon_handle* h, const float* d_img, float* d_grad, void* stream)
{
    if (!h || !d_img || !d_grad) return fail(RECON_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_tv_grad(d_img, d_grad, h->g.n, (float)h->p.tv_eps_per_mm, as_stream(stream)));
    return RECON_OK;
}

recon_status recon_os_iterate(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                              recon_state* state, double* d_trace, const double* d_lambda_schedule, void* stream)
{
    return recon_os_iterate_ex(h, d_counts, i0, d_img, n_iter, state, d_trace, d_lambda_schedule, nullptr, nullptr,
                               stream);
}

recon_status recon_os_iterate_ex(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                                 recon_state* state, double* d_trace, const double* d_lambda_schedule,
                                 double* d_f_hist, float* d_best, void* stream)
{
    return os_iterate_run(h, d_counts, i0, d_img, n_iter, state, d_trace, d_lambda_schedule, d_f_hist, d_best,
                          as_stream(stream), true);
}

}  // extern "C"

namespace recon {

recon_status os_iterate_run(recon_handle* h, const float* d_counts, float i0, float* d_img, int n_iter,
                            recon_state* state, double* d_trace, const double* d_lambda_schedule, double* d_f_hist,
                            float* d_best, hipStream_t s, bool new_graphs)
{
    if (!h || !d_counts || !d_img) return fail(RECON_INVALID_ARG, "NULL argument");
    if (!(i0 > 0) || !std::isfinite(i0)) return fail(RECON_INVALID_ARG, "i0 must be finite and > 0");
    if (n_iter < 0) return fail(RECON_INVALID_ARG, "n_iter must be >= 0");
    if (state && state->n_done < 0) return fail(RECON_INVALID_ARG, "state->n_done must be >= 0");
    if ((h->p.keep_best != 0) != (d_best != nullptr))
        return fail(RECON_INVALID_ARG, "d_best must be given exactly when keep_best is set");
    const int n_done = state ? state->n_done : 0;
    if (h->p.lambda_compare && h->M > 1 && n_done > 0 && !d_f_hist)
        return fail(RECON_INVALID_ARG, "a resumed run with lambda_compare needs the subset history d_f_hist");
    const Geo& G = h->geo;

    DevState v = fresh_state(h->p.lambda0);
    if (state && n_done > 0) {
        v.lambda = state->lambda;
        v.f_prev = state->f_prev;
        v.best_f = state->best_f;
        v.epoch_sum = state->epoch_sum;
        v.best_n = state->best_n;
    }
    v.flags = state ? state->flags : 0;
    v.n_global = n_done;
    v.trace = d_trace;
    v.schedule = d_lambda_schedule;
    v.fhist = h->p.lambda_compare ? (d_f_hist ? d_f_hist : h->d_fhist) : nullptr;
    v.best = d_best;

    HIP_TRY(launch_prep_counts(d_counts, h->d_views, G.nv, G.nch, i0, h->d_yt, h->d_p, s));
    HIP_TRY(launch_pad_image(d_img, h->d_img[0], h->d_imgT[0], G.n, G.P, s, true));
    HIP_TRY(launch_set_state(h->d_state, v, s));

    int in = 0;
    int n = 0;
    while (n < n_iter) {
        const int sub = (n_done + n) % h->M;
        if (sub == 0 && n_iter - n >= h->M && !h->graph_bad && (new_graphs || h->graph[in])) {
            hipGraphExec_t exec = nullptr;
            if (get_graph(h, in, &exec) == RECON_OK) {
                HIP_TRY(hipGraphLaunch(exec, s));
                n += h->M;
                if (h->M & 1) in = 1 - in;
                continue;
            }
            h->graph_bad = true;  // fall back to direct launches from now on
        }
        HIP_TRY(enqueue_subiter(h, sub, in, s));
        in = 1 - in;
        ++n;
    }
    if (v.fhist) HIP_TRY(launch_flush_hist(h->d_state + in, h->M, s));
    HIP_TRY(launch_unpad_image(h->d_img[in], d_img, G.n, G.P, s));
    if (state) {
        HIP_TRY(hipMemcpyAsync(h->h_state, h->d_state + in, sizeof(DevState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const DevState& r = *h->h_state;
        state->n_done = n_done + n_iter;
        state->flags = r.flags;
        state->lambda = r.lambda;
        state->f_prev = r.f_prev;
        state->best_f = r.best_f;
        state->epoch_sum = r.epoch_sum;
        state->best_n = r.best_n;
        state->reserved = 0;
        if (state->flags & 1) return fail(RECON_NUMERIC, "non-finite squared difference");
    }
    return RECON_OK;
}

}  // namespace recon

extern "C" {

recon_status recon_data_residual(recon_handle* h, const float* d_counts, float i0, const float* d_img,
                                 int32_t subset_stride, double* d_out, void* stream)
{
    if (!h || !d_counts || !d_img || !d_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (!(i0 > 0) || !std::isfinite(i0)) return fail(RECON_INVALID_ARG, "i0 must be finite and > 0");
    if (subset_stride < 1 || subset_stride > h->M ||
        (subset_stride > 1 && (h->M + subset_stride - 1) / subset_stride > RES_BLOCKS))
        return fail(RECON_INVALID_ARG, "subset_stride must be in [1, subsets], choosing at most 64 subsets if > 1");
    hipStream_t s = as_stream(stream);
    const Geo& G = h->geo;
    const long nrays = (long)G.nv * G.nch;
    HIP_TRY(launch_prep_counts(d_counts, h->d_views, G.nv, G.nch, i0, h->d_yt, h->d_p, s));
    HIP_TRY(launch_pad_image(d_img, h->d_img[0], h->d_imgT[0], G.n, G.P, s));
    if (subset_stride == 1) {
        // all views are one contiguous ray range in subset order
        HIP_TRY(launch_fp_os(G, h->fp_segments, h->d_img[0], h->d_imgT[0], h->d_raygeo, h->d_raymeta, 0, (int)nrays,
                             h->d_yt, h->d_p, h->d_w, h->d_part_all, s));
        HIP_TRY(launch_residual_final(h->d_part_all, (int)((nrays + SQ_GROUP - 1) / SQ_GROUP), d_counts, nrays,
                                      h->d_res_part, d_out, s));
        return RECON_OK;
    }
    // every subset_stride-th subset, one projection each
    long nchosen_rays = 0;
    int j = 0;
    for (int sub = 0; sub < h->M; sub += subset_stride, ++j) {
        const int ray0 = h->subset_start[sub] * G.nch, nr = h->subset_count[sub] * G.nch;
        HIP_TRY(launch_fp_os(G, h->fp_segments, h->d_img[0], h->d_imgT[0], h->d_raygeo, h->d_raymeta, ray0, nr,
                             h->d_yt, h->d_p, h->d_w, h->d_part, s));
        HIP_TRY(launch_residual_subset(h->d_part, (nr + SQ_GROUP - 1) / SQ_GROUP, h->d_res_part, j, s));
        nchosen_rays += nr;
    }
    HIP_TRY(launch_residual_strided_final(d_counts, G.nv, G.nch, h->M, subset_stride, j, nchosen_rays, h->d_res_part,
                                          d_out, s));
    return RECON_OK;
}

recon_status recon_count_pairs(recon_handle* h, int32_t subset, int32_t disc_only, int64_t* pairs)
{
    if (!h || !pairs) return fail(RECON_INVALID_ARG, "NULL argument");
    if (subset < -1 || subset >= h->M) return fail(RECON_INVALID_ARG, "subset out of range");
    const Geo& G = h->geo;
    const int q0 = subset < 0 ? 0 : h->subset_start[subset];
    const int nq = subset < 0 ? G.nv : h->subset_count[subset];
    int64_t total = 0;
    for (size_t r = (size_t)q0 * G.nch; r < (size_t)(q0 + nq) * G.nch; ++r) {
        const RayGeo g = h->h_raygeo[r];
        for (int t = 0; t < G.n; ++t) {
            const int fl = (int)std::floor(ray_offset(g, (float)t, 0.0f));
            for (int u = fl; u <= fl + 1; ++u)
                if (u >= 0 && u < G.n && (!disc_only || in_disc(t, u, G.n))) ++total;
        }
    }
    *pairs = total;
    return RECON_OK;
}

recon_status recon_read_bandwidth(int64_t bytes, int32_t reps, double* gbps_out, void* stream)
{
    if (!gbps_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (bytes < 16384 || bytes > (64L << 20) || (bytes & (bytes - 1)) != 0)
        return fail(RECON_INVALID_ARG, "bytes must be a power of two in [16 KiB, 64 MiB]");
    if (reps < 1 || reps > 100) return fail(RECON_INVALID_ARG, "reps must be in [1, 100]");
    hipStream_t s = as_stream(stream);
    constexpr int kBlocks = 2048;  // 8 blocks of 256 threads per compute unit
    float* buf = nullptr;
    float* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMalloc(&buf, (size_t)bytes);
    if (err == hipSuccess) err = hipMalloc(&out, (size_t)kBlocks * 256 * sizeof(float));
    if (err == hipSuccess) err = hipMemsetAsync(buf, 0, (size_t)bytes, s);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    const uint32_t n16 = (uint32_t)(bytes / 16);
    // one untimed launch brings the buffer into every XCD's L2
    if (err == hipSuccess) err = launch_read_probe(buf, n16, kBlocks, out, s);
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch_read_probe(buf, n16, kBlocks, out, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
    if (err != hipSuccess) return fail(RECON_DEVICE, std::string("read probe: ") + hipGetErrorString(err));
    *gbps_out = (double)kBlocks * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return RECON_OK;
}

recon_status recon_valu_rate(int32_t op, int32_t reps, double* lane_ops_out, void* stream)
{
    if (!lane_ops_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (op < 0 || op > 5) return fail(RECON_INVALID_ARG, "op must be in [0, 5]");
    if (reps < 1 || reps > 100) return fail(RECON_INVALID_ARG, "reps must be in [1, 100]");
    hipStream_t s = as_stream(stream);
    constexpr int kBlocks = 2048;  // 8 blocks of 4 waves per compute unit: 8 waves per SIMD
    uint32_t* seed = nullptr;
    float* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    long inst = 0;
    hipError_t err = hipMalloc(&seed, 256 * sizeof(uint32_t));
    if (err == hipSuccess) err = hipMalloc(&out, (size_t)kBlocks * 256 * sizeof(float));
    if (err == hipSuccess) err = hipMemsetAsync(seed, 0x5b, 256 * sizeof(uint32_t), s);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch_valu_probe(op, seed, kBlocks, out, &inst, s);  // untimed
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch_valu_probe(op, seed, kBlocks, out, &inst, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (seed) (void)hipFree(seed);
    if (out) (void)hipFree(out);
    if (err != hipSuccess) return fail(RECON_DEVICE, std::string("VALU probe: ") + hipGetErrorString(err));
    *lane_ops_out = (double)inst * 64.0 * reps / (ms * 1e-3);
    return RECON_OK;
}

recon_status recon_time_kernels(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                                double* ms_out, void* stream)
{
    if (!h || !d_counts || !d_img || !ms_out) return fail(RECON_INVALID_ARG, "NULL argument");
    if (n_iter < 1 || n_iter > 4096) return fail(RECON_INVALID_ARG, "n_iter must be in [1, 4096]");
    if (!(i0 > 0)) return fail(RECON_INVALID_ARG, "i0 must be > 0");
    hipStream_t s = as_stream(stream);
    const Geo& G = h->geo;
    HIP_TRY(launch_prep_counts(d_counts, h->d_views, G.nv, G.nch, i0, h->d_yt, h->d_p, s));
    HIP_TRY(launch_pad_image(d_img, h->d_img[0], h->d_imgT[0], G.n, G.P, s, true));
    HIP_TRY(launch_set_state(h->d_state, fresh_state(h->p.lambda0), s));
    // one sub-iteration of every subset first, so residuals and state are realistic
    for (int sub = 0; sub < h->M; ++sub) HIP_TRY(enqueue_subiter(h, sub, 0, s));
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    recon_status status = RECON_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) status = fail(RECON_DEVICE, "hipEventCreate failed");
    // each kernel n_iter times back to back (subsets in turn) between two events
    hipError_t err = status == RECON_OK ? hipEventRecord(ev[0], s) : hipSuccess;
    for (int n = 0; n < n_iter && status == RECON_OK && err == hipSuccess; ++n)
        err = enqueue_fp(h, n % h->M, 0, s);
    if (status == RECON_OK && err == hipSuccess) err = hipEventRecord(ev[1], s);
    // (the step rule has no launch of its own: it runs inside the update kernel)
    if (status == RECON_OK && err == hipSuccess) err = hipEventRecord(ev[2], s);
    for (int n = 0; n < n_iter && status == RECON_OK && err == hipSuccess; ++n)
        err = launch_bp_update(G, h->bp_variant, update_args(h, n % h->M, 0), s);
    if (status == RECON_OK && err == hipSuccess) err = hipEventRecord(ev[3], s);
    // then the kernels in their sub-iteration order (projector, update, subsets in turn), each
    // launch between two events of its own, as they meet each other's cache state in a run
    const int ns = std::min(n_iter, 256);
    std::vector<hipEvent_t> se(4 * (size_t)ns, nullptr);
    for (auto& e : se)
        if (status == RECON_OK && hipEventCreate(&e) != hipSuccess) status = fail(RECON_DEVICE, "hipEventCreate failed");
    for (int n = 0; n < ns && status == RECON_OK && err == hipSuccess; ++n) {
        err = hipEventRecord(se[4 * n], s);
        if (err == hipSuccess) err = enqueue_fp(h, n % h->M, 0, s);
        if (err == hipSuccess) err = hipEventRecord(se[4 * n + 1], s);
        if (err == hipSuccess) err = hipEventRecord(se[4 * n + 2], s);
        if (err == hipSuccess) err = launch_bp_update(G, h->bp_variant, update_args(h, n % h->M, 0), s);
        if (err == hipSuccess) err = hipEventRecord(se[4 * n + 3], s);
    }
    if (status == RECON_OK && err == hipSuccess) err = hipStreamSynchronize(s);
    if (status == RECON_OK && err != hipSuccess)
        status = fail(RECON_DEVICE, std::string("timing run: ") + hipGetErrorString(err));
    if (status == RECON_OK) {
        for (int k = 0; k < 3; ++k) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            ms_out[k] = ms / n_iter;
        }
        double fp_seq = 0.0, bp_seq = 0.0;
        for (int n = 0; n < ns; ++n) {
            float a = 0.0f, b = 0.0f;
            (void)hipEventElapsedTime(&a, se[4 * n], se[4 * n + 1]);
            (void)hipEventElapsedTime(&b, se[4 * n + 2], se[4 * n + 3]);
            fp_seq += a;
            bp_seq += b;
        }
        ms_out[3] = bp_seq / ns;
        ms_out[4] = fp_seq / ns;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : se)
        if (e) (void)hipEventDestroy(e);
    return status;
}

// Host-only check of the gather's candidate windows (no GPU needed): for every
// pixel and view, every ray of the view whose hat weight on the pixel is
// nonzero must lie inside the window the kernel enumerates, and every ray's
// sample range must hold all of its nonzero samples.  Returns the number of
// misses in *missed and the enumerated candidate count in *candidates.
recon_status recon_check_tables(const recon_geometry* geom, int32_t subsets, int32_t view_stride, int64_t* missed,
                                int64_t* candidates, int64_t* pairs)
{
    if (!missed || !candidates || !pairs) return fail(RECON_INVALID_ARG, "NULL argument");
    recon_status st = check_geometry(geom, subsets);
    if (st != RECON_OK) return st;
    Tables T;
    st = build_tables(geom, subsets, T);
    if (st != RECON_OK) return st;
    const Geo& G = T.geo;
    const int N = G.n, nch = G.nch;
    if (view_stride < 1) view_stride = 1;
    int64_t miss = 0, cand = 0, npairs = 0;
    for (int q = 0; q < G.nv; q += view_stride) {
        const ViewRec& v = T.views[q];
        // sample ranges: weight outside [lo, hi] must vanish
        for (int k = 0; k < nch; ++k) {
            const RayGeo g = T.rg[(size_t)q * nch + k];
            const uint32_t pk = T.rm[(size_t)q * nch + k].packed;
            const int lo = (int)(pk & 0x7fffu), hi = (int)((pk >> 15) & 0x7fffu);
            for (int t = 0; t < N; ++t) {
                const float u = ray_offset(g, (float)t, 0.0f);
                const bool touches = u > -1.0f && u < (float)N;
                if (touches && (t < lo || t > hi)) ++miss;
            }
        }
        int x0, x1, y0, y1;
        major_intervals(v, nch, x0, x1, y0, y1);
        // the staged gather's per-tile linear windows
        for (int tj0 = 0; tj0 < N; tj0 += 16)
            for (int ti0 = 0; ti0 < N; ti0 += 16) {
                const TileView tv = tile_view(G, v, (float)ti0 + 7.5f - G.c, (float)tj0 + 7.5f - G.c);
                // the staged channel range, when the view is staged, holds every window
                int k0, cnt;
                stage_range(tv, nch, STAGE_SLOTS, k0, cnt);
                auto outside_stage = [&](int lo, int hi) { return cnt > 0 && lo <= hi && (lo < k0 || hi >= k0 + cnt); };
                for (int j = tj0; j < std::min(N, tj0 + 16); ++j)
                    for (int i = ti0; i < std::min(N, ti0 + 16); ++i) {
                        const float dX = (float)(i - ti0) - 7.5f, dY = (float)(j - tj0) - 7.5f;
                        const float kp = fmaf(tv.gx, dX, fmaf(tv.gy, dY, tv.kpc));
                        int lo, hi;
                        candidate_range(kp, tv.hwx, x0, x1, lo, hi);
                        if (x0 < x1 && outside_stage(lo, hi)) ++miss;
                        for (int k = x0; k < x1; ++k)
                            if (hat(ray_offset(T.rg[(size_t)q * nch + k], (float)i, (float)j)) > 0.0f &&
                                (k < lo || k > hi))
                                ++miss;
                        candidate_range(kp, tv.hwy, y0, y1, lo, hi);
                        if (y0 < y1 && outside_stage(lo, hi)) ++miss;
                        for (int k = y0; k < y1; ++k)
                            if (hat(ray_offset(T.rg[(size_t)q * nch + k], (float)j, (float)i)) > 0.0f &&
                                (k < lo || k > hi))
                                ++miss;
                    }
                // the blocked gathers' windows (PX x PY pixels per thread): each holds the
                // windows of its pixels and lies in the staged range
                for (int shape = 0; shape < 3; ++shape) {
                    const int PX = shape == 0 ? 1 : 2, PY = shape == 1 ? 1 : 2;
                    const float spread = block_spread(tv, PX, PY);
                    for (int j0 = tj0; j0 < std::min(N, tj0 + 16); j0 += PY)
                        for (int i0 = ti0; i0 < std::min(N, ti0 + 16); i0 += PX) {
                            const float dXb = (float)(i0 - ti0) + 0.5f * (PX - 1) - 7.5f;
                            const float dYb = (float)(j0 - tj0) + 0.5f * (PY - 1) - 7.5f;
                            const float kpb = fmaf(tv.gx, dXb, fmaf(tv.gy, dYb, tv.kpc));
                            int bxl, bxh, byl, byh;
                            candidate_range(kpb, tv.hwx + spread, x0, x1, bxl, bxh);
                            candidate_range(kpb, tv.hwy + spread, y0, y1, byl, byh);
                            if (x0 < x1 && outside_stage(bxl, bxh)) ++miss;
                            if (y0 < y1 && outside_stage(byl, byh)) ++miss;
                            for (int b = 0; b < PY; ++b)
                                for (int a = 0; a < PX; ++a) {
                                    const int i = i0 + a, j = j0 + b;
                                    if (i >= N || j >= N) continue;
                                    const float kp = fmaf(tv.gx, (float)(i - ti0) - 7.5f,
                                                          fmaf(tv.gy, (float)(j - tj0) - 7.5f, tv.kpc));
                                    int lo, hi;
                                    candidate_range(kp, tv.hwx, x0, x1, lo, hi);
                                    if (x0 < x1 && lo <= hi && (lo < bxl || hi > bxh)) ++miss;
                                    candidate_range(kp, tv.hwy, y0, y1, lo, hi);
                                    if (y0 < y1 && lo <= hi && (lo < byl || hi > byh)) ++miss;
                                }
                        }
                }
            }
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const PixelView pv = pixel_view(G, v, (float)i - G.c, (float)j - G.c);
                int lo, hi;
                candidate_range(pv.kp, pv.hwx, x0, x1, lo, hi);
                if (x0 < x1) cand += std::max(0, hi - lo + 1);
                for (int k = x0; k < x1; ++k) {
                    const float wgt = hat(ray_offset(T.rg[(size_t)q * nch + k], (float)i, (float)j));
                    if (wgt > 0.0f) {
                        ++npairs;
                        if (k < lo || k > hi) ++miss;
                    }
                }
                candidate_range(pv.kp, pv.hwy, y0, y1, lo, hi);
                if (y0 < y1) cand += std::max(0, hi - lo + 1);
                for (int k = y0; k < y1; ++k) {
                    const float wgt = hat(ray_offset(T.rg[(size_t)q * nch + k], (float)j, (float)i));
                    if (wgt > 0.0f) {
                        ++npairs;
                        if (k < lo || k > hi) ++miss;
                    }
                }
            }
    }
    *missed = miss;
    *candidates = cand;
    *pairs = npairs;
    return RECON_OK;
}

}  // extern "C"
