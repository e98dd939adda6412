/*
 * FP64 CPU oracle for OS-TV statistical iterative reconstruction
 * (Ozaki et al., "Fast Statistical Iterative Reconstruction for MVCT in
 * TomoTherapy", arXiv:1903.10088).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant with the HIP
 * path: geometry, projector, transpose, TV, likelihood, step rule and the
 * ordered-subset loop are all written out here from their definitions.
 *
 * Plain and slow on purpose: every loop runs over the full index range with
 * explicit bounds tests, in double precision, in the paper's units (cm, 1/cm)
 * inside the iteration.  OpenMP is used only over independent rays (projection)
 * or fixed view chunks whose partial images are summed in chunk order
 * (transpose), so results do not depend on the thread count.
 *
 * Where the paper is silent (projector, geometry, likelihood normalisation,
 * TV discretisation, subset order, step floor) the readings are stated at the
 * function that takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Fan-beam geometry (lengths in mm, angles in rad). */
typedef struct {
    int32_t n;                  /* image is n x n */
    int32_t pad0;
    double pixel_mm;
    int32_t n_views, n_channels;
    double sad_mm, sdd_mm;
    double fan_half_angle_rad;  /* 0: asin(R/SAD), R = n*pixel/2 */
    double start_angle_rad;
    double scan_arc_rad;        /* angular range swept by the views; 0: a full turn (2 pi) */
} og_geometry;

/* Step-rule and prior parameters. */
typedef struct {
    double lambda0;        /* initial convergence parameter, 0.01 (section 3.C.2) */
    double lambda_inc;     /* added when the squared difference decreased, 1e-4 (Eq. 4) */
    double lambda_dec;     /* subtracted when it did not, 2e-4 (Eq. 5) */
    double lambda_min;     /* floor; the paper gives none (reading: 1e-4) */
    double mu0_per_mm;     /* homogeneous initial image, 0.05/cm = 0.005/mm (section 3.C.2) */
    double tv_eps_per_mm;  /* TV smoothing, 1e-5/mm (reading) */
    int32_t lambda_compare; /* 0: compare f_n with the previous sub-iteration's f (literal reading);
                               1: with the same subset's f one epoch earlier (during the first epoch,
                               with the previous sub-iteration's) */
    int32_t keep_best;      /* 1: keep the iterate that ends the epoch of least summed f (section 4.B) */
} og_params;

/* Resumable iteration state. */
typedef struct {
    int32_t n_done;   /* sub-iterations already run */
    int32_t flags;    /* bit 0: a non-finite value was met */
    double lambda;    /* lambda of the last sub-iteration */
    double f_prev;    /* squared difference of the last sub-iteration */
    double best_f;    /* least epoch sum of f so far (keep_best; +inf before the first epoch ends) */
    double epoch_sum; /* sum of f over the current, unfinished epoch */
    int32_t best_n;   /* sub-iterations that produced the kept iterate (0: none yet) */
    int32_t pad;
} og_state;

enum { OG_OK = 0, OG_INVALID = 1, OG_NUMERIC = 3 };

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

static int geometry_ok(const og_geometry* g)
{
    if (!g || g->n <= 0 || g->pixel_mm <= 0 || g->n_views <= 0 || g->n_channels <= 0) return 0;
    double half = 0.5 * g->n * g->pixel_mm;
    /* every pixel must lie between source and detector */
    if (g->sad_mm <= sqrt(2.0) * half) return 0;
    /* a partial arc (limited-angle data) lies in (0, 2 pi]; 0 selects the full turn */
    if (!(g->scan_arc_rad >= 0.0) || g->scan_arc_rad > 2.0 * M_PI) return 0;
    return 1;
}

/* Source angle of view v: the views step counter-clockwise from start_angle by
 * arc / n_views, arc = scan_arc_rad, or 2 pi for a full turn.  A partial arc
 * is the limited-data case (section 4, reconstructed images: fewer projection
 * data); its n_views views cover [start, start + arc) at the same spacing a
 * full turn of 2 pi n_views / arc views would have. */
static double view_angle(const og_geometry* g, int v)
{
    const double arc = g->scan_arc_rad > 0.0 ? g->scan_arc_rad : 2.0 * M_PI;
    return g->start_angle_rad + arc * (double)v / (double)g->n_views;
}

static double fan_half_angle(const og_geometry* g)
{
    if (g->fan_half_angle_rad > 0) return g->fan_half_angle_rad;
    return asin(0.5 * g->n * g->pixel_mm / g->sad_mm);
}

/* Source position and unit direction of ray (view v, channel k): the source
 * sits at angle view_angle(v);
 * channel k sits at fan angle (k - (n_ch-1)/2) * dgamma on an arc centred on
 * the source, dgamma = 2 gamma_max / n_ch; the ray leaves the source towards
 * angle beta + pi + gamma. */
static void ray_of(const og_geometry* g, int v, int k, double* sx, double* sy, double* dx, double* dy)
{
    double beta = view_angle(g, v);
    double dgam = 2.0 * fan_half_angle(g) / (double)g->n_channels;
    double gam = ((double)k - 0.5 * (double)(g->n_channels - 1)) * dgam;
    *sx = g->sad_mm * cos(beta);
    *sy = g->sad_mm * sin(beta);
    *dx = cos(beta + M_PI + gam);
    *dy = sin(beta + M_PI + gam);
}

/* Joseph's interpolation weights of one ray.  A ray with |dx| >= |dy| is
 * sampled once per image column (x-major; ties go to x), else once per row.
 * At column i it meets the line x = x_i at continuous row u; the two rows
 * floor(u) and floor(u)+1 receive (1-f) and f (f = u - floor u) times the
 * path length per column, delta / |dx|.  Rows outside the image hold zero and
 * get no entry.  `delta` is the pixel size in the caller's length unit; the
 * sampling positions depend only on the mm geometry.  Returns the count of
 * (pixel index, weight) pairs written. */
static int joseph_weights(const og_geometry* g, double delta, int v, int k, int32_t* idx, double* wt)
{
    const int N = g->n;
    const double c = 0.5 * (double)(N - 1);
    const double px = g->pixel_mm;
    double sx, sy, dx, dy;
    ray_of(g, v, k, &sx, &sy, &dx, &dy);
    int cnt = 0;
    if (fabs(dx) >= fabs(dy)) {
        double step = delta / fabs(dx);
        for (int i = 0; i < N; ++i) {
            double x = ((double)i - c) * px;
            double t = (x - sx) / dx;
            double y = sy + t * dy;
            double u = y / px + c;
            double fl = floor(u);
            double f = u - fl;
            long j = (long)fl;
            if (j >= 0 && j < N) { idx[cnt] = (int32_t)(j * N + i); wt[cnt++] = step * (1.0 - f); }
            if (j + 1 >= 0 && j + 1 < N) { idx[cnt] = (int32_t)((j + 1) * N + i); wt[cnt++] = step * f; }
        }
    } else {
        double step = delta / fabs(dy);
        for (int j = 0; j < N; ++j) {
            double y = ((double)j - c) * px;
            double t = (y - sy) / dy;
            double x = sx + t * dx;
            double u = x / px + c;
            double fl = floor(u);
            double f = u - fl;
            long i = (long)fl;
            if (i >= 0 && i < N) { idx[cnt] = (int32_t)(j * N + i); wt[cnt++] = step * (1.0 - f); }
            if (i + 1 >= 0 && i + 1 < N) { idx[cnt] = (int32_t)(j * N + i + 1); wt[cnt++] = step * f; }
        }
    }
    return cnt;
}

/* Major axis of every ray, [n_views][n_channels]: 0 = x-major, 1 = y-major. */
int oracle_ray_major(const og_geometry* g, int32_t* major)
{
    if (!geometry_ok(g) || !major) return OG_INVALID;
    for (int v = 0; v < g->n_views; ++v)
        for (int k = 0; k < g->n_channels; ++k) {
            double sx, sy, dx, dy;
            ray_of(g, v, k, &sx, &sy, &dx, &dy);
            major[(size_t)v * g->n_channels + k] = fabs(dx) >= fabs(dy) ? 0 : 1;
        }
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Projection and its transpose                                              */
/* ------------------------------------------------------------------------ */

/* l = A img over the listed views (output rows follow the list). */
static void project_views(const og_geometry* g, double delta, const double* img, double* sino,
                          const int32_t* views, int n_sel)
{
    const int nch = g->n_channels;
    const long total = (long)n_sel * nch;
#pragma omp parallel
    {
        int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)g->n);
        double* wt = (double*)malloc(sizeof(double) * 2 * (size_t)g->n);
#pragma omp for schedule(static)
        for (long r = 0; r < total; ++r) {
            int vs = (int)(r / nch), k = (int)(r % nch);
            int cnt = joseph_weights(g, delta, views[vs], k, idx, wt);
            double acc = 0.0;
            for (int e = 0; e < cnt; ++e) acc += wt[e] * img[idx[e]];
            sino[r] = acc;
        }
        free(idx);
        free(wt);
    }
}

/* img = A^T sino over the listed views, by scattering every ray's weights:
 * the same weights as the projection, so <A x, y> = <x, A^T y> up to
 * rounding.  Views are split into at most 16 fixed chunks; each chunk
 * accumulates its own image and the chunks are added in order. */
#define OG_BP_CHUNKS 16
static void backproject_views(const og_geometry* g, double delta, const double* sino, double* img,
                              const int32_t* views, int n_sel)
{
    const int N = g->n, nch = g->n_channels;
    const size_t npix = (size_t)N * N;
    int nchunk = n_sel < OG_BP_CHUNKS ? n_sel : OG_BP_CHUNKS;
    memset(img, 0, sizeof(double) * npix);
    if (nchunk <= 0) return;
    double* part = (double*)calloc((size_t)nchunk * npix, sizeof(double));
#pragma omp parallel
    {
        int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)N);
        double* wt = (double*)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < nchunk; ++c) {
            int v0 = (int)((long)c * n_sel / nchunk), v1 = (int)((long)(c + 1) * n_sel / nchunk);
            double* acc = part + (size_t)c * npix;
            for (int vs = v0; vs < v1; ++vs)
                for (int k = 0; k < nch; ++k) {
                    double y = sino[(size_t)vs * nch + k];
                    int cnt = joseph_weights(g, delta, views[vs], k, idx, wt);
                    for (int e = 0; e < cnt; ++e) acc[idx[e]] += wt[e] * y;
                }
        }
        free(idx);
        free(wt);
    }
    for (int c = 0; c < nchunk; ++c) {
        const double* p = part + (size_t)c * npix;
        for (size_t r = 0; r < npix; ++r) img[r] += p[r];
    }
    free(part);
}

static int32_t* all_views(const og_geometry* g, const int32_t* views, int n_sel, int* n_out)
{
    int32_t* v = NULL;
    if (views) {
        *n_out = n_sel;
        return NULL;
    }
    v = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n_views);
    for (int i = 0; i < g->n_views; ++i) v[i] = i;
    *n_out = g->n_views;
    return v;
}

/* Line integrals in mm geometry: sino[sel][k] = sum of path-length (mm)
 * weighted samples of img (1/mm).  views == NULL projects all views. */
int oracle_project(const og_geometry* g, const double* img, double* sino, const int32_t* views, int32_t n_sel)
{
    if (!geometry_ok(g) || !img || !sino) return OG_INVALID;
    int n;
    int32_t* own = all_views(g, views, n_sel, &n);
    const int32_t* vl = own ? own : views;
    for (int i = 0; i < n; ++i)
        if (vl[i] < 0 || vl[i] >= g->n_views) { free(own); return OG_INVALID; }
    project_views(g, g->pixel_mm, img, sino, vl, n);
    free(own);
    return OG_OK;
}

/* Transpose of oracle_project (weights in mm). */
int oracle_backproject(const og_geometry* g, const double* sino, double* img, const int32_t* views, int32_t n_sel)
{
    if (!geometry_ok(g) || !img || !sino) return OG_INVALID;
    int n;
    int32_t* own = all_views(g, views, n_sel, &n);
    const int32_t* vl = own ? own : views;
    for (int i = 0; i < n; ++i)
        if (vl[i] < 0 || vl[i] >= g->n_views) { free(own); return OG_INVALID; }
    backproject_views(g, g->pixel_mm, sino, img, vl, n);
    free(own);
    return OG_OK;
}

/* Nonzero pattern size of the listed views' rows of A: (ray, in-image pixel)
 * pairs.  It counts the pixel reads of the projection and the sinogram reads
 * of the gather transpose. */
int oracle_count_pairs(const og_geometry* g, const int32_t* views, int32_t n_sel, int64_t* pairs)
{
    if (!geometry_ok(g) || !pairs) return OG_INVALID;
    int n;
    int32_t* own = all_views(g, views, n_sel, &n);
    const int32_t* vl = own ? own : views;
    int64_t total = 0;
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)g->n);
    double* wt = (double*)malloc(sizeof(double) * 2 * (size_t)g->n);
    for (int vs = 0; vs < n; ++vs)
        for (int k = 0; k < g->n_channels; ++k) total += joseph_weights(g, 1.0, vl[vs], k, idx, wt);
    free(idx);
    free(wt);
    free(own);
    *pairs = total;
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Total variation (section 2: TV prior; discretisation is a reading)        */
/* ------------------------------------------------------------------------ */

/* TV(mu) = sum_r phi_r, phi_r = sqrt(dx_r^2 + dy_r^2 + eps^2), with forward
 * differences dx = mu[j][i+1]-mu[j][i], dy = mu[j+1][i]-mu[j][i] and a zero
 * difference past the last column / row.  Writes the value and
 * g_R = -dTV/dmu (the prior R = -TV, so g_R is the ascent direction of R). */
int oracle_tv(int32_t n, double eps, const double* img, double* tv_value, double* g_r)
{
    if (n <= 0 || !img || eps <= 0) return OG_INVALID;
    const size_t npix = (size_t)n * n;
    double* dxv = (double*)malloc(sizeof(double) * npix);
    double* dyv = (double*)malloc(sizeof(double) * npix);
    double* phi = (double*)malloc(sizeof(double) * npix);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            size_t r = (size_t)j * n + i;
            double dx = (i + 1 < n) ? img[r + 1] - img[r] : 0.0;
            double dy = (j + 1 < n) ? img[r + n] - img[r] : 0.0;
            dxv[r] = dx;
            dyv[r] = dy;
            phi[r] = sqrt(dx * dx + dy * dy + eps * eps);
        }
    if (tv_value) {
        double s = 0.0;
        for (size_t r = 0; r < npix; ++r) s += phi[r];
        *tv_value = s;
    }
    if (g_r) {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t r = (size_t)j * n + i;
                /* phi_r depends on mu_r through -dx_r and -dy_r */
                double d = -(dxv[r] + dyv[r]) / phi[r];
                /* phi at (j, i-1) depends on mu_r through +dx */
                if (i > 0) d += dxv[r - 1] / phi[r - 1];
                /* phi at (j-1, i) depends on mu_r through +dy */
                if (j > 0) d += dyv[r - n] / phi[r - n];
                g_r[r] = -d;
            }
    }
    free(dxv);
    free(dyv);
    free(phi);
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Likelihood (section 2: Poisson photon statistics)                         */
/* ------------------------------------------------------------------------ */

/* Transmission Poisson log-likelihood divided by the blank-scan count I0,
 * up to constants: L = sum_i [ -yt_i l_i - exp(-l_i) ], yt = y / I0 (a
 * reading: the paper gives no normalisation).  Its gradient with respect to
 * the image is A^T (exp(-l) - yt). */
double oracle_loglik(int64_t n_rays, const double* ell, const double* ytilde)
{
    double s = 0.0;
    for (int64_t i = 0; i < n_rays; ++i) s += -ytilde[i] * ell[i] - exp(-ell[i]);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Adaptive convergence parameter (Eqs. 4-5)                                 */
/* ------------------------------------------------------------------------ */

/* lambda_n from lambda_{n-1}: + lambda_inc when the squared difference
 * decreased strictly (Eq. 4), otherwise - lambda_dec (Eq. 5; a tie counts as
 * "not decreased"); then the floor lambda_min (reading).  At n = 0 there is
 * nothing to compare and lambda_0 is used. */
double oracle_lambda_next(const og_params* p, int32_t first, double lambda_prev, double f_n, double f_prev)
{
    if (first) return p->lambda0;
    double l = (f_n < f_prev) ? lambda_prev + p->lambda_inc : lambda_prev - p->lambda_dec;
    return l < p->lambda_min ? p->lambda_min : l;
}

/* ------------------------------------------------------------------------ */
/* Filtered backprojection (the comparison baseline of sections 1 and 4)     */
/* ------------------------------------------------------------------------ */

/* Fan-beam filtered backprojection over the full turn for the equiangular
 * arc geometry above (the paper compares with FBP but does not describe it;
 * this is the textbook algorithm of Kak and Slaney, Principles of
 * Computerized Tomographic Imaging, ch. 3, for equiangular rays):
 *   R'(v, k) = R(v, k) D cos(gamma_k)                        (D = sad_mm)
 *   Q(v, k)  = dgamma sum_k' R'(v, k') h(k - k'),   h(0) = 1 / (8 dgamma^2),
 *              h(m) = 0 for even m, -1 / (2 pi^2 sin^2(m dgamma)) for odd m
 *   f(x, y)  = dbeta sum_v Q(v, gamma') / L^2,   dbeta = 2 pi / n_views,
 * with gamma' the fan angle and L the distance from view v's source to
 * (x, y), Q linearly interpolated in gamma and zero outside the channels.
 * sino: [n_views][n_ch] line integrals (natural view order); img: [n][n],
 * 1/mm (no mask).  Full turns only: a partial arc would need redundancy
 * weights, which the comparison method is not stated to use. */
int oracle_fbp(const og_geometry* g, const double* sino, double* img)
{
    if (!geometry_ok(g) || !sino || !img) return OG_INVALID;
    if (g->scan_arc_rad != 0.0 && g->scan_arc_rad != 2.0 * M_PI) return OG_INVALID;
    const int N = g->n, nv = g->n_views, nch = g->n_channels;
    const double dgam = 2.0 * fan_half_angle(g) / (double)nch;
    const double D = g->sad_mm;
    double* h = (double*)malloc(sizeof(double) * (size_t)(2 * nch - 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)nv * nch);
    for (int m = -(nch - 1); m <= nch - 1; ++m) {
        double v;
        if (m == 0)
            v = 1.0 / (8.0 * dgam * dgam);
        else if (m % 2 == 0)
            v = 0.0;
        else {
            const double s = sin((double)m * dgam);
            v = -1.0 / (2.0 * M_PI * M_PI * s * s);
        }
        h[m + nch - 1] = v;
    }
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v)
        for (int k = 0; k < nch; ++k) {
            double acc = 0.0;
            for (int kk = 0; kk < nch; ++kk) {
                const double gam = ((double)kk - 0.5 * (double)(nch - 1)) * dgam;
                acc += sino[(size_t)v * nch + kk] * D * cos(gam) * h[k - kk + nch - 1];
            }
            q[(size_t)v * nch + k] = dgam * acc;
        }
    const double c = 0.5 * (double)(N - 1), dbeta = 2.0 * M_PI / (double)nv;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const double x = ((double)i - c) * g->pixel_mm, y = ((double)j - c) * g->pixel_mm;
            double acc = 0.0;
            for (int v = 0; v < nv; ++v) {
                const double beta = g->start_angle_rad + 2.0 * M_PI * (double)v / (double)nv;
                const double sx = D * cos(beta), sy = D * sin(beta);
                const double ux = -cos(beta), uy = -sin(beta); /* towards the origin */
                const double dx = x - sx, dy = y - sy;
                const double gam = atan2(ux * dy - uy * dx, ux * dx + uy * dy);
                const double kf = gam / dgam + 0.5 * (double)(nch - 1);
                const double k0 = floor(kf), f = kf - k0;
                const int ki = (int)k0;
                double val = 0.0;
                if (ki >= 0 && ki < nch) val += (1.0 - f) * q[(size_t)v * nch + ki];
                if (ki + 1 >= 0 && ki + 1 < nch) val += f * q[(size_t)v * nch + ki + 1];
                acc += val / (dx * dx + dy * dy);
            }
            img[(size_t)j * N + i] = dbeta * acc;
        }
    free(h);
    free(q);
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Ordered-subset gradient iteration (Eq. 3, section 3.D)                    */
/* ------------------------------------------------------------------------ */

/* Homogeneous initial image mu0 inside the reconstruction circle
 * x^2 + y^2 <= (N pixel / 2)^2, zero outside (section 3.C.2). */
int oracle_initial_image(const og_geometry* g, double mu0_per_mm, double* img)
{
    if (!geometry_ok(g) || !img) return OG_INVALID;
    const int N = g->n;
    const double c = 0.5 * (N - 1), R = 0.5 * N * g->pixel_mm;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double x = (i - c) * g->pixel_mm, y = (j - c) * g->pixel_mm;
            img[(size_t)j * N + i] = (x * x + y * y <= R * R) ? mu0_per_mm : 0.0;
        }
    return OG_OK;
}

/* Runs n_iter sub-iterations of
 *   mu^(n+1) = mask * max(0, mu^(n) + lambda_n [dL_s/dmu + (beta/M) dR/dmu])
 * (Eq. 3 with the TV weight times the thinning factor 1/M, section 3.D; the
 * positivity of Eq. 1 as a clamp), in cm and 1/cm.
 *
 * Subsets: subset s holds the views v with v mod M == s (equal-interval
 * thinning, section 3.D), visited in order s = n mod M; one sub-iteration is
 * one "iteration" of the paper.  f_n is the mean over the subset's rays of
 * (l_i - p_i)^2, p = ln(I0 / max(y, 1)): the squared difference between
 * reprojection and projection (section 3.C.2), compared with the previous
 * sub-iteration's f to step lambda (Eqs. 4-5).
 *
 * counts: [n_views][n_ch] in natural view order.  img: in/out, 1/mm; the
 * start image is taken as zero outside the reconstruction disc (the iterate is
 * held there at zero, reading of Eq. 1's support).
 *
 * Best iterate (section 4.B: the image at the minimum of the oscillating
 * squared difference is kept): with keep_best, f is summed over each complete
 * epoch (sub-iterations n with n mod M = 0 .. M-1, n counted from the fresh
 * start); when an epoch's sum is below every earlier one, the image that epoch
 * ends with, mu^(n+1), is copied to best_img (1/mm).  f_hist: NULL or [M]
 * in/out, f of each subset's latest sub-iteration (lambda_compare = 1 reads
 * it, so a resumed run passes it back).
 *
 * state: NULL for a fresh run, else resumed and updated.  trace: NULL or
 * [n_iter][2] = (f_n, lambda_n).  lambda_schedule: NULL, or [n_iter] values
 * that replace the step rule (f is still tracked). */
int oracle_os_iterate(const og_geometry* g, int32_t subsets, double beta, const og_params* p,
                      const double* counts, double i0, double* img, int32_t n_iter, og_state* state,
                      double* trace, const double* lambda_schedule, double* f_hist, double* best_img)
{
    if (!geometry_ok(g) || !p || !counts || !img || subsets < 1 || subsets > g->n_views || beta < 0 ||
        i0 <= 0 || n_iter < 0 || (p->keep_best && !best_img))
        return OG_INVALID;
    const int N = g->n, nch = g->n_channels, M = subsets;
    const size_t npix = (size_t)N * N;
    const double delta_cm = g->pixel_mm / 10.0;
    const double eps_cm = p->tv_eps_per_mm * 10.0;
    const double c = 0.5 * (N - 1), Rmm = 0.5 * N * g->pixel_mm;

    double* mu = (double*)malloc(sizeof(double) * npix);
    double* gl = (double*)malloc(sizeof(double) * npix);
    double* gr = (double*)malloc(sizeof(double) * npix);
    unsigned char* mask = (unsigned char*)malloc(npix);
    int32_t* views = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n_views / M + 1));
    double* ell = (double*)malloc(sizeof(double) * (size_t)(g->n_views / M + 1) * nch);
    double* w = (double*)malloc(sizeof(double) * (size_t)(g->n_views / M + 1) * nch);

    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double x = (i - c) * g->pixel_mm, y = (j - c) * g->pixel_mm;
            mask[(size_t)j * N + i] = (x * x + y * y <= Rmm * Rmm);
        }
    /* the iterate is held at zero outside the reconstruction disc, the start image included */
    for (size_t r = 0; r < npix; ++r) mu[r] = mask[r] ? 10.0 * img[r] : 0.0;

    int n_done = state ? state->n_done : 0;
    double lambda = state ? state->lambda : p->lambda0;
    double f_prev = state ? state->f_prev : 0.0;
    int flags = state ? state->flags : 0;
    double best_f = (state && n_done > 0) ? state->best_f : INFINITY;
    double epoch_sum = (state && n_done > 0) ? state->epoch_sum : 0.0;
    int best_n = (state && n_done > 0) ? state->best_n : 0;
    double* hist = f_hist ? f_hist : (double*)calloc((size_t)M, sizeof(double));
    int status = OG_OK;

    for (int it = 0; it < n_iter; ++it) {
        int n = n_done + it;
        int s = n % M;
        int nv = 0;
        for (int v = s; v < g->n_views; v += M) views[nv++] = v;

        /* reprojection of mu^(n) on subset s */
        project_views(g, delta_cm, mu, ell, views, nv);

        /* squared difference f_n, summed in ray order */
        double fsum = 0.0;
        for (int vs = 0; vs < nv; ++vs)
            for (int k = 0; k < nch; ++k) {
                double y = counts[(size_t)views[vs] * nch + k];
                double pr = log(i0 / (y > 1.0 ? y : 1.0));
                double d = ell[(size_t)vs * nch + k] - pr;
                fsum += d * d;
            }
        double f_n = fsum / ((double)nv * nch);

        const double f_ref = (p->lambda_compare && n >= M) ? hist[s] : f_prev;
        lambda = oracle_lambda_next(p, n == 0, lambda, f_n, f_ref);
        if (lambda_schedule) lambda = lambda_schedule[it];
        if (trace) {
            trace[2 * it] = f_n;
            trace[2 * it + 1] = lambda;
        }
        f_prev = f_n;
        hist[s] = f_n;
        if (!isfinite(f_n)) flags |= 1;
        int keep = 0;
        if ((n + 1) % M == 0) {
            const double e = epoch_sum + f_n;
            if (e < best_f) {
                best_f = e;
                best_n = n + 1;
                keep = 1;
            }
            epoch_sum = 0.0;
        } else {
            epoch_sum += f_n;
        }

        /* likelihood gradient A_s^T (exp(-l) - y/I0) */
        for (int vs = 0; vs < nv; ++vs)
            for (int k = 0; k < nch; ++k) {
                size_t q = (size_t)vs * nch + k;
                double yt = counts[(size_t)views[vs] * nch + k] / i0;
                w[q] = exp(-ell[q]) - yt;
            }
        backproject_views(g, delta_cm, w, gl, views, nv);

        /* prior gradient at mu^(n) */
        oracle_tv(N, eps_cm, mu, NULL, gr);

        /* update: all terms at mu^(n) */
        for (size_t r = 0; r < npix; ++r) {
            double v = mu[r] + lambda * (gl[r] + (beta / M) * gr[r]);
            if (!(v > 0.0)) v = 0.0;
            mu[r] = mask[r] ? v : 0.0;
        }
        if (keep && p->keep_best)
            for (size_t r = 0; r < npix; ++r) best_img[r] = mu[r] / 10.0;
    }

    for (size_t r = 0; r < npix; ++r) img[r] = mu[r] / 10.0;
    if (state) {
        state->n_done = n_done + n_iter;
        state->lambda = lambda;
        state->f_prev = f_prev;
        state->flags = flags;
        state->best_f = best_f;
        state->epoch_sum = epoch_sum;
        state->best_n = best_n;
    }
    if (!f_hist) free(hist);
    if (flags & 1) status = OG_NUMERIC;
    free(mu);
    free(gl);
    free(gr);
    free(mask);
    free(views);
    free(ell);
    free(w);
    return status;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int32_t n) { if (n > 0) omp_set_num_threads(n); }
