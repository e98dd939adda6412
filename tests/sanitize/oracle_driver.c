/* Drives every oracle entry point on tiny inputs; built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py (test infrastructure). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t n, pad0;
    double pixel_mm;
    int32_t n_views, n_channels;
    double sad_mm, sdd_mm, fan_half_angle_rad, start_angle_rad, scan_arc_rad;
} og_geometry;
typedef struct {
    double lambda0, lambda_inc, lambda_dec, lambda_min, mu0_per_mm, tv_eps_per_mm;
    int32_t lambda_compare, keep_best;
} og_params;
typedef struct {
    int32_t n_done, flags;
    double lambda, f_prev, best_f, epoch_sum;
    int32_t best_n, pad;
} og_state;

int oracle_project(const og_geometry*, const double*, double*, const int32_t*, int32_t);
int oracle_backproject(const og_geometry*, const double*, double*, const int32_t*, int32_t);
int oracle_tv(int32_t, double, const double*, double*, double*);
int oracle_initial_image(const og_geometry*, double, double*);
int oracle_os_iterate(const og_geometry*, int32_t, double, const og_params*, const double*, double, double*,
                      int32_t, og_state*, double*, const double*, double*, double*);
int oracle_fbp(const og_geometry*, const double*, double*);

int main(void)
{
    og_geometry g = {13, 0, 20.0, 17, 23, 850.0, 1450.0, 0.0, 0.4, 0.0};
    const int N = g.n, nv = g.n_views, nch = g.n_channels, M = 4;
    double* img = calloc((size_t)N * N, sizeof(double));
    double* img2 = calloc((size_t)N * N, sizeof(double));
    double* sino = calloc((size_t)nv * nch, sizeof(double));
    double* counts = calloc((size_t)nv * nch, sizeof(double));
    double* trace = calloc(2 * 9, sizeof(double));
    double* hist = calloc(M, sizeof(double));
    double tvv = 0.0;
    int rc = 0;
    for (int i = 0; i < N * N; ++i) img[i] = 0.001 * (double)(i % 7);
    rc |= oracle_project(&g, img, sino, NULL, nv);
    int32_t views[3] = {1, 5, 9};
    rc |= oracle_project(&g, img, sino, views, 3);
    rc |= oracle_backproject(&g, sino, img2, NULL, nv);
    rc |= oracle_backproject(&g, sino, img2, views, 3);
    rc |= oracle_tv(N, 1e-5, img, &tvv, img2);
    for (int r = 0; r < nv * nch; ++r) counts[r] = (double)(1000 + r % 50);
    og_params p = {0.01, 1e-4, 2e-4, 1e-4, 0.005, 1e-5, 1, 1};
    og_state st = {0};
    rc |= oracle_initial_image(&g, 0.005, img);
    rc |= oracle_os_iterate(&g, M, 1e-3, &p, counts, 2000.0, img, 9, &st, trace, NULL, hist, img2);
    rc |= oracle_fbp(&g, sino, img);
    /* a partial arc: the iteration runs, the filtered backprojection refuses it */
    og_geometry gs = g;
    gs.scan_arc_rad = 2.0;
    og_state st2 = {0};
    rc |= oracle_project(&gs, img, sino, NULL, nv);
    rc |= oracle_os_iterate(&gs, M, 1e-3, &p, counts, 2000.0, img, 5, &st2, NULL, NULL, hist, img2);
    rc |= oracle_fbp(&gs, sino, img) == 0;
    printf("rc %d f %.6e best_n %d\n", rc, trace[16], st.best_n);
    free(img); free(img2); free(sino); free(counts); free(trace); free(hist);
    return rc != 0;
}
