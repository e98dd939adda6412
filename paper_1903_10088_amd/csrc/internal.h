// Internal layout of the reconstruction library: device tables, workspace and
// kernel launchers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "recon.h"

namespace recon {

// Images live in the workspace with two zero columns on each side of every row
// (row stride P = n + 4, element (row, col) at row * P + col + PAD); each
// buffer holds the row-major copy followed by the transposed one (n P floats
// later), so the projector addresses both with 32-bit offsets from one base.
// The projector clamps its interpolation index to [-PAD, n] so that every read
// stays inside the row and reads zero outside the image.
constexpr int PAD = 2;

// The squared differences of a subset are summed in groups of this many
// consecutive rays (in ray order), then over groups in a fixed tree: the
// order, and so f_n to the last bit, is independent of launch shapes.
constexpr int SQ_GROUP = 16;

// One record per view, in subset order (subset 0's views first).  Kernels read
// it at a wave-uniform index, so the loads go through the scalar cache.
struct ViewRec {
    float sx, sy;      // source position in pixel units, relative to the grid centre
    float cb, sb;      // cos / sin of the source angle
    int32_t ray0;      // index of channel 0 of this view in the subset-ordered ray arrays
    int32_t k_split;   // channels [0, k_split) have major axis first_major, the rest the other
    int32_t first_major;  // 0 = x-major (sampled per column), 1 = y-major (per row)
    int32_t nat_view;  // natural view index
    float dist;        // source distance from the grid centre in pixels (SAD / pixel)
    int32_t pad[3];
};

// Per-ray sampling line: along the ray's major axis, sample line t (a column
// for x-major rays, a row for y-major rays) is crossed at continuous index
// u(t) = a + t * slope on the other axis.  In float32 an index near 512 only
// resolves 6e-5 pixel, so u is split into a lattice part and a small residual:
//   u(t) = (a_int + t * s_hi) + (a_frac + t * s_lo),
// with a_int an integer and s_hi a multiple of 2^-q chosen so that the first
// bracket, and its difference with any integer, is exact in float32; only the
// residual (|.| ~ 1) is rounded.
struct RayGeo {
    float a_int, a_frac, s_hi, s_lo;
};

// Per-ray constants of the projector: path length per sample line (mm) and the
// packed sample range lo | hi << 15 | major << 30 (lo > hi: the ray misses).
struct RayMeta {
    float scale;
    uint32_t packed;
};

// Device-resident iteration state, read and written only by kernels during a
// run, so that captured graphs replay without host involvement.
struct DevState {
    double lambda;          // lambda_n of the current sub-iteration (read by the update)
    double f_prev;          // f of the previous sub-iteration
    int32_t n_global;       // global index n of the next sub-iteration
    int32_t it;             // index into trace / schedule of the next sub-iteration
    int32_t flags;          // bit 0: non-finite f met
    int32_t best_n;         // sub-iterations behind the kept iterate (0: none)
    double best_f;          // least epoch sum of f so far
    double epoch_sum;       // sum of f over the current epoch's earlier sub-iterations
    double* trace;          // [n_iter][2] or null
    const double* schedule; // [n_iter] or null
    // [M] f of each subset's latest sub-iteration, or null.  Written one
    // sub-iteration late (sub-iteration n stores f_{n-1}, which it holds as
    // f_prev), so that a launch never reads the slot it writes.
    double* fhist;
    float* best;            // [n][n] kept iterate (1/mm) or null
};

// Step-rule constants handed to the update kernel by value.
struct StepRule {
    double lambda0, inc, dec, lmin;
    int M;        // subsets per epoch
    int compare;  // 1: compare with the same subset one epoch earlier
};

// Constants of the fused backprojection + TV + update kernel.
struct UpdateConst {
    float c_l;     // multiplies the likelihood gradient (mm): 1/100 for the cm-unit step
    float c_r;     // multiplies -dTV/dmu: beta / (10 M)
    float eps;     // TV smoothing (1/mm)
    float pad;
};

struct Geo {
    int n, P, nv, nch;
    float c;         // (n - 1) / 2
    float dg_inv;    // 1 / dgamma
    float kc;        // (n_channels - 1) / 2
    float margin;    // channel margin of the gather's candidate window
    int use_poly;    // 1: |tan| of every pixel's fan angle is small enough for the polynomial atan
};

// Everything a batched kernel needs about one slice (device memory, read at
// wave-uniform addresses).
struct SliceDesc {
    Geo geo;
    int pad0;
    const ViewRec* views;
    const RayGeo* rg;
    const RayMeta* rm;
    float* img[2];
    float* imgT[2];
    float* yt;  // written at the start of a run, read by the projector
    float* p;
    float* w;
    double* part;
    double* part_all;  // squared-difference sums per SQ_GROUP rays over all views
    double* res_part;  // [RES_BLOCKS][2] partial sums of the full-data residual
    DevState* state;   // two copies
    const int2* subs;  // per subset: (first subset-ordered view, number of views)
    UpdateConst uc;
};

// The full-data residual is reduced in RES_BLOCKS fixed ray ranges per slice,
// whose sums are then added in range order (a fixed order, so the result does
// not depend on batching).
constexpr int RES_BLOCKS = 64;

// Work items of the batched kernels: one per thread block.  slice < 0 = idle.
struct FpWork {
    int slice;
    int r0;  // first ray of the block within the slice's subset
};
struct BpWork {
    int slice;
    int ti0, tj0;  // first pixel of the tile
    int pad;
};

}  // namespace recon

struct recon_handle {
    recon_geometry g;
    recon_params p;
    int M;
    double beta;
    recon::Geo geo;
    int device;

    std::vector<int> subset_start;  // first subset-ordered view of subset s
    std::vector<int> subset_count;  // views in subset s
    std::vector<int> perm;          // subset-ordered view -> natural view
    int max_subset_views;

    // device tables
    recon::ViewRec* d_views = nullptr;
    recon::RayGeo* d_raygeo = nullptr;
    recon::RayMeta* d_raymeta = nullptr;

    // workspace
    float* d_img[2] = {nullptr, nullptr};   // padded [n][P], followed by the transposed copy
    float* d_imgT[2] = {nullptr, nullptr};  // padded transposed [n][P] (= d_img + n P, same allocation)
    float* d_yt = nullptr;                  // y / I0, subset order [nv * nch]
    float* d_p = nullptr;                   // ln(I0 / max(y, 1)), subset order
    float* d_w = nullptr;                   // weighted residual per ray, subset order
    double* d_part = nullptr;               // squared-difference sums per SQ_GROUP rays of a subset
    double* d_part_all = nullptr;           // the same over all views (full-data residual)
    double* d_res_part = nullptr;           // [RES_BLOCKS][2] partial sums of the full-data residual
    recon::DevState* d_state = nullptr;     // two copies: sub-iteration reads one, writes the other
    recon::DevState* h_state = nullptr;     // pinned read-back
    double* d_fhist = nullptr;              // [M] subset history of a fresh run with lambda_compare
    float* d_fbp = nullptr;                 // [n_ch] D cos(gamma_k), then [2 n_ch - 1] dgamma h(m) (fbp.hip)
    double* d_fbp_cs = nullptr;             // [n_views][2] cos / sin of the source angle, subset order (fbp.hip)

    int fp_segments = 8;
    int bp_variant = 5;      // update variant (launch_bp_update): 5 = 2x2 pixels per lane, views split over the waves

    // host copies of the ray tables (pair counts, checks)
    std::vector<recon::RayGeo> h_raygeo;
    std::vector<recon::RayMeta> h_raymeta;

    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_bad = false;
};

namespace recon {

// Source angle of view v (natural order): start + arc v / n_views, arc the
// geometry's scan arc or a full turn when that is 0.
inline double view_angle(const recon_geometry* g, int v)
{
    const double arc = g->scan_arc_rad > 0.0 ? g->scan_arc_rad : 2.0 * 3.14159265358979323846;
    return g->start_angle_rad + arc * (double)v / (double)g->n_views;
}

// Whether the views cover a full turn (scan arc 0 or exactly 2 pi).
inline bool full_turn(const recon_geometry* g)
{
    return g->scan_arc_rad == 0.0 || g->scan_arc_rad == 2.0 * 3.14159265358979323846;
}

// api.hip: error reporting and per-handle constants shared with batch.hip
recon_status fail(recon_status s, const std::string& msg);
hipStream_t as_stream(void* s);
// Argument checks of recon_create (geometry, subset count, beta, params), no device work.
recon_status validate_create(const recon_geometry* geom, int subsets, double beta, const recon_params* params);
StepRule rule_of(const recon_handle* h);
UpdateConst update_const(const recon_handle* h);
// recon_os_iterate_ex on a HIP stream; new_graphs = false replays only epoch
// graphs the handle has already instantiated and launches the rest directly
// (same kernels, same bits), so the call creates no graph.
recon_status os_iterate_run(recon_handle* h, const float* d_counts, float i0, float* d_img, int n_iter,
                            recon_state* state, double* d_trace, const double* d_lambda_schedule, double* d_f_hist,
                            float* d_best, hipStream_t s, bool new_graphs);

#define RECON_HIP_TRY(expr)                                                                              \
    do {                                                                                                 \
        hipError_t _e = (expr);                                                                          \
        if (_e != hipSuccess)                                                                            \
            return ::recon::fail(_e == hipErrorOutOfMemory ? RECON_OOM : RECON_DEVICE,                   \
                                 std::string(#expr) + ": " + hipGetErrorString(_e));                     \
    } while (0)

// kernels.hip
// mask_disc: zero outside the reconstruction disc (the iteration's start image)
hipError_t launch_pad_image(const float* src, float* dst, float* dstT, int n, int P, hipStream_t s,
                            bool mask_disc = false);
hipError_t launch_unpad_image(const float* src, float* dst, int n, int P, hipStream_t s);
hipError_t launch_initial_image(float* dst, int n, float mu0, hipStream_t s);
hipError_t launch_prep_counts(const float* counts, const ViewRec* views, int nv, int nch, float i0, float* yt,
                              float* p, hipStream_t s);
hipError_t launch_scale_sino(const float* sino, const RayMeta* meta, int ray0, int nrays, int nch,
                             const ViewRec* views, int q0, int natural_rows, float* w, hipStream_t s);
// Per-slice arguments of the batched layout kernels, passed by value (no
// upload): one launch covers up to BATCH_ARGS slices [first, first + count) of
// a slice table.  max_n / max_rays: the group's largest image side and
// views x channels, which size the grid.
constexpr int BATCH_ARGS = 64;
struct BatchRunArgs {
    const float* counts[BATCH_ARGS];
    float* img[BATCH_ARGS];
    double* trace[BATCH_ARGS];
    float i0[BATCH_ARGS];
    float mu0[BATCH_ARGS];
    int first, count;
    int max_n;
    long max_rays;
};
struct BatchCopyArgs {
    const float* src[BATCH_ARGS];
    float* dst[BATCH_ARGS];
    int count;
};
// passed by value: keep well inside the 4 KB of kernel arguments
static_assert(sizeof(BatchRunArgs) + sizeof(DevState) + 64 <= 4096, "batched layout arguments too large");
static_assert(sizeof(BatchCopyArgs) + 64 <= 4096, "batched copy arguments too large");
// Start of a batched run: counts -> yt, p; start image -> padded copies
// (masked to the disc); state[0] = fresh with the slice's trace and it = 0.
hipError_t launch_prepare_batch(const SliceDesc* slices, const BatchRunArgs& a, const DevState& fresh, bool counts,
                                hipStream_t s);
// img[k] = the unpadded image buffer `in` of slice first + k.
hipError_t launch_unpad_batch(const SliceDesc* slices, const BatchRunArgs& a, int in, hipStream_t s);
// img[k] = the homogeneous start image (mu0[k] in the disc, 0 outside).
hipError_t launch_initial_batch(const SliceDesc* slices, const BatchRunArgs& a, hipStream_t s);
// dst[k][0, len) = src[k][0, len) for k < count.
hipError_t launch_copy_batch(const BatchCopyArgs& a, long len, hipStream_t s);

hipError_t launch_fp_plain(const Geo& geo, int segments, const float* img, const float* imgT, const RayGeo* rg,
                           const RayMeta* rm, const ViewRec* views, int q0, int nq, int natural_rows, float* out,
                           hipStream_t s);
hipError_t launch_fp_os(const Geo& geo, int segments, const float* img, const float* imgT, const RayGeo* rg,
                        const RayMeta* rm, int ray0, int nrays, const float* yt, const float* p, float* w,
                        double* part, hipStream_t s);
// Writes v to *st on the stream (it = 0 at the start of every run).
hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s);
// State of a fresh run: lambda_0, no epoch ended yet, no trace, history or kept image.
DevState fresh_state(double lambda0);
// Completes the one-late history of the state st (fhist[(n - 1) mod M] = f_prev).
hipError_t launch_flush_hist(const DevState* st, int M, hipStream_t s);
hipError_t launch_bp_plain(const Geo& geo, const ViewRec* views, const RayGeo* rg, const float* w, int q0, int nq,
                           float* out, hipStream_t s);
// bp.hip; variant 0 = candidate reads from global memory, 1 = LDS-staged.
// Reads the step-rule state st_in and the group sums `part` of the subset's
// nrays rays, applies the step rule (block (0,0) writes st_out), then
// backprojects, takes the TV gradient and updates the image.
struct UpdateArgs {
    const ViewRec* views;
    const RayGeo* rg;
    const float* w;
    int q0, nq;
    const double* part;
    int nrays;
    const DevState* st_in;
    DevState* st_out;
    StepRule rule;
    const float* img;
    float* img_out;
    float* imgT_out;
    UpdateConst uc;
};
hipError_t launch_bp_update(const Geo& geo, int variant, const UpdateArgs& a, hipStream_t s);
// Batched sub-iteration after the projector: launch_step_batch takes every
// slice's step rule once (state in -> state 1 - in), then the batched update
// reads its step size from state 1 - in.
hipError_t launch_step_batch(const SliceDesc* slices, int n_slices, int sub, int in, StepRule rule, hipStream_t s);
hipError_t launch_bp_update_batch(int variant, const SliceDesc* slices, const BpWork* work, int nblocks, int sub,
                                  int in, StepRule rule, hipStream_t s);
// kernels.hip, batched projector: block b projects rays [r0, r0 + 256/segments)
// of slice work[b].slice's subset s (s = -1: all views, sums into part_all)
// from image buffer `in`.
hipError_t launch_fp_batch(int segments, const SliceDesc* slices, const FpWork* work, int nblocks, int sub, int in,
                           hipStream_t s);
int fp_rays_per_block(int segments);
hipError_t launch_tv_grad(const float* img, float* grad, int n, float eps, hipStream_t s);
// Read-bandwidth probe: `blocks` blocks of 256 threads each read the n16 16-byte
// words at buf (n16 a power of two >= 1024) once; out: blocks * 256 floats.
hipError_t launch_read_probe(const float* buf, uint32_t n16, int blocks, float* out, hipStream_t s);
hipError_t launch_valu_probe(int op, const uint32_t* seed, int blocks, float* out, long* instructions, hipStream_t s);
// fbp.hip: the filtered-backprojection tables of a geometry (host, double
// precision, stored as float): D cos(gamma_k) in pixel units for every channel,
// then dgamma h(m) for m = -(n_ch - 1) ... n_ch - 1.
std::vector<float> fbp_tables(const recon_geometry* g);
// kernels.hip: out[0] = (sum of part[0..ngroups)) / nrays, out[1] = mean of 1 / max(y, 1) over counts
// (partial sums of RES_BLOCKS ray ranges in res_part, then added in range order).
hipError_t launch_residual_final(const double* part, int ngroups, const float* counts, long nrays, double* res_part,
                                 double* out,
                                 hipStream_t s);
// kernels.hip: the same for every slice of a batch (block i -> out[2i], out[2i + 1]).
hipError_t launch_residual_final_batch(const SliceDesc* slices, const float* const* counts, int n_slices,
                                       double* out, hipStream_t s);
// kernels.hip, residual over every stride-th subset: res_part[2 j] = sum of part[0..ngroups) (the
// subset of rank j among the chosen ones), then the noise level over the chosen views' rows into
// res_part[2 b + 1] and out = (sum_j res_part[2 j], sum_b res_part[2 b + 1]) / nrays (chosen rays).
hipError_t launch_residual_subset(const double* part, int ngroups, double* res_part, int j, hipStream_t s);
hipError_t launch_residual_strided_final(const float* counts, int nv, int nch, int M, int stride, int nchosen,
                                         long nrays, double* res_part, double* out, hipStream_t s);
// Batched forms (each slice's subset buffer and res_part; subset counts from the slice table).
hipError_t launch_residual_subset_batch(const SliceDesc* slices, int n_slices, int sub, int j, hipStream_t s);
hipError_t launch_residual_strided_final_batch(const SliceDesc* slices, const float* const* counts, int n_slices,
                                               int M, int stride, double* out, hipStream_t s);

}  // namespace recon
