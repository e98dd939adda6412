// Batched reconstruction: many slices of different sizes (image size, views,
// channels, I0) advance together, one projector launch, one step-rule launch
// (a block per slice) and one update launch per sub-iteration for the whole
// batch, each subset epoch replayed from a captured HIP graph.
//
// Work tables map thread blocks to (slice, ray block) for the projector and to
// (slice, 16x16 tile) for the update.  Slices are placed on XCDs (the
// dispatcher hands block b to XCD b mod 8), so a slice's work in one kernel
// stays in one XCD's L2; the per-XCD lists are balanced by each kernel's own
// cost (the update's by pixels x views, the projector's by ray samples) and
// interleaved, with idle blocks padding the shorter lists.  When whole slices
// cannot be balanced (fewer slices than XCDs, or a few large ones), the
// largest are cut into 2, 4 or 8 parts (contiguous ranges of their tiles or
// ray blocks), each part placed like a slice.
//
// Every slice's arithmetic is exactly that of recon_os_iterate on its own
// handle (same device functions, same summation orders), so a batched slice
// is bitwise equal to the same slice reconstructed alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "recon.h"
#include "recon_cnn.h"

using namespace recon;

constexpr int BATCH_FP_SEGMENTS = 4;

struct recon_batch_handle {
    std::vector<recon_handle*> h;  // one handle (tables + workspace) per slice
    bool owns = true;              // destroy the handles with the batch
    int M = 1;
    int last_in = 0;               // image / state buffer holding the last run's result
    // launch shapes until recon_batch_tune or recon_batch_set_launch: what the
    // tuner picks for batches of 512^2 slices (4 threads per projector ray, the
    // 2x2-pixel update with the views split over a tile's waves); results are
    // identical for every choice
    int fp_segments = BATCH_FP_SEGMENTS;
    int bp_variant = 5;
    std::vector<std::vector<int>> xcd;     // update: XCD of each part of each slice (1, 2, 4 or 8 parts)
    std::vector<std::vector<int>> xcd_fp;  // projector: the same, placed by the projector's cost

    SliceDesc* d_slices = nullptr;
    int2* d_subs = nullptr;
    BpWork* d_bp = nullptr;
    int n_bp = 0;
    std::vector<FpWork*> d_fp;  // per subset
    std::vector<int> n_fp;
    FpWork* d_fp_all = nullptr;  // every ray of every slice (full-data residual)
    int n_fp_all = 0;

    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_bad = false;

    // recon_warm_start's staging, allocated by its first call and kept for the next ones
    float* ws_stage = nullptr;
    size_t ws_stage_floats = 0;
    double* ws_res = nullptr;        // 2 per slice
    const float** ws_cptr = nullptr;  // one per slice

    // recon_warm_start_async: cold starts left running on the batch's own stream
    hipStream_t side = nullptr;
    hipEvent_t side_ready = nullptr, side_done = nullptr;
    bool pending = false;                       // side_done not yet waited for
    recon_batch_handle* pending_sub = nullptr;  // the sub-batch they ran as, freed once they are done
};

namespace {

constexpr int NXCD = 8;

void drop_graphs(recon_batch_handle* b)
{
    for (auto& g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

void free_batch(recon_batch_handle* b)
{
    if (!b) return;
    if (b->pending) (void)hipEventSynchronize(b->side_done);
    if (b->pending_sub) free_batch(b->pending_sub);
    if (b->side_ready) (void)hipEventDestroy(b->side_ready);
    if (b->side_done) (void)hipEventDestroy(b->side_done);
    if (b->side) (void)hipStreamDestroy(b->side);
    drop_graphs(b);
    for (FpWork* p : b->d_fp)
        if (p) (void)hipFree(p);
    if (b->d_fp_all) (void)hipFree(b->d_fp_all);
    if (b->d_bp) (void)hipFree(b->d_bp);
    if (b->d_subs) (void)hipFree(b->d_subs);
    if (b->d_slices) (void)hipFree(b->d_slices);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ws_stage) (void)hipFree(b->ws_stage);
    if (b->ws_res) (void)hipFree(b->ws_res);
    if (b->ws_cptr) (void)hipFree(b->ws_cptr);
    if (b->owns)
        for (recon_handle* h : b->h) recon_destroy(h);
    delete b;
}

// Waits for the cold starts a recon_warm_start_async call left running on the
// batch's stream; their sub-batch is freed then unless free_sub is false (the
// allocation-free entry point), in which case a later call frees it.
recon_status wait_pending(recon_batch_handle* b, bool free_sub = true)
{
    hipError_t e = hipSuccess;
    if (b->pending) {
        e = hipEventSynchronize(b->side_done);
        b->pending = false;
    }
    if (free_sub && b->pending_sub) {
        free_batch(b->pending_sub);
        b->pending_sub = nullptr;
    }
    if (e != hipSuccess) return fail(RECON_DEVICE, std::string("pending cold starts: ") + hipGetErrorString(e));
    return RECON_OK;
}

// What the work tables need to know of a slice.
struct SliceShape {
    int n, nch, nv;
    std::vector<int> subset_count;  // views per subset
    int max_subset_views;
};

std::vector<SliceShape> shapes_of(const recon_batch_handle* b)
{
    std::vector<SliceShape> sh;
    for (const recon_handle* h : b->h)
        sh.push_back(SliceShape{h->geo.n, h->geo.nch, h->geo.nv, h->subset_count, h->max_subset_views});
    return sh;
}

// Placement of slices on XCDs.  A slice costs, in the update, pixels x views
// per subset and, in the projector (`projector`), image edge x channels x
// views per subset (its rays' samples); it is cut into k in {1, 2, 4, 8}
// equal parts, and the parts are placed greedily, largest first, each on the
// least loaded XCD.  Starting from whole slices,
// the slice with the largest part is cut in twice as many parts while the
// busiest XCD carries more than SPLIT_TOLERANCE times the mean load (a batch
// of one slice ends in 8 parts; batches of many similar slices stay whole).
// Which block computes a tile or a ray block does not change its arithmetic,
// so the placement never changes a result.
constexpr double SPLIT_TOLERANCE = 1.03;

std::vector<std::vector<int>> assign_xcds(const std::vector<SliceShape>& sh, bool projector)
{
    const int n = (int)sh.size();
    std::vector<double> cost(n);
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        cost[i] = (double)sh[i].n * (projector ? sh[i].nch : sh[i].n) * sh[i].max_subset_views;
        total += cost[i];
    }
    std::vector<int> k(n, 1);
    std::vector<std::vector<int>> xcd(n);
    for (;;) {
        struct Part {
            double c;
            int slice, p;
        };
        std::vector<Part> parts;
        for (int i = 0; i < n; ++i) {
            xcd[i].assign(k[i], 0);
            for (int p = 0; p < k[i]; ++p) parts.push_back(Part{cost[i] / k[i], i, p});
        }
        std::stable_sort(parts.begin(), parts.end(), [](const Part& a, const Part& c) { return a.c > c.c; });
        std::vector<double> load(NXCD, 0.0);
        for (const Part& q : parts) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            xcd[q.slice][q.p] = x;
            load[x] += q.c;
        }
        if (*std::max_element(load.begin(), load.end()) <= SPLIT_TOLERANCE * total / NXCD) break;
        int j = -1;
        for (int i = 0; i < n; ++i)
            if (k[i] < NXCD && (j < 0 || cost[i] / k[i] > cost[j] / k[j])) j = i;
        if (j < 0) break;
        k[j] *= 2;
    }
    return xcd;
}

// Part of item t of a slice whose `count` items are cut into `parts` equal
// contiguous ranges: the p with floor(p count / parts) <= t < floor((p+1) count / parts).
int part_of(long t, long count, int parts)
{
    int p = (int)((t * parts) / count);
    while (p + 1 < parts && (long)(p + 1) * count / parts <= t) ++p;
    while (p > 0 && (long)p * count / parts > t) --p;
    return p;
}

// Interleaves per-XCD lists so that block p runs on XCD p mod 8.
template <class W>
std::vector<W> interleave(const std::vector<std::vector<W>>& lists, const W& idle)
{
    size_t len = 0;
    for (const auto& l : lists) len = std::max(len, l.size());
    std::vector<W> out(len * NXCD, idle);
    for (int x = 0; x < NXCD; ++x)
        for (size_t k = 0; k < lists[x].size(); ++k) out[k * NXCD + x] = lists[x][k];
    return out;
}

// Update work: every 16x16 tile of every slice (row-major, each part's range
// of tiles on that part's XCD), slice by slice within an XCD.
std::vector<BpWork> bp_work_table(const std::vector<SliceShape>& sh, const std::vector<std::vector<int>>& xcd)
{
    std::vector<std::vector<BpWork>> bl(NXCD);
    for (size_t i = 0; i < sh.size(); ++i) {
        const int T = (sh[i].n + 15) / 16, parts = (int)xcd[i].size();
        const long nt = (long)T * T;
        for (long t = 0; t < nt; ++t) {
            const int ty = (int)(t / T), tx = (int)(t % T);
            bl[xcd[i][part_of(t, nt, parts)]].push_back(BpWork{(int)i, tx * 16, ty * 16, 0});
        }
    }
    return interleave(bl, BpWork{-1, 0, 0, 0});
}

// Projector work of subset s (-1: every view) in blocks of rpb rays, each
// part's range of ray blocks on that part's XCD.
std::vector<FpWork> fp_work_table(const std::vector<SliceShape>& sh, const std::vector<std::vector<int>>& xcd, int s,
                                  int rpb)
{
    std::vector<std::vector<FpWork>> fl(NXCD);
    for (size_t i = 0; i < sh.size(); ++i) {
        const int nrays = (s < 0 ? sh[i].nv : sh[i].subset_count[s]) * sh[i].nch, parts = (int)xcd[i].size();
        const long nb = (nrays + rpb - 1) / rpb;
        for (long b = 0; b < nb; ++b) fl[xcd[i][part_of(b, nb, parts)]].push_back(FpWork{(int)i, (int)(b * rpb)});
    }
    return interleave(fl, FpWork{-1, 0});
}

recon_status upload_work(recon_batch_handle* b)
{
    drop_graphs(b);
    const std::vector<SliceShape> sh = shapes_of(b);
    const std::vector<BpWork> bp = bp_work_table(sh, b->xcd);
    if (b->d_bp) (void)hipFree(b->d_bp);
    b->d_bp = nullptr;
    RECON_HIP_TRY(hipMalloc(&b->d_bp, std::max<size_t>(1, bp.size()) * sizeof(BpWork)));
    RECON_HIP_TRY(hipMemcpy(b->d_bp, bp.data(), bp.size() * sizeof(BpWork), hipMemcpyHostToDevice));
    b->n_bp = (int)bp.size();
    // projector: per subset, the subset's rays in blocks of 256 / segments
    const int rpb = fp_rays_per_block(b->fp_segments);
    for (FpWork* p : b->d_fp)
        if (p) (void)hipFree(p);
    b->d_fp.assign(b->M, nullptr);
    b->n_fp.assign(b->M, 0);
    for (int s = 0; s < b->M; ++s) {
        const std::vector<FpWork> fp = fp_work_table(sh, b->xcd_fp, s, rpb);
        RECON_HIP_TRY(hipMalloc(&b->d_fp[s], std::max<size_t>(1, fp.size()) * sizeof(FpWork)));
        RECON_HIP_TRY(hipMemcpy(b->d_fp[s], fp.data(), fp.size() * sizeof(FpWork), hipMemcpyHostToDevice));
        b->n_fp[s] = (int)fp.size();
    }
    {
        const std::vector<FpWork> fp = fp_work_table(sh, b->xcd_fp, -1, rpb);
        if (b->d_fp_all) (void)hipFree(b->d_fp_all);
        b->d_fp_all = nullptr;
        RECON_HIP_TRY(hipMalloc(&b->d_fp_all, std::max<size_t>(1, fp.size()) * sizeof(FpWork)));
        RECON_HIP_TRY(hipMemcpy(b->d_fp_all, fp.data(), fp.size() * sizeof(FpWork), hipMemcpyHostToDevice));
        b->n_fp_all = (int)fp.size();
    }
    return RECON_OK;
}

// Default threads per projector ray: BATCH_FP_SEGMENTS, doubled (up to 16)
// while a subset's rays over the whole batch, at that many threads each, would
// not give every compute unit 2048 threads (a batch of one or two 512^2
// slices gets 16, as a single slice does).
int default_fp_segments(const recon_batch_handle* b)
{
    double rays = 0.0;  // rays of an average subset, all slices
    for (const recon_handle* h : b->h) rays += (double)h->geo.nv * h->geo.nch / b->M;
    int seg = BATCH_FP_SEGMENTS;
    while (seg < 16 && rays * seg < 256.0 * 2048.0) seg *= 2;
    return seg;
}

// Slice descriptors, subset tables, XCD placement and work tables of a batch
// whose handles are in b->h; fp_segments 0 takes the batch default.
recon_status setup_batch(recon_batch_handle* b, int fp_segments)
{
    const int n_slices = (int)b->h.size(), subsets = b->M;
    b->fp_segments = fp_segments > 0 ? fp_segments : default_fp_segments(b);
    b->xcd = assign_xcds(shapes_of(b), false);
    b->xcd_fp = assign_xcds(shapes_of(b), true);
    std::vector<int2> subs((size_t)n_slices * subsets);
    for (int i = 0; i < n_slices; ++i)
        for (int s = 0; s < subsets; ++s)
            subs[(size_t)i * subsets + s] = make_int2(b->h[i]->subset_start[s], b->h[i]->subset_count[s]);
    RECON_HIP_TRY(hipMalloc(&b->d_subs, subs.size() * sizeof(int2)));
    RECON_HIP_TRY(hipMemcpy(b->d_subs, subs.data(), subs.size() * sizeof(int2), hipMemcpyHostToDevice));
    std::vector<SliceDesc> desc(n_slices);
    for (int i = 0; i < n_slices; ++i) {
        recon_handle* h = b->h[i];
        SliceDesc& D = desc[i];
        D.geo = h->geo;
        D.pad0 = 0;
        D.views = h->d_views;
        D.rg = h->d_raygeo;
        D.rm = h->d_raymeta;
        D.img[0] = h->d_img[0];
        D.img[1] = h->d_img[1];
        D.imgT[0] = h->d_imgT[0];
        D.imgT[1] = h->d_imgT[1];
        D.yt = h->d_yt;
        D.p = h->d_p;
        D.w = h->d_w;
        D.part = h->d_part;
        D.part_all = h->d_part_all;
        D.res_part = h->d_res_part;
        D.state = h->d_state;
        D.subs = b->d_subs + (size_t)i * subsets;
        D.uc = update_const(h);
    }
    RECON_HIP_TRY(hipMalloc(&b->d_slices, desc.size() * sizeof(SliceDesc)));
    RECON_HIP_TRY(hipMemcpy(b->d_slices, desc.data(), desc.size() * sizeof(SliceDesc), hipMemcpyHostToDevice));
    RECON_HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    return upload_work(b);
}

hipError_t enqueue_batch_subiter(recon_batch_handle* b, int s, int in, hipStream_t st)
{
    hipError_t e = launch_fp_batch(b->fp_segments, b->d_slices, b->d_fp[s], b->n_fp[s], s, in, st);
    if (e == hipSuccess) e = launch_step_batch(b->d_slices, (int)b->h.size(), s, in, rule_of(b->h[0]), st);
    if (e != hipSuccess) return e;
    return launch_bp_update_batch(b->bp_variant, b->d_slices, b->d_bp, b->n_bp, s, in, rule_of(b->h[0]), st);
}

recon_status get_graph(recon_batch_handle* b, int parity, hipGraphExec_t* out)
{
    if (b->graph[parity]) {
        *out = b->graph[parity];
        return RECON_OK;
    }
    hipGraph_t graph = nullptr;
    RECON_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    int in = parity;
    for (int s = 0; s < b->M && err == hipSuccess; ++s) {
        err = enqueue_batch_subiter(b, s, in, b->cap_stream);
        in = 1 - in;
    }
    hipError_t end = hipStreamEndCapture(b->cap_stream, &graph);
    if (err != hipSuccess || end != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(RECON_DEVICE,
                    std::string("batch graph capture failed: ") + hipGetErrorString(err != hipSuccess ? err : end));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(RECON_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    b->graph[parity] = exec;
    *out = exec;
    return RECON_OK;
}

// Groups of up to BATCH_ARGS consecutive slices for the batched layout kernels.
template <class F>
recon_status for_groups(const recon_batch_handle* b, F&& f)
{
    const int n = (int)b->h.size();
    for (int first = 0; first < n; first += BATCH_ARGS) {
        BatchRunArgs a{};
        a.first = first;
        a.count = std::min(BATCH_ARGS, n - first);
        for (int k = 0; k < a.count; ++k) {
            const Geo& G = b->h[first + k]->geo;
            a.max_n = std::max(a.max_n, G.n);
            a.max_rays = std::max(a.max_rays, (long)G.nv * G.nch);
        }
        recon_status st = f(a);
        if (st != RECON_OK) return st;
    }
    return RECON_OK;
}

// Start of a run of every slice: counts, start image, fresh step-rule state
// (one launch per group of slices).
recon_status prepare(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                     double* const* d_traces, hipStream_t s, bool counts_ready = false)
{
    for (size_t i = 0; i < b->h.size(); ++i)
        if (!d_counts[i] || !d_imgs[i] || !(i0[i] > 0) || !std::isfinite(i0[i]))
            return fail(RECON_INVALID_ARG, "slice " + std::to_string(i) + ": NULL buffer or bad i0");
    const DevState fresh = fresh_state(b->h[0]->p.lambda0);
    return for_groups(b, [&](BatchRunArgs& a) -> recon_status {
        for (int k = 0; k < a.count; ++k) {
            a.counts[k] = d_counts[a.first + k];
            a.img[k] = d_imgs[a.first + k];
            a.trace[k] = d_traces ? d_traces[a.first + k] : nullptr;
            a.i0[k] = i0[a.first + k];
        }
        RECON_HIP_TRY(launch_prepare_batch(b->d_slices, a, fresh, !counts_ready, s));
        return RECON_OK;
    });
}

// Copies images of side sz between the slices' buffers and a contiguous stage
// (to_stage: d_imgs[i] -> stage slot, else back): the slices of that size
// numbered [skip, skip + take) in batch order, to slots 0, 1, ...
recon_status stage_copy(const recon_batch_handle* b, float* const* d_imgs, float* d_stage, int sz, bool to_stage,
                        hipStream_t s, int skip = 0, int take = INT_MAX)
{
    const size_t img = (size_t)sz * sz;
    BatchCopyArgs c{};
    int slot = 0, seen = 0;
    for (size_t i = 0; i <= b->h.size(); ++i) {
        if (c.count == BATCH_ARGS || (i == b->h.size() && c.count > 0)) {
            RECON_HIP_TRY(launch_copy_batch(c, (long)img, s));
            c.count = 0;
        }
        if (i == b->h.size()) break;
        if (b->h[i]->geo.n != sz) continue;
        const int k = seen++;
        if (k < skip || k - skip >= take) continue;
        float* st = d_stage + (size_t)(slot++) * img;
        c.src[c.count] = to_stage ? d_imgs[i] : st;
        c.dst[c.count] = to_stage ? st : d_imgs[i];
        ++c.count;
    }
    return RECON_OK;
}

// counts_ready: the slices' y/I0 and p were prepared from these same counts by the previous run.
recon_status batch_run(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                       int n_iter, double* const* d_traces, hipStream_t s, bool new_graphs, bool counts_ready = false);

// The homogeneous start image of every slice into d_imgs (host array of device pointers).
recon_status initial_images(recon_batch_handle* b, float* const* d_imgs, hipStream_t s)
{
    for (size_t i = 0; i < b->h.size(); ++i)
        if (!d_imgs[i]) return fail(RECON_INVALID_ARG, "slice " + std::to_string(i) + ": NULL image");
    return for_groups(b, [&](BatchRunArgs& a) -> recon_status {
        for (int k = 0; k < a.count; ++k) {
            a.img[k] = d_imgs[a.first + k];
            a.mu0[k] = (float)b->h[a.first + k]->p.mu0_per_mm;
        }
        RECON_HIP_TRY(launch_initial_batch(b->d_slices, a, s));
        return RECON_OK;
    });
}

}  // namespace

extern "C" {

recon_status recon_batch_check_work(const recon_geometry* geoms, int32_t n_slices, int32_t subsets,
                                    int32_t fp_segments, int64_t* errors, int64_t* blocks)
{
    if (!geoms || !errors || !blocks) return fail(RECON_INVALID_ARG, "NULL argument");
    if (n_slices < 1) return fail(RECON_INVALID_ARG, "n_slices must be >= 1");
    if (fp_segments != 1 && fp_segments != 2 && fp_segments != 4 && fp_segments != 8 && fp_segments != 16)
        return fail(RECON_INVALID_ARG, "fp_segments must be 1, 2, 4, 8 or 16");
    std::vector<SliceShape> sh;
    for (int i = 0; i < n_slices; ++i) {
        recon_status st = validate_create(&geoms[i], subsets, 0.0, nullptr);
        if (st != RECON_OK) return fail(st, "slice " + std::to_string(i) + ": " + recon_last_error());
        const recon_geometry& g = geoms[i];
        SliceShape s{g.n, g.n_channels, g.n_views, std::vector<int>(subsets, 0), 0};
        for (int v = 0; v < g.n_views; ++v) ++s.subset_count[v % subsets];  // V_s = {v : v mod M = s}
        s.max_subset_views = *std::max_element(s.subset_count.begin(), s.subset_count.end());
        sh.push_back(s);
    }
    const std::vector<std::vector<int>> xcd = assign_xcds(sh, false), xfp = assign_xcds(sh, true);
    int64_t bad = 0, nblk = 0;
    for (const auto* pl : {&xcd, &xfp})
        for (int i = 0; i < n_slices; ++i) {
            const size_t k = (*pl)[i].size();
            if (k != 1 && k != 2 && k != 4 && k != 8) ++bad;
            for (int x : (*pl)[i]) bad += x < 0 || x >= NXCD;
        }
    // every tile of every slice exactly once, each on the XCD of its part of the slice
    const std::vector<BpWork> bp = bp_work_table(sh, xcd);
    std::vector<std::vector<int>> seen(n_slices);
    for (int i = 0; i < n_slices; ++i) seen[i].assign((size_t)((sh[i].n + 15) / 16) * ((sh[i].n + 15) / 16), 0);
    for (size_t p = 0; p < bp.size(); ++p) {
        const BpWork& w = bp[p];
        if (w.slice < 0) continue;
        if (w.slice >= n_slices) {
            ++bad;
            continue;
        }
        const int T = (sh[w.slice].n + 15) / 16;
        if (w.ti0 % 16 || w.tj0 % 16 || w.ti0 / 16 >= T || w.tj0 / 16 >= T) {
            ++bad;
            continue;
        }
        const long t = (long)(w.tj0 / 16) * T + w.ti0 / 16;
        if (xcd[w.slice][part_of(t, (long)T * T, (int)xcd[w.slice].size())] != (int)(p % NXCD)) {
            ++bad;
            continue;
        }
        ++seen[w.slice][(size_t)(w.tj0 / 16) * T + w.ti0 / 16];
    }
    for (const auto& v : seen)
        for (int c : v) bad += c != 1;
    nblk += (int64_t)bp.size();
    // every ray block of every subset (and of all views) exactly once, on the XCD of its part of the slice
    const int rpb = fp_rays_per_block(fp_segments);
    for (int s = -1; s < subsets; ++s) {
        const std::vector<FpWork> fp = fp_work_table(sh, xfp, s, rpb);
        for (int i = 0; i < n_slices; ++i) {
            const int nrays = (s < 0 ? sh[i].nv : sh[i].subset_count[s]) * sh[i].nch;
            seen[i].assign((size_t)((nrays + rpb - 1) / rpb), 0);
        }
        for (size_t p = 0; p < fp.size(); ++p) {
            const FpWork& w = fp[p];
            if (w.slice < 0) continue;
            if (w.slice >= n_slices) {
                ++bad;
                continue;
            }
            const int nrays = (s < 0 ? sh[w.slice].nv : sh[w.slice].subset_count[s]) * sh[w.slice].nch;
            const long nb = (nrays + rpb - 1) / rpb;
            if (w.r0 % rpb || w.r0 >= nrays ||
                xfp[w.slice][part_of(w.r0 / rpb, nb, (int)xfp[w.slice].size())] != (int)(p % NXCD)) {
                ++bad;
                continue;
            }
            ++seen[w.slice][w.r0 / rpb];
        }
        for (const auto& v : seen)
            for (int c : v) bad += c != 1;
        nblk += (int64_t)fp.size();
    }
    *errors = bad;
    *blocks = nblk;
    return RECON_OK;
}

recon_status recon_batch_create(const recon_geometry* geoms, int32_t n_slices, int32_t subsets, double beta,
                                const recon_params* params, recon_batch_handle** out)
{
    if (!out || !geoms) return fail(RECON_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (n_slices < 1) return fail(RECON_INVALID_ARG, "n_slices must be >= 1");
    if (params && (params->lambda_compare || params->keep_best))
        return fail(RECON_INVALID_ARG, "lambda_compare and keep_best are single-slice options (recon_os_iterate_ex)");
    for (int i = 0; i < n_slices; ++i) {
        recon_status st = validate_create(&geoms[i], subsets, beta, params);
        if (st != RECON_OK) return fail(st, "slice " + std::to_string(i) + ": " + recon_last_error());
    }
    recon_batch_handle* b = new (std::nothrow) recon_batch_handle();
    if (!b) return fail(RECON_OOM, "host allocation failed");
    b->M = subsets;
    for (int i = 0; i < n_slices; ++i) {
        recon_handle* h = nullptr;
        recon_status st = recon_create(&geoms[i], subsets, beta, params, &h);
        if (st != RECON_OK) {
            std::string msg = recon_last_error();
            free_batch(b);
            return fail(st, "slice " + std::to_string(i) + ": " + msg);
        }
        b->h.push_back(h);
    }
    recon_status st = setup_batch(b, 0);
    if (st != RECON_OK) {
        free_batch(b);
        return st;
    }
    *out = b;
    return RECON_OK;
}

recon_status recon_batch_initial_images(recon_batch_handle* b, float* const* d_imgs, void* stream)
{
    if (!b || !d_imgs) return fail(RECON_INVALID_ARG, "NULL argument");
    recon_status pst = wait_pending(b);
    if (pst != RECON_OK) return pst;
    return initial_images(b, d_imgs, as_stream(stream));
}

recon_status recon_batch_destroy(recon_batch_handle* b)
{
    if (!b) return RECON_OK;
    (void)hipDeviceSynchronize();
    free_batch(b);
    return RECON_OK;
}

recon_status recon_batch_set_launch(recon_batch_handle* b, int32_t fp_segments, int32_t bp_variant)
{
    if (!b) return fail(RECON_INVALID_ARG, "NULL batch");
    recon_status pst = wait_pending(b);
    if (pst != RECON_OK) return pst;
    if (fp_segments != 0) {
        if (fp_segments != 1 && fp_segments != 2 && fp_segments != 4 && fp_segments != 8 && fp_segments != 16)
            return fail(RECON_INVALID_ARG, "fp_segments must be 1, 2, 4, 8 or 16");
        b->fp_segments = fp_segments;
    }
    if (bp_variant != 0) {
        if (bp_variant < 1 || bp_variant > 6) return fail(RECON_INVALID_ARG, "bp_variant must be in [0, 6]");
        b->bp_variant = bp_variant - 1;
    }
    return upload_work(b);
}

recon_status recon_batch_run(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                             int32_t n_iter, double* const* d_traces, void* stream)
{
    if (!b) return fail(RECON_INVALID_ARG, "NULL argument");
    recon_status pst = wait_pending(b);
    if (pst != RECON_OK) return pst;
    return batch_run(b, d_counts, i0, d_imgs, n_iter, d_traces, as_stream(stream), true);
}

}  // extern "C"

namespace {

// recon_batch_run on a HIP stream; new_graphs = false replays only the epoch
// graphs the batch has already instantiated and launches the rest directly
// (same kernels, same bits).
recon_status batch_run(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                       int n_iter, double* const* d_traces, hipStream_t s, bool new_graphs, bool counts_ready)
{
    if (!b || !d_counts || !i0 || !d_imgs) return fail(RECON_INVALID_ARG, "NULL argument");
    if (n_iter < 0) return fail(RECON_INVALID_ARG, "n_iter must be >= 0");
    recon_status st = prepare(b, d_counts, i0, d_imgs, d_traces, s, counts_ready);
    if (st != RECON_OK) return st;
    int in = 0, n = 0;
    while (n < n_iter) {
        const int sub = n % b->M;
        if (sub == 0 && n_iter - n >= b->M && !b->graph_bad && (new_graphs || b->graph[in])) {
            hipGraphExec_t exec = nullptr;
            if (get_graph(b, in, &exec) == RECON_OK) {
                RECON_HIP_TRY(hipGraphLaunch(exec, s));
                n += b->M;
                if (b->M & 1) in = 1 - in;
                continue;
            }
            b->graph_bad = true;
        }
        RECON_HIP_TRY(enqueue_batch_subiter(b, sub, in, s));
        in = 1 - in;
        ++n;
    }
    st = for_groups(b, [&](BatchRunArgs& a) -> recon_status {
        for (int k = 0; k < a.count; ++k) a.img[k] = d_imgs[a.first + k];
        RECON_HIP_TRY(launch_unpad_batch(b->d_slices, a, in, s));
        return RECON_OK;
    });
    if (st != RECON_OK) return st;
    b->last_in = in;
    return RECON_OK;
}

}  // namespace

extern "C" {

recon_status recon_batch_tune(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                              int32_t reps, int32_t* fp_segments_out, int32_t* bp_variant_out, void* stream)
{
    if (!b || !d_counts || !i0 || !d_imgs) return fail(RECON_INVALID_ARG, "NULL argument");
    if (reps < 1 || reps > 1000) return fail(RECON_INVALID_ARG, "reps must be in [1, 1000]");
    recon_status pst = wait_pending(b);
    if (pst != RECON_OK) return pst;
    hipStream_t s = as_stream(stream);
    recon_status st = prepare(b, d_counts, i0, d_imgs, nullptr, s);
    if (st != RECON_OK) return st;
    for (int sub = 0; sub < b->M; ++sub) RECON_HIP_TRY(enqueue_batch_subiter(b, sub, 0, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RECON_HIP_TRY(hipEventCreate(&e0));
    RECON_HIP_TRY(hipEventCreate(&e1));
    auto timed = [&](auto&& launch, float* ms) -> hipError_t {
        hipError_t err = launch(0);  // warm
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch(r % b->M);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
        return err;
    };
    hipError_t err = hipSuccess;
    const int segs[] = {4, 8, 16};
    int best_seg = b->fp_segments;
    float best_ms = 3.0e38f;
    for (int seg : segs) {
        b->fp_segments = seg;
        st = upload_work(b);
        if (st != RECON_OK) break;
        float ms = 0.0f;
        err = timed([&](int sub) { return launch_fp_batch(seg, b->d_slices, b->d_fp[sub], b->n_fp[sub], sub, 0, s); },
                    &ms);
        if (err != hipSuccess) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_seg = seg;
        }
    }
    int best_var = b->bp_variant;
    if (st == RECON_OK && err == hipSuccess) {
        best_ms = 3.0e38f;
        for (int var = 0; var < 6; ++var) {
            float ms = 0.0f;
            err = timed(
                [&](int sub) {
                    return launch_bp_update_batch(var, b->d_slices, b->d_bp, b->n_bp, sub, 0, rule_of(b->h[0]), s);
                },
                &ms);
            if (err != hipSuccess) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_var = var;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RECON_OK) return st;
    if (err != hipSuccess) return fail(RECON_DEVICE, std::string("tuning run: ") + hipGetErrorString(err));
    b->fp_segments = best_seg;
    b->bp_variant = best_var;
    st = upload_work(b);
    if (st != RECON_OK) return st;
    if (fp_segments_out) *fp_segments_out = best_seg;
    if (bp_variant_out) *bp_variant_out = best_var + 1;
    return RECON_OK;
}

recon_status recon_batch(const recon_geometry* geoms, int32_t n_slices, int32_t subsets, double beta,
                         const recon_params* params, const float* const* d_counts, const float* i0,
                         float* const* d_imgs, int32_t n_iter, void* stream)
{
    recon_batch_handle* b = nullptr;
    recon_status st = recon_batch_create(geoms, n_slices, subsets, beta, params, &b);
    if (st != RECON_OK) return st;
    st = recon_batch_run(b, d_counts, i0, d_imgs, n_iter, nullptr, stream);
    if (st == RECON_OK) {
        hipError_t e = hipStreamSynchronize(as_stream(stream));
        if (e != hipSuccess) st = fail(RECON_DEVICE, std::string("recon_batch: ") + hipGetErrorString(e));
    }
    recon_batch_destroy(b);
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned warm start.  With a null scratch the stage, the residuals and the
// device copy of the count pointers are allocated for the call, the epoch
// graphs are built on first use and many fallback slices run as a sub-batch.
// With a scratch buffer (the allocation-free entry point) the images pass
// through the network in chunks that fit the scratch stage, only graphs that
// already exist are replayed, and fallback slices run one by one on their own
// handles: the same kernels in the same order, so the same bits.
// ---------------------------------------------------------------------------

namespace {

// Allocation-free warm start: the scratch holds a stage of NOALLOC_STAGE_FLOATS
// floats (16 MiB: 16 slices of 512^2, one of 2048^2), then per slice two
// doubles (residual, noise level) and one count pointer.
constexpr size_t NOALLOC_STAGE_FLOATS = (size_t)4 << 20;
constexpr int NOALLOC_MAX_SLICES = 4096;
constexpr size_t NOALLOC_RES_OFFSET = NOALLOC_STAGE_FLOATS * sizeof(float);
constexpr size_t NOALLOC_CPTR_OFFSET = NOALLOC_RES_OFFSET + 2 * sizeof(double) * NOALLOC_MAX_SLICES;
constexpr size_t NOALLOC_BYTES = NOALLOC_CPTR_OFFSET + sizeof(float*) * NOALLOC_MAX_SLICES;

recon_status warm_start_impl(recon_batch_handle* b, recon_cnn* net, const float* const* d_counts, const float* i0,
                             float* const* d_imgs, int n_pre, int n_refine, int n_cold, double residual_ratio,
                             int check_stride, double* h_residual, double* h_floor, int32_t* h_fallback,
                             hipStream_t s, unsigned char* ws, bool async = false)
{
    const bool noalloc = ws != nullptr;
    const int n = (int)b->h.size();
    // the cold starts an earlier asynchronous call left running use this batch's handles
    recon_status pst = wait_pending(b, !noalloc);
    if (pst != RECON_OK) return pst;
    // 1. early iterate of every slice from the homogeneous start
    recon_status st = initial_images(b, d_imgs, s);
    if (st == RECON_OK) st = batch_run(b, d_counts, i0, d_imgs, n_pre, nullptr, s, !noalloc);
    if (st != RECON_OK) return st;
    // 2. network estimate of the converged image, projected onto the constraints:
    //    slices of one size go through the network together (staged contiguously)
    std::vector<int> sizes, per_size;
    for (recon_handle* h : b->h) {
        auto it = std::find(sizes.begin(), sizes.end(), h->geo.n);
        if (it == sizes.end()) {
            sizes.push_back(h->geo.n);
            per_size.push_back(1);
        } else {
            ++per_size[it - sizes.begin()];
        }
    }
    float* d_stage = nullptr;
    double* d_res = nullptr;
    const float** d_cptr = nullptr;
    hipError_t e = hipSuccess;
    if (noalloc) {
        d_stage = reinterpret_cast<float*>(ws);
        d_res = reinterpret_cast<double*>(ws + NOALLOC_RES_OFFSET);
        d_cptr = reinterpret_cast<const float**>(ws + NOALLOC_CPTR_OFFSET);
    } else {
        // kept with the batch: a stream of calls on one batch allocates once (a free here would
        // wait for the whole device between one call's check and the next call's first kernel)
        size_t stage_floats = 0;
        for (size_t k = 0; k < sizes.size(); ++k)
            stage_floats = std::max(stage_floats, (size_t)per_size[k] * sizes[k] * sizes[k]);
        if (b->ws_stage_floats < stage_floats) {
            if (b->ws_stage) (void)hipFree(b->ws_stage);
            b->ws_stage = nullptr;
            b->ws_stage_floats = 0;
            e = hipMalloc(&b->ws_stage, stage_floats * sizeof(float));
            if (e == hipSuccess) b->ws_stage_floats = stage_floats;
        }
        if (e == hipSuccess && !b->ws_res) e = hipMalloc(&b->ws_res, 2 * sizeof(double) * n);
        if (e == hipSuccess && !b->ws_cptr) e = hipMalloc((void**)&b->ws_cptr, sizeof(float*) * n);
        d_stage = b->ws_stage;
        d_res = b->ws_res;
        d_cptr = b->ws_cptr;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d_cptr, d_counts, sizeof(float*) * n, hipMemcpyHostToDevice, s);
    for (size_t k = 0; k < sizes.size() && e == hipSuccess && st == RECON_OK; ++k) {
        const int sz = sizes[k];
        const int chunk = noalloc ? (int)std::min<size_t>(per_size[k], NOALLOC_STAGE_FLOATS / ((size_t)sz * sz))
                                  : per_size[k];
        for (int first = 0; first < per_size[k] && st == RECON_OK; first += chunk) {
            const int cnt = std::min(chunk, per_size[k] - first);
            st = stage_copy(b, d_imgs, d_stage, sz, true, s, first, cnt);
            if (st == RECON_OK) st = recon_cnn_forward(net, d_stage, d_stage, cnt, sz, 1, s);
            if (st == RECON_OK) st = stage_copy(b, d_imgs, d_stage, sz, false, s, first, cnt);
        }
    }
    // 3. refinement by the plain iteration, fresh step-rule state
    // (the same counts as step 1: their y/I0 and p are still in place)
    if (e == hipSuccess && st == RECON_OK)
        st = batch_run(b, d_counts, i0, d_imgs, n_refine, nullptr, s, !noalloc, /*counts_ready=*/true);
    // 4. residual and its noise level, every slice at once from the final iterate, over every
    //    view or every check_stride-th subset (fresh projections: the refining sub-iterations'
    //    own squared differences lag the still-moving iterate and would not be comparable with
    //    the plain method's images)
    if (check_stride == 1) {
        if (e == hipSuccess && st == RECON_OK)
            e = launch_fp_batch(b->fp_segments, b->d_slices, b->d_fp_all, b->n_fp_all, -1, b->last_in, s);
        if (e == hipSuccess && st == RECON_OK) e = launch_residual_final_batch(b->d_slices, d_cptr, n, d_res, s);
    } else {
        for (int sub = 0, j = 0; sub < b->M && e == hipSuccess && st == RECON_OK; sub += check_stride, ++j) {
            e = launch_fp_batch(b->fp_segments, b->d_slices, b->d_fp[sub], b->n_fp[sub], sub, b->last_in, s);
            if (e == hipSuccess) e = launch_residual_subset_batch(b->d_slices, n, sub, j, s);
        }
        if (e == hipSuccess && st == RECON_OK)
            e = launch_residual_strided_final_batch(b->d_slices, d_cptr, n, b->M, check_stride, d_res, s);
    }
    std::vector<double> res(2 * (size_t)n);
    if (e == hipSuccess && st == RECON_OK)
        e = hipMemcpyAsync(res.data(), d_res, 2 * sizeof(double) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && st == RECON_OK) e = hipStreamSynchronize(s);
    if (st != RECON_OK) return st;
    if (e != hipSuccess) return fail(RECON_DEVICE, std::string("warm start: ") + hipGetErrorString(e));
    // 5. cold start for every slice whose data residual exceeds the limit
    std::vector<int> fb;
    for (int i = 0; i < n; ++i) {
        const bool bad = !(res[2 * i] <= residual_ratio * res[2 * i + 1]);
        if (h_residual) h_residual[i] = res[2 * i];
        if (h_floor) h_floor[i] = res[2 * i + 1];
        if (h_fallback) h_fallback[i] = bad ? 1 : 0;
        if (bad) fb.push_back(i);
    }
    if (fb.empty()) return RECON_OK;
    // The cold starts run on `s`, or (async) on the batch's own stream, after
    // the check's reads of the images on `s`, and the call returns once they are
    // enqueued.
    hipStream_t fs = s;
    if (async) {
        if (!b->side) {
            RECON_HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
            RECON_HIP_TRY(hipEventCreateWithFlags(&b->side_ready, hipEventDisableTiming));
            RECON_HIP_TRY(hipEventCreateWithFlags(&b->side_done, hipEventDisableTiming));
        }
        RECON_HIP_TRY(hipEventRecord(b->side_ready, s));
        RECON_HIP_TRY(hipStreamWaitEvent(b->side, b->side_ready, 0));
        fs = b->side;
    }
    auto leave_pending = [&]() -> recon_status {
        const hipError_t re = hipEventRecord(b->side_done, fs);
        if (re != hipSuccess) {
            (void)hipStreamSynchronize(fs);
            return fail(RECON_DEVICE, std::string("cold start: ") + hipGetErrorString(re));
        }
        b->pending = true;
        return RECON_OK;
    };
    // A few slices (or any number, without allocation) run alone on their own
    // handles; many go through a batch over their handles.  Both give the same bits.
    constexpr size_t kSubBatchMin = 2;  // one slice runs faster on its own handle; two or more as a batch
    if (noalloc || fb.size() < kSubBatchMin) {
        for (int i : fb) {
            st = recon_initial_image(b->h[i], d_imgs[i], fs);
            if (st == RECON_OK)
                st = os_iterate_run(b->h[i], d_counts[i], i0[i], d_imgs[i], n_cold, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, fs, !noalloc);
            if (st != RECON_OK) {
                if (async) (void)hipStreamSynchronize(fs);
                return st;
            }
        }
        if (async) return leave_pending();
        RECON_HIP_TRY(hipStreamSynchronize(s));
        return RECON_OK;
    }
    recon_batch_handle* sub = new (std::nothrow) recon_batch_handle();
    if (!sub) return fail(RECON_OOM, "host allocation failed");
    sub->owns = false;
    sub->M = b->M;
    sub->bp_variant = b->bp_variant;
    std::vector<const float*> c_sub;
    std::vector<float> i0_sub;
    std::vector<float*> img_sub;
    for (int i : fb) {
        sub->h.push_back(b->h[i]);
        c_sub.push_back(d_counts[i]);
        i0_sub.push_back(i0[i]);
        img_sub.push_back(d_imgs[i]);
    }
    st = setup_batch(sub, 0);
    if (st == RECON_OK) st = recon_batch_initial_images(sub, img_sub.data(), fs);
    if (st == RECON_OK) st = recon_batch_run(sub, c_sub.data(), i0_sub.data(), img_sub.data(), n_cold, nullptr, fs);
    if (async && st == RECON_OK) {
        st = leave_pending();
        if (st == RECON_OK) {
            b->pending_sub = sub;  // freed once the cold starts are done
            return RECON_OK;
        }
    }
    hipError_t se = hipStreamSynchronize(fs);
    free_batch(sub);
    if (st != RECON_OK) return st;
    if (se != hipSuccess) return fail(RECON_DEVICE, std::string("cold start: ") + hipGetErrorString(se));
    return RECON_OK;
}

recon_status check_warm_args(recon_batch_handle* b, recon_cnn* net, const float* const* d_counts, const float* i0,
                             float* const* d_imgs, int n_pre, int n_refine, int n_cold, double residual_ratio,
                             int check_stride)
{
    if (!b || !net || !d_counts || !i0 || !d_imgs) return fail(RECON_INVALID_ARG, "NULL argument");
    if (n_pre < 0 || n_refine < 0 || n_cold < 0) return fail(RECON_INVALID_ARG, "iteration counts must be >= 0");
    if (!(residual_ratio > 0)) return fail(RECON_INVALID_ARG, "residual_ratio must be > 0");
    if (check_stride < 1 || check_stride > b->M ||
        (check_stride > 1 && (b->M + check_stride - 1) / check_stride > RES_BLOCKS))
        return fail(RECON_INVALID_ARG, "check_stride must be in [1, subsets], choosing at most 64 subsets if > 1");
    return RECON_OK;
}

}  // namespace

// The allocation-free warm start's scratch: one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel or a copy (on
// the host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device.
recon_status scratch_of_current_device(unsigned char** out)
{
    int dev = -1;
    RECON_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RECON_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RECON_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RECON_OK;
}

}  // namespace

extern "C" {

recon_status recon_warm_start(recon_batch_handle* b, recon_cnn* net, const float* const* d_counts, const float* i0,
                              float* const* d_imgs, int32_t n_pre, int32_t n_refine, int32_t n_cold,
                              double residual_ratio, int32_t check_stride, double* h_residual, double* h_floor,
                              int32_t* h_fallback, void* stream)
{
    recon_status st =
        check_warm_args(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride);
    if (st != RECON_OK) return st;
    return warm_start_impl(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride,
                           h_residual, h_floor, h_fallback, as_stream(stream), nullptr);
}

recon_status recon_warm_start_async(recon_batch_handle* b, recon_cnn* net, const float* const* d_counts,
                                    const float* i0, float* const* d_imgs, int32_t n_pre, int32_t n_refine,
                                    int32_t n_cold, double residual_ratio, int32_t check_stride, double* h_residual,
                                    double* h_floor, int32_t* h_fallback, void* stream)
{
    recon_status st =
        check_warm_args(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride);
    if (st != RECON_OK) return st;
    return warm_start_impl(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride,
                           h_residual, h_floor, h_fallback, as_stream(stream), nullptr, /*async=*/true);
}

recon_status recon_batch_wait(recon_batch_handle* b)
{
    if (!b) return fail(RECON_INVALID_ARG, "NULL batch");
    return wait_pending(b);
}

recon_status recon_warm_start_noalloc(recon_batch_handle* b, recon_cnn* net, const float* const* d_counts,
                                      const float* i0, float* const* d_imgs, int32_t n_pre, int32_t n_refine,
                                      int32_t n_cold, double residual_ratio, int32_t check_stride, double* h_residual,
                                      double* h_floor, int32_t* h_fallback, void* stream)
{
    recon_status st =
        check_warm_args(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride);
    if (st != RECON_OK) return st;
    if ((int)b->h.size() > NOALLOC_MAX_SLICES)
        return fail(RECON_INVALID_ARG, "recon_warm_start_noalloc takes at most 4096 slices per call");
    for (recon_handle* h : b->h)
        if ((size_t)h->geo.n * h->geo.n > NOALLOC_STAGE_FLOATS)
            return fail(RECON_INVALID_ARG, "recon_warm_start_noalloc takes images of at most 2048 x 2048");
    int dev = -1;
    RECON_HIP_TRY(hipGetDevice(&dev));
    if (dev != b->h[0]->device)
        return fail(RECON_INVALID_ARG, "the batch's device must be the current device");
    unsigned char* sp = nullptr;
    st = scratch_of_current_device(&sp);
    if (st != RECON_OK) return st;
    return warm_start_impl(b, net, d_counts, i0, d_imgs, n_pre, n_refine, n_cold, residual_ratio, check_stride,
                           h_residual, h_floor, h_fallback, as_stream(stream), sp);
}

}  // extern "C"
