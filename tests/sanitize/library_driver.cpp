// Host-only code of the reconstruction library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the ray tables and the gather's window check
// (recon_check_tables), the batched kernels' work tables
// (recon_batch_check_work), and the argument checks every entry point runs
// before it touches the device.  No GPU is used; every call here returns
// before any device work.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "recon.h"
#include "recon_cnn.h"

namespace {

recon_geometry geom(int n, double px, int nv, int nch, double start = 0.0, double arc = 0.0)
{
    recon_geometry g{};
    g.n = n;
    g.pixel_mm = px;
    g.n_views = nv;
    g.n_channels = nch;
    g.sad_mm = 850.0;
    g.sdd_mm = 1450.0;
    g.fan_half_angle_rad = 0.0;
    g.start_angle_rad = start;
    g.scan_arc_rad = arc;
    return g;
}

int failures = 0;

void expect(bool ok, const char* what)
{
    if (!ok) {
        std::printf("FAIL %s (%s)\n", what, recon_last_error());
        ++failures;
    }
}

}  // namespace

int main()
{
    recon_params p;
    recon_default_params(&p);
    expect(p.lambda0 == 0.01, "default params");
    for (int s = 0; s <= 5; ++s) expect(recon_status_string((recon_status)s) != nullptr, "status string");

    // tables and windows of odd, rotated, limited-angle and larger geometries
    const recon_geometry tab[] = {geom(37, 10.0, 33, 51, 0.3), geom(64, 6.25, 36, 48, 0.37, 3.6),
                                  geom(128, 3.125, 180, 192), geom(200, 2.0, 45, 301, 1.1, 2.5),
                                  geom(96, 400.0 / 96, 21, 150)};
    for (const recon_geometry& g : tab) {
        int64_t missed = -1, cand = 0, pairs = 0;
        expect(recon_check_tables(&g, 4, 1, &missed, &cand, &pairs) == RECON_OK, "check_tables");
        expect(missed == 0 && pairs > 0 && cand >= pairs, "windows hold every ray");
    }
    {
        const recon_geometry big = geom(256, 1.5625, 700, 600);
        int64_t missed = -1, cand = 0, pairs = 0;
        expect(recon_check_tables(&big, 20, 139, &missed, &cand, &pairs) == RECON_OK, "check_tables 256");
        expect(missed == 0, "windows hold every ray (256)");
    }

    // batched work tables: a mix of sizes, view and channel counts, every projector shape
    std::vector<recon_geometry> batch;
    for (int i = 0; i < 19; ++i)
        batch.push_back(geom(i % 3 == 0 ? 64 : (i % 3 == 1 ? 48 : 37), 4.0, 30 + 7 * i, 41 + 13 * i, 0.1 * i,
                             i % 4 == 0 ? 4.0 : 0.0));
    for (int seg : {1, 2, 4, 8, 16})
        for (int M : {1, 5, 20}) {
            int64_t errors = -1, blocks = 0;
            expect(recon_batch_check_work(batch.data(), (int)batch.size(), M, seg, &errors, &blocks) == RECON_OK,
                   "batch_check_work");
            expect(errors == 0 && blocks > 0, "work tables cover every tile and ray block once");
        }

    // argument checks that return before the device is touched
    recon_handle* h = nullptr;
    recon_geometry bad = geom(1, 1.0, 10, 10);
    expect(recon_create(&bad, 2, 1e-3, nullptr, &h) == RECON_INVALID_ARG && h == nullptr, "create n = 1");
    bad = geom(64, 6.25, 36, 48, 0.0, 7.0);
    expect(recon_create(&bad, 2, 1e-3, nullptr, &h) == RECON_INVALID_ARG, "create arc > 2 pi");
    const recon_geometry good = geom(64, 6.25, 36, 48);
    expect(recon_create(&good, 37, 1e-3, nullptr, &h) == RECON_INVALID_ARG, "create M > n_views");
    expect(recon_create(&good, 4, -1.0, nullptr, &h) == RECON_INVALID_ARG, "create beta < 0");
    expect(recon_create(nullptr, 4, 1e-3, nullptr, &h) == RECON_INVALID_ARG, "create NULL geometry");
    recon_batch_handle* b = nullptr;
    recon_geometry two[2] = {good, geom(64, 6.25, 36, 48, 0.0, -1.0)};
    expect(recon_batch_create(two, 2, 4, 1e-3, nullptr, &b) == RECON_INVALID_ARG && b == nullptr, "batch create");
    double gbps = 0.0;
    expect(recon_read_bandwidth(3000, 5, &gbps, nullptr) == RECON_INVALID_ARG, "read probe size");
    expect(recon_valu_rate(6, 5, &gbps, nullptr) == RECON_INVALID_ARG, "VALU probe op");
    expect(recon_valu_rate(0, 0, &gbps, nullptr) == RECON_INVALID_ARG, "VALU probe reps");
    expect(recon_warm_start_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr, 1, 1, 1, 1.0, 1, nullptr, nullptr,
                                    nullptr, nullptr) == RECON_INVALID_ARG,
           "warm start NULL");
    expect(recon_warm_start_async(nullptr, nullptr, nullptr, nullptr, nullptr, 1, 1, 1, 1.0, 1, nullptr, nullptr,
                                  nullptr, nullptr) == RECON_INVALID_ARG,
           "async warm start NULL");
    expect(recon_batch_wait(nullptr) == RECON_INVALID_ARG, "batch wait NULL");
    const double z[1] = {0.0};
    expect(recon_rebin_helical(&good, 72, 10.0, 0.0, nullptr, 1e4f, z, 0, nullptr, nullptr) == RECON_OK,
           "rebin zero slices");
    expect(recon_rebin_helical(&good, 72, -1.0, 0.0, (const float*)8, 1e4f, z, 1, (float*)8, nullptr) ==
               RECON_INVALID_ARG,
           "rebin pitch");
    expect(recon_rebin_helical(&good, 72, 10.0, 0.0, (const float*)8, 1e4f, z, 1, (float*)8, nullptr) ==
               RECON_INVALID_ARG,
           "rebin slice outside the helix");
    int64_t e = 0, nb = 0;
    expect(recon_batch_check_work(batch.data(), 0, 4, 4, &e, &nb) == RECON_INVALID_ARG, "check_work n = 0");
    expect(recon_batch_check_work(batch.data(), 3, 4, 3, &e, &nb) == RECON_INVALID_ARG, "check_work segments");

    std::printf("failures %d\n", failures);
    return failures != 0;
}
