// Helical rebinning (gfx950): single-row helical fan data -> per-slice
// full-turn fan sinograms by 360-degree linear interpolation along z (the
// textbook 360LI method; the paper reconstructs helical MVCT slices without
// stating its rebinning).  Helical view h has the angle of view h mod n_views
// of a turn and source z0 + pitch h / n_views.  For slice z and view v the
// two helical views at that angle whose z bracket z are interpolated on the
// measured line integrals ln(I0 / max(y, 1)); the result is written back as
// counts I0 exp(-l), the input of the iterative method.
//
// One thread per output element, consecutive threads on consecutive channels
// (coalesced reads of the two bracketing rows and the write), up to 64 slices
// per launch; 12 bytes of HBM traffic per output element.  The bracket,
// weight and the interpolation, written as y0 exp(w ln(y1 / y0)) (the same
// value as the line-integral form, one logarithm instead of two), are in
// double precision, whose logarithm, exponential and divisions make the
// kernel ALU-bound rather than HBM-bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"
#include "recon.h"

namespace recon {
namespace {

// Slices of one launch (blockIdx.y), passed by value: q0 = (z - z0) / pitch,
// the turns from the first helical view to each slice.
constexpr int REBIN_SLICES = 64;
struct RebinSlices {
    double q0[REBIN_SLICES];
};

__global__ __launch_bounds__(256) void rebin_kernel(const float* __restrict__ counts, int nv, int nch, int nh,
                                                    RebinSlices sl, float* __restrict__ out)
{
    const int per = nv * nch;  // < 2^31 (checked on the host)
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int v = idx / nch, k = idx - v * nch;
    const double q = sl.q0[blockIdx.y] - (double)v / nv;  // turns since the first helical view at this angle
    const double m = floor(q);
    const double w = q - m;  // (z - z_lower) / pitch
    long h = v + (long)m * nv;
    // the host has checked that every view is bracketed; this only keeps the reads in bounds
    h = min(max(h, 0L), (long)nh - 1 - nv);
    const double y0 = fmax((double)counts[h * nch + k], 1.0);
    const double y1 = fmax((double)counts[(h + nv) * nch + k], 1.0);
    // I0 exp(-((1 - w) ln(I0 / y0) + w ln(I0 / y1))) = y0 exp(w ln(y1 / y0))
    out[(size_t)blockIdx.y * per + idx] = (float)(y0 * exp(w * log(y1 / y0)));
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace
}  // namespace recon

using namespace recon;

extern "C" recon_status recon_rebin_helical(const recon_geometry* g, int32_t n_helical_views, double pitch_mm,
                                            double z0_mm, const float* d_counts, float i0, const double* z_slices,
                                            int32_t n_slices, float* d_out, void* stream)
{
    if (!g) return fail(RECON_INVALID_ARG, "NULL geometry");
    if (n_slices < 0) return fail(RECON_INVALID_ARG, "n_slices must be >= 0");
    if (n_slices == 0) return RECON_OK;
    if (!d_counts || !d_out || !z_slices) return fail(RECON_INVALID_ARG, "NULL argument");
    const int nv = g->n_views, nch = g->n_channels, nh = n_helical_views;
    if (nv < 1 || nch < 1) return fail(RECON_INVALID_ARG, "n_views and n_channels must be >= 1");
    if (nh <= nv) return fail(RECON_INVALID_ARG, "n_helical_views must exceed n_views (more than one turn)");
    if (!full_turn(g)) return fail(RECON_INVALID_ARG, "the rebinned views must cover a full turn");
    if ((long)nh * nch >= (1L << 40) || (long)nv * nch >= (1L << 31))
        return fail(RECON_INVALID_ARG, "helical data too large");
    if (!(pitch_mm > 0) || !std::isfinite(pitch_mm) || !std::isfinite(z0_mm))
        return fail(RECON_INVALID_ARG, "pitch_mm must be finite and > 0, z0_mm finite");
    if (!(i0 > 0) || !std::isfinite(i0)) return fail(RECON_INVALID_ARG, "i0 must be finite and > 0");
    // every view of every slice must have a helical view on both sides, with the
    // bracket formed exactly as the kernel forms it
    for (int s = 0; s < n_slices; ++s) {
        const double q0 = (z_slices[s] - z0_mm) / pitch_mm;
        if (!std::isfinite(q0)) return fail(RECON_INVALID_ARG, "slice position not finite");
        for (int v = 0; v < nv; ++v) {
            const double m = std::floor(q0 - (double)v / nv);
            const bool inside = m >= 0.0 && m <= (double)nh && v + (long)m * nv + nv <= (long)nh - 1;
            if (!inside)
                return fail(RECON_INVALID_ARG, "slice " + std::to_string(s) + " (z = " +
                                                   std::to_string(z_slices[s]) +
                                                   " mm) is not bracketed by the helical views");
        }
    }
    hipStream_t st = as_stream(stream);
    const long per = (long)nv * nch;
    for (int first = 0; first < n_slices; first += REBIN_SLICES) {
        const int cnt = std::min(REBIN_SLICES, n_slices - first);
        RebinSlices sl{};
        for (int j = 0; j < cnt; ++j) sl.q0[j] = (z_slices[first + j] - z0_mm) / pitch_mm;
        rebin_kernel<<<dim3(cdiv(per, 256), cnt), 256, 0, st>>>(d_counts, nv, nch, nh, sl,
                                                               d_out + (size_t)first * per);
        RECON_HIP_TRY(hipGetLastError());
    }
    return RECON_OK;
}
