// Kernel parameter block and launchers of the gfx950 Katsevich kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace kats {

// Scalars and table pointers every kernel reads; passed by value (kernel argument).
struct KParams {
    // detector / geometry (float32 copies of float64 plan values)
    float R, D;
    float inv_dalpha, col_c;      // column coordinate = alpha * inv_dalpha + col_c
    float inv_dw, row_c;          // row coordinate    = w * inv_dw + row_c
    float dz;
    float x_first, y_first, dx, dy;
    float scale;                  // dlambda / (2 pi)
    float inv_2dlam, inv_2dalpha;
    int nx, ny, nz, ns, n_tab;
    int rows, cols, n_psi, fft_len, log2n;
    int Nv, n_lo, W, n_pitches;
    long long n_views, first_view, n_filt;
    // sinogram as acquired: with the half-sample derivative (half = 1) views and columns of
    // the filtered grid sit between those of the sinogram (sino_views = n_views + 1,
    // sino_cols = cols + 1); otherwise the two grids coincide
    int half, sino_cols;
    long long sino_views;
    // device tables (inside the caller's bound table buffer)
    const float4 *view;
    const FrEntry *fr;
    const int *br_k;
    const float *br_w;
    const float *lw;
    const float *cos_alpha;
    const float2 *twiddle;
    const float *hil_im;
    // Hilbert on the matrix cores (hil_mode 2): reversed odd taps times 2^14 (256 hil_f + 32
    // floats), 2^-14, 32-column fragments per wave quarter
    const float *hil_u;
    float hil_uinv;
    int hil_f, hil_mode;
    const PiEntry *pi;
    const BpBox *boxes;
    const TileRay *tref;
    int bp_tiles_x, bp_tiles_y, bp_runs, bp_kz;
    int bp_all_fit;                    // every footprint box fits the LDS tile
    int gf_rows, gf_cols;              // padded g^F view (zero border kPad)
    int atan_deg;                      // < 0: atan2f
    float atan_coef[9];                // alpha/dalpha = t * sum_k atan_coef[k] t^(2k)
};

KParams make_params(const PlanHost &P);

// Sparse-detector data path and image metrics (data.hip).
uint64_t data_scratch_bytes();
hipError_t launch_upsample(const float *sp, float *full, long long lines, int cols, int ns, int step,
                           hipStream_t s);
hipError_t launch_max(const float *x, unsigned long long n, float *out, void *scratch, hipStream_t s);
hipError_t launch_noise(const float *in, float *out, unsigned long long n, const float *d_max, float I0,
                        float sd_e, uint64_t seed, hipStream_t s);
hipError_t launch_rmse_ssim(const float *f, const float *g, unsigned long long n, double *result,
                            void *scratch, hipStream_t s);
// Device address (for the current device) and size of the library-owned static reduction
// scratch; the address is looked up with hipGetSymbolAddress on a device's first call.
hipError_t static_scratch(void **out, uint64_t *bytes);

// Hilbert filter on the matrix cores, in place on the rebinned kappa rows g4 (vmax: the
// per-(view, column block) maxima above).
hipError_t launch_hilbert_mfma(const KParams &k, float *g4, const float *vmax, hipStream_t s);

// Forward filter chain on views first_view..last_view:
//   g2 = deriv+LW(sino); g4 = Hilbert(FR(g2)); gF = cos * BR(g4).
// Matrix-core Hilbert path: the forward rebinning runs as a kernel of its own (one thread per
// (4 views, column, group of kRebinLines kappa lines)) and leaves one max |g3| per (4 views,
// line group, block of kDRThreads columns) for the Hilbert's range scaling.
constexpr int kDRThreads = 128;
constexpr int kRebinLines = 16;
constexpr int kRebinViews = 4;
inline uint64_t rebin_max_count(long long n_filt, int n_psi, int cols) {
    return (uint64_t)((n_filt + kRebinViews - 1) / kRebinViews) * ((n_psi + kRebinLines - 1) / kRebinLines) *
           ((cols + kDRThreads - 1) / kDRThreads);
}
// vmax: those maxima (MFMA path only).
hipError_t launch_filter(const KParams &k, const float *sino, float *g2, float *g4, float *gF,
                         float *vmax, hipStream_t s);
// Backprojection of every pitch (reusing the first pitch's tables).
hipError_t launch_backproject(const KParams &k, const float *gF, float *vol, hipStream_t s);
// Grouped backprojection of n bound plans (one launch per group of up to 16 plans, the
// plans whose boxes fit the LDS tile grouped apart); kz: the plans' common slice run.
hipError_t launch_backproject_batch(const KParams *ks, const float *const *gF, float *const *vol,
                                    int n, int kz, hipStream_t s);
// Adjoint pieces.
hipError_t launch_backproject_T(const KParams &k, const float *gvol, float *gFbar, hipStream_t s);
// Deterministic adjoint backprojection: max |gvol| -> power-of-two scale S (bound * max * S
// < 2^62) kept in the scratch (fixed_scale_ptr), 64-bit fixed-point accumulation into gF64
// (zeroed here); launch_fixed_to_float turns a range of it into g^F-bar = gF64 / S.
constexpr int kFixedScaleBlocks = 4096;     // partial maxima of the scale reduction
inline uint64_t fixed_scratch_bytes() { return (uint64_t)kFixedScaleBlocks * 4 + 256; }
hipError_t launch_backproject_T_fixed(const KParams &k, const float *gvol, unsigned long long *gF64,
                                      void *scratch, double bound, hipStream_t s);
const double *fixed_scale_ptr(const void *scratch);
hipError_t launch_fixed_to_float(const unsigned long long *in, unsigned long long n, const double *S,
                                 float *out, hipStream_t s);
hipError_t launch_zero(void *ptr, uint64_t bytes, hipStream_t s);
hipError_t launch_filter_T(const KParams &k, const float *gFbar, float *g4bar, float *g2bar,
                           float *gsino, hipStream_t s);
// The per-view transposes (BR^T + cos, Hilbert^T, FR^T + LW) of views first_view ..
// first_view + n_filt - 1 of k, and the derivative transpose of sinogram views n0 ..
// n0 + count - 1 from the g2bar of k's views (zero outside them).
hipError_t launch_filter_T_views(const KParams &k, const float *gFbar, float *g4bar, float *g2bar,
                                 hipStream_t s);
hipError_t launch_deriv_T(const KParams &k, const float *g2bar, float *gsino, long long n0,
                          long long count, hipStream_t s);

// ---- Device plan builder (plan_gpu.hip): float64 scalars of the plan, exactly as the host
// builder holds them.
struct DevPlanArgs {
    double R, D, h, lambda0, z0, lambda_first, dlam;
    double dalpha, col_offset, dw, row_offset;
    double kscale, psi_max, dpsi, r_fov;
    double x_first, dx, y_first, dy, z_first, dz;
    long long n_views;
    int cols, rows, n_psi, fft_len;
    int nx, ny, nz, n_tab, ns, Nv;
    int tiles_x, tiles_y, runs, kz, W_cap;
    int hil_f;
};

// Counts the device builder reduces (in scratch; read back once at the end).
struct DevPlanStats {
    int nmin, nmax;                  // over voxels in the field of view: first / last covered view
    int box_rows, box_cols;          // largest footprint box over the tiles' hulls
    long long vmin, vmax;            // first / last view any valid voxel uses
    unsigned long long n_vv, n_valid;
};

struct DevPlanPtrs {
    // scratch: float64 PI limits (view units) and integer PI tables of the table pitch,
    // the counts, and float64 copies of the rebinning tables for the host
    double *li, *lo;
    int *nf, *nl;
    unsigned char *fov;
    DevPlanStats *stats;
    int *fr_row;
    double *fr_w, *psi_hat;
    int *br_k;
    double *br_w;
    // the caller's table buffer
    float4 *view;
    FrEntry *fr;
    int *t_br_k;
    float *t_br_w, *lw, *cos_alpha;
    float2 *twiddle;
    float *hil_im;
    float *hil_u;
    PiEntry *pi;
    BpBox *boxes;
    TileRay *tref;
};

hipError_t launch_plan_device(const DevPlanArgs &a, const DevPlanPtrs &p, hipStream_t s);

}  // namespace kats
