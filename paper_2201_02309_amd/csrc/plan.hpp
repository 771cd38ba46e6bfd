// Host-side float64 plan of the pitch-by-pitch Katsevich reconstruction.
//
// Everything that depends only on the scan geometry and the grid of one pitch is
// computed here once (Sec. II pre-calculating step): kappa-line forward-rebinning
// rows/weights (eqs. FR, w_k), psi_hat and backward-rebinning indices/weights (eq. BR),
// PI-line limits of every voxel of the first pitch (pre-calculating step 2), the pitch
// view window (eq. maxvalue), per-view trigonometry and the Hilbert kernel spectrum
// (eqs. HF, e4).  The periodicity relations of Sec. II let every later pitch reuse them.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/katsevich.h"

namespace kats {

// One voxel of the PI table, packed for a single 16-byte load in the backprojector.
// li/lo: PI limits in view units relative to the pitch window start n_lo;
// nf/nl: first/last view (same origin) with non-zero coverage weight; an empty range
// (nf > nl) marks a voxel outside the field of view.
struct PiEntry {
    float li, lo;
    int32_t nf, nl;
};
static_assert(sizeof(PiEntry) == 16, "PiEntry must be 16 bytes");

// Backprojection tiling: a workgroup owns a kBpTile x kBpTile (x, y) tile and a run of
// bp_kz consecutive slices of one pitch (8, 16 or 32; kBpKZ by default).
constexpr int kBpTile = 16;
constexpr int kBpKZ = 16;
// Rows / columns of zero padding around every filtered view g^F (so that clamped
// bilinear taps outside the detector read exact zeros).
constexpr int kPad = 2;
// Largest footprint box the backprojector stages in LDS (rows x columns); a plan whose
// boxes all fit lets the kernel drop its HBM fallback path.
constexpr int kBpBoxRows = 32;
constexpr int kBpBoxCols = 64;

// Detector footprint (absolute row/col origin, may be -kPad, and extent) of one
// backprojection tile x slice run at one pitch-relative view: every bilinear tap of
// every voxel of the tile lies inside it (float64 bound plus a one-cell margin),
// clipped to the zero-padded detector.
struct BpBox {
    int16_t r0, nr, c0, nc;
};
static_assert(sizeof(BpBox) == 8, "BpBox must be 8 bytes");

// Forward height rebinning of one (kappa-line, column): rows r0, r0+1 with weight w on r0+1.
struct FrEntry {
    int32_t r0;
    float w;
};
static_assert(sizeof(FrEntry) == 8, "FrEntry must be 8 bytes");

// Byte offsets of the sub-tables inside the caller's device table buffer.
struct TableLayout {
    uint64_t view = 0;       // float4 [W]   cos(beta), sin(beta), e_m, 0
    uint64_t fr = 0;         // FrEntry [n_psi][cols]  forward-rebin row and weight
    uint64_t br_k = 0;       // int32  [rows][cols]
    uint64_t br_w = 0;       // float  [rows][cols]
    uint64_t lw = 0;         // float  [rows]
    uint64_t cos_alpha = 0;  // float  [cols]
    uint64_t twiddle = 0;    // float2 [fft_len]  exp(-2 pi i k / N)
    uint64_t hil_im = 0;     // float  [fft_len]  Im(DFT of the Hilbert taps) / N
    uint64_t pi = 0;         // PiEntry [n_tab][ny][nx]
    uint64_t boxes = 0;      // BpBox   [runs][tiles_y][tiles_x][W]
    uint64_t total = 0;
};

struct PlanHost {
    katsevich_geometry geom{};       // grid of the filtered data (see build_plan)
    bool half = false;               // half-sample derivative (KATS_FLAG_HALF_SAMPLE_DERIVATIVE)
    int64_t sino_views = 0;          // sinogram views and columns as acquired
    int sino_cols = 0;
    katsevich_grid grid{};
    katsevich_options opts{};

    // derived scalars
    double h = 0, dlam = 0, alpha_m = 0, r_fov = 0, psi_max = 0, dpsi = 0;
    int n_psi = 0;
    std::vector<double> alpha, w, psi;

    // kappa rebinning
    std::vector<int32_t> fr_row;     // [n_psi][cols]
    std::vector<double> fr_w;
    std::vector<double> psi_hat;     // [rows][cols]
    std::vector<int32_t> br_k;
    std::vector<double> br_w;

    // pitches and PI limits (first pitch)
    bool commensurate = false;
    int ns = 0, n_tab = 0, n_pitches = 0;
    std::vector<double> pi_li, pi_lo;      // global view units, pitch 0
    std::vector<int32_t> pi_nf, pi_nl;     // global view indices, pitch 0
    std::vector<uint8_t> fov;
    int32_t n_lo = 0, n_hi = 0, W = 0;
    int bp_tiles_x = 0, bp_tiles_y = 0, bp_runs = 0, bp_kz = kBpKZ;
    int bp_box_rows = 0, bp_box_cols = 0;  // largest footprint box
    int64_t first_view = 0, last_view = -1, n_vv = 0, n_valid = 0;

    // Hilbert
    int fft_len = 0;
    std::vector<double> hil_im;            // [fft_len], already divided by fft_len

    // device image
    TableLayout layout;
    std::vector<unsigned char> image;      // table_bytes, copied by katsevich_plan_bind
    void *d_tables = nullptr;              // caller memory after bind

    // padded g^F view: [gf_rows][gf_cols], gf_cols a multiple of 4 (16-byte rows)
    int gf_rows = 0, gf_cols = 0;

    // column coordinate alpha*/dalpha as an odd polynomial t * P(t^2) of t = tan(alpha*)
    // (fitted on the detector's fan range); atan_deg < 0: use the library atan2f
    float atan_coef[9] = {0};
    int atan_deg = -1;

    // workspace layout (bytes)
    uint64_t g4_bytes = 0, g2_bytes = 0, gF_bytes = 0;   // gF: padded [n][rows+2kPad][cols+2kPad]
};

// Device resources for solving the PI lines on the GPU (scratch of pi_scratch_bytes()).
struct DevicePiSolve {
    void *scratch;
    uint64_t bytes;
    void *stream;
};

// Build the plan; returns a KATS_* status and fills err on failure.  With dev, the PI lines
// of one pitch are solved on the GPU (float64, same iteration) and the rest on the host.
int build_plan(const katsevich_geometry &g, const katsevich_grid &grid,
               const katsevich_options &opts, PlanHost &P, std::string &err,
               const DevicePiSolve *dev = nullptr);

// Device scratch the GPU PI solve needs for this geometry and grid (two float64 per voxel
// of one pitch's slices).
uint64_t pi_scratch_bytes(const katsevich_geometry &g, const katsevich_grid &grid);

// Validity of voxel (iz, iy, ix) (integer decision taken from the float64 tables).
bool voxel_valid(const PlanHost &P, int iz, int iy, int ix);

}  // namespace kats
