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
// Views per chunk of the filter chains: as many as kFilterChunkBytes of intermediates
// (kappa-rows + detector rows) hold, at least kFilterChunk (the clinical 736-column detector
// takes 398 views, 0.22 GB, cut to 381 for whole rounds of the matrix-core Hilbert's tiles; a
// narrow detector gets longer chunks, whose launches would otherwise be too short to fill
// the GPU).  Measured on the clinical filter: 381-view chunks 1.76 ms, 508 1.79, 1016 1.84,
// 254 1.79 (half-sample plan 1.90, 1.97, 2.10, 1.87).
constexpr int kFilterChunk = 384;
constexpr uint64_t kFilterChunkBytes = 216ull << 20;
// Scale of the matrix-core Hilbert's taps: |K[m]| <= 2/pi, so 2^14 K stays below the float16
// maximum and the smallest taps' low halves stay normal numbers.
constexpr double kHilTapScale = 16384.0;
// Matrix-core Hilbert: kappa rows per tile and persistent workgroups (two per CU of the
// MI355X), so one round of tiles holds kHilTileRows x kHilBlocks rows; its chunks of views are
// cut to whole rounds (a chunk of 512 clinical views is 4.03 rounds: the 0.03 takes a fifth).
constexpr int kHilTileRows = 32;
constexpr int kHilBlocks = 512;

// Detector footprint (absolute row/col origin, may be -kPad, and extent) of one
// backprojection tile x slice run at one pitch-relative view: every bilinear tap of
// every voxel of the tile lies inside it (float64 bound plus a one-cell margin),
// clipped to the zero-padded detector.
struct BpBox {
    int16_t r0, nr, c0, nc;
};
static_assert(sizeof(BpBox) == 8, "BpBox must be 8 bytes");

// The ray from the source to the centre (x_c, y_c) of a backprojection tile at one window
// view, from float64: u_c = -x_c sin(beta) + y_c cos(beta), v_c = R - x_c cos(beta) - y_c
// sin(beta), col = its column coordinate atan2(u_c, v_c)/dalpha + col_c relative to the
// tile's footprint box column c0.  The adjoint backprojector measures a voxel's column from
// it (small in-tile offsets in float32) instead of from the detector centre.
struct TileRay {
    float col, uc, vc, rho2;   // rho2 = u_c^2 + v_c^2
};
static_assert(sizeof(TileRay) == 16, "TileRay must be 16 bytes");

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
    uint64_t hil_u = 0;      // float  [256 hil_f + 32]  reversed odd Hilbert taps x 2^14
    uint64_t pi = 0;         // PiEntry [n_tab][ny][nx]
    uint64_t boxes = 0;      // BpBox   [runs][tiles_y][tiles_x][W]
    uint64_t tref = 0;       // float4  [tiles_y][tiles_x][W]  the tile centre's ray (see below)
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
    int hil_mode = 1;                      // KATS_HILBERT_FFT or KATS_HILBERT_MFMA
    int hil_f = 1;                         // 128-column groups of one output parity (matrix cores)
    std::vector<double> hil_im;            // [fft_len], already divided by fft_len

    // device image
    TableLayout layout;
    std::vector<unsigned char> image;      // table_bytes, copied by katsevich_plan_bind
    void *d_tables = nullptr;              // caller memory after bind
    // device-built plan: the tables were computed in place in d_tables (no host image, no
    // host PI tables); W_cap is the window bound its view and box tables are laid out for
    bool device_built = false;
    int W_cap = 0;

    // padded g^F view: [gf_rows][gf_cols], gf_cols a multiple of 4 (16-byte rows)
    int gf_rows = 0, gf_cols = 0;

    // column coordinate alpha*/dalpha as an odd polynomial t * P(t^2) of t = tan(alpha*)
    // (fitted on the detector's fan range); atan_deg < 0: use the library atan2f
    float atan_coef[9] = {0};
    int atan_deg = -1;

    // workspace layout (bytes).  The filter chains run over chunks of at most chunk_views
    // views (plus one view each side for the adjoint's derivative): g4 and g2 hold one
    // chunk's kappa-rows and detector rows; gF the padded g^F of every filtered view
    // [n][rows+2kPad][cols+2kPad]; gbar the adjoint's g^F-bar of every filtered view (float,
    // or 64-bit fixed point in the deterministic mode, which also takes conv_bytes for one
    // chunk's conversion to float and det_bytes of scale scratch).
    int64_t chunk_views = 0;
    uint64_t vmax_off = 0;                 // per-view maxima (matrix-core Hilbert) inside the g2 region
    uint64_t g4_bytes = 0, g2_bytes = 0, gF_bytes = 0, gbar_bytes = 0;
    bool det_adjoint = false;                           // KATS_FLAG_DETERMINISTIC_ADJOINT
    uint64_t conv_bytes = 0, det_bytes = 0;
};

// Build the plan on the host in float64; returns a KATS_* status and fills err on failure.
int build_plan(const katsevich_geometry &g, const katsevich_grid &grid,
               const katsevich_options &opts, PlanHost &P, std::string &err);

// Caller buffers of the device plan builder (sizes from device_plan_sizes).
struct DevicePlanBuffers {
    void *scratch;
    uint64_t scratch_bytes;
    void *tables;
    uint64_t table_bytes;
    void *stream;
};

// Scratch and table bytes the device builder needs for this geometry, grid and options.
int device_plan_sizes(const katsevich_geometry &g, const katsevich_grid &grid,
                      const katsevich_options &opts, uint64_t &scratch_bytes,
                      uint64_t &table_bytes, std::string &err);

// Offsets in the device builder's scratch of its float64 PI limits (view units) li, lo,
// int32 first / last covered views nf, nl and uint8 field-of-view flags, each
// [n_tab][ny][nx]; they hold the table pitch's values when build_plan_device returns.
int device_plan_scratch_offsets(const katsevich_geometry &g, const katsevich_grid &grid,
                                const katsevich_options &opts, uint64_t off[5], int &n_tab,
                                std::string &err);

// Build the plan on the GPU in float64, straight into buf.tables (the plan is bound to it);
// one synchronisation of buf.stream at the end.
int build_plan_device(const katsevich_geometry &g, const katsevich_grid &grid,
                      const katsevich_options &opts, PlanHost &P, std::string &err,
                      const DevicePlanBuffers &buf);

// Validity of voxel (iz, iy, ix) (integer decision taken from the float64 tables).
bool voxel_valid(const PlanHost &P, int iz, int iy, int ix);

}  // namespace kats
