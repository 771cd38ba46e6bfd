// C ABI of the Katsevich library (include/katsevich.h): argument checks, plan lifetime,
// workspace carving and the launch sequence on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/katsevich.h"
#include "kernels.hpp"
#include "plan.hpp"

struct katsevich_plan_s {
    kats::PlanHost P;
};

namespace {

thread_local std::string g_err;

int fail(int status, const std::string &msg) {
    g_err = msg;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return KATS_EHIP;
}

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace

namespace kats {

KParams make_params(const PlanHost &P) {
    KParams k{};
    const katsevich_geometry &g = P.geom;
    const katsevich_grid &gr = P.grid;
    k.R = (float)g.R;
    k.D = (float)g.D;
    k.inv_dalpha = (float)(1.0 / g.dalpha);
    k.col_c = (float)(0.5 * (g.det_cols - 1) - g.col_offset);
    k.inv_dw = (float)(1.0 / g.dw);
    k.row_c = (float)(0.5 * (g.det_rows - 1) - g.row_offset);
    k.dz = (float)gr.dz;
    k.x_first = (float)gr.x_first;
    k.y_first = (float)gr.y_first;
    k.dx = (float)gr.dx;
    k.dy = (float)gr.dy;
    k.scale = (float)(P.dlam / (2.0 * 3.14159265358979323846));
    k.inv_2dlam = (float)(1.0 / (2.0 * P.dlam));
    k.inv_2dalpha = (float)(1.0 / (2.0 * g.dalpha));
    k.nx = gr.nx;
    k.ny = gr.ny;
    k.nz = gr.nz;
    k.ns = P.ns;
    k.n_tab = P.n_tab;
    k.rows = g.det_rows;
    k.cols = g.det_cols;
    k.n_psi = P.n_psi;
    k.fft_len = P.fft_len;
    int l2 = 0;
    while ((1 << l2) < P.fft_len) ++l2;
    k.log2n = l2;
    k.Nv = g.views_per_turn;
    k.n_lo = P.n_lo;
    k.W = P.W;
    k.n_pitches = P.n_pitches;
    k.n_views = g.n_views;
    k.half = P.half ? 1 : 0;
    k.sino_cols = P.sino_cols;
    k.sino_views = P.sino_views;
    k.first_view = P.first_view;
    k.n_filt = P.last_view >= P.first_view ? P.last_view - P.first_view + 1 : 0;
    const unsigned char *base = static_cast<const unsigned char *>(P.d_tables);
    const TableLayout &L = P.layout;
    k.view = reinterpret_cast<const float4 *>(base + L.view);
    k.fr = reinterpret_cast<const FrEntry *>(base + L.fr);
    k.br_k = reinterpret_cast<const int *>(base + L.br_k);
    k.br_w = reinterpret_cast<const float *>(base + L.br_w);
    k.lw = reinterpret_cast<const float *>(base + L.lw);
    k.cos_alpha = reinterpret_cast<const float *>(base + L.cos_alpha);
    k.twiddle = reinterpret_cast<const float2 *>(base + L.twiddle);
    k.hil_im = reinterpret_cast<const float *>(base + L.hil_im);
    k.hil_u = reinterpret_cast<const float *>(base + L.hil_u);
    k.hil_uinv = (float)(1.0 / kHilTapScale);
    k.hil_f = P.hil_f;
    k.hil_mode = P.hil_mode;
    k.pi = reinterpret_cast<const PiEntry *>(base + L.pi);
    k.boxes = reinterpret_cast<const BpBox *>(base + L.boxes);
    k.tref = reinterpret_cast<const TileRay *>(base + L.tref);
    k.bp_tiles_x = P.bp_tiles_x;
    k.bp_tiles_y = P.bp_tiles_y;
    k.bp_runs = P.bp_runs;
    k.bp_kz = P.bp_kz;
    k.bp_all_fit = P.bp_box_rows <= (P.bp_kz >= 32 ? 2 : 1) * kBpBoxRows && P.bp_box_cols <= kBpBoxCols;
    k.gf_rows = P.gf_rows;
    k.gf_cols = P.gf_cols;
    k.atan_deg = P.atan_deg;
    for (int i = 0; i < 9; ++i) k.atan_coef[i] = P.atan_coef[i];
    return k;
}

// Workspace of katsevich_recon: [g4 chunk | g2 chunk | g^F of every filtered view].
uint64_t recon_ws(const PlanHost &P) { return P.g4_bytes + P.g2_bytes + P.gF_bytes; }

// Workspace of katsevich_recon_backward: [g4 chunk | g2 chunk | g^F-bar (float or fixed
// point) | conversion chunk | scale scratch].
uint64_t backward_ws(const PlanHost &P) {
    return P.g4_bytes + P.g2_bytes + P.gbar_bytes + P.conv_bytes + P.det_bytes;
}

// The forward filter chain over chunks of views: g2 / g4 hold one chunk, g^F every view.
static hipError_t filter_chunks(const PlanHost &P, const KParams &k, const float *sino, float *g2,
                                float *g4, float *gF, hipStream_t s) {
    const size_t gfv = (size_t)k.gf_rows * k.gf_cols;
    for (long long a = 0; a < k.n_filt; a += P.chunk_views) {
        KParams kc = k;
        kc.first_view = k.first_view + a;
        kc.n_filt = std::min<long long>(P.chunk_views, k.n_filt - a);
        float *vmax = reinterpret_cast<float *>(reinterpret_cast<unsigned char *>(g2) + P.vmax_off);
        const hipError_t e = launch_filter(kc, sino, g2, g4, gF + (size_t)a * gfv, vmax, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The adjoint filter chain over chunks, each with one view of halo on both sides (the
// derivative transpose of a sinogram view reads its neighbours); sinogram views no filtered
// view reaches are zeroed.  g64 / S (deterministic mode): g^F-bar in fixed point, each
// chunk converted to float into conv first; otherwise gbar is float.
static hipError_t filter_T_chunks(const PlanHost &P, const KParams &k, const float *gbar,
                                  const unsigned long long *g64, const double *S, float *conv,
                                  float *g4, float *g2, float *gsino, hipStream_t s) {
    const size_t rc = (size_t)k.rows * k.cols;
    const long long sv = k.half ? k.sino_views : k.n_views;
    const size_t srow = (size_t)k.rows * (k.half ? k.sino_cols : k.cols) * 4;   // bytes per view
    const long long n = k.n_filt, fv = k.first_view;
    long long out_lo = 0, out_hi = 0;
    if (n > 0) {
        out_lo = k.half ? fv : fv - 1;
        out_hi = fv + n + 1;
    }
    hipError_t e = hipSuccess;
    if (out_lo > 0) e = launch_zero(gsino, (uint64_t)out_lo * srow, s);
    if (e == hipSuccess && out_hi < sv)
        e = launch_zero(reinterpret_cast<unsigned char *>(gsino) + (size_t)out_hi * srow,
                        (uint64_t)(sv - out_hi) * srow, s);
    for (long long a = 0; a < n && e == hipSuccess; a += P.chunk_views) {
        const long long b = std::min<long long>(n, a + P.chunk_views);
        const long long a1 = a > 0 ? a - 1 : 0, b1 = b < n ? b + 1 : n;
        KParams kc = k;
        kc.first_view = fv + a1;
        kc.n_filt = b1 - a1;
        const float *src = gbar + (size_t)a1 * rc;
        if (g64) {
            e = launch_fixed_to_float(g64 + (size_t)a1 * rc, (unsigned long long)(b1 - a1) * rc, S, conv, s);
            src = conv;
        }
        if (e == hipSuccess) e = launch_filter_T_views(kc, src, g4, g2, s);
        const long long lo = a > 0 ? fv + a : out_lo, hi = b < n ? fv + b : out_hi;
        if (e == hipSuccess) e = launch_deriv_T(kc, g2, gsino, lo, hi - lo, s);
    }
    return e;
}

}  // namespace kats

extern "C" {

const char *katsevich_status_string(int status) {
    switch (status) {
        case KATS_OK: return "ok";
        case KATS_EINVAL: return "invalid argument";
        case KATS_EINVAL_GEOMETRY: return "invalid geometry or grid";
        case KATS_ESHAPE: return "buffer size does not match the plan";
        case KATS_EWORKSPACE: return "workspace too small";
        case KATS_ENOTBOUND: return "plan has no bound device tables";
        case KATS_EHIP: return "HIP runtime error";
        case KATS_ENOMEM: return "out of host memory";
        default: return "unknown status";
    }
}

const char *katsevich_last_error(void) { return g_err.c_str(); }

int katsevich_plan(const katsevich_geometry *geom, const katsevich_grid *grid,
                   const katsevich_options *opts, katsevich_plan_t *out) {
    g_err.clear();
    if (!geom || !grid || !out) return fail(KATS_EINVAL, "katsevich_plan: null argument");
    *out = nullptr;
    katsevich_options o{};
    if (opts) o = *opts;
    katsevich_plan_s *p = new (std::nothrow) katsevich_plan_s();
    if (!p) return fail(KATS_ENOMEM, "katsevich_plan: out of host memory");
    std::string err;
    int st;
    try {
        st = kats::build_plan(*geom, *grid, o, p->P, err);
    } catch (const std::bad_alloc &) {
        st = KATS_ENOMEM;
        err = "out of host memory while planning";
    } catch (...) {
        st = KATS_EINVAL;
        err = "unexpected failure while planning";
    }
    if (st != KATS_OK) {
        delete p;
        return fail(st, "katsevich_plan: " + err);
    }
    *out = p;
    return KATS_OK;
}

int katsevich_plan_device_sizes(const katsevich_geometry *geom, const katsevich_grid *grid,
                                const katsevich_options *opts, katsevich_device_plan_sizes *out) {
    g_err.clear();
    if (!geom || !grid || !out) return fail(KATS_EINVAL, "katsevich_plan_device_sizes: null argument");
    katsevich_options o{};
    if (opts) o = *opts;
    katsevich_device_plan_sizes z{};
    std::string err;
    uint64_t off[5] = {0, 0, 0, 0, 0};
    int n_tab = 0;
    int st;
    try {
        st = kats::device_plan_sizes(*geom, *grid, o, z.scratch_bytes, z.table_bytes, err);
        if (st == KATS_OK) st = kats::device_plan_scratch_offsets(*geom, *grid, o, off, n_tab, err);
    } catch (const std::bad_alloc &) {
        st = KATS_ENOMEM;
        err = "out of host memory";
    }
    if (st != KATS_OK) return fail(st, "katsevich_plan_device_sizes: " + err);
    z.pi_li_offset = off[0];
    z.pi_lo_offset = off[1];
    z.pi_nfirst_offset = off[2];
    z.pi_nlast_offset = off[3];
    z.fov_offset = off[4];
    z.n_table_slices = n_tab;
    *out = z;
    return KATS_OK;
}

int katsevich_plan_device(const katsevich_geometry *geom, const katsevich_grid *grid,
                          const katsevich_options *opts, void *d_scratch, uint64_t scratch_bytes,
                          void *d_tables, uint64_t table_bytes, void *stream, katsevich_plan_t *out) {
    g_err.clear();
    if (!geom || !grid || !out || !d_scratch || !d_tables)
        return fail(KATS_EINVAL, "katsevich_plan_device: null argument");
    *out = nullptr;
    if (!aligned256(d_scratch) || !aligned256(d_tables))
        return fail(KATS_EINVAL, "katsevich_plan_device: scratch or table buffer not 256-byte aligned");
    katsevich_options o{};
    if (opts) o = *opts;
    katsevich_plan_s *p = new (std::nothrow) katsevich_plan_s();
    if (!p) return fail(KATS_ENOMEM, "katsevich_plan_device: out of host memory");
    const kats::DevicePlanBuffers buf{d_scratch, scratch_bytes, d_tables, table_bytes, stream};
    std::string err;
    int st;
    try {
        st = kats::build_plan_device(*geom, *grid, o, p->P, err, buf);
    } catch (const std::bad_alloc &) {
        st = KATS_ENOMEM;
        err = "out of host memory while planning";
    } catch (...) {
        st = KATS_EINVAL;
        err = "unexpected failure while planning";
    }
    if (st != KATS_OK) {
        delete p;
        return fail(st, "katsevich_plan_device: " + err);
    }
    *out = p;
    return KATS_OK;
}

int katsevich_plan_query(katsevich_plan_t plan, katsevich_plan_info *out) {
    g_err.clear();
    if (!plan || !out) return fail(KATS_EINVAL, "katsevich_plan_query: null argument");
    const kats::PlanHost &P = plan->P;
    katsevich_plan_info i{};
    i.table_bytes = P.layout.total;
    i.workspace_bytes = kats::recon_ws(P) > kats::backward_ws(P) ? kats::recon_ws(P) : kats::backward_ws(P);
    i.filtered_bytes = P.gF_bytes;
    i.workspace_bytes_filter = P.g4_bytes + P.g2_bytes;
    i.first_view = P.first_view;
    i.last_view = P.last_view;
    i.n_vv = P.n_vv;
    i.n_valid_voxels = P.n_valid;
    i.n_pitches = P.n_pitches;
    i.slices_per_pitch = P.ns;
    i.n_table_slices = P.n_tab;
    i.n_psi = P.n_psi;
    i.window_views = P.W;
    i.window_lo = P.n_lo;
    i.fft_len = P.fft_len;
    i.commensurate = P.commensurate ? 1 : 0;
    i.hilbert_mode = P.hil_mode;
    i.gf_rows = P.gf_rows;
    i.gf_cols = P.gf_cols;
    i.atan_degree = P.atan_deg;
    i.bp_slices = P.bp_kz;
    i.bp_box_rows = P.bp_box_rows;
    i.bp_box_cols = P.bp_box_cols;
    i.half_sample = P.half ? 1 : 0;
    *out = i;
    return KATS_OK;
}

int katsevich_plan_bind(katsevich_plan_t plan, void *d_tables, uint64_t bytes, void *stream) {
    g_err.clear();
    if (!plan || !d_tables) return fail(KATS_EINVAL, "katsevich_plan_bind: null argument");
    kats::PlanHost &P = plan->P;
    if (bytes < P.layout.total)
        return fail(KATS_ESHAPE, "katsevich_plan_bind: table buffer smaller than table_bytes");
    if (!aligned256(d_tables)) return fail(KATS_EINVAL, "katsevich_plan_bind: buffer not 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (P.device_built && d_tables == P.d_tables) return KATS_OK;
    // a device-built plan has no host image: its tables move from the buffer they were built in
    hipError_t e = P.device_built
        ? hipMemcpyAsync(d_tables, P.d_tables, P.layout.total, hipMemcpyDeviceToDevice, s)
        : hipMemcpyAsync(d_tables, P.image.data(), P.layout.total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "katsevich_plan_bind: hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "katsevich_plan_bind: hipStreamSynchronize");
    P.d_tables = d_tables;
    return KATS_OK;
}

int katsevich_plan_export(katsevich_plan_t plan, int which, void *host_dst, uint64_t bytes) {
    g_err.clear();
    if (!plan || !host_dst) return fail(KATS_EINVAL, "katsevich_plan_export: null argument");
    const kats::PlanHost &P = plan->P;
    const void *src = nullptr;
    uint64_t n = 0;
    std::vector<uint8_t> valid;
    if (P.device_built && which >= KATS_TABLE_PI_LI && which <= KATS_TABLE_FOV)
        return fail(KATS_EINVAL, "katsevich_plan_export: a device-built plan keeps its PI tables on the "
                                 "device (the scratch of katsevich_plan_device holds them on return)");
    if (P.device_built && which == KATS_TABLE_VALID) {
        // from the device PI table: entries relative to the window start, empty outside the FOV
        const katsevich_grid &gr = P.grid;
        const size_t plane = (size_t)gr.ny * gr.nx;
        std::vector<kats::PiEntry> pe((size_t)P.n_tab * plane);
        hipError_t e = hipMemcpy(pe.data(), static_cast<const unsigned char *>(P.d_tables) + P.layout.pi,
                                 pe.size() * sizeof(kats::PiEntry), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "katsevich_plan_export: hipMemcpy");
        const uint64_t need = (uint64_t)gr.nz * plane;
        if (bytes != need) return fail(KATS_ESHAPE, "katsevich_plan_export: size mismatch (need " + std::to_string(need) + ")");
        uint8_t *dst = static_cast<uint8_t *>(host_dst);
        for (int iz = 0; iz < gr.nz; ++iz) {
            const int k = iz / P.ns, j = iz % P.ns;
            const int64_t shift = (int64_t)k * P.geom.views_per_turn + P.n_lo;
            for (size_t q = 0; q < plane; ++q) {
                const kats::PiEntry &x = pe[(size_t)j * plane + q];
                dst[(size_t)iz * plane + q] = (x.nf <= x.nl && x.nf + shift - 1 >= 0 &&
                                               x.nl + shift + 1 <= P.geom.n_views - 1) ? 1 : 0;
            }
        }
        return KATS_OK;
    }
    switch (which) {
        case KATS_TABLE_FR_ROW: src = P.fr_row.data(); n = P.fr_row.size() * 4; break;
        case KATS_TABLE_FR_WEIGHT: src = P.fr_w.data(); n = P.fr_w.size() * 8; break;
        case KATS_TABLE_BR_KAPPA: src = P.br_k.data(); n = P.br_k.size() * 4; break;
        case KATS_TABLE_BR_WEIGHT: src = P.br_w.data(); n = P.br_w.size() * 8; break;
        case KATS_TABLE_PSI_HAT: src = P.psi_hat.data(); n = P.psi_hat.size() * 8; break;
        case KATS_TABLE_PI_LI: src = P.pi_li.data(); n = P.pi_li.size() * 8; break;
        case KATS_TABLE_PI_LO: src = P.pi_lo.data(); n = P.pi_lo.size() * 8; break;
        case KATS_TABLE_PI_NFIRST: src = P.pi_nf.data(); n = P.pi_nf.size() * 4; break;
        case KATS_TABLE_PI_NLAST: src = P.pi_nl.data(); n = P.pi_nl.size() * 4; break;
        case KATS_TABLE_FOV: src = P.fov.data(); n = P.fov.size(); break;
        case KATS_TABLE_VALID: {
            const katsevich_grid &gr = P.grid;
            valid.resize((size_t)gr.nz * gr.ny * gr.nx);
            for (int iz = 0; iz < gr.nz; ++iz)
                for (int iy = 0; iy < gr.ny; ++iy)
                    for (int ix = 0; ix < gr.nx; ++ix)
                        valid[((size_t)iz * gr.ny + iy) * gr.nx + ix] = kats::voxel_valid(P, iz, iy, ix) ? 1 : 0;
            src = valid.data();
            n = valid.size();
            break;
        }
        default: return fail(KATS_EINVAL, "katsevich_plan_export: unknown table id");
    }
    if (bytes != n) return fail(KATS_ESHAPE, "katsevich_plan_export: size mismatch (need " + std::to_string(n) + ")");
    std::memcpy(host_dst, src, n);
    return KATS_OK;
}

static int check_compute(katsevich_plan_t plan, const void *a, const void *b, const char *who) {
    if (!plan || !a || !b) return fail(KATS_EINVAL, std::string(who) + ": null argument");
    if (!plan->P.d_tables) return fail(KATS_ENOTBOUND, std::string(who) + ": plan not bound");
    return KATS_OK;
}

int katsevich_filter(katsevich_plan_t plan, const float *d_sino, float *d_gF, void *d_ws,
                     uint64_t ws_bytes, void *stream) {
    g_err.clear();
    int st = check_compute(plan, d_sino, d_gF, "katsevich_filter");
    if (st) return st;
    const kats::PlanHost &P = plan->P;
    if (P.g4_bytes + P.g2_bytes > 0 && (!d_ws || ws_bytes < P.g4_bytes + P.g2_bytes))
        return fail(KATS_EWORKSPACE, "katsevich_filter: workspace too small");
    if (d_ws && !aligned256(d_ws)) return fail(KATS_EINVAL, "katsevich_filter: workspace not 256-byte aligned");
    const kats::KParams k = kats::make_params(P);
    float *g4 = static_cast<float *>(d_ws);
    float *g2 = reinterpret_cast<float *>(static_cast<unsigned char *>(d_ws) + P.g4_bytes);
    hipError_t e = kats::filter_chunks(P, k, d_sino, g2, g4, d_gF, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_filter: launch");
    return KATS_OK;
}

int katsevich_backproject(katsevich_plan_t plan, const float *d_gF, float *d_vol, void *stream) {
    g_err.clear();
    int st = check_compute(plan, d_gF, d_vol, "katsevich_backproject");
    if (st) return st;
    const kats::KParams k = kats::make_params(plan->P);
    hipError_t e = kats::launch_backproject(k, d_gF, d_vol, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_backproject: launch");
    return KATS_OK;
}

int katsevich_recon(katsevich_plan_t plan, const float *d_sino, float *d_vol, void *d_ws,
                    uint64_t ws_bytes, void *stream) {
    g_err.clear();
    int st = check_compute(plan, d_sino, d_vol, "katsevich_recon");
    if (st) return st;
    const kats::PlanHost &P = plan->P;
    const uint64_t need = kats::recon_ws(P);
    if (need > 0 && (!d_ws || ws_bytes < need))
        return fail(KATS_EWORKSPACE, "katsevich_recon: workspace too small");
    if (d_ws && !aligned256(d_ws)) return fail(KATS_EINVAL, "katsevich_recon: workspace not 256-byte aligned");
    const kats::KParams k = kats::make_params(P);
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(d_ws);
    float *g4 = reinterpret_cast<float *>(w);
    float *g2 = reinterpret_cast<float *>(w + P.g4_bytes);
    float *gF = reinterpret_cast<float *>(w + P.g4_bytes + P.g2_bytes);
    hipError_t e = kats::filter_chunks(P, k, d_sino, g2, g4, gF, s);
    if (e != hipSuccess) return hip_fail(e, "katsevich_recon: filter launch");
    e = kats::launch_backproject(k, gF, d_vol, s);
    if (e != hipSuccess) return hip_fail(e, "katsevich_recon: backprojection launch");
    return KATS_OK;
}

int katsevich_recon_backward(katsevich_plan_t plan, const float *d_grad_vol, float *d_grad_sino,
                             void *d_ws, uint64_t ws_bytes, void *stream) {
    g_err.clear();
    int st = check_compute(plan, d_grad_vol, d_grad_sino, "katsevich_recon_backward");
    if (st) return st;
    const kats::PlanHost &P = plan->P;
    const uint64_t need = kats::backward_ws(P);
    if (need > 0 && (!d_ws || ws_bytes < need))
        return fail(KATS_EWORKSPACE, "katsevich_recon_backward: workspace too small");
    if (d_ws && !aligned256(d_ws)) return fail(KATS_EINVAL, "katsevich_recon_backward: workspace not 256-byte aligned");
    const kats::KParams k = kats::make_params(P);
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(d_ws);
    float *g4 = reinterpret_cast<float *>(w);
    float *g2 = reinterpret_cast<float *>(w + P.g4_bytes);
    void *gbar = w + P.g4_bytes + P.g2_bytes;
    hipError_t e = hipSuccess;
    if (P.det_adjoint) {
        // bound: every valid voxel adding at most max|fbar| dlambda/(2 pi) / v* to a cell,
        // v* >= R - r_fov for voxels in the field of view
        float *conv = reinterpret_cast<float *>(w + P.g4_bytes + P.g2_bytes + P.gbar_bytes);
        void *scr = w + P.g4_bytes + P.g2_bytes + P.gbar_bytes + P.conv_bytes;
        const double bound = (double)std::max<int64_t>(P.n_valid, 1) * (P.dlam / (2.0 * 3.14159265358979323846)) /
                             (P.geom.R - P.r_fov);
        unsigned long long *g64 = static_cast<unsigned long long *>(gbar);
        e = kats::launch_backproject_T_fixed(k, d_grad_vol, g64, scr, bound, s);
        if (e == hipSuccess)
            e = kats::filter_T_chunks(P, k, nullptr, g64, kats::fixed_scale_ptr(scr), conv, g4, g2, d_grad_sino, s);
    } else {
        float *gb = static_cast<float *>(gbar);
        e = kats::launch_zero(gb, P.gbar_bytes, s);
        if (e == hipSuccess) e = kats::launch_backproject_T(k, d_grad_vol, gb, s);
        if (e == hipSuccess) e = kats::filter_T_chunks(P, k, gb, nullptr, nullptr, nullptr, g4, g2, d_grad_sino, s);
    }
    if (e != hipSuccess) return hip_fail(e, "katsevich_recon_backward: launch");
    return KATS_OK;
}

int katsevich_sparse_upsample(const float *d_sparse, float *d_full, int64_t n_lines, int32_t cols,
                              int32_t step, void *stream) {
    g_err.clear();
    if (n_lines < 0 || cols < 1 || step < 1)
        return fail(KATS_EINVAL, "katsevich_sparse_upsample: need n_lines >= 0, cols >= 1, step >= 1");
    if (n_lines == 0) return KATS_OK;                 // nothing to read or write
    if (!d_sparse || !d_full) return fail(KATS_EINVAL, "katsevich_sparse_upsample: null pointer");
    if ((uint64_t)n_lines * (((uint64_t)cols + 3) / 4) >= (1ull << 32))
        return fail(KATS_EINVAL, "katsevich_sparse_upsample: more than 2^34 output samples");
    const int ns = (cols + step - 1) / step;
    hipError_t e = kats::launch_upsample(d_sparse, d_full, n_lines, cols, ns, step,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_sparse_upsample: launch");
    return KATS_OK;
}

uint64_t katsevich_data_scratch_bytes(void) { return kats::data_scratch_bytes(); }

int katsevich_max(const float *d_x, uint64_t n, float *d_max, void *d_scratch, uint64_t scratch_bytes,
                  void *stream) {
    g_err.clear();
    if (!d_x || !d_max || !d_scratch || n < 1) return fail(KATS_EINVAL, "katsevich_max: null pointer or n < 1");
    if (scratch_bytes < kats::data_scratch_bytes()) return fail(KATS_EWORKSPACE, "katsevich_max: scratch too small");
    if (!aligned256(d_scratch)) return fail(KATS_EINVAL, "katsevich_max: scratch not 256-byte aligned");
    hipError_t e = kats::launch_max(d_x, n, d_max, d_scratch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_max: launch");
    return KATS_OK;
}

int katsevich_add_noise(const float *d_in, float *d_out, uint64_t n, const float *d_max, double I0,
                        double var, uint64_t seed, void *stream) {
    g_err.clear();
    if (!(I0 > 1.0) || !(var >= 0.0)) return fail(KATS_EINVAL, "katsevich_add_noise: need I0 > 1 and var >= 0");
    if (n == 0) return KATS_OK;                       // nothing to read or write
    if (!d_in || !d_out || !d_max) return fail(KATS_EINVAL, "katsevich_add_noise: null pointer");
    hipError_t e = kats::launch_noise(d_in, d_out, n, d_max, (float)I0, (float)std::sqrt(var), seed,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_add_noise: launch");
    return KATS_OK;
}

int katsevich_rmse_ssim(const float *d_f, const float *d_ref, uint64_t n, double *d_result,
                        void *d_scratch, uint64_t scratch_bytes, void *stream) {
    g_err.clear();
    if (!d_f || !d_ref || !d_result || !d_scratch || n < 1)
        return fail(KATS_EINVAL, "katsevich_rmse_ssim: null pointer or n < 1");
    if (scratch_bytes < kats::data_scratch_bytes())
        return fail(KATS_EWORKSPACE, "katsevich_rmse_ssim: scratch too small");
    if (!aligned256(d_scratch)) return fail(KATS_EINVAL, "katsevich_rmse_ssim: scratch not 256-byte aligned");
    hipError_t e = kats::launch_rmse_ssim(d_f, d_ref, n, d_result, d_scratch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_rmse_ssim: launch");
    return KATS_OK;
}

int katsevich_rmse_ssim_noscratch(const float *d_f, const float *d_ref, uint64_t n, double *d_result,
                                  void *stream) {
    g_err.clear();
    if (!d_f || !d_ref || !d_result || n < 1)
        return fail(KATS_EINVAL, "katsevich_rmse_ssim_noscratch: null pointer or n < 1");
    void *scr = nullptr;
    uint64_t scr_bytes = 0;
    hipError_t e = kats::static_scratch(&scr, &scr_bytes);
    if (e != hipSuccess) return hip_fail(e, "katsevich_rmse_ssim_noscratch: static scratch address");
    if (scr_bytes < kats::data_scratch_bytes())
        return fail(KATS_EWORKSPACE, "katsevich_rmse_ssim_noscratch: reduction needs " +
                                         std::to_string(kats::data_scratch_bytes()) +
                                         " bytes of scratch, the static array holds " +
                                         std::to_string(scr_bytes));
    e = kats::launch_rmse_ssim(d_f, d_ref, n, d_result, scr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_rmse_ssim_noscratch: launch");
    return KATS_OK;
}

int katsevich_backproject_batch(const katsevich_plan_t *plans, const float *const *d_gF,
                                float *const *d_vol, int n, void *stream) {
    g_err.clear();
    if (!plans || !d_gF || !d_vol || n < 1)
        return fail(KATS_EINVAL, "katsevich_backproject_batch: null argument or n < 1");
    std::vector<kats::KParams> ks((size_t)n);
    int kz = -1;
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !d_gF[i] || !d_vol[i])
            return fail(KATS_EINVAL, "katsevich_backproject_batch: null plan or buffer at item " + std::to_string(i));
        if (!plans[i]->P.d_tables)
            return fail(KATS_ENOTBOUND, "katsevich_backproject_batch: plan " + std::to_string(i) + " not bound");
        if (kz < 0) kz = plans[i]->P.bp_kz;
        if (plans[i]->P.bp_kz != kz)
            return fail(KATS_EINVAL, "katsevich_backproject_batch: plans use different bp_slices");
        ks[(size_t)i] = kats::make_params(plans[i]->P);
    }
    hipError_t e = kats::launch_backproject_batch(ks.data(), d_gF, d_vol, n, kz,
                                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "katsevich_backproject_batch: launch");
    return KATS_OK;
}

void katsevich_plan_destroy(katsevich_plan_t plan) { delete plan; }

}  // extern "C"
