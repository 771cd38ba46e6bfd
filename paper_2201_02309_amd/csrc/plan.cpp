// Host float64 plan builder: see plan.hpp.
#include "plan.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

namespace kats {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

// ---------------------------------------------------------------------------------
// kappa-lines (eqs. FR and w_k; R_o read as R, P as the feed per turn)
// ---------------------------------------------------------------------------------
struct Kappa {
    double scale;   // D P / (2 pi R)
    double wk(double a, double p) const {
        const double pc = (p == 0.0) ? 1.0 : p / std::tan(p);   // psi cot psi -> 1 at 0
        return scale * (p * std::cos(a) + pc * std::sin(a));
    }
    // d w_kappa / d psi; the bracket is psi-derivative of psi cot psi
    double dwk(double a, double p) const {
        const double s = std::sin(p);
        return scale * (std::cos(a) + std::sin(a) * (std::cos(p) / s - p / (s * s)));
    }
};

// Bisection for an increasing function on [lo, hi], run to the end of float64
// resolution (until the midpoint no longer lies strictly inside the bracket).
template <class F>
double bisect_increasing(F f, double lo, double hi) {
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        const double v = f(mid);
        if (v < 0) lo = mid;
        else if (v > 0) hi = mid;
        else { lo = hi = mid; break; }
    }
    return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------------
// PI lines.  For source angle b1 = s + lambda0 and X = (x, y) = rho (cos phi, sin phi),
// d = phi - b1, the in-plane chord from the source through X ends at b1 + 2 theta with
// theta = atan2(A, B), A = R - rho cos d, B = rho sin d (the chord lies at distance
// R cos(theta) from the axis, normal direction b1 + theta).  Along the chord direction
// e(b1 + theta + pi/2), X sits at fraction t = 1/2 + rho (B cos d ... ) / (2 R sin theta),
// i.e. t = 1/2 + rho (sin d * B - cos d * A) / (2 R A).  lambda_i = s solves
// z0 + h (s + 2 theta t) = z.
// ---------------------------------------------------------------------------------
struct PiSolver {
    double R, h, lambda0, z0;

    double height_gap(double s, double rho, double phi, double z, double &span) const {
        const double d = phi - (s + lambda0);
        const double sd = std::sin(d), cd = std::cos(d);
        const double A = R - rho * cd, B = rho * sd;
        span = 2.0 * std::atan2(A, B);                      // (0, 2 pi)
        const double t = 0.5 + rho * (sd * B - cd * A) / (2.0 * R * A);
        return z0 + h * (s + t * span) - z;
    }

    // height gap and its derivative in s (dd/ds = -1):
    // dA/ds = -rho sin d, dB/ds = -rho cos d, dtheta/ds = rho (A cos d - B sin d)/(A^2+B^2),
    // N = sin d B - cos d A, dN/ds = -(cos d B + sin d A), t = 1/2 + rho N / (2 R A).
    double height_gap_d(double s, double rho, double phi, double z, double &span,
                        double &deriv) const {
        const double d = phi - (s + lambda0);
        const double sd = std::sin(d), cd = std::cos(d);
        const double A = R - rho * cd, B = rho * sd;
        const double th = std::atan2(A, B);
        span = 2.0 * th;
        const double N = sd * B - cd * A;
        const double t = 0.5 + rho * N / (2.0 * R * A);
        const double dth = rho * (A * cd - B * sd) / (A * A + B * B);
        const double dA = -rho * sd;
        const double dN = -(cd * B + sd * A);
        const double dt = rho / (2.0 * R) * (dN * A - N * dA) / (A * A);
        deriv = h * (1.0 + dt * span + t * 2.0 * dth);
        return z0 + h * (s + t * span) - z;
    }

    // Newton from a close guess, kept inside the domain; false if it does not settle
    // within a few steps (the caller then brackets).
    bool newton(double guess, double rho, double phi, double z, double &root) const {
        const double zr = (z - z0) / h;
        double s = guess, span, der;
        for (int it = 0; it < 8; ++it) {
            const double f = height_gap_d(s, rho, phi, z, span, der);
            if (f == 0.0) { root = s; return true; }
            if (!(der > 0.0)) return false;
            const double sn = s - f / der;
            if (!(sn > zr - kTwoPi && sn < zr)) return false;
            // quadratic convergence: after a step of 1e-9 the error is ~1e-18, below the
            // float64 resolution of s, so the update is final
            if (std::fabs(sn - s) <= 1e-9 * std::max(1.0, std::fabs(s))) { root = sn; return true; }
            s = sn;
        }
        return false;
    }

    // Illinois-modified regula falsi on a bracket [a, b] with F(a) < 0 < F(b).
    double illinois(double a, double fa, double b, double fb, double rho, double phi,
                    double z) const {
        double s = 0.5 * (a + b), span;
        int side = 0;
        for (int it = 0; it < 200; ++it) {
            s = b - fb * (b - a) / (fb - fa);
            if (!(s > a && s < b)) s = 0.5 * (a + b);
            if (!(s > a && s < b)) break;                 // bracket at float64 resolution
            const double fs = height_gap(s, rho, phi, z, span);
            if (fs == 0.0) return s;
            if (fs < 0) {
                a = s; fa = fs;
                if (side == -1) fb *= 0.5;
                side = -1;
            } else {
                b = s; fb = fs;
                if (side == +1) fa *= 0.5;
                side = +1;
            }
            if (b - a <= 4e-16 * std::max(1.0, std::fabs(s))) break;
        }
        return s;
    }

    // Root on ((z-z0)/h - 2pi, (z-z0)/h); a previous root s_prev of a lower z (same
    // x, y) is a lower bound, since lambda_i increases with z.
    void solve(double x, double y, double z, double &li, double &lo, const double *s_prev,
               double step, const double *guess = nullptr) const {
        const double rho = std::hypot(x, y), phi = std::atan2(y, x);
        const double zr = (z - z0) / h;
        double span;
        double root;
        if (guess && newton(*guess, rho, phi, z, root)) {
            height_gap(root, rho, phi, z, span);
            li = root;
            lo = root + span;
            return;
        }
        double a = zr - kTwoPi, b = zr;
        double fa, fb;
        bool have = false;
        if (s_prev && *s_prev > a && *s_prev < b) {
            fa = height_gap(*s_prev, rho, phi, z, span);
            if (fa < 0) {
                a = *s_prev;
                for (double w = step; !have; w *= 4.0) {
                    const double hi = std::min(a + w, zr);
                    fb = height_gap(hi, rho, phi, z, span);
                    if (fb > 0) { b = hi; have = true; }
                    else if (hi >= zr) break;
                    else { a = hi; fa = fb; }
                }
            }
        }
        if (!have) {
            a = zr - kTwoPi;
            b = zr;
            fa = height_gap(a, rho, phi, z, span);
            fb = height_gap(b, rho, phi, z, span);
        }
        const double s = (fa < 0 && fb > 0) ? illinois(a, fa, b, fb, rho, phi, z) : 0.5 * (a + b);
        height_gap(s, rho, phi, z, span);
        li = s;
        lo = s + span;
    }
};

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

int threads_for(const katsevich_options &o) {
    int n = o.n_threads > 0 ? o.n_threads : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 256));
}

template <class Fn>
void parallel_for(int n, int threads, Fn fn) {
    std::atomic<int> next(0);
    auto worker = [&]() {
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= n) break;
            fn(i);
        }
    };
    std::vector<std::thread> pool;
    const int t = std::min(threads, n);
    for (int k = 1; k < t; ++k) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
}

// Odd polynomial for alpha / dalpha = atan(t) / dalpha on |t| <= T: interpolate
// f(sigma) = atan(t)/t, s = t^2 = sigma T^2, at the d+1 Chebyshev points of sigma in [0, 1]
// (Vandermonde solve in long double), scale by 1/dalpha, round to float32, and accept the
// lowest degree whose float32 Horner evaluation t * (c0 + s (c1 + ...)) stays within 4 ulp
// of the largest column coordinate over a dense grid of t.
bool fit_atan_columns(double T, double inv_dalpha, float coef[9], int &deg) {
    const double S = T * T;
    const double ymax = std::atan(T) * inv_dalpha;
    const double tol = 4.0 * std::ldexp(1.0, std::ilogb(ymax) - 23);
    for (int d = 2; d <= 8; ++d) {
        const int n = d + 1;
        long double M[9][10];
        for (int i = 0; i < n; ++i) {
            const long double sig = 0.5L + 0.5L * std::cos((2.0L * i + 1.0L) * (long double)kPi / (2.0L * n));
            const long double t = std::sqrt(sig * (long double)S);
            const long double f = (t == 0.0L) ? 1.0L : std::atan(t) / t;
            long double pw = 1.0L;
            for (int k = 0; k < n; ++k) { M[i][k] = pw; pw *= sig; }
            M[i][n] = f;
        }
        for (int c = 0; c < n; ++c) {                 // Gaussian elimination, partial pivoting
            int piv = c;
            for (int r = c + 1; r < n; ++r)
                if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
            for (int k = 0; k <= n; ++k) std::swap(M[c][k], M[piv][k]);
            for (int r = 0; r < n; ++r) {
                if (r == c) continue;
                const long double fct = M[r][c] / M[c][c];
                for (int k = c; k <= n; ++k) M[r][k] -= fct * M[c][k];
            }
        }
        float cf[9] = {0};
        long double sk = 1.0L;
        for (int k = 0; k < n; ++k) {                 // sigma^k = s^k / S^k
            cf[k] = (float)((M[k][n] / M[k][k]) / sk * (long double)inv_dalpha);
            sk *= (long double)S;
        }
        double err = 0.0;
        for (int i = 0; i <= 20000; ++i) {
            const float t = (float)(-T + 2.0 * T * i / 20000.0);
            const float ss = t * t;
            float q = cf[d];
            for (int k = d - 1; k >= 0; --k) q = std::fmaf(q, ss, cf[k]);
            const float y = t * q;
            err = std::max(err, std::fabs((double)y - std::atan((double)t) * inv_dalpha));
        }
        if (err <= tol) {
            for (int k = 0; k < 9; ++k) coef[k] = cf[k];
            deg = d;
            return true;
        }
    }
    deg = -1;
    return false;
}

}  // namespace

bool voxel_valid(const PlanHost &P, int iz, int iy, int ix) {
    const int k = iz / P.ns, j = iz % P.ns;
    const size_t e = ((size_t)j * P.grid.ny + iy) * P.grid.nx + ix;
    if (!P.fov[e]) return false;
    const int64_t shift = (int64_t)k * P.geom.views_per_turn;
    return P.pi_nf[e] + shift - 1 >= 0 && P.pi_nl[e] + shift + 1 <= P.geom.n_views - 1;
}

static int table_slices(const katsevich_geometry &g, const katsevich_grid &gr, int *ns_out,
                        bool *comm_out) {
    const int ns_round = (int)std::llround(g.feed_per_turn / gr.dz);
    const bool comm = ns_round >= 1 && std::fabs(ns_round * gr.dz - g.feed_per_turn) <= 1e-9 * g.feed_per_turn;
    const int ns = comm ? ns_round : gr.nz;
    if (ns_out) *ns_out = ns;
    if (comm_out) *comm_out = comm;
    return std::min(ns, gr.nz);
}


// Validation, detector coordinates, kappa-line sampling, pitch structure and the Hilbert
// FFT length: everything both builders share, all of it O(rows + cols + n_psi).
static int plan_setup(const katsevich_geometry &g_in, const katsevich_grid &gr,
                      const katsevich_options &opts, PlanHost &P, std::string &err) {
    auto bad = [&](const std::string &m) { err = m; return KATS_EINVAL_GEOMETRY; };
    if (opts.flags & ~(KATS_FLAG_HALF_SAMPLE_DERIVATIVE | KATS_FLAG_DETERMINISTIC_ADJOINT))
        return bad("unknown option flags");
    P.det_adjoint = (opts.flags & KATS_FLAG_DETERMINISTIC_ADJOINT) != 0;
    // Half-sample derivative: eq. Deriv is taken at the centre of each 2 x 2 cell of the
    // sinogram's (lambda, alpha) samples, so the filtered data live on views lambda_{n+1/2}
    // and columns alpha_{c+1/2}: one view and one column fewer, the same column offset
    // (columns are centred on the detector).  Every later step runs on that grid; only the
    // derivative reads the sinogram's own grid.
    P.half = (opts.flags & KATS_FLAG_HALF_SAMPLE_DERIVATIVE) != 0;
    P.sino_views = g_in.n_views;
    P.sino_cols = g_in.det_cols;
    katsevich_geometry g = g_in;
    if (P.half) {
        if (g_in.n_views < 4 || g_in.det_cols < 3)
            return bad("the half-sample derivative needs n_views >= 4 and det_cols >= 3");
        if (g_in.views_per_turn < 4) return bad("views_per_turn must be >= 4");
        g.lambda_first += kPi / g_in.views_per_turn;
        g.det_cols -= 1;
        g.n_views -= 1;
    }
    P.geom = g;
    P.grid = gr;
    P.opts = opts;
    // ------------------------------------------------------------------ validation
    if (!(g.R > 0) || !(g.D > 0) || !(g.feed_per_turn > 0)) return bad("R, D and feed_per_turn must be > 0");
    if (g.views_per_turn < 4) return bad("views_per_turn must be >= 4");
    if (g.n_views < 3) return bad("n_views must be >= 3");
    if (g.det_cols < 2 || g.det_rows < 2) return bad("detector needs >= 2 columns and rows");
    if (g.det_cols > 1024) return bad("det_cols > 1024 is not supported (Hilbert FFT length <= 2048)");
    if (!(g.dalpha > 0) || !(g.dw > 0)) return bad("dalpha and dw must be > 0");
    if (gr.nx < 1 || gr.ny < 1 || gr.nz < 1) return bad("grid sizes must be >= 1");
    if (!(gr.dx > 0) || !(gr.dy > 0) || !(gr.dz > 0)) return bad("grid spacings must be > 0");
    if (opts.n_psi != 0 && opts.n_psi < 3) return bad("n_psi must be 0 or >= 3");
    if (opts.bp_slices != 0 && opts.bp_slices != 8 && opts.bp_slices != 16 && opts.bp_slices != 32)
        return bad("bp_slices must be 0, 8, 16 or 32");
    P.bp_kz = opts.bp_slices ? opts.bp_slices : kBpKZ;
    if (opts.hilbert_mode < KATS_HILBERT_AUTO || opts.hilbert_mode > KATS_HILBERT_MFMA)
        return bad("hilbert_mode must be 0 (auto), 1 (FFT) or 2 (matrix cores)");
    // auto: the matrix-core product, measured faster than the register FFT on the clinical
    // workload (whole filter 1.87 against 2.16 ms)
    P.hil_mode = opts.hilbert_mode == KATS_HILBERT_FFT ? KATS_HILBERT_FFT : KATS_HILBERT_MFMA;
    P.hil_f = ((g.det_cols + 1) / 2 + 127) / 128;            // <= 4 for det_cols <= 1024

    const int cols = g.det_cols, rows = g.det_rows;
    P.h = g.feed_per_turn / kTwoPi;
    P.dlam = kTwoPi / g.views_per_turn;
    P.alpha.resize(cols);
    P.w.resize(rows);
    for (int c = 0; c < cols; ++c) P.alpha[c] = (c - 0.5 * (cols - 1) + g.col_offset) * g.dalpha;
    for (int r = 0; r < rows; ++r) P.w[r] = (r - 0.5 * (rows - 1) + g.row_offset) * g.dw;
    const double a_first = P.alpha.front(), a_last = P.alpha.back();
    if (!(a_first < 0 && a_last > 0)) return bad("detector columns must straddle alpha = 0");
    if (!(a_last < 0.5 * kPi && -a_first < 0.5 * kPi)) return bad("|alpha| must stay below pi/2");
    P.alpha_m = std::max(std::fabs(a_first), std::fabs(a_last));
    P.r_fov = g.R * std::sin(std::min(-a_first, a_last));
    {
        // every lane of a backprojection tile (the grid rounded up to whole tiles) must see
        // the source in front of it (v* > 0): keep that extent well inside the helix radius
        const int ex = ((gr.nx + kBpTile - 1) / kBpTile) * kBpTile - 1;
        const int ey = ((gr.ny + kBpTile - 1) / kBpTile) * kBpTile - 1;
        const double xs[2] = {gr.x_first, gr.x_first + ex * gr.dx};
        const double ys[2] = {gr.y_first, gr.y_first + ey * gr.dy};
        double rmax = 0.0;
        for (double xv : xs)
            for (double yv : ys) rmax = std::max(rmax, std::hypot(xv, yv));
        if (rmax >= 0.9 * g.R) return bad("grid extends beyond 0.9 R from the axis");
    }

    // Tam-Danielsson window of the curved detector: w_top(a) = (D P/2pi R)(pi/2 - a)/cos a,
    // w_bot(a) = -(D P/2pi R)(pi/2 + a)/cos a, must lie inside the row range.
    const Kappa K{g.D * P.h / g.R};
    for (int c = 0; c < cols; ++c) {
        const double a = P.alpha[c];
        const double top = K.scale * (0.5 * kPi - a) / std::cos(a);
        const double bot = -K.scale * (0.5 * kPi + a) / std::cos(a);
        if (top > P.w.back() || bot < P.w.front()) {
            return bad("detector rows do not cover the Tam-Danielsson window (need w from " +
                       std::to_string(bot) + " to " + std::to_string(top) + " mm at column " +
                       std::to_string(c) + ")");
        }
    }

    // ------------------------------------------------------------------ kappa-lines
    P.n_psi = opts.n_psi ? opts.n_psi : 2 * rows + 1;
    P.psi_max = 0.5 * kPi + P.alpha_m;
    P.dpsi = 2.0 * P.psi_max / (P.n_psi - 1);
    P.psi.resize(P.n_psi);
    for (int k = 0; k < P.n_psi; ++k) P.psi[k] = (k - 0.5 * (P.n_psi - 1)) * P.dpsi;

    // ------------------------------------------------------------------ pitches, FFT length
    P.n_tab = table_slices(g, gr, &P.ns, &P.commensurate);
    P.n_pitches = (gr.nz + P.ns - 1) / P.ns;
    P.bp_tiles_x = (gr.nx + kBpTile - 1) / kBpTile;
    P.bp_tiles_y = (gr.ny + kBpTile - 1) / kBpTile;
    P.bp_runs = (P.n_tab + P.bp_kz - 1) / P.bp_kz;
    P.fft_len = 1;
    while (P.fft_len < 2 * cols - 1) P.fft_len *= 2;
    P.fft_len = std::max(P.fft_len, 64);          // smallest register-FFT shape
    P.gf_rows = rows + 2 * kPad;
    P.gf_cols = (cols + 2 * kPad + 3) & ~3;
    // |tan(alpha*)| <= tan(alpha_m) for every voxel inside the field of view; other lanes
    // are discarded (and clamped into their box), so a fit on that range is exact enough
    fit_atan_columns(std::tan(P.alpha_m) * (1.0 + 1e-4), 1.0 / g.dalpha, P.atan_coef, P.atan_deg);
    return KATS_OK;
}

// Byte offsets of the device tables for a pitch window of W views (the host builder knows
// W exactly, the device builder lays the tables out for an upper bound of it).
static void make_layout(PlanHost &P, int W) {
    const katsevich_geometry &g = P.geom;
    const uint64_t nvox = (uint64_t)P.n_tab * P.grid.ny * P.grid.nx;
    TableLayout &L = P.layout;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { const uint64_t o = off; off = align256(off + bytes); return o; };
    L.view = take((uint64_t)W * 16);
    L.fr = take((uint64_t)P.n_psi * g.det_cols * sizeof(FrEntry));
    L.br_k = take((uint64_t)g.det_rows * g.det_cols * 4);
    L.br_w = take((uint64_t)g.det_rows * g.det_cols * 4);
    L.lw = take((uint64_t)g.det_rows * 4);
    L.cos_alpha = take((uint64_t)g.det_cols * 4);
    L.twiddle = take((uint64_t)P.fft_len * 8);
    L.hil_im = take((uint64_t)P.fft_len * 4);
    L.hil_u = take((uint64_t)(256 * P.hil_f + 32) * 4);
    L.pi = take(nvox * sizeof(PiEntry));
    L.boxes = take((uint64_t)P.bp_runs * P.bp_tiles_y * P.bp_tiles_x * W * sizeof(BpBox));
    L.tref = take((uint64_t)P.bp_tiles_y * P.bp_tiles_x * W * sizeof(TileRay));
    L.total = off;
}

// Workspace sizes once the filtered view range is known.
static void set_workspace(PlanHost &P) {
    const katsevich_geometry &g = P.geom;
    const int64_t nfilt = std::max<int64_t>(0, P.last_view - P.first_view + 1);
    const uint64_t rc = (uint64_t)g.det_rows * g.det_cols;
    const uint64_t per_view = (uint64_t)(P.n_psi + g.det_rows) * g.det_cols * 4;
    P.chunk_views = std::min<int64_t>(nfilt, std::max<int64_t>(kFilterChunk, (int64_t)(kFilterChunkBytes / per_view)));
    if (P.hil_mode == KATS_HILBERT_MFMA) {
        const int64_t round = (int64_t)kHilTileRows * kHilBlocks;
        const int64_t rounds = P.chunk_views * P.n_psi / round;
        if (rounds >= 1) P.chunk_views = std::min<int64_t>(P.chunk_views, rounds * round / P.n_psi);
    }
    const uint64_t cv = nfilt > 0 ? (uint64_t)P.chunk_views + 2 : 0;     // + the adjoint's halo
    P.g4_bytes = align256(cv * P.n_psi * g.det_cols * 4);
    P.vmax_off = align256(cv * rc * 4);                 // then the rebinning's maxima
    P.g2_bytes = P.vmax_off + align256(rebin_max_count((long long)cv, P.n_psi, g.det_cols) * 4);
    P.gF_bytes = align256((uint64_t)nfilt * P.gf_rows * P.gf_cols * 4);
    P.gbar_bytes = align256((uint64_t)nfilt * rc * (P.det_adjoint ? 8 : 4));
    P.conv_bytes = P.det_adjoint ? align256(cv * rc * 4) : 0;
    P.det_bytes = P.det_adjoint ? align256(fixed_scratch_bytes()) : 0;
}

int build_plan(const katsevich_geometry &g_in, const katsevich_grid &gr,
               const katsevich_options &opts, PlanHost &P, std::string &err) {
    auto bad = [&](const std::string &m) { err = m; return KATS_EINVAL_GEOMETRY; };
    const int st0 = plan_setup(g_in, gr, opts, P, err);
    if (st0 != KATS_OK) return st0;
    const katsevich_geometry &g = P.geom;
    const int cols = g.det_cols, rows = g.det_rows;
    const Kappa K{g.D * P.h / g.R};

    P.fr_row.resize((size_t)P.n_psi * cols);
    P.fr_w.resize((size_t)P.n_psi * cols);
    for (int k = 0; k < P.n_psi; ++k)
        for (int c = 0; c < cols; ++c) {
            const double s = K.wk(P.alpha[c], P.psi[k]) / g.dw + 0.5 * (rows - 1) - g.row_offset;
            const double f = std::floor(s);
            P.fr_row[(size_t)k * cols + c] = (int32_t)f;
            P.fr_w[(size_t)k * cols + c] = s - f;
        }

    // psi_hat: root of w = w_kappa(alpha, psi) on the branch through psi = 0 where
    // w_kappa increases; the branch ends at a turning point (d w_kappa/d psi = 0) or at
    // +-psi_max.  d w_kappa/d psi decreases in |psi| on the side where sin(alpha) psi > 0.
    P.psi_hat.resize((size_t)rows * cols);
    P.br_k.resize((size_t)rows * cols);
    P.br_w.resize((size_t)rows * cols);
    for (int c = 0; c < cols; ++c) {
        const double a = P.alpha[c];
        double lo = -P.psi_max, hi = P.psi_max;
        if (a > 0 && K.dwk(a, P.psi_max) < 0)
            hi = bisect_increasing([&](double p) { return -K.dwk(a, p); }, 1e-3, P.psi_max);
        if (a < 0 && K.dwk(a, -P.psi_max) < 0)
            lo = bisect_increasing([&](double p) { return K.dwk(a, p); }, -P.psi_max, -1e-3);
        const double wlo = K.wk(a, lo), whi = K.wk(a, hi);
        for (int r = 0; r < rows; ++r) {
            const double wr = P.w[r];
            double ph;
            if (wr <= wlo) ph = lo;
            else if (wr >= whi) ph = hi;
            else ph = bisect_increasing([&](double p) { return K.wk(a, p) - wr; }, lo, hi);
            double q = ph / P.dpsi + 0.5 * (P.n_psi - 1);
            q = std::min(std::max(q, 0.0), (double)(P.n_psi - 1));
            const double k0 = std::min(std::floor(q), (double)(P.n_psi - 2));
            const size_t e = (size_t)r * cols + c;
            P.psi_hat[e] = ph;
            P.br_k[e] = (int32_t)k0;
            P.br_w[e] = q - k0;
        }
    }

    // ------------------------------------------------------------------ PI limits
    const size_t plane = (size_t)gr.ny * gr.nx;
    const size_t nvox = (size_t)P.n_tab * plane;
    try {
        P.pi_li.resize(nvox);
        P.pi_lo.resize(nvox);
        P.pi_nf.resize(nvox);
        P.pi_nl.resize(nvox);
        P.fov.resize(nvox);
    } catch (...) {
        err = "out of host memory for PI tables";
        return KATS_ENOMEM;
    }
    {
        const PiSolver S{g.R, P.h, g.lambda0, g.z0};
        // per voxel column (x, y), slices in increasing z so each root brackets the next
        const double step = 2.0 * gr.dz / P.h;
        parallel_for(gr.ny, threads_for(opts), [&](int iy) {
            const double y = gr.y_first + iy * gr.dy;
            for (int ix = 0; ix < gr.nx; ++ix) {
                const double x = gr.x_first + ix * gr.dx;
                double prev = 0.0, prev2 = 0.0;
                for (int j = 0; j < P.n_tab; ++j) {
                    const double z = gr.z_first + j * gr.dz;
                    const size_t e = (size_t)j * plane + (size_t)iy * gr.nx + ix;
                    double li, lo;
                    const double guess = 2.0 * prev - prev2;     // linear extrapolation in z
                    S.solve(x, y, z, li, lo, j > 0 ? &prev : nullptr, step, j > 1 ? &guess : nullptr);
                    prev2 = prev;
                    prev = li;
                    P.pi_li[e] = li;
                    P.pi_lo[e] = lo;
                }
            }
        });
    }
    // view units, first / last covered views, field of view
    const double r2 = P.r_fov * P.r_fov;
    parallel_for(P.n_tab * gr.ny, threads_for(opts), [&](int jy) {
        const int iy = jy % gr.ny;
        const double y = gr.y_first + iy * gr.dy;
        for (int ix = 0; ix < gr.nx; ++ix) {
            const double x = gr.x_first + ix * gr.dx;
            const size_t e = (size_t)jy * gr.nx + ix;
            const double vi = (P.pi_li[e] - g.lambda_first) / P.dlam;
            const double vo = (P.pi_lo[e] - g.lambda_first) / P.dlam;
            P.pi_li[e] = vi;
            P.pi_lo[e] = vo;
            P.pi_nf[e] = (int32_t)(std::floor(vi - 0.5) + 1.0);
            P.pi_nl[e] = (int32_t)(std::ceil(vo + 0.5) - 1.0);
            P.fov[e] = (x * x + y * y <= r2) ? 1 : 0;
        }
    });

    int64_t nmin = std::numeric_limits<int64_t>::max(), nmax = std::numeric_limits<int64_t>::min();
    for (size_t e = 0; e < nvox; ++e)
        if (P.fov[e]) {
            nmin = std::min<int64_t>(nmin, P.pi_nf[e]);
            nmax = std::max<int64_t>(nmax, P.pi_nl[e]);
        }
    if (nmin > nmax) return bad("no voxel of the grid lies inside the field of view");
    P.n_lo = (int32_t)(nmin - 1);
    P.n_hi = (int32_t)(nmax + 1);
    P.W = P.n_hi - P.n_lo + 1;

    // valid voxels, (voxel, view) pairs, filtered view range
    P.n_vv = 0;
    P.n_valid = 0;
    int64_t vmin = std::numeric_limits<int64_t>::max(), vmax = std::numeric_limits<int64_t>::min();
    {
        struct Part {
            int64_t n_vv = 0, n_valid = 0;
            int64_t vmin = std::numeric_limits<int64_t>::max();
            int64_t vmax = std::numeric_limits<int64_t>::min();
        };
        std::vector<Part> part((size_t)gr.nz);          // one per slice, summed in order
        parallel_for(gr.nz, threads_for(opts), [&](int iz) {
            const int k = iz / P.ns, j = iz % P.ns;
            const int64_t shift = (int64_t)k * g.views_per_turn;
            Part &pt = part[(size_t)iz];
            for (size_t q = 0; q < plane; ++q) {
                const size_t e = (size_t)j * plane + q;
                if (!P.fov[e]) continue;
                const int64_t nf = P.pi_nf[e] + shift, nl = P.pi_nl[e] + shift;
                if (nf - 1 < 0 || nl + 1 > g.n_views - 1) continue;
                pt.n_valid += 1;
                pt.n_vv += nl - nf + 1;
                pt.vmin = std::min(pt.vmin, nf);
                pt.vmax = std::max(pt.vmax, nl);
            }
        });
        for (const Part &pt : part) {
            P.n_valid += pt.n_valid;
            P.n_vv += pt.n_vv;
            vmin = std::min(vmin, pt.vmin);
            vmax = std::max(vmax, pt.vmax);
        }
    }
    if (P.n_valid == 0) {
        P.first_view = 1;
        P.last_view = 0;   // empty
    } else {
        P.first_view = vmin;
        P.last_view = vmax;
    }

    // ------------------------------------------------------------------ Hilbert spectrum
    // taps K[m] = 2 dalpha / (pi sin(m dalpha)) for odd m, 0 for even m; real and odd, so the
    // length-N DFT of the wrapped taps is i * Im with Im[f] = -2 sum_{m odd} K[m] sin(2 pi f m/N).
    const int N = P.fft_len;
    P.hil_im.assign(N, 0.0);
    for (int f = 0; f < N; ++f) {
        double acc = 0.0;
        for (int m = 1; m < cols; m += 2) {
            const double Km = 2.0 * g.dalpha / (kPi * std::sin(m * g.dalpha));
            const long long ph = ((long long)f * m) % N;
            acc += Km * std::sin(kTwoPi * (double)ph / N);
        }
        P.hil_im[f] = -2.0 * acc / N;
    }

    // ------------------------------------------------------------------ device image
    make_layout(P, P.W);
    const TableLayout &L = P.layout;
    try {
        P.image.assign(L.total, 0);
    } catch (...) {
        err = "out of host memory for the device table image";
        return KATS_ENOMEM;
    }
    unsigned char *img = P.image.data();
    {
        float *v = reinterpret_cast<float *>(img + L.view);
        for (int m = 0; m < P.W; ++m) {
            const double lam = g.lambda_first + (double)(P.n_lo + m) * P.dlam;
            const double b = lam + g.lambda0;
            v[4 * m + 0] = (float)std::cos(b);
            v[4 * m + 1] = (float)std::sin(b);
            v[4 * m + 2] = (float)(gr.z_first - g.z0 - P.h * lam);
            v[4 * m + 3] = 0.0f;
        }
    }
    {
        FrEntry *d = reinterpret_cast<FrEntry *>(img + L.fr);
        for (size_t i = 0; i < P.fr_w.size(); ++i) d[i] = FrEntry{P.fr_row[i], (float)P.fr_w[i]};
    }
    std::memcpy(img + L.br_k, P.br_k.data(), P.br_k.size() * 4);
    {
        float *d = reinterpret_cast<float *>(img + L.br_w);
        for (size_t i = 0; i < P.br_w.size(); ++i) d[i] = (float)P.br_w[i];
        float *lw = reinterpret_cast<float *>(img + L.lw);
        for (int r = 0; r < rows; ++r) lw[r] = (float)(g.D / std::sqrt(g.D * g.D + P.w[r] * P.w[r]));
        float *ca = reinterpret_cast<float *>(img + L.cos_alpha);
        for (int c = 0; c < cols; ++c) ca[c] = (float)std::cos(P.alpha[c]);
        float *tw = reinterpret_cast<float *>(img + L.twiddle);
        for (int k = 0; k < N; ++k) {
            tw[2 * k + 0] = (float)std::cos(kTwoPi * k / N);
            tw[2 * k + 1] = (float)(-std::sin(kTwoPi * k / N));
        }
        float *hi = reinterpret_cast<float *>(img + L.hil_im);
        for (int f = 0; f < N; ++f) hi[f] = (float)P.hil_im[f];
        // odd taps u[d] = K[2d + 1] reversed, q = Q0 - d with Q0 = 128 hil_f + 7, times 2^14
        // (the matrix-core Hilbert's operand; zero where |2d + 1| > cols - 1)
        float *hu = reinterpret_cast<float *>(img + L.hil_u);
        const int nq = 256 * P.hil_f + 32, q0 = 128 * P.hil_f + 7;
        for (int q = 0; q < nq; ++q) {
            const int m = 2 * (q0 - q) + 1;
            hu[q] = std::abs(m) <= cols - 1
                        ? (float)(kHilTapScale * 2.0 * g.dalpha / (kPi * std::sin(m * g.dalpha)))
                        : 0.0f;
        }
    }
    {
        PiEntry *pe = reinterpret_cast<PiEntry *>(img + L.pi);
        constexpr int32_t kEmptyLo = 1 << 29;
        const int chunks = 64;
        parallel_for(chunks, threads_for(opts), [&](int ch) {
        const size_t e0 = nvox * ch / chunks, e1 = nvox * (ch + 1) / chunks;
        for (size_t e = e0; e < e1; ++e) {
            if (P.fov[e]) {
                pe[e].li = (float)(P.pi_li[e] - P.n_lo);
                pe[e].lo = (float)(P.pi_lo[e] - P.n_lo);
                pe[e].nf = P.pi_nf[e] - P.n_lo;
                pe[e].nl = P.pi_nl[e] - P.n_lo;
            } else {
                pe[e].li = 0.f;
                pe[e].lo = 0.f;
                pe[e].nf = kEmptyLo;
                pe[e].nl = -kEmptyLo;
            }
        }
        });
    }

    // ------------------------------------------------------------------ footprint boxes
    // Columns: alpha* over a rectangle seen from an outside point is extremal at a corner
    // (its level sets are rays from the source).  Rows: w* = D dz / rho with rho between the
    // distance from the source to the rectangle and to its farthest corner, dz between
    // the run's first and last slice.  One extra cell each side absorbs float32 rounding
    // in the kernel; the box is clipped to the zero-padded detector.
    {
        BpBox *bx = reinterpret_cast<BpBox *>(img + L.boxes);
        TileRay *tr = reinterpret_cast<TileRay *>(img + L.tref);
        const double col_c = 0.5 * (cols - 1) - g.col_offset;
        const double row_c = 0.5 * (rows - 1) - g.row_offset;
        const int tiles = P.bp_tiles_y * P.bp_tiles_x;
        parallel_for(tiles, threads_for(opts), [&](int t) {
            const int tx = t % P.bp_tiles_x;
            const int ty = t / P.bp_tiles_x;
            const double x0 = gr.x_first + (double)tx * kBpTile * gr.dx;
            const double x1 = gr.x_first + (double)(tx * kBpTile + kBpTile - 1) * gr.dx;
            const double y0 = gr.y_first + (double)ty * kBpTile * gr.dy;
            const double y1 = gr.y_first + (double)(ty * kBpTile + kBpTile - 1) * gr.dy;
            const double cx[4] = {x0, x1, x0, x1}, cy[4] = {y0, y0, y1, y1};
            const double xc = gr.x_first + (tx * kBpTile + 0.5 * (kBpTile - 1)) * gr.dx;
            const double yc = gr.y_first + (ty * kBpTile + 0.5 * (kBpTile - 1)) * gr.dy;
            auto clip = [](double lo, double hi, int n) {
                // cells [lo, hi] clipped to [-kPad, n-1+kPad], at least two cells
                double a = std::floor(lo) - 1.0, c = std::floor(hi) + 2.0;
                a = std::max(a, (double)-kPad);
                c = std::min(c, (double)(n - 1 + kPad));
                int ia = (int)std::min(a, 1e6), ic = (int)std::max(c, -1e6);
                if (ic - ia < 1) {
                    if (ia >= n) { ia = n + kPad - 2; ic = n + kPad - 1; }
                    else { ia = -kPad; ic = -kPad + 1; }
                }
                return std::make_pair(ia, ic - ia + 1);
            };
            for (int m = 0; m < P.W; ++m) {
                const double lam = g.lambda_first + (double)(P.n_lo + m) * P.dlam;
                const double b = lam + g.lambda0;
                const double cb = std::cos(b), sb = std::sin(b);
                const double Sx = g.R * cb, Sy = g.R * sb;
                double amin = 1e300, amax = -1e300, rmax = 0.0;
                for (int k = 0; k < 4; ++k) {
                    const double u = -cx[k] * sb + cy[k] * cb;
                    const double v = g.R - cx[k] * cb - cy[k] * sb;
                    const double a = std::atan2(u, v);
                    amin = std::min(amin, a);
                    amax = std::max(amax, a);
                    rmax = std::max(rmax, std::hypot(cx[k] - Sx, cy[k] - Sy));
                }
                const double ddx = std::max({x0 - Sx, 0.0, Sx - x1});
                const double ddy = std::max({y0 - Sy, 0.0, Sy - y1});
                const double rmin = std::max(std::hypot(ddx, ddy), 1e-9);
                auto cc = clip(amin / g.dalpha + col_c, amax / g.dalpha + col_c, cols);
                // start the columns on a 16-byte boundary of the padded view row
                const int shift = (cc.first + kPad) & 3;
                cc.first -= shift;
                cc.second += shift;
                {
                    const double uc = -xc * sb + yc * cb, vc = g.R - xc * cb - yc * sb;
                    const double col = std::atan2(uc, vc) / g.dalpha + col_c - cc.first;
                    tr[(size_t)t * P.W + m] = TileRay{(float)col, (float)uc, (float)vc,
                                                      (float)(uc * uc + vc * vc)};
                }
                const double e = gr.z_first - g.z0 - P.h * lam;
                for (int run = 0; run < P.bp_runs; ++run) {
                    const double dz0 = e + (double)(run * P.bp_kz) * gr.dz;
                    const double dz1 = e + (double)(run * P.bp_kz + P.bp_kz - 1) * gr.dz;
                    const double wlo = g.D * dz0 / (dz0 >= 0 ? rmax : rmin);
                    const double whi = g.D * dz1 / (dz1 >= 0 ? rmin : rmax);
                    const auto rr = clip(wlo / g.dw + row_c, whi / g.dw + row_c, rows);
                    BpBox &o = bx[((size_t)run * tiles + t) * P.W + m];
                    o.r0 = (int16_t)rr.first;
                    o.nr = (int16_t)rr.second;
                    o.c0 = (int16_t)cc.first;
                    o.nc = (int16_t)cc.second;
                }
            }
        });
    }

    {
        // Largest box a workgroup can stage: a workgroup only walks the views of its hull,
        // the union of the PI windows (pitch-relative [nf, nl]) of the voxels of its tile and
        // slice run that lie in the field of view; the kernels' own hull is a subset (it
        // also drops voxels whose window leaves the scan), so tiles and views outside these
        // hulls never touch their boxes.
        const BpBox *bx = reinterpret_cast<const BpBox *>(img + L.boxes);
        const PiEntry *pe = reinterpret_cast<const PiEntry *>(img + L.pi);
        const int tiles = P.bp_tiles_y * P.bp_tiles_x;
        std::vector<int> tmr((size_t)P.bp_runs * tiles, 0), tmc((size_t)P.bp_runs * tiles, 0);
        parallel_for(P.bp_runs * tiles, threads_for(opts), [&](int rt) {
            const int run = rt / tiles, t = rt % tiles;
            const int tx = t % P.bp_tiles_x, ty = t / P.bp_tiles_x;
            int hlo = INT32_MAX, hhi = INT32_MIN;
            const int j1 = std::min(P.n_tab, (run + 1) * P.bp_kz);
            for (int j = run * P.bp_kz; j < j1; ++j)
                for (int iy = ty * kBpTile; iy < std::min(gr.ny, (ty + 1) * kBpTile); ++iy)
                    for (int ix = tx * kBpTile; ix < std::min(gr.nx, (tx + 1) * kBpTile); ++ix) {
                        const PiEntry &q = pe[((size_t)j * gr.ny + iy) * gr.nx + ix];
                        if (q.nf <= q.nl) {
                            hlo = std::min(hlo, q.nf);
                            hhi = std::max(hhi, q.nl);
                        }
                    }
            int mr = 0, mc = 0;
            for (int m = std::max(hlo, 0); m <= std::min(hhi, P.W - 1); ++m) {
                const BpBox &b = bx[(size_t)rt * P.W + m];
                mr = std::max(mr, (int)b.nr);
                mc = std::max(mc, (int)b.nc);
            }
            tmr[(size_t)rt] = mr;
            tmc[(size_t)rt] = mc;
        });
        P.bp_box_rows = *std::max_element(tmr.begin(), tmr.end());
        P.bp_box_cols = *std::max_element(tmc.begin(), tmc.end());
    }

    // ------------------------------------------------------------------ workspace sizes
    set_workspace(P);
    return KATS_OK;
}

// ---------------------------------------------------------------------------------
// Device builder (kernels in plan_gpu.hip)
// ---------------------------------------------------------------------------------

// Byte offsets inside the device builder's scratch buffer.
struct ScratchLayout {
    uint64_t li, lo, nf, nl, fov, stats, fr_row, fr_w, psi_hat, br_k, br_w, total;
};

static ScratchLayout scratch_layout(const PlanHost &P) {
    const uint64_t nvox = (uint64_t)P.n_tab * P.grid.ny * P.grid.nx;
    const uint64_t rc = (uint64_t)P.geom.det_rows * P.geom.det_cols;
    const uint64_t pc = (uint64_t)P.n_psi * P.geom.det_cols;
    ScratchLayout S{};
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { const uint64_t o = off; off = align256(off + bytes); return o; };
    S.li = take(nvox * 8);
    S.lo = take(nvox * 8);
    S.nf = take(nvox * 4);
    S.nl = take(nvox * 4);
    S.fov = take(nvox);
    S.stats = take(sizeof(DevPlanStats));
    S.fr_row = take(pc * 4);
    S.fr_w = take(pc * 8);
    S.psi_hat = take(rc * 8);
    S.br_k = take(rc * 4);
    S.br_w = take(rc * 8);
    S.total = off;
    return S;
}

// Upper bound of the pitch window W over the voxels in the field of view (r <= r_fov):
// on the PI line of a point at height z, lambda_i = z_r - g (1 + tau) and lambda_o =
// z_r + g (1 - tau) with z_r = (z - z0)/h, half-span g <= pi/2 + asin(r_fov/R) and
// |tau| <= r_fov/R, so the covered views of the table slices lie within
// [z_r(first) - G, z_r(last) + G], G = (pi/2 + asin(s))(1 + s), s = r_fov/R, plus the
// rounding of the first / last covered view and the two margin views.
static int window_cap(const PlanHost &P) {
    const katsevich_geometry &g = P.geom;
    const katsevich_grid &gr = P.grid;
    const double zr0 = (gr.z_first - g.z0) / P.h;
    const double zr1 = (gr.z_first + (P.n_tab - 1) * gr.dz - g.z0) / P.h;
    const double s = std::min(P.r_fov / g.R, 1.0);
    const double G = (0.5 * kPi + std::asin(s)) * (1.0 + s);
    const double span = (zr1 - zr0) + 2.0 * G;
    return (int)std::ceil(span / P.dlam) + 8;
}

int device_plan_sizes(const katsevich_geometry &g, const katsevich_grid &gr,
                      const katsevich_options &opts, uint64_t &scratch_bytes,
                      uint64_t &table_bytes, std::string &err) {
    PlanHost P;
    const int st = plan_setup(g, gr, opts, P, err);
    if (st != KATS_OK) return st;
    make_layout(P, window_cap(P));
    scratch_bytes = scratch_layout(P).total;
    table_bytes = P.layout.total;
    return KATS_OK;
}

int device_plan_scratch_offsets(const katsevich_geometry &g, const katsevich_grid &gr,
                                const katsevich_options &opts, uint64_t off[5], int &n_tab,
                                std::string &err) {
    PlanHost P;
    const int st = plan_setup(g, gr, opts, P, err);
    if (st != KATS_OK) return st;
    const ScratchLayout S = scratch_layout(P);
    off[0] = S.li;
    off[1] = S.lo;
    off[2] = S.nf;
    off[3] = S.nl;
    off[4] = S.fov;
    n_tab = P.n_tab;
    return KATS_OK;
}

int build_plan_device(const katsevich_geometry &g_in, const katsevich_grid &gr,
                      const katsevich_options &opts, PlanHost &P, std::string &err,
                      const DevicePlanBuffers &buf) {
    const int st0 = plan_setup(g_in, gr, opts, P, err);
    if (st0 != KATS_OK) return st0;
    const katsevich_geometry &g = P.geom;
    const int W_cap = window_cap(P);
    make_layout(P, W_cap);
    const ScratchLayout S = scratch_layout(P);
    if (!buf.scratch || buf.scratch_bytes < S.total) {
        err = "scratch smaller than katsevich_plan_device_sizes says";
        return KATS_EWORKSPACE;
    }
    if (!buf.tables || buf.table_bytes < P.layout.total) {
        err = "table buffer smaller than katsevich_plan_device_sizes says";
        return KATS_ESHAPE;
    }
    DevPlanArgs a{};
    a.R = g.R;
    a.D = g.D;
    a.h = P.h;
    a.lambda0 = g.lambda0;
    a.z0 = g.z0;
    a.lambda_first = g.lambda_first;
    a.dlam = P.dlam;
    a.dalpha = g.dalpha;
    a.col_offset = g.col_offset;
    a.dw = g.dw;
    a.row_offset = g.row_offset;
    a.kscale = g.D * P.h / g.R;
    a.psi_max = P.psi_max;
    a.dpsi = P.dpsi;
    a.r_fov = P.r_fov;
    a.x_first = gr.x_first;
    a.dx = gr.dx;
    a.y_first = gr.y_first;
    a.dy = gr.dy;
    a.z_first = gr.z_first;
    a.dz = gr.dz;
    a.n_views = g.n_views;
    a.cols = g.det_cols;
    a.rows = g.det_rows;
    a.n_psi = P.n_psi;
    a.fft_len = P.fft_len;
    a.hil_f = P.hil_f;
    a.nx = gr.nx;
    a.ny = gr.ny;
    a.nz = gr.nz;
    a.n_tab = P.n_tab;
    a.ns = P.ns;
    a.Nv = g.views_per_turn;
    a.tiles_x = P.bp_tiles_x;
    a.tiles_y = P.bp_tiles_y;
    a.runs = P.bp_runs;
    a.kz = P.bp_kz;
    a.W_cap = W_cap;
    unsigned char *sc = static_cast<unsigned char *>(buf.scratch);
    unsigned char *tb = static_cast<unsigned char *>(buf.tables);
    const TableLayout &L = P.layout;
    DevPlanPtrs p{};
    p.li = reinterpret_cast<double *>(sc + S.li);
    p.lo = reinterpret_cast<double *>(sc + S.lo);
    p.nf = reinterpret_cast<int *>(sc + S.nf);
    p.nl = reinterpret_cast<int *>(sc + S.nl);
    p.fov = sc + S.fov;
    p.stats = reinterpret_cast<DevPlanStats *>(sc + S.stats);
    p.fr_row = reinterpret_cast<int *>(sc + S.fr_row);
    p.fr_w = reinterpret_cast<double *>(sc + S.fr_w);
    p.psi_hat = reinterpret_cast<double *>(sc + S.psi_hat);
    p.br_k = reinterpret_cast<int *>(sc + S.br_k);
    p.br_w = reinterpret_cast<double *>(sc + S.br_w);
    p.view = reinterpret_cast<float4 *>(tb + L.view);
    p.fr = reinterpret_cast<FrEntry *>(tb + L.fr);
    p.t_br_k = reinterpret_cast<int *>(tb + L.br_k);
    p.t_br_w = reinterpret_cast<float *>(tb + L.br_w);
    p.lw = reinterpret_cast<float *>(tb + L.lw);
    p.cos_alpha = reinterpret_cast<float *>(tb + L.cos_alpha);
    p.twiddle = reinterpret_cast<float2 *>(tb + L.twiddle);
    p.hil_im = reinterpret_cast<float *>(tb + L.hil_im);
    p.hil_u = reinterpret_cast<float *>(tb + L.hil_u);
    p.pi = reinterpret_cast<PiEntry *>(tb + L.pi);
    p.boxes = reinterpret_cast<BpBox *>(tb + L.boxes);
    p.tref = reinterpret_cast<TileRay *>(tb + L.tref);

    const size_t pc = (size_t)P.n_psi * g.det_cols, rc = (size_t)g.det_rows * g.det_cols;
    P.fr_row.resize(pc);
    P.fr_w.resize(pc);
    P.psi_hat.resize(rc);
    P.br_k.resize(rc);
    P.br_w.resize(rc);
    DevPlanStats stats{};
    hipStream_t s = static_cast<hipStream_t>(buf.stream);
    hipError_t e = launch_plan_device(a, p, s);
    // the counts and the float64 rebinning tables (kept on the host for export) come back
    if (e == hipSuccess) e = hipMemcpyAsync(&stats, p.stats, sizeof(stats), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.fr_row.data(), p.fr_row, pc * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.fr_w.data(), p.fr_w, pc * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.psi_hat.data(), p.psi_hat, rc * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.br_k.data(), p.br_k, rc * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.br_w.data(), p.br_w, rc * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        err = std::string("device plan: ") + hipGetErrorString(e);
        return KATS_EHIP;
    }
    if (stats.nmin > stats.nmax) {
        err = "no voxel of the grid lies inside the field of view";
        return KATS_EINVAL_GEOMETRY;
    }
    P.n_lo = stats.nmin - 1;
    P.n_hi = stats.nmax + 1;
    P.W = P.n_hi - P.n_lo + 1;
    if (P.W > W_cap) {   // excluded by window_cap's bound; refuse rather than overrun the tables
        err = "pitch window " + std::to_string(P.W) + " exceeds its bound " + std::to_string(W_cap);
        return KATS_EINVAL_GEOMETRY;
    }
    P.n_vv = (int64_t)stats.n_vv;
    P.n_valid = (int64_t)stats.n_valid;
    if (P.n_valid == 0) {
        P.first_view = 1;
        P.last_view = 0;   // empty
    } else {
        P.first_view = stats.vmin;
        P.last_view = stats.vmax;
    }
    P.bp_box_rows = stats.box_rows;
    P.bp_box_cols = stats.box_cols;
    set_workspace(P);
    P.d_tables = buf.tables;
    P.device_built = true;
    P.W_cap = W_cap;
    return KATS_OK;
}

}  // namespace kats
