// The plan of the pitch-by-pitch reconstruction built on the GPU in float64 (Sec. II
// pre-calculating step): the kappa-line forward-rebinning table (eqs. FR, w_k), psi_hat and
// the backward-rebinning table (eq. BR), the Hilbert kernel spectrum (eqs. HF, e4), the PI
// limits of every voxel of one pitch (pre-calculating step 2), the pitch window (eq.
// maxvalue), the per-view trigonometry, the backprojector's footprint boxes and the plan's
// counts, each kernel writing its table straight into the caller's table buffer.  The
// arithmetic is the host builder's, term for term; only the PI lines are solved another
// way (below), so every table agrees with the host plan's to the last bits of the libm
// functions and the integer tables bit for bit.
//
// PI lines.  For x = (rho cos phi, rho sin phi, z) let the PI chord run from in-plane angle
// mu - g to mu + g (mu = its midpoint direction, 2 g its angular span, 0 < g < pi) and let
// theta = phi - mu.  In the plane x lies on the chord where rho cos(theta) = R cos(g), at
// the signed fraction tau = rho sin(theta) / (R sin g) of its half-length from the middle;
// the chord's height there is z0 + h (mu - lambda0 + g tau).  With c = (z - z0)/h + lambda0
// - phi the PI line of x is the root of the one-variable equation
//     F(theta) = g(theta) tau(theta) - theta - c = 0,  g(theta) = acos(rho cos(theta) / R),
// whose derivative F'(theta) = (1 - tau^2)(g cot g - 1) is negative inside the helix
// cylinder (rho < R gives |tau| < 1 and g cot g < 1 on (0, pi)), so the root is unique,
// and it lies in (-c - pi, -c + pi) because |g tau| < pi.  It is found by Newton's method
// from the root on the axis (theta = -c) with the iterate projected onto [-pi, pi] at every
// step (a whole turn moved into c, which leaves the equation unchanged), inside a shrinking
// bracket that takes a bisection step whenever Newton leaves it.  Then
//     lambda_i = (z - z0)/h - g (1 + tau),   lambda_o = (z - z0)/h + g (1 - tau).
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

// float64 plan arithmetic as written (no fused multiply-adds), like the host builder's
#pragma clang fp contract(off)

namespace kats {

namespace {

constexpr double kPiD = 3.14159265358979323846;
constexpr double kTwoPiD = 2.0 * kPiD;
constexpr int kTB = 256;
constexpr int32_t kEmptyLo = 1 << 29;     // PiEntry of a voxel outside the field of view

__device__ inline double alpha_c(const DevPlanArgs &a, int c) {
    return (c - 0.5 * (a.cols - 1) + a.col_offset) * a.dalpha;
}
__device__ inline double w_r(const DevPlanArgs &a, int r) {
    return (r - 0.5 * (a.rows - 1) + a.row_offset) * a.dw;
}
// w_kappa(alpha, psi) of eq. w_k (R_o = R, P = the feed per turn) and its psi-derivative
__device__ inline double wk(const DevPlanArgs &a, double al, double p) {
    const double pc = (p == 0.0) ? 1.0 : p / tan(p);
    return a.kscale * (p * cos(al) + pc * sin(al));
}
__device__ inline double dwk(const DevPlanArgs &a, double al, double p) {
    const double s = sin(p);
    return a.kscale * (cos(al) + sin(al) * (cos(p) / s - p / (s * s)));
}

// bisection of an increasing function on [lo, hi] to the end of float64 resolution
template <class F>
__device__ double bisect_increasing(F f, double lo, double hi) {
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

__device__ inline int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline long long wave_min_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, (long long)__shfl_xor(v, o, 64));
    return v;
}
__device__ inline long long wave_max_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (long long)__shfl_xor(v, o, 64));
    return v;
}
__device__ inline unsigned long long wave_sum_ull(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor(v, o, 64);
    return v;
}

// the pitch window W = n_hi - n_lo + 1 = nmax - nmin + 3 (0 while no voxel is in the FOV)
__device__ inline int window(const DevPlanStats *st) {
    const int nmin = st->nmin, nmax = st->nmax;
    return nmin <= nmax ? nmax - nmin + 3 : 0;
}

__global__ __launch_bounds__(kTB) void k_plan_init(DevPlanStats *st) {
    if (threadIdx.x == 0) {
        st->nmin = INT_MAX;
        st->nmax = INT_MIN;
        st->box_rows = 0;
        st->box_cols = 0;
        st->vmin = LLONG_MAX;
        st->vmax = LLONG_MIN;
        st->n_vv = 0;
        st->n_valid = 0;
    }
}

// forward rebinning (eqs. FR, w_k): row coordinate of w_kappa(alpha_c, psi_k), floor + fraction
__global__ __launch_bounds__(kTB) void k_plan_fr(DevPlanArgs a, DevPlanPtrs p) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= a.n_psi * a.cols) return;
    const int k = i / a.cols, c = i - k * a.cols;
    const double psi = (k - 0.5 * (a.n_psi - 1)) * a.dpsi;
    const double s = wk(a, alpha_c(a, c), psi) / a.dw + 0.5 * (a.rows - 1) - a.row_offset;
    const double f = floor(s);
    p.fr_row[i] = (int)f;
    p.fr_w[i] = s - f;
    p.fr[i] = FrEntry{(int)f, (float)(s - f)};
}

// psi_hat (eq. BR): the root of w_r = w_kappa(alpha_c, psi) on the branch through psi = 0
// where w_kappa increases (ending at a turning point d w_kappa / d psi = 0 or at +-psi_max),
// clamped to that branch; kappa index and weight of the linear interpolation in psi
__global__ __launch_bounds__(kTB) void k_plan_br(DevPlanArgs a, DevPlanPtrs p) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= a.rows * a.cols) return;
    const int r = i / a.cols, c = i - r * a.cols;
    const double al = alpha_c(a, c);
    double lo = -a.psi_max, hi = a.psi_max;
    if (al > 0 && dwk(a, al, a.psi_max) < 0)
        hi = bisect_increasing([&](double q) { return -dwk(a, al, q); }, 1e-3, a.psi_max);
    if (al < 0 && dwk(a, al, -a.psi_max) < 0)
        lo = bisect_increasing([&](double q) { return dwk(a, al, q); }, -a.psi_max, -1e-3);
    const double wlo = wk(a, al, lo), whi = wk(a, al, hi);
    const double wr = w_r(a, r);
    double ph;
    if (wr <= wlo) ph = lo;
    else if (wr >= whi) ph = hi;
    else ph = bisect_increasing([&](double q) { return wk(a, al, q) - wr; }, lo, hi);
    double q = ph / a.dpsi + 0.5 * (a.n_psi - 1);
    q = fmin(fmax(q, 0.0), (double)(a.n_psi - 1));
    const double k0 = fmin(floor(q), (double)(a.n_psi - 2));
    p.psi_hat[i] = ph;
    p.br_k[i] = (int)k0;
    p.br_w[i] = q - k0;
    p.t_br_k[i] = (int)k0;
    p.t_br_w[i] = (float)(q - k0);
}

// length-correction weights (eq. LW), post-cosine weights (eq. PW), FFT twiddles
__global__ __launch_bounds__(kTB) void k_plan_small(DevPlanArgs a, DevPlanPtrs p) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i < a.rows) {
        const double w = w_r(a, i);
        p.lw[i] = (float)(a.D / sqrt(a.D * a.D + w * w));
    }
    if (i < a.cols) p.cos_alpha[i] = (float)cos(alpha_c(a, i));
    if (i < a.fft_len) {
        const int N = a.fft_len;
        p.twiddle[i] = make_float2((float)cos(kTwoPiD * i / N), (float)(-sin(kTwoPiD * i / N)));
    }
}

// Hilbert kernel spectrum (eqs. HF, e4): taps K[m] = 2 dalpha / (pi sin(m dalpha)) for odd m,
// 0 for even m, real and odd, so the length-N DFT of the wrapped taps is i Im with
// Im[f] = -2 sum_{m odd} K[m] sin(2 pi f m / N); stored divided by N
__global__ __launch_bounds__(kTB) void k_plan_hilbert(DevPlanArgs a, DevPlanPtrs p) {
    const int f = blockIdx.x * kTB + threadIdx.x;
    const int N = a.fft_len;
    // the matrix-core path's operand: odd taps u[d] = K[2d + 1] reversed (q = Q0 - d,
    // Q0 = 128 hil_f + 7) times 2^14, zero where |2d + 1| > cols - 1
    if (f < 256 * a.hil_f + 32) {
        const int m = 2 * (128 * a.hil_f + 7 - f) + 1;
        p.hil_u[f] = abs(m) <= a.cols - 1
                         ? (float)(kHilTapScale * 2.0 * a.dalpha / (kPiD * sin(m * a.dalpha)))
                         : 0.0f;
    }
    if (f >= N) return;
    double acc = 0.0;
    for (int m = 1; m < a.cols; m += 2) {
        const double Km = 2.0 * a.dalpha / (kPiD * sin(m * a.dalpha));
        const long long ph = ((long long)f * m) % N;
        acc += Km * sin(kTwoPiD * (double)ph / N);
    }
    p.hil_im[f] = (float)(-2.0 * acc / N);
}

// PI line of one point (see the head of this file): g and tau at the root of F
__device__ void pi_line(double R, double rho, double phi, double zr_l0, double &g, double &tau) {
    double c = zr_l0 - phi;
    c -= kTwoPiD * rint(c / kTwoPiD);             // a whole number of turns moved into phi
    double lo = -c - kPiD, hi = -c + kPiD;         // F(lo) > 0 > F(hi)
    double th = -c;                                // the root on the axis
    auto project = [&]() {                         // keep the iterate in [-pi, pi]
        if (th > kPiD) {
            th -= kTwoPiD; c += kTwoPiD; lo -= kTwoPiD; hi -= kTwoPiD;
        } else if (th < -kPiD) {
            th += kTwoPiD; c -= kTwoPiD; lo += kTwoPiD; hi += kTwoPiD;
        }
    };
    project();
    for (int it = 0; it < 120; ++it) {
        double st, ct;
        sincos(th, &st, &ct);
        const double q = rho * ct / R;
        const double gg = acos(q);
        const double sg = sqrt((1.0 - q) * (1.0 + q));
        const double t = rho * st / (R * sg);
        const double F = gg * t - th - c;
        if (F == 0.0) break;
        if (F > 0.0) lo = th;
        else hi = th;
        const double dF = (1.0 - t * t) * (gg * q / sg - 1.0);
        const double step = F / dF;
        double tn = th - step;
        // after a Newton step of 1e-10 the error is ~1e-20: the new iterate is final
        const bool done = fabs(step) <= 1e-10 * fmax(1.0, fabs(th)) && tn >= lo && tn <= hi;
        if (!done && !(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        th = tn;
        project();
        if (done || !(hi - lo > 4e-16 * fmax(1.0, fabs(th)))) break;
    }
    double st, ct;
    sincos(th, &st, &ct);
    const double q = rho * ct / R;
    g = acos(q);
    tau = rho * st / (R * sqrt((1.0 - q) * (1.0 + q)));
}

// PI limits of every voxel of the table pitch in view units, first / last covered view,
// field of view; the FOV's first / last covered views reduced into the counts
__global__ __launch_bounds__(kTB) void k_plan_pi(DevPlanArgs a, DevPlanPtrs p) {
    const long long nvox = (long long)a.n_tab * a.ny * a.nx;
    const long long e = (long long)blockIdx.x * kTB + threadIdx.x;
    int nfv = INT_MAX, nlv = INT_MIN;
    if (e < nvox) {
        const int ix = (int)(e % a.nx);
        const long long t = e / a.nx;
        const int iy = (int)(t % a.ny), j = (int)(t / a.ny);
        const double x = a.x_first + ix * a.dx, y = a.y_first + iy * a.dy;
        const double z = a.z_first + j * a.dz;
        const double rho = hypot(x, y), phi = atan2(y, x);
        const double zr = (z - a.z0) / a.h;
        double g, tau;
        pi_line(a.R, rho, phi, zr + a.lambda0, g, tau);
        const double li = zr - g * (1.0 + tau), lo = zr + g * (1.0 - tau);
        const double vi = (li - a.lambda_first) / a.dlam;
        const double vo = (lo - a.lambda_first) / a.dlam;
        const int nf = (int)(floor(vi - 0.5) + 1.0);
        const int nl = (int)(ceil(vo + 0.5) - 1.0);
        const bool in = x * x + y * y <= a.r_fov * a.r_fov;
        p.li[e] = vi;
        p.lo[e] = vo;
        p.nf[e] = nf;
        p.nl[e] = nl;
        p.fov[e] = in ? 1 : 0;
        if (in) {
            nfv = nf;
            nlv = nl;
        }
    }
    nfv = wave_min_i(nfv);
    nlv = wave_max_i(nlv);
    if ((threadIdx.x & 63) == 0 && nfv <= nlv) {
        atomicMin(&p.stats->nmin, nfv);
        atomicMax(&p.stats->nmax, nlv);
    }
}

// PI table of the backprojector: limits and covered views relative to the window start
// n_lo = nmin - 1
__global__ __launch_bounds__(kTB) void k_plan_pack(DevPlanArgs a, DevPlanPtrs p) {
    const long long nvox = (long long)a.n_tab * a.ny * a.nx;
    const long long e = (long long)blockIdx.x * kTB + threadIdx.x;
    if (e >= nvox) return;
    const int n_lo = p.stats->nmin - 1;
    PiEntry q;
    if (p.fov[e]) {
        q.li = (float)(p.li[e] - n_lo);
        q.lo = (float)(p.lo[e] - n_lo);
        q.nf = p.nf[e] - n_lo;
        q.nl = p.nl[e] - n_lo;
    } else {
        q.li = 0.f;
        q.lo = 0.f;
        q.nf = kEmptyLo;
        q.nl = -kEmptyLo;
    }
    p.pi[e] = q;
}

// valid voxels of the whole grid (every pitch), their (voxel, view) pairs and the views they use
__global__ __launch_bounds__(kTB) void k_plan_count(DevPlanArgs a, DevPlanPtrs p) {
    const long long plane = (long long)a.ny * a.nx;
    const long long total = (long long)a.nz * plane;
    unsigned long long vv = 0, nvalid = 0;
    long long vmin = LLONG_MAX, vmax = LLONG_MIN;
    for (long long i = (long long)blockIdx.x * kTB + threadIdx.x; i < total;
         i += (long long)gridDim.x * kTB) {
        const int iz = (int)(i / plane);
        const long long qv = i - (long long)iz * plane;
        const int k = iz / a.ns, j = iz - k * a.ns;
        const long long e = (long long)j * plane + qv;
        if (!p.fov[e]) continue;
        const long long shift = (long long)k * a.Nv;
        const long long nf = p.nf[e] + shift, nl = p.nl[e] + shift;
        if (nf - 1 < 0 || nl + 1 > a.n_views - 1) continue;
        nvalid += 1;
        vv += (unsigned long long)(nl - nf + 1);
        vmin = min(vmin, nf);
        vmax = max(vmax, nl);
    }
    vv = wave_sum_ull(vv);
    nvalid = wave_sum_ull(nvalid);
    vmin = wave_min_ll(vmin);
    vmax = wave_max_ll(vmax);
    if ((threadIdx.x & 63) == 0 && nvalid > 0) {
        atomicAdd(&p.stats->n_vv, vv);
        atomicAdd(&p.stats->n_valid, nvalid);
        atomicMin(&p.stats->vmin, vmin);
        atomicMax(&p.stats->vmax, vmax);
    }
}

// per-view trigonometry of the pitch window: cos(beta), sin(beta), z_first - z0 - h lambda
__global__ __launch_bounds__(kTB) void k_plan_view(DevPlanArgs a, DevPlanPtrs p) {
    const int m = blockIdx.x * kTB + threadIdx.x;
    if (m >= a.W_cap || m >= window(p.stats)) return;
    const int n_lo = p.stats->nmin - 1;
    const double lam = a.lambda_first + (double)(n_lo + m) * a.dlam;
    const double b = lam + a.lambda0;
    p.view[m] = make_float4((float)cos(b), (float)sin(b), (float)(a.z_first - a.z0 - a.h * lam), 0.0f);
}

// cells [lo, hi] widened by one cell, clipped to [-kPad, n-1+kPad], at least two cells
__device__ inline int2 clip_cells(double lo, double hi, int n) {
    double a = floor(lo) - 1.0, c = floor(hi) + 2.0;
    a = fmax(a, (double)-kPad);
    c = fmin(c, (double)(n - 1 + kPad));
    int ia = (int)fmin(a, 1e6), ic = (int)fmax(c, -1e6);
    if (ic - ia < 1) {
        if (ia >= n) { ia = n + kPad - 2; ic = n + kPad - 1; }
        else { ia = -kPad; ic = -kPad + 1; }
    }
    return make_int2(ia, ic - ia + 1);
}

// Footprint box of one backprojection tile at one window view, for every slice run, and
// the ray to the tile's centre (TileRay).
// Columns: alpha* over a rectangle seen from an outside point is extremal at a corner (its
// level sets are rays from the source).  Rows: w* = D dz / rho with rho between the
// distance from the source to the rectangle and to its farthest corner, dz between the
// run's first and last slice.  One extra cell each side absorbs float32 rounding in the
// kernel; the box is clipped to the zero-padded detector.
__global__ __launch_bounds__(kTB) void k_plan_boxes(DevPlanArgs a, DevPlanPtrs p) {
    const long long i = (long long)blockIdx.x * kTB + threadIdx.x;
    const int tiles = a.tiles_x * a.tiles_y;
    if (i >= (long long)tiles * a.W_cap) return;
    const int W = window(p.stats);
    if (W > a.W_cap) return;                        // bound exceeded: the host refuses the plan
    const int t = (int)(i / a.W_cap), m = (int)(i - (long long)t * a.W_cap);
    if (m >= W) return;
    const int n_lo = p.stats->nmin - 1;
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const double x0 = a.x_first + (double)tx * kBpTile * a.dx;
    const double x1 = a.x_first + (double)(tx * kBpTile + kBpTile - 1) * a.dx;
    const double y0 = a.y_first + (double)ty * kBpTile * a.dy;
    const double y1 = a.y_first + (double)(ty * kBpTile + kBpTile - 1) * a.dy;
    const double cx[4] = {x0, x1, x0, x1}, cy[4] = {y0, y0, y1, y1};
    const double xc = a.x_first + (tx * kBpTile + 0.5 * (kBpTile - 1)) * a.dx;
    const double yc = a.y_first + (ty * kBpTile + 0.5 * (kBpTile - 1)) * a.dy;
    const double col_c = 0.5 * (a.cols - 1) - a.col_offset;
    const double row_c = 0.5 * (a.rows - 1) - a.row_offset;
    const double lam = a.lambda_first + (double)(n_lo + m) * a.dlam;
    const double b = lam + a.lambda0;
    const double cb = cos(b), sb = sin(b);
    const double Sx = a.R * cb, Sy = a.R * sb;
    double amin = 1e300, amax = -1e300, rmax = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double u = -cx[k] * sb + cy[k] * cb;
        const double v = a.R - cx[k] * cb - cy[k] * sb;
        const double al = atan2(u, v);
        amin = fmin(amin, al);
        amax = fmax(amax, al);
        rmax = fmax(rmax, hypot(cx[k] - Sx, cy[k] - Sy));
    }
    const double ddx = fmax(fmax(x0 - Sx, 0.0), Sx - x1);
    const double ddy = fmax(fmax(y0 - Sy, 0.0), Sy - y1);
    const double rmin = fmax(hypot(ddx, ddy), 1e-9);
    int2 cc = clip_cells(amin / a.dalpha + col_c, amax / a.dalpha + col_c, a.cols);
    const int shift = (cc.x + kPad) & 3;            // columns from a 16-byte boundary of the row
    cc.x -= shift;
    cc.y += shift;
    {
        // the tile centre's ray, for the adjoint's column coordinate
        const double uc = -xc * sb + yc * cb, vc = a.R - xc * cb - yc * sb;
        const double col = atan2(uc, vc) / a.dalpha + col_c - cc.x;
        p.tref[(size_t)t * W + m] = TileRay{(float)col, (float)uc, (float)vc, (float)(uc * uc + vc * vc)};
    }
    const double e = a.z_first - a.z0 - a.h * lam;
    for (int run = 0; run < a.runs; ++run) {
        const double dz0 = e + (double)(run * a.kz) * a.dz;
        const double dz1 = e + (double)(run * a.kz + a.kz - 1) * a.dz;
        const double wlo = a.D * dz0 / (dz0 >= 0 ? rmax : rmin);
        const double whi = a.D * dz1 / (dz1 >= 0 ? rmin : rmax);
        const int2 rr = clip_cells(wlo / a.dw + row_c, whi / a.dw + row_c, a.rows);
        BpBox o;
        o.r0 = (int16_t)rr.x;
        o.nr = (int16_t)rr.y;
        o.c0 = (int16_t)cc.x;
        o.nc = (int16_t)cc.y;
        p.boxes[((size_t)run * tiles + t) * W + m] = o;
    }
}

// Largest box a workgroup stages: over the views of each tile x run's hull (the union of
// the covered views of its voxels in the field of view).  One workgroup per (run, tile).
__global__ __launch_bounds__(kTB) void k_plan_box_stats(DevPlanArgs a, DevPlanPtrs p) {
    __shared__ int sh[2][kTB / 64];
    const int tiles = a.tiles_x * a.tiles_y;
    const int rt = blockIdx.x;
    const int run = rt / tiles, t = rt - run * tiles;
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int W = min(window(p.stats), a.W_cap);
    const int ix = tx * kBpTile + (threadIdx.x & (kBpTile - 1));
    const int iy = ty * kBpTile + (threadIdx.x / kBpTile);
    int hlo = INT_MAX, hhi = INT_MIN;
    if (ix < a.nx && iy < a.ny) {
        const int j1 = min(a.n_tab, (run + 1) * a.kz);
        for (int j = run * a.kz; j < j1; ++j) {
            const PiEntry q = p.pi[((size_t)j * a.ny + iy) * a.nx + ix];
            if (q.nf <= q.nl) {
                hlo = min(hlo, q.nf);
                hhi = max(hhi, q.nl);
            }
        }
    }
    hlo = wave_min_i(hlo);
    hhi = wave_max_i(hhi);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][wave] = hlo;
        sh[1][wave] = hhi;
    }
    __syncthreads();
    hlo = min(min(sh[0][0], sh[0][1]), min(sh[0][2], sh[0][3]));
    hhi = max(max(sh[1][0], sh[1][1]), max(sh[1][2], sh[1][3]));
    int mr = 0, mc = 0;
    if (hlo <= hhi) {
        const BpBox *bx = p.boxes + (size_t)rt * W;
        for (int m = max(hlo, 0) + threadIdx.x; m <= min(hhi, W - 1); m += kTB) {
            const BpBox b = bx[m];
            mr = max(mr, (int)b.nr);
            mc = max(mc, (int)b.nc);
        }
    }
    mr = wave_max_i(mr);
    mc = wave_max_i(mc);
    if ((threadIdx.x & 63) == 0 && (mr > 0 || mc > 0)) {
        atomicMax(&p.stats->box_rows, mr);
        atomicMax(&p.stats->box_cols, mc);
    }
}

unsigned blocks_for(long long n) { return (unsigned)((n + kTB - 1) / kTB); }

}  // namespace

hipError_t launch_plan_device(const DevPlanArgs &a, const DevPlanPtrs &p, hipStream_t s) {
    const long long nvox = (long long)a.n_tab * a.ny * a.nx;
    const long long tiles = (long long)a.tiles_x * a.tiles_y;
    const long long total = (long long)a.nz * a.ny * a.nx;
    const int small = a.rows > a.cols ? a.rows : a.cols;
    hipLaunchKernelGGL(k_plan_init, dim3(1), dim3(kTB), 0, s, p.stats);
    hipLaunchKernelGGL(k_plan_fr, dim3(blocks_for((long long)a.n_psi * a.cols)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_br, dim3(blocks_for((long long)a.rows * a.cols)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_small, dim3(blocks_for(small > a.fft_len ? small : a.fft_len)), dim3(kTB), 0, s, a, p);
    const int nq = 256 * a.hil_f + 32;
    hipLaunchKernelGGL(k_plan_hilbert, dim3(blocks_for(a.fft_len > nq ? a.fft_len : nq)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_pi, dim3(blocks_for(nvox)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_pack, dim3(blocks_for(nvox)), dim3(kTB), 0, s, a, p);
    const long long cb = blocks_for(total);
    hipLaunchKernelGGL(k_plan_count, dim3((unsigned)(cb < 8192 ? cb : 8192)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_view, dim3(blocks_for(a.W_cap)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_boxes, dim3(blocks_for(tiles * a.W_cap)), dim3(kTB), 0, s, a, p);
    hipLaunchKernelGGL(k_plan_box_stats, dim3((unsigned)(tiles * a.runs)), dim3(kTB), 0, s, a, p);
    return hipGetLastError();
}

}  // namespace kats
