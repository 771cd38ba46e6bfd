// PI lines of every voxel of one pitch on the GPU, in float64 (pre-calculating step 2 of
// Sec. II): the plan's dominant cost, solved per voxel column on the device with the same
// formulation and iteration as the host plan builder.
//
// The PI line of x is the chord of the helix through x whose end points a(lambda_i),
// a(lambda_o) are less than one turn apart.  With the lower end parametrised by s and
// d = phi - (s + lambda0) the in-plane angle from the source to x, the chord's in-plane
// half-span theta = atan2(R - rho cos d, rho sin d) gives lambda_o = s + 2 theta and the
// fraction t of the chord at which x sits; x lies on it when z0 + h (s + t 2 theta) = z.
// That height gap rises monotonically with s on ((z - z0)/h - 2 pi, (z - z0)/h).
// Each thread takes one (x, y) column and walks the slices of the pitch in increasing z:
// Newton from the linear extrapolation of the two previous roots, an Illinois bracket
// search from the previous root when Newton does not settle.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kats {

namespace {

constexpr double kTwoPiD = 6.283185307179586476925286766559;

struct PiArgs {
    double R, h, lambda0, z0;
    double x_first, dx, y_first, dy, z_first, dz;
    int nx, ny, n_tab;
};

__device__ inline double gap(const PiArgs &a, double s, double rho, double phi, double z,
                             double &span) {
    const double d = phi - (s + a.lambda0);
    double sd, cd;
    sincos(d, &sd, &cd);
    const double A = a.R - rho * cd, B = rho * sd;
    span = 2.0 * atan2(A, B);
    const double t = 0.5 + rho * (sd * B - cd * A) / (2.0 * a.R * A);
    return a.z0 + a.h * (s + t * span) - z;
}

// height gap and its s-derivative (see the host builder for the terms)
__device__ inline double gap_d(const PiArgs &a, double s, double rho, double phi, double z,
                               double &span, double &deriv) {
    const double d = phi - (s + a.lambda0);
    double sd, cd;
    sincos(d, &sd, &cd);
    const double A = a.R - rho * cd, B = rho * sd;
    const double th = atan2(A, B);
    span = 2.0 * th;
    const double N = sd * B - cd * A;
    const double t = 0.5 + rho * N / (2.0 * a.R * A);
    const double dth = rho * (A * cd - B * sd) / (A * A + B * B);
    const double dA = -rho * sd;
    const double dN = -(cd * B + sd * A);
    const double dt = rho / (2.0 * a.R) * (dN * A - N * dA) / (A * A);
    deriv = a.h * (1.0 + dt * span + t * 2.0 * dth);
    return a.z0 + a.h * (s + t * span) - z;
}

__device__ bool newton(const PiArgs &a, double guess, double rho, double phi, double z,
                       double &root) {
    const double zr = (z - a.z0) / a.h;
    double s = guess, span, der;
    for (int it = 0; it < 8; ++it) {
        const double f = gap_d(a, s, rho, phi, z, span, der);
        if (f == 0.0) { root = s; return true; }
        if (!(der > 0.0)) return false;
        const double sn = s - f / der;
        if (!(sn > zr - kTwoPiD && sn < zr)) return false;
        if (fabs(sn - s) <= 1e-9 * fmax(1.0, fabs(s))) { root = sn; return true; }
        s = sn;
    }
    return false;
}

__device__ double illinois(const PiArgs &a, double lo, double flo, double hi, double fhi,
                           double rho, double phi, double z) {
    double s = 0.5 * (lo + hi), span;
    int side = 0;
    for (int it = 0; it < 200; ++it) {
        s = hi - fhi * (hi - lo) / (fhi - flo);
        if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
        if (!(s > lo && s < hi)) break;
        const double fs = gap(a, s, rho, phi, z, span);
        if (fs == 0.0) return s;
        if (fs < 0) {
            lo = s; flo = fs;
            if (side == -1) fhi *= 0.5;
            side = -1;
        } else {
            hi = s; fhi = fs;
            if (side == +1) flo *= 0.5;
            side = +1;
        }
        if (hi - lo <= 4e-16 * fmax(1.0, fabs(s))) break;
    }
    return s;
}

__global__ __launch_bounds__(256) void k_pi_solve(PiArgs a, double *__restrict__ li_out,
                                                  double *__restrict__ lo_out) {
    const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
    if (col >= (long long)a.nx * a.ny) return;
    const int ix = (int)(col % a.nx), iy = (int)(col / a.nx);
    const double x = a.x_first + ix * a.dx, y = a.y_first + iy * a.dy;
    const double rho = hypot(x, y), phi = atan2(y, x);
    const double step = 2.0 * a.dz / a.h;
    const size_t plane = (size_t)a.nx * a.ny;
    double prev = 0.0, prev2 = 0.0;
    for (int j = 0; j < a.n_tab; ++j) {
        const double z = a.z_first + j * a.dz;
        const double zr = (z - a.z0) / a.h;
        double span, root = 0.0;
        bool done = false;
        if (j > 1) done = newton(a, 2.0 * prev - prev2, rho, phi, z, root);
        if (!done) {
            // bracket from the previous root (lambda_i rises with z), else the whole domain
            double lo = zr - kTwoPiD, hi = zr, flo = 0.0, fhi = 0.0;
            bool have = false;
            if (j > 0 && prev > lo && prev < hi) {
                flo = gap(a, prev, rho, phi, z, span);
                if (flo < 0) {
                    lo = prev;
                    for (double w = step; !have; w *= 4.0) {
                        const double b = fmin(lo + w, zr);
                        fhi = gap(a, b, rho, phi, z, span);
                        if (fhi > 0) { hi = b; have = true; }
                        else if (b >= zr) break;
                        else { lo = b; flo = fhi; }
                    }
                }
            }
            if (!have) {
                lo = zr - kTwoPiD;
                hi = zr;
                flo = gap(a, lo, rho, phi, z, span);
                fhi = gap(a, hi, rho, phi, z, span);
            }
            root = (flo < 0 && fhi > 0) ? illinois(a, lo, flo, hi, fhi, rho, phi, z) : 0.5 * (lo + hi);
        }
        gap(a, root, rho, phi, z, span);
        const size_t e = (size_t)j * plane + (size_t)col;
        li_out[e] = root;
        lo_out[e] = root + span;
        prev2 = prev;
        prev = root;
    }
}

}  // namespace

hipError_t launch_pi_solve(const katsevich_geometry &g, const katsevich_grid &gr, double h,
                           int n_tab, double *d_li, double *d_lo, hipStream_t s) {
    PiArgs a;
    a.R = g.R;
    a.h = h;
    a.lambda0 = g.lambda0;
    a.z0 = g.z0;
    a.x_first = gr.x_first;
    a.dx = gr.dx;
    a.y_first = gr.y_first;
    a.dy = gr.dy;
    a.z_first = gr.z_first;
    a.dz = gr.dz;
    a.nx = gr.nx;
    a.ny = gr.ny;
    a.n_tab = n_tab;
    const long long cols = (long long)gr.nx * gr.ny;
    hipLaunchKernelGGL(k_pi_solve, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, a, d_li, d_lo);
    return hipGetLastError();
}

}  // namespace kats
