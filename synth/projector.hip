// FP64 closed-form projector of additive ellipsoids for large synthetic scans (test and
// benchmark harness only; not part of the reconstruction library).  Same ray model as
// synth/phantom.py: ray from a(lambda_n) towards the curved-detector cell (alpha_c, w_r),
// line integral = density |d| 2 sqrt(max(B^2 - A C, 0)) / A in the ellipsoid's unit-sphere
// frame.  One thread per detector sample.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct ScanArgs {
    double R, D, h, lambda0, z0, lambda_first, dlam, dalpha, col_offset, dw, row_offset;
    int rows, cols;
};

// ellipsoid record: centre (3), M = Q diag(1/a) row-major (9), density (1), pad (3)
constexpr int kRec = 16;

__global__ __launch_bounds__(256) void k_project(ScanArgs s, const double *__restrict__ ell, int n_ell,
                                                 long long view0, long long n_views,
                                                 float *__restrict__ out) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long per_view = (long long)s.rows * s.cols;
    if (idx >= n_views * per_view) return;
    const long long v = idx / per_view;
    const int rc = (int)(idx % per_view);
    const int r = rc / s.cols, c = rc % s.cols;
    const double lam = s.lambda_first + (double)(view0 + v) * s.dlam;
    const double b = lam + s.lambda0;
    double sb, cb;
    sincos(b, &sb, &cb);
    const double alpha = (c - 0.5 * (s.cols - 1) + s.col_offset) * s.dalpha;
    const double w = (r - 0.5 * (s.rows - 1) + s.row_offset) * s.dw;
    double sa, ca;
    sincos(alpha, &sa, &ca);
    const double src[3] = {s.R * cb, s.R * sb, s.z0 + s.h * lam};
    // d = D sin(a) e_u + D cos(a) e_v + w e_z, e_u = (-sb, cb, 0), e_v = (-cb, -sb, 0)
    const double d[3] = {-s.D * sa * sb - s.D * ca * cb, s.D * sa * cb - s.D * ca * sb, w};
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double acc = 0.0;
    for (int e = 0; e < n_ell; ++e) {
        const double *q = ell + (size_t)e * kRec;
        const double p0 = src[0] - q[0], p1 = src[1] - q[1], p2 = src[2] - q[2];
        // (p @ M)_k = sum_i p_i M[i][k]
        double sp[3], dp[3];
        for (int k = 0; k < 3; ++k) {
            sp[k] = p0 * q[3 + k] + p1 * q[6 + k] + p2 * q[9 + k];
            dp[k] = d[0] * q[3 + k] + d[1] * q[6 + k] + d[2] * q[9 + k];
        }
        const double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
        const double B = sp[0] * dp[0] + sp[1] * dp[1] + sp[2] * dp[2];
        const double C = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
        const double disc = B * B - A * C;
        if (disc > 0.0) acc += q[12] * dn * 2.0 * sqrt(disc) / A;
    }
    out[idx] = (float)acc;
}

}  // namespace

extern "C" int synth_project_ellipsoids(const double *scan11, int rows, int cols,
                                        const double *d_ell, int n_ell, long long view0,
                                        long long n_views, float *d_out, void *stream) {
    ScanArgs s;
    s.R = scan11[0]; s.D = scan11[1]; s.h = scan11[2]; s.lambda0 = scan11[3]; s.z0 = scan11[4];
    s.lambda_first = scan11[5]; s.dlam = scan11[6]; s.dalpha = scan11[7]; s.col_offset = scan11[8];
    s.dw = scan11[9]; s.row_offset = scan11[10];
    s.rows = rows;
    s.cols = cols;
    const long long total = n_views * (long long)rows * cols;
    if (total <= 0) return 0;
    const long long blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       s, d_ell, n_ell, view0, n_views, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
