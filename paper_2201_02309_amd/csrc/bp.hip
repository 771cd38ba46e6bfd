// Backprojection over the PI interval (Sec. II backprojection step) for gfx950.
//
// f(x) = dlambda/(2 pi) sum_n c_n(x) / v*_n(x) g^F(lambda_n, alpha*_n(x), w*_n(x)),
// v* = R - x cos(b) - y sin(b), alpha* = atan(u / v*), u = -x sin(b) + y cos(b),
// w* = D cos(alpha*) / v* (z - z0 - P lambda / 2 pi) = D (z - z0 - P lambda / 2 pi) / sqrt(u^2+v*^2),
// with b = lambda + lambda0 and c_n the overlap of view cell [n-1/2, n+1/2] with the PI
// interval [l_i, l_o] (view units).
//
// Every pitch k reuses the first pitch's tables (Sec. II periodicity): slice j of pitch k
// sees view n = n_lo + k Nv + m exactly as slice j of pitch 0 sees view n_lo + m, so the
// per-view table (cos b, sin b, e_m = z_first - z0 - h lambda_{n_lo+m}) and the PI table
// (l_i, l_o, n_first, n_last relative to n_lo) are indexed by the pitch-relative view m
// and slice j only.  The geometry is therefore bit-identical for every pitch.
//
// Thread layout: one wave (64 lanes) = an 8 x 8 (x, y) tile; each lane owns a run of
// KZ consecutive slices of one pitch and keeps their accumulators in registers.  The
// wave walks the hull of its lanes' PI windows (a wave-uniform loop, view table read
// through scalar loads); alpha*, 1/v* and 1/rho are computed once per (lane, view) and
// shared by the KZ slices, whose detector rows advance by dz D / rho per slice.  Each
// voxel is written exactly once, no atomics.
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace kats {

namespace {

constexpr int kTile = 8;          // 8 x 8 lanes per wave
constexpr int kKZ = 8;            // slices per lane

__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// detector sample with zero outside [0, rows) x [0, cols)
__device__ inline float tap(const float *__restrict__ img, int r, int c, int rows, int cols) {
    return ((unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols) ? img[r * cols + c] : 0.0f;
}

template <int KZ>
__global__ __launch_bounds__(64) void k_backproject(KParams p, const float *__restrict__ gF,
                                                    float *__restrict__ vol, int runs_per_pitch) {
    const int lane = threadIdx.x;
    const int ix = blockIdx.x * kTile + (lane & (kTile - 1));
    const int iy = blockIdx.y * kTile + (lane >> 3);
    const int pitch = blockIdx.z / runs_per_pitch;
    const int j0 = (blockIdx.z % runs_per_pitch) * KZ;
    const int slices = min(p.ns, p.nz - pitch * p.ns);
    const int nrun = min(KZ, slices - j0);
    if (nrun <= 0) return;                                   // whole wave: uniform
    const bool inxy = ix < p.nx && iy < p.ny;
    const long long base = (long long)p.n_lo + (long long)pitch * p.Nv;   // view of m = 0

    float A[KZ], B[KZ], acc[KZ];
    unsigned valid = 0;
    int mlo = INT_MAX, mhi = INT_MIN;
#pragma unroll
    for (int jj = 0; jj < KZ; ++jj) {
        A[jj] = 3.0e38f;
        B[jj] = -3.0e38f;
        acc[jj] = 0.0f;
        if (inxy && jj < nrun) {
            const PiEntry e = p.pi[((size_t)(j0 + jj) * p.ny + iy) * p.nx + ix];
            const long long nf = base + e.nf, nl = base + e.nl;
            if (e.nf <= e.nl && nf - 1 >= 0 && nl + 1 <= p.n_views - 1) {
                A[jj] = e.li - 0.5f;           // c_n = clamp(min(m - A, B - m), 0, 1)
                B[jj] = e.lo + 0.5f;
                valid |= 1u << jj;
                mlo = min(mlo, e.nf);
                mhi = max(mhi, e.nl);
            }
        }
    }
    mlo = __builtin_amdgcn_readfirstlane(wave_min(mlo));
    mhi = __builtin_amdgcn_readfirstlane(wave_max(mhi));

    const float x = fmaf((float)ix, p.dx, p.x_first);
    const float y = fmaf((float)iy, p.dy, p.y_first);
    const float zoff = (float)j0 * p.dz;
    const size_t rc = (size_t)p.rows * p.cols;
    for (int m = mlo; m <= mhi; ++m) {
        const float4 vt = p.view[m];
        const float u = fmaf(-x, vt.y, y * vt.x);
        const float v = p.R - fmaf(x, vt.x, y * vt.y);
        const float vinv = 1.0f / v;
        const float rinv = rsqrtf(fmaf(u, u, v * v));
        const float cc = fmaf(atan2f(u, v), p.inv_dalpha, p.col_c);
        const float ccl = fminf(fmaxf(cc, -2.0f), (float)p.cols);
        const float c0f = floorf(ccl);
        const float tc = ccl - c0f;
        const int c0 = (int)c0f;
        const float q = p.D * rinv * p.inv_dw;               // rows per mm of z
        const float ez = vt.z + zoff;                        // z - z0 - h lambda at slice j0
        const float *img = gF + (size_t)(base + m - p.first_view) * rc;
        const float mf = (float)m;
#pragma unroll
        for (int jj = 0; jj < KZ; ++jj) {
            const float rr = fmaf(q, fmaf((float)jj, p.dz, ez), p.row_c);
            const float rrl = fminf(fmaxf(rr, -2.0f), (float)p.rows);
            const float r0f = floorf(rrl);
            const float tr = rrl - r0f;
            const int r0 = (int)r0f;
            const float v00 = tap(img, r0, c0, p.rows, p.cols);
            const float v01 = tap(img, r0, c0 + 1, p.rows, p.cols);
            const float v10 = tap(img, r0 + 1, c0, p.rows, p.cols);
            const float v11 = tap(img, r0 + 1, c0 + 1, p.rows, p.cols);
            const float top = fmaf(tc, v01 - v00, v00);
            const float bot = fmaf(tc, v11 - v10, v10);
            const float val = fmaf(tr, bot - top, top);
            const float cw = fminf(fmaxf(fminf(mf - A[jj], B[jj] - mf), 0.0f), 1.0f);
            acc[jj] = fmaf(cw * vinv, val, acc[jj]);
        }
    }
    if (!inxy) return;
    const int iz0 = pitch * p.ns + j0;
#pragma unroll
    for (int jj = 0; jj < KZ; ++jj) {
        if (jj < nrun)
            vol[((size_t)(iz0 + jj) * p.ny + iy) * p.nx + ix] =
                ((valid >> jj) & 1u) ? acc[jj] * p.scale : 0.0f;
    }
}

// Transpose: gFbar[n] += dlambda/(2 pi) c_n / v*_n * fbar(x) spread over the four bilinear
// taps (global float atomics; the adjoint's only non-deterministic summation order).
template <int KZ>
__global__ __launch_bounds__(64) void k_backproject_T(KParams p, const float *__restrict__ gvol,
                                                      float *__restrict__ gFbar, int runs_per_pitch) {
    const int lane = threadIdx.x;
    const int ix = blockIdx.x * kTile + (lane & (kTile - 1));
    const int iy = blockIdx.y * kTile + (lane >> 3);
    const int pitch = blockIdx.z / runs_per_pitch;
    const int j0 = (blockIdx.z % runs_per_pitch) * KZ;
    const int slices = min(p.ns, p.nz - pitch * p.ns);
    const int nrun = min(KZ, slices - j0);
    if (nrun <= 0) return;
    const bool inxy = ix < p.nx && iy < p.ny;
    const long long base = (long long)p.n_lo + (long long)pitch * p.Nv;
    float A[KZ], B[KZ], g[KZ];
    int mlo = INT_MAX, mhi = INT_MIN;
    const int iz0 = pitch * p.ns + j0;
#pragma unroll
    for (int jj = 0; jj < KZ; ++jj) {
        A[jj] = 3.0e38f;
        B[jj] = -3.0e38f;
        g[jj] = 0.0f;
        if (inxy && jj < nrun) {
            const PiEntry e = p.pi[((size_t)(j0 + jj) * p.ny + iy) * p.nx + ix];
            const long long nf = base + e.nf, nl = base + e.nl;
            if (e.nf <= e.nl && nf - 1 >= 0 && nl + 1 <= p.n_views - 1) {
                A[jj] = e.li - 0.5f;
                B[jj] = e.lo + 0.5f;
                g[jj] = gvol[((size_t)(iz0 + jj) * p.ny + iy) * p.nx + ix] * p.scale;
                mlo = min(mlo, e.nf);
                mhi = max(mhi, e.nl);
            }
        }
    }
    mlo = __builtin_amdgcn_readfirstlane(wave_min(mlo));
    mhi = __builtin_amdgcn_readfirstlane(wave_max(mhi));
    const float x = fmaf((float)ix, p.dx, p.x_first);
    const float y = fmaf((float)iy, p.dy, p.y_first);
    const float zoff = (float)j0 * p.dz;
    const size_t rc = (size_t)p.rows * p.cols;
    for (int m = mlo; m <= mhi; ++m) {
        const float4 vt = p.view[m];
        const float u = fmaf(-x, vt.y, y * vt.x);
        const float v = p.R - fmaf(x, vt.x, y * vt.y);
        const float vinv = 1.0f / v;
        const float rinv = rsqrtf(fmaf(u, u, v * v));
        const float cc = fmaf(atan2f(u, v), p.inv_dalpha, p.col_c);
        const float ccl = fminf(fmaxf(cc, -2.0f), (float)p.cols);
        const float c0f = floorf(ccl);
        const float tc = ccl - c0f;
        const int c0 = (int)c0f;
        const float q = p.D * rinv * p.inv_dw;
        const float ez = vt.z + zoff;
        float *img = gFbar + (size_t)(base + m - p.first_view) * rc;
        const float mf = (float)m;
#pragma unroll
        for (int jj = 0; jj < KZ; ++jj) {
            const float cw = fminf(fmaxf(fminf(mf - A[jj], B[jj] - mf), 0.0f), 1.0f);
            const float amp = cw * vinv * g[jj];
            if (amp == 0.0f) continue;
            const float rr = fmaf(q, fmaf((float)jj, p.dz, ez), p.row_c);
            const float rrl = fminf(fmaxf(rr, -2.0f), (float)p.rows);
            const float r0f = floorf(rrl);
            const float tr = rrl - r0f;
            const int r0 = (int)r0f;
            const float w00 = (1.0f - tr) * (1.0f - tc), w01 = (1.0f - tr) * tc;
            const float w10 = tr * (1.0f - tc), w11 = tr * tc;
            if ((unsigned)r0 < (unsigned)p.rows) {
                if ((unsigned)c0 < (unsigned)p.cols) atomicAdd(img + r0 * p.cols + c0, amp * w00);
                if ((unsigned)(c0 + 1) < (unsigned)p.cols) atomicAdd(img + r0 * p.cols + c0 + 1, amp * w01);
            }
            if ((unsigned)(r0 + 1) < (unsigned)p.rows) {
                if ((unsigned)c0 < (unsigned)p.cols) atomicAdd(img + (r0 + 1) * p.cols + c0, amp * w10);
                if ((unsigned)(c0 + 1) < (unsigned)p.cols)
                    atomicAdd(img + (r0 + 1) * p.cols + c0 + 1, amp * w11);
            }
        }
    }
}

}  // namespace

hipError_t launch_backproject(const KParams &k, const float *gF, float *vol, hipStream_t s) {
    const int ns_eff = k.ns < k.nz ? k.ns : k.nz;
    const int runs = (ns_eff + kKZ - 1) / kKZ;
    dim3 grid((k.nx + kTile - 1) / kTile, (k.ny + kTile - 1) / kTile, (unsigned)(k.n_pitches * runs));
    hipLaunchKernelGGL(k_backproject<kKZ>, grid, dim3(64), 0, s, k, gF, vol, runs);
    return hipGetLastError();
}

hipError_t launch_backproject_T(const KParams &k, const float *gvol, float *gFbar, hipStream_t s) {
    const int ns_eff = k.ns < k.nz ? k.ns : k.nz;
    const int runs = (ns_eff + kKZ - 1) / kKZ;
    dim3 grid((k.nx + kTile - 1) / kTile, (k.ny + kTile - 1) / kTile, (unsigned)(k.n_pitches * runs));
    hipLaunchKernelGGL(k_backproject_T<kKZ>, grid, dim3(64), 0, s, k, gvol, gFbar, runs);
    return hipGetLastError();
}

}  // namespace kats
