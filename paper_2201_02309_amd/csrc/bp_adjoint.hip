// Adjoint of the backprojection (the transpose of the operator in bp.hip), for the
// gradient of a reconstruction loss with respect to the filtered data.
#include <algorithm>
#include <cmath>

#include "bp_common.hpp"

namespace kats {

namespace {

using namespace bpdev;

// ---------------------------------------------------------------------------------
// Adjoint of the backprojection, tiled like the forward kernel: the workgroup's 16 x 16
// voxel columns x KZ slices, the same PI-window hull, group words and footprint boxes.  At
// each view every lane scatters its four bilinear weights times
// dlambda/(2 pi) c_n / v* fbar(x) into the view's box held in LDS (LDS float64 atomics); the
// box of the previous view is flushed meanwhile from the other buffer to g^F-bar with one
// global float atomic per non-zero detector cell (cells of the zero padding are dropped,
// as the forward reads zeros there), and left zeroed for its next use.
// ---------------------------------------------------------------------------------
// The adjoint's LDS boxes accumulate in float64: the hardware's LDS float64 atomic add is
// several times faster here than its float32 one, and exact enough that the flushed float32
// sums round once.  Group words are bytes while the groups fit in 4 bits, so that the
// double-buffered boxes still leave room for four workgroups per CU.
constexpr int kLPT = kLP;         // box columns
// LDS row pitch of the boxes (doubles): 64 would put a column's cells of every row in one
// bank pair, so lanes scattering to one column at different rows would conflict; 66 moves
// each row by four banks (65, 68, 70, 72 and 80 were slower).  The hull's word table is
// sized so that a 16-slice workgroup still takes exactly 40960 bytes, four per CU: views
// of hulls up to 1784 long (the largest hull of the 512^3 / 55296-view workload is 1649).
// Whole adjoint against 64-double rows: clinical 512^2 x 128 workload 44.3 ms against
// 56.8 ms, 16-row network window 2.82 against 3.30 ms, 184-column sparse detector 51.1
// against 51.7 ms.
constexpr int kRowT = 66;
constexpr int kHullT = 1784;

// DET: the deterministic mode's accumulators are 64-bit fixed point (integer adds are
// associative, so the result does not depend on the order of the atomics).
template <int KZ, bool DET>
struct BpTShared {
    static constexpr int NG = KZ / kKG;
    using Word = typename std::conditional<(NG <= 4), unsigned char, unsigned short>::type;
    using Acc = typename std::conditional<DET, unsigned long long, double>::type;
    static constexpr int kFull = NG <= 4 ? 4 : 8;
    __attribute__((aligned(16))) Acc box[2][kRowT * lds_rows<KZ>()];
    Word words[4][kHullT];
    int red[8];
};

// v * S rounded to the nearest integer, two's complement (|v| S < 2^62 by the choice of S)
__device__ inline unsigned long long to_fixed(float v, double S) {
    return (unsigned long long)__double2ll_rn((double)v * S);
}

// FB: some box of the plan may exceed the LDS tile; those views scatter their taps
// straight into g^F-bar with global atomics (the cells the forward's HBM path reads).
//
// Column coordinate.  The cotangent scattered here is arbitrary (random in the dot-product
// and oracle tests, a residual in training), so the bilinear weights themselves must be
// accurate, not only the interpolated value: a column coordinate formed in float32 at the
// detector's scale (|alpha*/dalpha| up to ~370 cells, ulp 3e-5) plus the float32 rounding
// of u, v from coordinates of ~180 mm moves the weights by ~3e-5, which is what a random
// cotangent sees.  Each lane therefore measures its angle from the ray to its tile's centre
// (TileRay, float64 from the plan): with small in-tile offsets (du, dv) of (u, v),
//     alpha* - alpha_c = atan2(du v_c - u_c dv, rho_c^2 + u_c du + v_c dv),
// an angle of a few cells whose float32 error is ~1e-6 cell, and atan of its small tangent
// is the odd series through t^11 (remainder below t^13/13: ~1e-17 at the tangents of
// voxels in the field of view).  Geometries whose tiles subtend wide angles from the source
// (helix radius not large against the tile; see series_serves) take atan2f of the same two
// terms instead.
//
// DET (deterministic mode): the boxes accumulate 64-bit integers, each contribution v
// entering as round(v S) (the split between the two columns taken in integers, so that
// it sums exactly), and g^F-bar is accumulated the same way in a 64-bit buffer (global
// integer atomics); S = *fscale, a power of two chosen from max |fbar| so that no sum can
// reach 2^62.  Integer sums do not depend on their order: the result is the same bits on
// every run.
template <int KZ, bool FB, bool DET>
__device__ void bpT_tile(const BpArgs p, const float *__restrict__ fvol, void *__restrict__ gFout,
                         const double *__restrict__ fscale, int rows, int cols, long long first_view,
                         const float4 *__restrict__ view_tab, const uint2 *__restrict__ box_tab,
                         const float4 *__restrict__ ray_tab, int series, int bxi, int byi, int bz,
                         BpTShared<KZ, DET> &S) {
    using Acc = typename BpTShared<KZ, DET>::Acc;
    typedef __attribute__((address_space(3))) Acc LdsAcc;
    float *gFbar = static_cast<float *>(gFout);
    unsigned long long *gFbar64 = static_cast<unsigned long long *>(gFout);
    const double fx = DET ? *fscale : 0.0;
    static_assert(KZ % kKG == 0 && KZ / kKG <= 8, "groups use 8-bit masks");
    constexpr int kLR = lds_rows<KZ>();
    constexpr int NG = KZ / kKG;
    auto &box = S.box;
    auto &words = S.words;
    auto &red = S.red;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ix = bxi * kT + (tid & (kT - 1));
    const int iy = byi * kT + (tid >> 4);
    const int pitch = bz / p.runs;
    const int run = bz % p.runs;
    const int j0 = run * KZ;
    const int slices = min(p.ns, p.nz - pitch * p.ns);
    const int nrun = min(KZ, slices - j0);
    if (nrun <= 0) return;                                   // uniform over the workgroup
    const bool inxy = ix < p.nx && iy < p.ny;
    const long long base = (long long)p.n_lo + (long long)pitch * p.Nv;   // view of m = 0
    const int iz0 = pitch * p.ns + j0;

    // register r of a lane holds slice (r + off) mod KZ: lanes of a wave that lie on one ray
    // then scatter slices of different z (different detector rows) in the same instruction
    const int off = ((tid & 15) + 4 * ((tid >> 4) & 3)) & (KZ - 1);
    float A[KZ], B[KZ], fb[KZ];
    int wlo = INT_MAX, whi = INT_MIN;
    int g_alo[NG], g_ahi[NG], g_flo[NG], g_fhi[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        int alo = INT_MAX, ahi = INT_MIN, flo = INT_MIN, fhi = INT_MAX;
#pragma unroll
        for (int s = 0; s < kKG; ++s) {
            const int r = g * kKG + s;                      // register
            const int jj = (r + off) & (KZ - 1);            // slice
            A[r] = 3.0e38f;
            B[r] = -3.0e38f;
            fb[r] = 0.0f;
            if (inxy && jj < nrun) {
                const PiEntry e = ldg(p.pi + ((size_t)(j0 + jj) * p.ny + iy) * p.nx + ix);
                const long long nf = base + e.nf, nl = base + e.nl;
                if (e.nf <= e.nl && nf - 1 >= 0 && nl + 1 <= p.n_views - 1) {
                    A[r] = e.li - 0.5f;
                    B[r] = e.lo + 0.5f;
                    fb[r] = ldg(fvol + ((size_t)(iz0 + jj) * p.ny + iy) * p.nx + ix) * p.scale;
                    alo = min(alo, e.nf);
                    ahi = max(ahi, e.nl);
                    flo = max(flo, (int)ceilf(A[r] + 1.0f) + 1);
                    fhi = min(fhi, (int)floorf(B[r] - 1.0f) - 1);
                }
            }
        }
        g_alo[g] = wave_min(alo);
        g_ahi[g] = wave_max(ahi);
        g_flo[g] = wave_max(flo);
        g_fhi[g] = wave_min(fhi);
        wlo = min(wlo, g_alo[g]);
        whi = max(whi, g_ahi[g]);
    }
    if (lane == 0) {
        red[wave] = wlo;
        red[4 + wave] = whi;
    }
    // both box buffers start zeroed (every flush leaves its cells zero again)
    for (int i = tid; i < 2 * kRowT * kLR; i += kNT) (&box[0][0])[i] = 0;
    __syncthreads();
    const int mlo = __builtin_amdgcn_readfirstlane(min(min(red[0], red[1]), min(red[2], red[3])));
    const int mhi = __builtin_amdgcn_readfirstlane(max(max(red[4], red[5]), max(red[6], red[7])));
    using Word = typename BpTShared<KZ, DET>::Word;
    constexpr int kFull = BpTShared<KZ, DET>::kFull;
    // (an empty hull, mlo = INT_MAX > mhi = INT_MIN, takes no words: mhi - mlo would overflow)
    const bool use_words = mlo <= mhi && mhi - mlo < kHullT;
    if (use_words) {
        for (int w = lane; w <= mhi - mlo; w += 64) {
            const int m = mlo + w;
            unsigned word = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (m >= g_alo[g] && m <= g_ahi[g]) word |= 1u << g;
                if (m >= g_flo[g] && m <= g_fhi[g]) word |= 1u << (kFull + g);
            }
            words[wave][w] = (Word)word;
        }
    }
    __syncthreads();

    // offsets from the tile centre (half-integers of the grid steps)
    const float ddx = ((float)(tid & (kT - 1)) - 0.5f * (kT - 1)) * p.dx;
    const float ddy = ((float)(tid >> 4) - 0.5f * (kT - 1)) * p.dy;
    const float zoff = (float)j0 * p.dz;
    const uint2 *__restrict__ boxes =
        box_tab + ((size_t)(run * p.tiles_y + byi) * p.tiles_x + bxi) * p.W;
    const float4 *__restrict__ rays = ray_tab + ((size_t)byi * p.tiles_x + bxi) * p.W;
    const size_t vstride = (size_t)rows * cols;
    auto fits = [](const BpBox &b) { return !FB || (b.nr <= kLR && b.nc <= kLPT); };
    // flush of view m's box from buffer buf: lanes over 4 rows x 64 columns per pass
    auto flush = [&](int m, const BpBox &b, int buf) {
        LdsAcc *bx = (LdsAcc *)box[buf];
        const size_t vo = (size_t)(base + m - first_view) * vstride;
        const int cc = tid & 63;
        for (int rr = tid >> 6; rr < b.nr; rr += 4) {
            LdsAcc *cell = bx + __mul24(rr, kRowT) + cc;
            const Acc v = *cell;
            if (v != 0) {
                *cell = 0;
                const int r = b.r0 + rr, c = b.c0 + cc;
                if ((unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols) {
                    if constexpr (DET) atomicAdd(gFbar64 + vo + (size_t)r * cols + c, v);
                    else atomicAdd(gFbar + vo + (size_t)r * cols + c, (float)v);
                }
            }
        }
    };
    BpBox prev_b = unpack_box(ldg(boxes + (mlo <= mhi ? mlo : 0)));
    for (int m = mlo; m <= mhi; ++m) {
        const int buf = (m - mlo) & 1;
        const BpBox b = unpack_box(ldg(boxes + m));
        const float4 vt = ldg(view_tab + m);
        const float4 ray = ldg(rays + m);          // col, u_c, v_c, rho_c^2
        const float du = fmaf(-ddx, vt.y, ddy * vt.x);
        const float dv = -fmaf(ddx, vt.x, ddy * vt.y);
        const float u = ray.y + du, v = ray.z + dv;
        const float vinv = __builtin_amdgcn_rcpf(v);
        const float rinv = __builtin_amdgcn_rsqf(fmaf(u, u, v * v));
        const float tn = fmaf(du, ray.z, -ray.y * dv);
        const float td = fmaf(ray.y, du, fmaf(ray.z, dv, ray.w));
        float dang;                                 // alpha* - alpha_c
        if (series) {
            const float t = tn * __builtin_amdgcn_rcpf(td);
            const float s2 = t * t;
            float qa = fmaf(s2, -1.0f / 11.0f, 1.0f / 9.0f);
            qa = fmaf(qa, s2, -1.0f / 7.0f);
            qa = fmaf(qa, s2, 1.0f / 5.0f);
            qa = fmaf(qa, s2, -1.0f / 3.0f);
            qa = fmaf(qa, s2, 1.0f);
            dang = t * qa;
        } else {
            dang = atan2f(tn, td);
        }
        const float cc = med3(fmaf(dang, p.inv_dalpha, ray.x), 0.0f, (float)(b.nc - 2));
        const int c0 = (int)cc;
        const float tc = cc - (float)c0;
        const float q = p.q_scale * rinv;
        const float rb = fmaf(q, vt.z + zoff, p.row_c - (float)b.r0);
        const float st = q * p.dz;
        const float rmax = (float)(b.nr - 2);
        const float mf = (float)m;
        unsigned word = (1u << NG) - 1u;
        if (use_words) word = __builtin_amdgcn_readfirstlane(words[wave][m - mlo]);
        // the view's active slices in register order: each slice adds its row weights to
        // two pending rows (R, R+1) kept in registers; a row's two taps (columns c0, c0+1)
        // are scattered once the walk has moved past it, so slices that share detector
        // rows (row steps of 0 or 1) meet in registers first
        auto walk = [&](auto emit) {
            int R = -1;                                       // -1: nothing pending yet
            float P = 0.0f, Q = 0.0f;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (!(word & (1u << g))) continue;
                const bool full = word & (1u << (kFull + g));
#pragma unroll
                for (int s = 0; s < kKG; ++s) {
                    const int r = g * kKG + s;                // register
                    const float sl = (float)((r + off) & (KZ - 1));     // its slice
                    float a = vinv * fb[r];
                    if (!full) a *= med3(fminf(mf - A[r], B[r] - mf), 0.0f, 1.0f);
                    const float rr = med3(fmaf(sl, st, rb), 0.0f, rmax);
                    const int Rk = (int)rr;
                    const float a1 = a * __builtin_amdgcn_fractf(rr), a0 = a - a1;   // rows Rk, Rk+1
                    const bool same = Rk == R, next = Rk == R + 1;
                    if (!same && R >= 0) emit(R, P);
                    if (!same && !next && R >= 0) emit(R + 1, Q);
                    P = same ? P + a0 : (next ? Q + a0 : a0);
                    Q = same ? Q + a1 : a1;
                    R = Rk;
                }
            }
            if (R >= 0) {
                emit(R, P);
                emit(R + 1, Q);
            }
        };
        if (fits(b)) {
            // LDS addresses in 32 bits (the box is shared memory)
            LdsAcc *bx = (LdsAcc *)box[buf] + c0;
            walk([&](int row, float v) {
                if (v != 0.0f) {
                    const float v1 = v * tc;
                    LdsAcc *cell = bx + __mul24(row, kRowT);
                    if constexpr (DET) {
                        const unsigned long long q = to_fixed(v, fx), q1 = to_fixed(v1, fx);
                        __hip_atomic_fetch_add(cell, q - q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(cell + 1, q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else {
                        __hip_atomic_fetch_add(cell, (double)(v - v1), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(cell + 1, (double)v1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            });
        } else {
            // rows and columns relative to the box, which is clipped to the zero-padded
            // detector; cells of the padding are dropped (the forward reads zeros there)
            const size_t vo = (size_t)(base + m - first_view) * vstride;
            const int c = b.c0 + c0;
            walk([&](int row, float v) {
                const int rd = b.r0 + row;
                if (v != 0.0f && (unsigned)rd < (unsigned)rows) {
                    const float v1 = v * tc;
                    const size_t q = vo + (size_t)rd * cols;
                    if constexpr (DET) {
                        const unsigned long long f = to_fixed(v, fx), f1 = to_fixed(v1, fx);
                        if ((unsigned)c < (unsigned)cols) atomicAdd(gFbar64 + q + c, f - f1);
                        if ((unsigned)(c + 1) < (unsigned)cols) atomicAdd(gFbar64 + q + c + 1, f1);
                    } else {
                        if ((unsigned)c < (unsigned)cols) atomicAdd(gFbar + q + c, v - v1);
                        if ((unsigned)(c + 1) < (unsigned)cols) atomicAdd(gFbar + q + c + 1, v1);
                    }
                }
            });
        }
        if (m > mlo && fits(prev_b)) flush(m - 1, prev_b, buf ^ 1);
        prev_b = b;
        __syncthreads();
    }
    if (mlo <= mhi && fits(prev_b)) flush(mhi, prev_b, (mhi - mlo) & 1);
}

template <int KZ, bool FB, bool DET>
__global__ __launch_bounds__(kNT) void k_bpT_lds(BpArgs p, const float *__restrict__ fvol,
                                                 void *__restrict__ gFout,
                                                 const double *__restrict__ fscale, int rows,
                                                 int cols, long long first_view,
                                                 const float4 *__restrict__ view_tab,
                                                 const uint2 *__restrict__ box_tab,
                                                 const float4 *__restrict__ ray_tab, int series) {
    __shared__ BpTShared<KZ, DET> S;
    bpT_tile<KZ, FB, DET>(p, fvol, gFout, fscale, rows, cols, first_view, view_tab, box_tab, ray_tab, series,
                          blockIdx.x, blockIdx.y, blockIdx.z, S);
}

// Whether the odd series serves every voxel's angle from its tile centre's ray: a voxel lies
// within h (the tile's half-diagonal) of its tile centre, which is at least d = R - rho_c from
// the source (rho_c: the largest distance of a tile centre from the axis), so |tan delta| <=
// h / sqrt(d^2 - h^2); at most 0.2 keeps the series' remainder below 1e-10 rad.  Wider angles
// (short helix radii against the tile) take atan2f.
int series_serves(const KParams &k) {
    const double h = 0.5 * (kT - 1) * std::hypot(k.dx, k.dy);
    double rc = 0.0;
    for (int tx : {0, k.bp_tiles_x - 1})
        for (int ty : {0, k.bp_tiles_y - 1}) {
            const double xc = k.x_first + (tx * kT + 0.5 * (kT - 1)) * k.dx;
            const double yc = k.y_first + (ty * kT + 0.5 * (kT - 1)) * k.dy;
            rc = std::max(rc, std::hypot(xc, yc));
        }
    const double d = k.R - rc;
    return d > h && h <= 0.2 * std::sqrt(d * d - h * h) ? 1 : 0;
}

template <int KZ, bool DET>
void launch_bpT(bool fb, dim3 grid, hipStream_t s, const BpArgs &a, const float *gvol, void *gFout,
                const double *fscale, int rows, int cols, long long first_view, const float4 *view,
                const uint2 *boxes, const float4 *rays, int series) {
    // fb: HBM path for boxes beyond the LDS tile
    if (fb)
        hipLaunchKernelGGL((k_bpT_lds<KZ, true, DET>), grid, dim3(kNT), 0, s, a, gvol, gFout, fscale, rows,
                           cols, first_view, view, boxes, rays, series);
    else
        hipLaunchKernelGGL((k_bpT_lds<KZ, false, DET>), grid, dim3(kNT), 0, s, a, gvol, gFout, fscale, rows,
                           cols, first_view, view, boxes, rays, series);
}

// ----------------------------------------------------------------------------- fixed point

// partial maxima of |fbar| (grid-stride)
__global__ __launch_bounds__(kNT) void k_absmax_partial(const float *__restrict__ x, unsigned long long n,
                                                        float *__restrict__ part) {
    __shared__ float sh[kNT / 64];
    float m = 0.0f;
    for (unsigned long long i = (unsigned long long)blockIdx.x * kNT + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * kNT)
        m = fmaxf(m, fabsf(x[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// S = 2^e with bound * max|fbar| * S < 2^62 (bound: the largest possible |g^F-bar| cell per
// unit of max|fbar|); S = 1 when fbar is zero
__global__ __launch_bounds__(kNT) void k_fixed_scale(const float *__restrict__ part, int np, double bound,
                                                     double *__restrict__ S) {
    __shared__ float sh[kNT / 64];
    float m = 0.0f;
    for (int i = threadIdx.x; i < np; i += kNT) m = fmaxf(m, part[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = (double)fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3])) * bound;
        *S = mx > 0.0 ? ldexp(1.0, 61 - ilogb(mx)) : 1.0;       // mx S in [2^61, 2^62)
    }
}

// g^F-bar = fixed-point sums / S, rounded once to float32
__global__ __launch_bounds__(kNT) void k_fixed_to_float(const unsigned long long *__restrict__ in,
                                                        unsigned long long n, const double *__restrict__ S,
                                                        float *__restrict__ out) {
    const double inv = 1.0 / *S;
    for (unsigned long long i = (unsigned long long)blockIdx.x * kNT + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * kNT)
        out[i] = (float)((double)(long long)in[i] * inv);
}

}  // namespace

hipError_t launch_backproject_T(const KParams &k, const float *gvol, float *gFbar, hipStream_t s) {
    const dim3 grid((unsigned)k.bp_tiles_x, (unsigned)k.bp_tiles_y, (unsigned)(k.n_pitches * k.bp_runs));
    const BpArgs a = bp_args(k);
    const uint2 *boxes = reinterpret_cast<const uint2 *>(k.boxes);
    const float4 *rays = reinterpret_cast<const float4 *>(k.tref);
    const bool fb = !k.bp_all_fit;
    const int ser = series_serves(k);
    switch (k.bp_kz) {
        case 8: launch_bpT<8, false>(fb, grid, s, a, gvol, gFbar, nullptr, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
        case 32: launch_bpT<32, false>(fb, grid, s, a, gvol, gFbar, nullptr, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
        default: launch_bpT<16, false>(fb, grid, s, a, gvol, gFbar, nullptr, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
    }
    return hipGetLastError();
}

hipError_t launch_backproject_T_fixed(const KParams &k, const float *gvol, unsigned long long *gF64,
                                      void *scratch, double bound, hipStream_t s) {
    const unsigned long long nvol = (unsigned long long)k.nx * k.ny * k.nz;
    const unsigned long long ngf = (unsigned long long)k.n_filt * k.rows * k.cols;
    float *part = static_cast<float *>(scratch);
    double *S = reinterpret_cast<double *>(static_cast<unsigned char *>(scratch) + (uint64_t)kFixedScaleBlocks * 4);
    const unsigned long long pb = (nvol + kNT * 16ull - 1) / (kNT * 16ull);
    const int np = (int)(pb < 1 ? 1 : (pb > (unsigned long long)kFixedScaleBlocks ? kFixedScaleBlocks : pb));
    hipLaunchKernelGGL(k_absmax_partial, dim3(np), dim3(kNT), 0, s, gvol, nvol, part);
    hipLaunchKernelGGL(k_fixed_scale, dim3(1), dim3(kNT), 0, s, (const float *)part, np, bound, S);
    hipError_t e = launch_zero(gF64, ngf * 8, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)k.bp_tiles_x, (unsigned)k.bp_tiles_y, (unsigned)(k.n_pitches * k.bp_runs));
    const BpArgs a = bp_args(k);
    const uint2 *boxes = reinterpret_cast<const uint2 *>(k.boxes);
    const float4 *rays = reinterpret_cast<const float4 *>(k.tref);
    const bool fb = !k.bp_all_fit;
    const int ser = series_serves(k);
    switch (k.bp_kz) {
        case 8: launch_bpT<8, true>(fb, grid, s, a, gvol, gF64, S, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
        case 32: launch_bpT<32, true>(fb, grid, s, a, gvol, gF64, S, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
        default: launch_bpT<16, true>(fb, grid, s, a, gvol, gF64, S, k.rows, k.cols, k.first_view, k.view, boxes, rays, ser); break;
    }
    return hipGetLastError();
}

const double *fixed_scale_ptr(const void *scratch) {
    return reinterpret_cast<const double *>(static_cast<const unsigned char *>(scratch) +
                                            (uint64_t)kFixedScaleBlocks * 4);
}

hipError_t launch_fixed_to_float(const unsigned long long *in, unsigned long long n, const double *S,
                                 float *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned long long cb = (n + kNT - 1) / kNT;
    hipLaunchKernelGGL(k_fixed_to_float, dim3((unsigned)(cb < 16384 ? cb : 16384)), dim3(kNT), 0, s, in, n, S,
                       out);
    return hipGetLastError();
}

}  // namespace kats
