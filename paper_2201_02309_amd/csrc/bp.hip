// Backprojection over the PI interval (Sec. II backprojection step) for gfx950.
//
// f(x) = dlambda/(2 pi) sum_n c_n(x) / v*_n(x) g^F(lambda_n, alpha*_n(x), w*_n(x)),
// v* = R - x cos(b) - y sin(b), alpha* = atan(u / v*), u = -x sin(b) + y cos(b),
// w* = D cos(alpha*) / v* (z - z0 - P lambda / 2 pi) = D (z - z0 - P lambda / 2 pi) / sqrt(u^2+v*^2),
// with b = lambda + lambda0 and c_n the overlap of view cell [n-1/2, n+1/2] with the PI
// interval [l_i, l_o] (view units); c_n differs from 0 and 1 only at the first and last
// view of the interval.
//
// Every pitch k reuses the first pitch's tables (Sec. II periodicity): slice j of pitch k
// sees view n = n_lo + k Nv + m exactly as slice j of pitch 0 sees view n_lo + m, so the
// per-view table (cos b, sin b, e_m = z_first - z0 - h lambda_{n_lo+m}), the PI table
// (l_i, l_o, n_first, n_last relative to n_lo) and the footprint boxes are indexed by the
// pitch-relative view m and slice j only: the geometry is bit-identical for every pitch.
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace kats {

namespace {

__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline float med3(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

// Pointers read from memory (the packed launch's request descriptors) carry no address
// space, so loads through them would be flat (slower, and ordered with LDS traffic);
// every table / g^F / volume access goes through a global-address-space pointer instead.
template <class T>
__device__ inline __attribute__((address_space(1))) T *glb(T *ptr) {
    return (__attribute__((address_space(1))) T *)ptr;
}
// Load of a 4-, 8- or 16-byte value through a global-address-space pointer.
template <class T>
__device__ inline T ldg(const T *ptr) {
    static_assert(sizeof(T) % 4 == 0 && sizeof(T) <= 16, "whole dwords");
    typedef unsigned int W __attribute__((ext_vector_type(sizeof(T) / 4)));
    const W w = *(const __attribute__((address_space(1))) W *)ptr;
    T out;
    __builtin_memcpy(&out, &w, sizeof(T));
    return out;
}

// ---------------------------------------------------------------------------------
// Forward backprojection.  Workgroup = 256 lanes = a 16 x 16 (x, y) tile (4 waves of
// 16 x 4) x a run of KZ consecutive slices of one pitch; every lane keeps KZ accumulators.
// The workgroup walks the hull of its voxels' PI windows view by view.  For each view the
// plan gives the tile's detector footprint box (float64 bound); the box of view m+1 is
// loaded from HBM into registers while view m is backprojected from LDS, then stored into
// the other LDS buffer (one barrier per view).  Per (lane, view): v*, 1/v*, 1/rho and the
// column coordinate (atan); per (lane, view, slice): the row coordinate (one FMA: rows
// advance by dz D / (rho dw) per slice), two ds_read2 of the 2 x 2 taps, three lerps and
// one FMA into the accumulator.  Slices are handled in groups of kKG: before the view
// loop every wave classifies each view of the hull into a 16-bit word (bit g: some voxel
// of group g is active; bit 8+g: every valid voxel of group g has c_n = 1): inactive
// groups are skipped by a wave-uniform branch and fully covered ones skip the coverage
// arithmetic.  When the plan has boxes larger than the LDS tile, the kernel instance with
// the fallback reads those views' taps from the zero-padded g^F in HBM instead.
// ---------------------------------------------------------------------------------
constexpr int kT = kBpTile;       // 16
constexpr int kNT = kT * kT;      // 256 lanes
constexpr int kLP = kBpBoxCols;   // LDS tile row pitch (floats) = max box columns
// LDS tile depth (max box rows) of a slice run: runs of 32 slices span up to ~60 detector
// rows, shorter runs fit 32.
template <int KZ>
constexpr int lds_rows() { return KZ >= 32 ? 2 * kBpBoxRows : kBpBoxRows; }
constexpr int kHull = 2048;       // max views of a workgroup hull with per-view group words
constexpr int kKG = 4;            // slices per branch group

// The scalars the backprojector needs (a slim kernel argument keeps SGPR pressure low).
struct BpArgs {
    const float4 *view;
    const PiEntry *pi;
    const BpBox *boxes;
    long long n_views, first_view;
    float R, inv_dalpha, col_c, q_scale, row_c, dz, x_first, y_first, dx, dy, scale;
    int nx, ny, nz, ns, Nv, n_lo, W, runs, tiles_x, tiles_y, gf_rows, gf_cols;
    int atan_deg;
    float atan_coef[9];
};

template <class P>
__device__ inline float lerp_bilinear(P t, int pitch_f, float tc, float tr) {
    const float v00 = t[0], v01 = t[1], v10 = t[pitch_f], v11 = t[pitch_f + 1];
    const float top = fmaf(tc, v01 - v00, v00);
    const float bot = fmaf(tc, v11 - v10, v10);
    return fmaf(tr, bot - top, top);
}

// Shared memory of one backprojection workgroup.
template <int KZ>
struct BpShared {
    __attribute__((aligned(16))) float tile[2][kLP * lds_rows<KZ>()];   // double-buffered box
    unsigned short words[4][kHull];  // per wave and view: active groups | full groups << 8
    int red[8];
};

// One workgroup task: tile (bx, by) of the grid, slice run / pitch bz = pitch * runs + run.
// Shared by the one-plan kernel (task = block index) and the packed multi-plan kernel.
// FB: some box of the plan may exceed the LDS tile (those views read their taps from HBM);
// without it the view loop has a single path, which keeps the accumulators in place.
// P4: the plan's atan polynomial has degree <= 4 in t^2 (otherwise degree 8, or atan2f).
template <int KZ, bool FB, bool P4>
__device__ void bp_tile(const BpArgs p, const float *__restrict__ gF, float *__restrict__ vol,
                        const float4 *__restrict__ view_tab, const uint2 *__restrict__ box_tab,
                        int bxi, int byi, int bz, BpShared<KZ> &S) {
    static_assert(KZ % kKG == 0 && KZ / kKG <= 8, "groups use 8-bit masks");
    constexpr int kLR = lds_rows<KZ>();
    constexpr int NP = kLR / 16;          // staging passes of 16 rows x 16 float4 lanes
    static_assert(NP == 2 || NP == 4, "box staging passes");
    constexpr int NG = KZ / kKG;
    auto &lds = S.tile;
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

    float A[KZ], B[KZ], acc[KZ];
    unsigned valid = 0;
    int wlo = INT_MAX, whi = INT_MIN;
    int g_alo[NG], g_ahi[NG], g_flo[NG], g_fhi[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        int alo = INT_MAX, ahi = INT_MIN, flo = INT_MIN, fhi = INT_MAX;
#pragma unroll
        for (int s = 0; s < kKG; ++s) {
            const int jj = g * kKG + s;
            A[jj] = 3.0e38f;
            B[jj] = -3.0e38f;
            acc[jj] = 0.0f;
            if (inxy && jj < nrun) {
                const PiEntry e = ldg(p.pi + ((size_t)(j0 + jj) * p.ny + iy) * p.nx + ix);
                const long long nf = base + e.nf, nl = base + e.nl;
                if (e.nf <= e.nl && nf - 1 >= 0 && nl + 1 <= p.n_views - 1) {
                    A[jj] = e.li - 0.5f;      // c_n = clamp(min(m - A, B - m), 0, 1)
                    B[jj] = e.lo + 0.5f;
                    valid |= 1u << jj;
                    alo = min(alo, e.nf);
                    ahi = max(ahi, e.nl);
                    // views with c_n = 1 for certain (one view of margin against rounding)
                    flo = max(flo, (int)ceilf(A[jj] + 1.0f) + 1);
                    fhi = min(fhi, (int)floorf(B[jj] - 1.0f) - 1);
                }
            }
        }
        // a group is active at m if one of its voxels is; full if every valid voxel of the
        // group has c_n = 1 at m
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
    __syncthreads();
    // wave-uniform (scalar) so that the per-view box and view-table reads are scalar loads
    const int mlo = __builtin_amdgcn_readfirstlane(min(min(red[0], red[1]), min(red[2], red[3])));
    const int mhi = __builtin_amdgcn_readfirstlane(max(max(red[4], red[5]), max(red[6], red[7])));
    // Per-view group classification of this wave.  A hull longer than kHull views
    // takes the coverage path for every group at every view, which is exact.
    const bool use_words = mhi - mlo + 1 <= kHull;
    if (use_words) {
        for (int w = lane; w <= mhi - mlo; w += 64) {
            const int m = mlo + w;
            unsigned word = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (m >= g_alo[g] && m <= g_ahi[g]) word |= 1u << g;
                if (m >= g_flo[g] && m <= g_fhi[g]) word |= 1u << (8 + g);
            }
            words[wave][w] = (unsigned short)word;
        }
    }

    const float x = fmaf((float)ix, p.dx, p.x_first);
    const float y = fmaf((float)iy, p.dy, p.y_first);
    const float zoff = (float)j0 * p.dz;
    const int cpitch = p.gf_cols;
    const size_t vstride = (size_t)p.gf_rows * cpitch;
    // boxes read as two dwords (scalar loads) and unpacked: {r0 | nr << 16, c0 | nc << 16}
    const uint2 *__restrict__ boxes =
        box_tab + ((size_t)(run * p.tiles_y + byi) * p.tiles_x + bxi) * p.W;
    auto unpack = [](uint2 w) {
        BpBox b;
        b.r0 = (int16_t)(w.x & 0xffffu);
        b.nr = (int16_t)(w.x >> 16);
        b.c0 = (int16_t)(w.y & 0xffffu);
        b.nc = (int16_t)(w.y >> 16);
        return b;
    };
    // g^F of pitch-relative view 0; element (0, 0) of a view is detector cell (-kPad, -kPad)
    const float *gF0 = gF + (size_t)(base - p.first_view) * vstride;
    auto fits = [](const BpBox &b) { return !FB || (b.nr <= kLR && b.nc <= kLP); };

    // Box staging: 16 lanes per LDS row, one aligned float4 each (the plan starts every box
    // on a 16-byte boundary of the padded row; columns past the box land in unused LDS).
    const int srow = tid >> 4, scol = (tid & 15) * 4;
    uint2 bw_next = make_uint2(0u, 0u);   // box of the view after the current one
    if (mlo <= mhi) {
        const BpBox b = unpack(ldg(boxes + mlo));
        if (mlo < mhi) bw_next = ldg(boxes + mlo + 1);
        if (fits(b)) {
            const float *src = gF0 + (size_t)mlo * vstride + (b.r0 + kPad) * cpitch + (b.c0 + kPad);
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (srow + 16 * k < b.nr && scol < b.nc)
                    *reinterpret_cast<float4 *>(&lds[0][(srow + 16 * k) * kLP + scol]) =
                        ldg(reinterpret_cast<const float4 *>(src + (srow + 16 * k) * cpitch + scol));
        }
    }
    __syncthreads();
    BpBox b = unpack(ldg(boxes + (mlo <= mhi ? mlo : 0)));
    for (int m = mlo; m <= mhi; ++m) {
        const int buf = (m - mlo) & 1;
        // box of view m+2, loaded one iteration ahead of its use
        uint2 bw_after = make_uint2(0u, 0u);
        if (m + 2 <= mhi) bw_after = ldg(boxes + m + 2);
        // prefetch the next view's box into registers (NP rows of 16 float4 lanes)
        float4 pf[NP];
        BpBox bn = b;
        bool next_fits = false, stg[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) stg[k] = false;
        if (m < mhi) {
            bn = unpack(bw_next);
            next_fits = fits(bn);
            if (next_fits) {
                const float *src = gF0 + (size_t)(m + 1) * vstride + (bn.r0 + kPad) * cpitch + (bn.c0 + kPad);
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    stg[k] = srow + 16 * k < bn.nr && scol < bn.nc;
                    if (stg[k]) pf[k] = ldg(reinterpret_cast<const float4 *>(src + (srow + 16 * k) * cpitch + scol));
                }
            }
        }
        // per (lane, view) geometry; coordinates relative to the box origin, clamped into
        // the box (only voxels projecting outside the zero-padded detector are clamped)
        const float4 vt = ldg(view_tab + m);
        const float u = fmaf(-x, vt.y, y * vt.x);
        const float v = p.R - fmaf(x, vt.x, y * vt.y);
        const float vinv = __builtin_amdgcn_rcpf(v);
        const float rinv = __builtin_amdgcn_rsqf(fmaf(u, u, v * v));
        float acol;                                          // alpha* / dalpha
        if (P4 || p.atan_deg >= 0) {
            const float t = u * vinv;                        // tan(alpha*)
            const float s2 = t * t;
            constexpr int deg = P4 ? 4 : 8;
            float qa = p.atan_coef[deg];
#pragma unroll
            for (int k = deg - 1; k >= 0; --k) qa = fmaf(qa, s2, p.atan_coef[k]);
            acol = t * qa;
        } else {
            acol = atan2f(u, v) * p.inv_dalpha;
        }
        const float cc = med3(acol + (p.col_c - (float)b.c0), 0.0f, (float)(b.nc - 2));
        const int c0 = (int)cc;
        const float tc = cc - (float)c0;
        const float q = p.q_scale * rinv;                   // detector rows per mm of z
        const float rb = fmaf(q, vt.z + zoff, p.row_c - (float)b.r0);
        const float st = q * p.dz;
        const float rmax = (float)(b.nr - 2);
        const float mf = (float)m;
        unsigned word = (1u << NG) - 1u;                    // all groups active, none full
        if (use_words) word = __builtin_amdgcn_readfirstlane(words[wave][m - mlo]);
        // one group of kKG slices: taps of all its slices first (independent LDS / HBM
        // loads), then the accumulation with or without the coverage weight
        auto group = [&](auto T, int tp, int g) {         // T: LDS or global taps
            float val[kKG];
#pragma unroll
            for (int s = 0; s < kKG; ++s) {
                const float rr = med3(fmaf((float)(g * kKG + s), st, rb), 0.0f, rmax);
                const int r0 = (int)rr;               // rr >= 0: truncation = floor
                val[s] = lerp_bilinear(T + r0 * tp, tp, tc, __builtin_amdgcn_fractf(rr));
            }
            // the coverage weight scales the taps in place, so that both paths end in
            // the same FMA on the accumulators
            if (!(word & (1u << (8 + g)))) {
#pragma unroll
                for (int s = 0; s < kKG; ++s) {
                    const int jj = g * kKG + s;
                    val[s] *= med3(fminf(mf - A[jj], B[jj] - mf), 0.0f, 1.0f);
                }
            }
#pragma unroll
            for (int s = 0; s < kKG; ++s) acc[g * kKG + s] = fmaf(vinv, val[s], acc[g * kKG + s]);
        };
        if (fits(b)) {
            const float *T = &lds[buf][c0];
#pragma unroll
            for (int g = 0; g < NG; ++g)
                if (word & (1u << g)) group(T, kLP, g);
        } else {
            const auto T = glb(gF0 + (size_t)m * vstride + (b.r0 + kPad) * cpitch + (b.c0 + kPad) + c0);
#pragma unroll
            for (int g = 0; g < NG; ++g)
                if (word & (1u << g)) group(T, cpitch, g);
        }
        {
            float *Dst = lds[buf ^ 1];
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (stg[k]) *reinterpret_cast<float4 *>(&Dst[(srow + 16 * k) * kLP + scol]) = pf[k];
        }
        b = bn;
        bw_next = bw_after;
        __syncthreads();
    }
    if (!inxy) return;
    const int iz0 = pitch * p.ns + j0;
#pragma unroll
    for (int jj = 0; jj < KZ; ++jj) {
        if (jj < nrun)
            glb(vol)[((size_t)(iz0 + jj) * p.ny + iy) * p.nx + ix] =
                ((valid >> jj) & 1u) ? acc[jj] * p.scale : 0.0f;
    }
}

template <int KZ, bool FB, bool P4>
__global__ __launch_bounds__(kNT) void k_bp_lds(BpArgs p, const float *__restrict__ gF,
                                                float *__restrict__ vol,
                                                const float4 *__restrict__ view_tab,
                                                const uint2 *__restrict__ box_tab) {
    __shared__ BpShared<KZ> S;
    bp_tile<KZ, FB, P4>(p, gF, vol, view_tab, box_tab, blockIdx.x, blockIdx.y, blockIdx.z, S);
}

// ---------------------------------------------------------------------------------
// Grouped backprojection of several plans in one launch (serving): the grid enumerates
// the (pitch, slice run, tile) tasks of up to kGroupMax requests back to back; a block
// finds its request from the task prefix held in the kernel argument (a wave-uniform scan)
// and runs that request's tile exactly as the one-plan kernel does.  Descriptors travel as
// kernel arguments, so the compiler sees them as constant memory (scalar loads, global
// pointers), as for the one-plan kernel.
// ---------------------------------------------------------------------------------
struct BpRequest {
    BpArgs a;
    const float *gF;
    float *vol;
    const float4 *view;
    const uint2 *boxes;
    long long first_task;          // prefix of the task counts of earlier requests
};

constexpr int kGroupMax = 16;
struct BpGroup {
    BpRequest r[kGroupMax];
    int n;
};
static_assert(sizeof(BpGroup) <= 4000, "kernel argument segment");

template <int KZ, bool FB, bool P4>
__global__ __launch_bounds__(kNT) void k_bp_group(const BpGroup g) {
    __shared__ BpShared<KZ> S;
    const long long task = blockIdx.x;
    int r = 0;
    while (r + 1 < g.n && g.r[r + 1].first_task <= task) ++r;
    const BpRequest &q = g.r[r];
    long long local = task - q.first_task;
    const int bxi = (int)(local % q.a.tiles_x);
    local /= q.a.tiles_x;
    const int byi = (int)(local % q.a.tiles_y);
    const int bz = (int)(local / q.a.tiles_y);
    bp_tile<KZ, FB, P4>(q.a, q.gF, q.vol, q.view, q.boxes, bxi, byi, bz, S);
}

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
constexpr int kLPT = kLP;
constexpr int kHullT = 2000;

template <int KZ>
struct BpTShared {
    static constexpr int NG = KZ / kKG;
    using Word = typename std::conditional<(NG <= 4), unsigned char, unsigned short>::type;
    static constexpr int kFull = NG <= 4 ? 4 : 8;
    __attribute__((aligned(16))) double box[2][kLPT * lds_rows<KZ>()];
    Word words[4][kHullT];
    int red[8];
};

template <int KZ, bool P4>
__device__ void bpT_tile(const BpArgs p, const float *__restrict__ fvol, float *__restrict__ gFbar,
                         int rows, int cols, long long first_view,
                         const float4 *__restrict__ view_tab, const uint2 *__restrict__ box_tab,
                         int bxi, int byi, int bz, BpTShared<KZ> &S) {
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

    float A[KZ], B[KZ], fb[KZ];
    int wlo = INT_MAX, whi = INT_MIN;
    int g_alo[NG], g_ahi[NG], g_flo[NG], g_fhi[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        int alo = INT_MAX, ahi = INT_MIN, flo = INT_MIN, fhi = INT_MAX;
#pragma unroll
        for (int s = 0; s < kKG; ++s) {
            const int jj = g * kKG + s;
            A[jj] = 3.0e38f;
            B[jj] = -3.0e38f;
            fb[jj] = 0.0f;
            if (inxy && jj < nrun) {
                const PiEntry e = ldg(p.pi + ((size_t)(j0 + jj) * p.ny + iy) * p.nx + ix);
                const long long nf = base + e.nf, nl = base + e.nl;
                if (e.nf <= e.nl && nf - 1 >= 0 && nl + 1 <= p.n_views - 1) {
                    A[jj] = e.li - 0.5f;
                    B[jj] = e.lo + 0.5f;
                    fb[jj] = ldg(fvol + ((size_t)(iz0 + jj) * p.ny + iy) * p.nx + ix) * p.scale;
                    alo = min(alo, e.nf);
                    ahi = max(ahi, e.nl);
                    flo = max(flo, (int)ceilf(A[jj] + 1.0f) + 1);
                    fhi = min(fhi, (int)floorf(B[jj] - 1.0f) - 1);
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
    for (int i = tid; i < 2 * kLPT * kLR; i += kNT) (&box[0][0])[i] = 0.0;
    __syncthreads();
    const int mlo = __builtin_amdgcn_readfirstlane(min(min(red[0], red[1]), min(red[2], red[3])));
    const int mhi = __builtin_amdgcn_readfirstlane(max(max(red[4], red[5]), max(red[6], red[7])));
    using Word = typename BpTShared<KZ>::Word;
    constexpr int kFull = BpTShared<KZ>::kFull;
    const bool use_words = mhi - mlo + 1 <= kHullT;
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

    const float x = fmaf((float)ix, p.dx, p.x_first);
    const float y = fmaf((float)iy, p.dy, p.y_first);
    const float zoff = (float)j0 * p.dz;
    const uint2 *__restrict__ boxes =
        box_tab + ((size_t)(run * p.tiles_y + byi) * p.tiles_x + bxi) * p.W;
    auto unpack = [](uint2 w) {
        BpBox b;
        b.r0 = (int16_t)(w.x & 0xffffu);
        b.nr = (int16_t)(w.x >> 16);
        b.c0 = (int16_t)(w.y & 0xffffu);
        b.nc = (int16_t)(w.y >> 16);
        return b;
    };
    const size_t vstride = (size_t)rows * cols;
    // flush of view m's box from buffer buf: lanes over 4 rows x 64 columns per pass
    auto flush = [&](int m, const BpBox &b, int buf) {
        double *bx = box[buf];
        float *img = gFbar + (size_t)(base + m - first_view) * vstride;
        const int cc = tid & 63;
        for (int rr = tid >> 6; rr < b.nr; rr += 4) {
            double *cell = bx + rr * kLPT + cc;
            const double v = *cell;
            if (v != 0.0) {
                *cell = 0.0;
                const int r = b.r0 + rr, c = b.c0 + cc;
                if ((unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols)
                    atomicAdd(img + (size_t)r * cols + c, (float)v);
            }
        }
    };
    BpBox prev_b = unpack(ldg(boxes + (mlo <= mhi ? mlo : 0)));
    for (int m = mlo; m <= mhi; ++m) {
        const int buf = (m - mlo) & 1;
        const BpBox b = unpack(ldg(boxes + m));
        const float4 vt = ldg(view_tab + m);
        const float u = fmaf(-x, vt.y, y * vt.x);
        const float v = p.R - fmaf(x, vt.x, y * vt.y);
        const float vinv = __builtin_amdgcn_rcpf(v);
        const float rinv = __builtin_amdgcn_rsqf(fmaf(u, u, v * v));
        float acol;
        if (P4 || p.atan_deg >= 0) {
            const float t = u * vinv;
            const float s2 = t * t;
            constexpr int deg = P4 ? 4 : 8;
            float qa = p.atan_coef[deg];
#pragma unroll
            for (int k = deg - 1; k >= 0; --k) qa = fmaf(qa, s2, p.atan_coef[k]);
            acol = t * qa;
        } else {
            acol = atan2f(u, v) * p.inv_dalpha;
        }
        const float cc = med3(acol + (p.col_c - (float)b.c0), 0.0f, (float)(b.nc - 2));
        const int c0 = (int)cc;
        const float tc = cc - (float)c0;
        const float q = p.q_scale * rinv;
        const float rb = fmaf(q, vt.z + zoff, p.row_c - (float)b.r0);
        const float st = q * p.dz;
        const float rmax = (float)(b.nr - 2);
        const float mf = (float)m;
        unsigned word = (1u << NG) - 1u;
        if (use_words) word = __builtin_amdgcn_readfirstlane(words[wave][m - mlo]);
        double *bx = box[buf] + c0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (!(word & (1u << g))) continue;
            const bool full = word & (1u << (kFull + g));
#pragma unroll
            for (int s = 0; s < kKG; ++s) {
                const int jj = g * kKG + s;
                float a = vinv * fb[jj];
                if (!full) a *= med3(fminf(mf - A[jj], B[jj] - mf), 0.0f, 1.0f);
                if (a != 0.0f) {
                    const float rr = med3(fmaf((float)jj, st, rb), 0.0f, rmax);
                    const int r0 = (int)rr;
                    const float tr = __builtin_amdgcn_fractf(rr);
                    const float a1 = a * tr, a0 = a - a1;          // rows r0, r0 + 1
                    const float a01 = a0 * tc, a11 = a1 * tc;        // column c0 + 1
                    double *cell = bx + r0 * kLPT;
                    atomicAdd(cell, (double)(a0 - a01));
                    atomicAdd(cell + 1, (double)a01);
                    atomicAdd(cell + kLPT, (double)(a1 - a11));
                    atomicAdd(cell + kLPT + 1, (double)a11);
                }
            }
        }
        if (m > mlo) flush(m - 1, prev_b, buf ^ 1);
        prev_b = b;
        __syncthreads();
    }
    if (mlo <= mhi) flush(mhi, prev_b, (mhi - mlo) & 1);
}

template <int KZ, bool P4>
__global__ __launch_bounds__(kNT) void k_bpT_lds(BpArgs p, const float *__restrict__ fvol,
                                                 float *__restrict__ gFbar, int rows, int cols,
                                                 long long first_view,
                                                 const float4 *__restrict__ view_tab,
                                                 const uint2 *__restrict__ box_tab) {
    __shared__ BpTShared<KZ> S;
    bpT_tile<KZ, P4>(p, fvol, gFbar, rows, cols, first_view, view_tab, box_tab, blockIdx.x,
                     blockIdx.y, blockIdx.z, S);
}

// ---------------------------------------------------------------------------------
// Adjoint of the backprojection (the transpose of the operator above, acting on an
// unpadded g^F cotangent).
// ---------------------------------------------------------------------------------
constexpr int kTile = 8;          // 8 x 8 lanes per wave
constexpr int kKZ = 8;            // slices per lane

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

static BpArgs bp_args(const KParams &k) {
    BpArgs a;
    a.view = k.view;
    a.pi = k.pi;
    a.boxes = k.boxes;
    a.n_views = k.n_views;
    a.first_view = k.first_view;
    a.R = k.R;
    a.inv_dalpha = k.inv_dalpha;
    a.col_c = k.col_c;
    a.q_scale = k.D * k.inv_dw;
    a.row_c = k.row_c;
    a.dz = k.dz;
    a.x_first = k.x_first;
    a.y_first = k.y_first;
    a.dx = k.dx;
    a.dy = k.dy;
    a.scale = k.scale;
    a.nx = k.nx;
    a.ny = k.ny;
    a.nz = k.nz;
    a.ns = k.ns;
    a.Nv = k.Nv;
    a.n_lo = k.n_lo;
    a.W = k.W;
    a.runs = k.bp_runs;
    a.tiles_x = k.bp_tiles_x;
    a.tiles_y = k.bp_tiles_y;
    a.gf_rows = k.gf_rows;
    a.gf_cols = k.gf_cols;
    a.atan_deg = k.atan_deg;
    for (int i = 0; i < 9; ++i) a.atan_coef[i] = k.atan_coef[i];
    return a;
}

// Kernel instance of a plan: bit 0 = HBM fallback path, bit 1 = short atan polynomial.
static int kernel_class(const KParams &k) {
    return (k.bp_all_fit ? 0 : 1) | ((k.atan_deg >= 0 && k.atan_deg <= 4) ? 2 : 0);
}

template <int KZ>
static void launch_lds(int cls, dim3 grid, hipStream_t s, const BpArgs &a, const float *gF,
                       float *vol, const float4 *view, const uint2 *boxes) {
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_bp_lds<KZ, false, false>), grid, dim3(kNT), 0, s, a, gF, vol, view, boxes); break;
        case 1: hipLaunchKernelGGL((k_bp_lds<KZ, true, false>), grid, dim3(kNT), 0, s, a, gF, vol, view, boxes); break;
        case 2: hipLaunchKernelGGL((k_bp_lds<KZ, false, true>), grid, dim3(kNT), 0, s, a, gF, vol, view, boxes); break;
        default: hipLaunchKernelGGL((k_bp_lds<KZ, true, true>), grid, dim3(kNT), 0, s, a, gF, vol, view, boxes); break;
    }
}

template <int KZ>
static void launch_group(int cls, dim3 grid, hipStream_t s, const BpGroup &g) {
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_bp_group<KZ, false, false>), grid, dim3(kNT), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_bp_group<KZ, true, false>), grid, dim3(kNT), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_bp_group<KZ, false, true>), grid, dim3(kNT), 0, s, g); break;
        default: hipLaunchKernelGGL((k_bp_group<KZ, true, true>), grid, dim3(kNT), 0, s, g); break;
    }
}

hipError_t launch_backproject(const KParams &k, const float *gF, float *vol, hipStream_t s) {
    dim3 grid((unsigned)k.bp_tiles_x, (unsigned)k.bp_tiles_y, (unsigned)(k.n_pitches * k.bp_runs));
    const BpArgs a = bp_args(k);
    const uint2 *boxes = reinterpret_cast<const uint2 *>(k.boxes);
    const int cls = kernel_class(k);
    switch (k.bp_kz) {
        case 8: launch_lds<8>(cls, grid, s, a, gF, vol, k.view, boxes); break;
        case 32: launch_lds<32>(cls, grid, s, a, gF, vol, k.view, boxes); break;
        default: launch_lds<16>(cls, grid, s, a, gF, vol, k.view, boxes); break;
    }
    return hipGetLastError();
}

// Requests are grouped by kernel instance (HBM fallback path or not, atan polynomial
// length); each launch takes up to kGroupMax requests of one class.
hipError_t launch_backproject_batch(const KParams *ks, const float *const *gF, float *const *vol,
                                    int n, int kz, hipStream_t s) {
    for (int cls = 0; cls < 4; ++cls) {
        BpGroup grp{};
        long long total = 0;
        auto flush = [&]() {
            if (grp.n == 0) return;
            const dim3 grid((unsigned)total);
            switch (kz) {
                case 8: launch_group<8>(cls, grid, s, grp); break;
                case 32: launch_group<32>(cls, grid, s, grp); break;
                default: launch_group<16>(cls, grid, s, grp); break;
            }
            grp = BpGroup{};
            total = 0;
        };
        for (int i = 0; i < n; ++i) {
            const KParams &k = ks[i];
            if (kernel_class(k) != cls) continue;
            const long long tasks = (long long)k.bp_tiles_x * k.bp_tiles_y * k.n_pitches * k.bp_runs;
            if (tasks == 0) continue;
            if (grp.n == kGroupMax || total + tasks > 0x7fffffffLL) flush();
            BpRequest &q = grp.r[grp.n++];
            q.a = bp_args(k);
            q.gF = gF[i];
            q.vol = vol[i];
            q.view = k.view;
            q.boxes = reinterpret_cast<const uint2 *>(k.boxes);
            q.first_task = total;
            total += tasks;
        }
        flush();
    }
    return hipGetLastError();
}

hipError_t launch_backproject_T(const KParams &k, const float *gvol, float *gFbar, hipStream_t s) {
    if (k.bp_all_fit) {
        // tiled adjoint: LDS-accumulated boxes, one global atomic per cell and view
        const dim3 grid((unsigned)k.bp_tiles_x, (unsigned)k.bp_tiles_y, (unsigned)(k.n_pitches * k.bp_runs));
        const BpArgs a = bp_args(k);
        const uint2 *boxes = reinterpret_cast<const uint2 *>(k.boxes);
        const bool p4 = k.atan_deg >= 0 && k.atan_deg <= 4;
#define KATS_BPT(KZ, P4) hipLaunchKernelGGL((k_bpT_lds<KZ, P4>), grid, dim3(kNT), 0, s, a, gvol, gFbar, \
                                            k.rows, k.cols, k.first_view, k.view, boxes)
        switch (k.bp_kz) {
            case 8: if (p4) KATS_BPT(8, true); else KATS_BPT(8, false); break;
            case 32: if (p4) KATS_BPT(32, true); else KATS_BPT(32, false); break;
            default: if (p4) KATS_BPT(16, true); else KATS_BPT(16, false); break;
        }
#undef KATS_BPT
        return hipGetLastError();
    }
    // plans with boxes beyond the LDS tile: per-tap global atomics
    const int ns_eff = k.ns < k.nz ? k.ns : k.nz;
    const int runs = (ns_eff + kKZ - 1) / kKZ;
    dim3 grid((k.nx + kTile - 1) / kTile, (k.ny + kTile - 1) / kTile, (unsigned)(k.n_pitches * runs));
    hipLaunchKernelGGL(k_backproject_T<kKZ>, grid, dim3(64), 0, s, k, gvol, gFbar, runs);
    return hipGetLastError();
}

}  // namespace kats
