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
#include "bp_common.hpp"

namespace kats {

namespace {

using namespace bpdev;

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
constexpr int kHull = 2048;       // max views of a workgroup hull with per-view group words
// LDS row pitch of the box tile (floats): 72 instead of the 64 box columns moves each row
// by eight banks, so lanes reading one column at different rows meet fewer conflicts
// (9.11 ms against 9.15 ms on the clinical workload; the adjoint gains far more from the
// same padding)
constexpr int kRowF = 72;

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
    __attribute__((aligned(16))) float tile[2][kRowF * lds_rows<KZ>()];   // double-buffered box
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
    // (an empty hull, mlo = INT_MAX > mhi = INT_MIN, takes no words: mhi - mlo would overflow)
    const bool use_words = mlo <= mhi && mhi - mlo < kHull;
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
    // g^F of pitch-relative view 0; element (0, 0) of a view is detector cell (-kPad, -kPad)
    const float *gF0 = gF + (size_t)(base - p.first_view) * vstride;
    auto fits = [](const BpBox &b) { return !FB || (b.nr <= kLR && b.nc <= kLP); };

    // Box staging: 16 lanes per LDS row, one aligned float4 each (the plan starts every box
    // on a 16-byte boundary of the padded row; columns past the box land in unused LDS).
    const int srow = tid >> 4, scol = (tid & 15) * 4;
    uint2 bw_next = make_uint2(0u, 0u);   // box of the view after the current one
    if (mlo <= mhi) {
        const BpBox b = unpack_box(ldg(boxes + mlo));
        if (mlo < mhi) bw_next = ldg(boxes + mlo + 1);
        if (fits(b)) {
            const float *src = gF0 + (size_t)mlo * vstride + (b.r0 + kPad) * cpitch + (b.c0 + kPad);
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (srow + 16 * k < b.nr && scol < b.nc)
                    *reinterpret_cast<float4 *>(&lds[0][(srow + 16 * k) * kRowF + scol]) =
                        ldg(reinterpret_cast<const float4 *>(src + (srow + 16 * k) * cpitch + scol));
        }
    }
    __syncthreads();
    BpBox b = unpack_box(ldg(boxes + (mlo <= mhi ? mlo : 0)));
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
            bn = unpack_box(bw_next);
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
                if (word & (1u << g)) group(T, kRowF, g);
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
                if (stg[k]) *reinterpret_cast<float4 *>(&Dst[(srow + 16 * k) * kRowF + scol]) = pf[k];
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

}  // namespace

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

}  // namespace kats
