// Filtering kernels of the Katsevich reconstruction for gfx950 (Sec. II steps 1-6):
//   k_deriv_lw    derivative at constant direction (eq. Deriv) + length weighting (eq. LW)
//   k_hilbert_fft forward height rebinning onto two kappa-lines (eqs. FR, w_k) packed as one
//                 complex row, then the Hilbert transform in alpha (eq. HF, kernel of e4) as a
//                 zero-padded linear convolution by register Stockham FFTs
//   k_br_cos      backward height rebinning (eq. BR) + post-cosine weighting (eq. PW)
// All kernels are HBM-streaming: one pass over their input and output, coalesced along
// detector columns.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kats {

namespace {

constexpr int kElemThreads = 256;
constexpr int kFftThreads = 256;

constexpr int kDerivRun = 16;     // filtered views per thread in k_deriv_lw
constexpr int kBrBlocks = 8;      // row blocks of a view in k_br_cos
constexpr int kBrUnroll = 12;     // rows per thread with every load issued first

// One thread per (detector row, column) takes a run of consecutive views, so each sinogram
// sample comes from HBM about once: the run's samples (plus one view on each side) are loaded
// into registers, every load issued before the first use (0.03 ms faster over the clinical
// filter than a walk keeping the previous / current / next views).  The neighbouring
// columns' samples come from the neighbouring lanes (wave shuffles): a wave loads 64
// consecutive columns and writes the 62 inner ones, its first and last lanes loading the
// halo columns only.
constexpr int kDerivColsPerWave = 62;
__global__ __launch_bounds__(kElemThreads) void k_deriv_lw(KParams p, const float *__restrict__ sino,
                                                           float *__restrict__ g2) {
    const int lane = threadIdx.x & 63;
    const int c = (blockIdx.x * (kElemThreads / 64) + (threadIdx.x >> 6)) * kDerivColsPerWave + lane - 1;
    const bool inc = c >= 0 && c < p.cols;                      // a column of the detector
    const bool out = inc && lane > 0 && lane < 63;              // written by this lane
    const int r = blockIdx.y;
    const long long i0 = (long long)blockIdx.z * kDerivRun;   // first filtered view of the run
    const long long i1 = i0 + kDerivRun < p.n_filt ? i0 + kDerivRun : p.n_filt;
    const size_t rc = (size_t)p.rows * p.cols;
    const float *col = sino + (size_t)r * p.cols + (inc ? c : 0);   // sample (view 0, r, c)
    const float w = p.lw[r];
    long long n = p.first_view + i0;                           // 1 <= n <= n_views-2
    // all of the run's loads issued before the first use
    float x[kDerivRun + 2];
    const int nr = (int)(i1 - i0);
#pragma unroll
    for (int j = 0; j < kDerivRun + 2; ++j) x[j] = (inc && j < nr + 2) ? col[(size_t)(n - 1 + j) * rc] : 0.0f;
#pragma unroll
    for (int j = 0; j < kDerivRun; ++j) {
        // columns c - 1 and c + 1 of view n + j (zero outside the detector: those lanes hold 0)
        const float lf = __shfl_up(x[j + 1], 1, 64), rt = __shfl_down(x[j + 1], 1, 64);
        if (out && j < nr)
            g2[(size_t)(i0 + j) * rc + (size_t)r * p.cols + c] =
                w * ((x[j + 2] - x[j]) * p.inv_2dlam + (rt - lf) * p.inv_2dalpha);
    }
}

// Half-sample derivative: filtered view i (cell-centre view n = first_view + i, between
// sinogram views n and n+1) and column c (between sinogram columns c and c+1).  Each partial
// derivative is the mean of the two forward differences across the 2 x 2 cell; the thread
// loads the two columns of its run of views (plus the next view) before the first use.
__global__ __launch_bounds__(kElemThreads) void k_deriv_lw_half(KParams p, const float *__restrict__ sino,
                                                                float *__restrict__ g2) {
    // a wave loads 64 consecutive sinogram columns and writes the 63 cells between them; the
    // right column of each cell comes from the next lane (wave shuffle)
    const int lane = threadIdx.x & 63;
    const int c = (blockIdx.x * (kElemThreads / 64) + (threadIdx.x >> 6)) * (kDerivColsPerWave + 1) + lane;
    const bool inc = c < p.sino_cols;                          // a sinogram column
    const bool out = lane < 63 && c < p.cols;                  // a cell written by this lane
    const int r = blockIdx.y;
    const long long i0 = (long long)blockIdx.z * kDerivRun;
    const long long i1 = i0 + kDerivRun < p.n_filt ? i0 + kDerivRun : p.n_filt;
    const size_t src = (size_t)p.rows * p.sino_cols;          // sinogram view stride
    const size_t rc = (size_t)p.rows * p.cols;
    const float *col = sino + (size_t)r * p.sino_cols + (inc ? c : 0);   // sinogram (view 0, r, c)
    const float w = p.lw[r];
    long long n = p.first_view + i0;                          // 0 <= n, n+1 <= sino_views-1
    // all of the run's loads issued before the first use
    float x0[kDerivRun + 1];
    const int nr = (int)(i1 - i0);
#pragma unroll
    for (int j = 0; j < kDerivRun + 1; ++j) x0[j] = (inc && j < nr + 1) ? col[(size_t)(n + j) * src] : 0.0f;
    float x1[kDerivRun + 1];
#pragma unroll
    for (int j = 0; j < kDerivRun + 1; ++j) x1[j] = __shfl_down(x0[j], 1, 64);
#pragma unroll
    for (int j = 0; j < kDerivRun; ++j) {
        if (out && j < nr) {
            const float dl = ((x0[j + 1] - x0[j]) + (x1[j + 1] - x1[j])) * p.inv_2dlam;
            const float da = ((x1[j] - x0[j]) + (x1[j + 1] - x0[j + 1])) * p.inv_2dalpha;
            g2[(size_t)(i0 + j) * rc + (size_t)r * p.cols + c] = w * (dl + da);
        }
    }
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 conj2(float2 a) { return make_float2(a.x, -a.y); }
// times -i (forward transform) or +i (inverse)
template <bool INV>
__device__ inline float2 rot(float2 a) { return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }

// ---------------------------------------------------------------------------------
// Hilbert filtering along detector columns (eq. HF) as a zero-padded linear convolution:
// y = IDFT_N(i Im[K^](f) / N * DFT_N(x)), N = fft_len >= 2 cols - 1 (a power of two).
// Two real kappa rows are transformed together as one complex row (real and imaginary
// parts); the kernel spectrum is purely imaginary (odd kernel), so the two stay separate.
//
// Each transform is spread over T = N / 16 threads holding 16 complex values in
// registers.  Stockham radix passes: a radix-R pass of span L maps butterfly i
// (k = i mod L) with inputs x[i + j N/R] (times w_{RL}^{jk}) to outputs at
// (i - k) R + k + m L.  Forward: one radix-RF pass (RF = N / 16^q in {2, 4, 8}, or 16)
// reading the rebinned input straight from global memory, then radix-16 passes; the
// last leaves X[t + m T] in thread t, which is exactly the input distribution of the
// inverse's first radix-16 pass, so the spectrum product needs no exchange.  Inverse:
// radix-16 passes of span 1, 16, ..., then the radix-RF pass writing the result to global
// memory.  Passes exchange through LDS with the bijective swizzle x ^ ((x >> 4) & 31)
// (the exchange patterns are free of bank conflicts up to two-way).  Twiddles are the
// plan's exp(-2 pi i n / N) table, read through the cache.  N >= 2 cols - 1 puts every
// column c >= N / 2 in the zero padding: the edge passes' inputs (and outputs) j >= RF / 2
// are zero (unused) at compile time, so their butterflies drop that half.
// ---------------------------------------------------------------------------------
template <bool INV>
__device__ inline void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 s0 = cadd(a0, a2), d0 = csub(a0, a2);
    const float2 s1 = cadd(a1, a3), d1 = rot<INV>(csub(a1, a3));
    a0 = cadd(s0, s1);
    a2 = csub(s0, s1);
    a1 = cadd(d0, d1);
    a3 = csub(d0, d1);
}

// w_16^e (forward) or its conjugate, e in 0..9 known at compile time
template <bool INV>
__device__ inline float2 tw16(float2 v, int e) {
    constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f;
    constexpr float r2 = 0.707106781186547524f;
    float c = 1.0f, s = 0.0f;           // w = c - i s  (forward)
    switch (e) {
        case 0: return v;
        case 4: return rot<INV>(v);
        case 1: c = c1; s = s1; break;
        case 2: c = r2; s = r2; break;
        case 3: c = s1; s = c1; break;
        case 6: c = -r2; s = r2; break;
        case 9: c = -c1; s = -s1; break;
        default: break;
    }
    return cmul(v, make_float2(c, INV ? s : -s));
}

// In-place DFT of v[0..R-1] in natural order, R in {2, 4, 8, 16}.
template <int R, bool INV>
__device__ inline void dft(float2 *v) {
    if constexpr (R == 2) {
        const float2 a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        // index j = 2 j1 + j2, m = m1 + 4 m2
        float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        o1 = tw16<INV>(o1, 2);          // w_8^1 = w_16^2
        o2 = tw16<INV>(o2, 4);          // w_8^2 = w_16^4
        o3 = tw16<INV>(o3, 6);          // w_8^3 = w_16^6
        v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
    } else {
        static_assert(R == 16, "radix");
        // index j = 4 j1 + j2, m = m1 + 4 m2: DFT4 over j1, twiddle w_16^(j2 m1), DFT4 over j2
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) dft4<INV>(v[j2], v[4 + j2], v[8 + j2], v[12 + j2]);
#pragma unroll
        for (int j2 = 1; j2 < 4; ++j2)
#pragma unroll
            for (int m1 = 1; m1 < 4; ++m1) v[j2 + 4 * m1] = tw16<INV>(v[j2 + 4 * m1], j2 * m1);
#pragma unroll
        for (int m1 = 0; m1 < 4; ++m1) dft4<INV>(v[4 * m1], v[4 * m1 + 1], v[4 * m1 + 2], v[4 * m1 + 3]);
        // y[m1 + 4 m2] now sits in v[4 m1 + m2]: transpose the 4 x 4 index
        float2 t[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) t[m] = v[4 * (m & 3) + (m >> 2)];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = t[m];
    }
}

__device__ inline int fft_swz(int x) { return x ^ ((x >> 4) & 31); }

template <int LOG2N>
struct FftShape {
    static constexpr int N = 1 << LOG2N;
    static constexpr int T = N / 16;                                   // threads per transform
    static constexpr int RF = (LOG2N % 4) ? (1 << (LOG2N % 4)) : 16;   // edge pass radix
    static constexpr int NP16 = (LOG2N - ((LOG2N % 4) ? (LOG2N % 4) : 4)) / 4;
    static constexpr int F = kFftThreads / T;                          // transforms per block
    static_assert(LOG2N >= 6 && LOG2N <= 11, "fft length 64 .. 2048");
};

// Twiddles w^j, j = 1 .. R-1, of w = tw[step] (conjugated for the inverse): the powers
// 1, 2, 4, 8 come from the table, the others are products of at most three of them (a few
// ulp), which trades table reads (latency) for cheap VALU.
template <int R, bool INV>
__device__ inline void twiddles(const float2 *__restrict__ tw, int step, float2 *w) {
    auto ld = [&](int e) { const float2 x = tw[e * step]; return INV ? conj2(x) : x; };
    w[1] = ld(1);
    if constexpr (R > 2) {
        w[2] = ld(2);
        w[3] = cmul(w[2], w[1]);
    }
    if constexpr (R > 4) {
        w[4] = ld(4);
#pragma unroll
        for (int j = 5; j < 8; ++j) w[j] = cmul(w[4], w[j - 4]);
    }
    if constexpr (R > 8) {
        w[8] = ld(8);
#pragma unroll
        for (int j = 9; j < 16; ++j) w[j] = cmul(w[8], w[j - 8]);
    }
}

// A middle radix-16 pass of span L on this thread's butterfly i = t: twiddles then DFT.
template <int LOG2N, bool INV>
__device__ inline void pass16(float2 *v, int t, int L, const float2 *__restrict__ tw) {
    constexpr int N = FftShape<LOG2N>::N;
    const int k = t % L;
    float2 w[16];
    twiddles<16, INV>(tw, k * (N / (16 * L)), w);
#pragma unroll
    for (int j = 1; j < 16; ++j) v[j] = cmul(v[j], w[j]);
    dft<16, INV>(v);
}

// Filter (ADJ = false): rebin kappa rows ka, kb from g2, convolve, write g4.
// Adjoint Hilbert (ADJ = true): rows ka, kb of g4bar convolved with the negated spectrum
// (H^T = -H), in place.
template <int LOG2N, bool ADJ>
__global__ __launch_bounds__(kFftThreads) void k_hilbert_fft(KParams p, const float *__restrict__ g2,
                                                             float *__restrict__ g4) {
    using S = FftShape<LOG2N>;
    constexpr int N = S::N, T = S::T, RF = S::RF, NB = 16 / RF;
    __shared__ float2 lds[S::F * N];
    const int tid = threadIdx.x;
    const int t = tid % T;
    float2 *X = lds + (tid / T) * N;
    const int n_pairs = (p.n_psi + 1) >> 1;
    const long long xf = (long long)blockIdx.x * S::F + tid / T;     // transform index
    const bool live = xf < (long long)p.n_filt * n_pairs;
    const long long i = live ? xf / n_pairs : 0;
    const int ka = live ? 2 * (int)(xf % n_pairs) : 0;
    const int kb = ka + 1;
    const bool has_b = live && kb < p.n_psi;
    const int cols = p.cols, rows = p.rows;
    const float2 *__restrict__ tw = p.twiddle;
    float *row = g4 + (size_t)i * p.n_psi * cols;                     // output / in-place rows
    const float *v2 = g2 + (size_t)i * rows * cols;
    auto rebin = [&](int k, int c) -> float {
        const FrEntry e = p.fr[k * cols + c];
        const int r0 = e.r0;
        const float w = e.w;
        const float x0 = (r0 >= 0 && r0 < rows) ? v2[r0 * cols + c] : 0.0f;
        const float x1 = (r0 + 1 >= 0 && r0 + 1 < rows) ? v2[(r0 + 1) * cols + c] : 0.0f;
        return (1.0f - w) * x0 + w * x1;
    };
    float2 v[16];
    // forward edge pass (span 1): butterflies i = t + T b, inputs x[i + j N/RF]
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int j = 0; j < RF; ++j) {
            const int c = t + T * b + j * (N / RF);
            float a = 0.0f, bb = 0.0f;
            if (j < RF / 2 && live && c < cols) {          // c >= N/2 >= cols for j >= RF/2
                if constexpr (ADJ) {
                    a = row[ka * cols + c];
                    if (has_b) bb = row[kb * cols + c];
                } else {
                    a = rebin(ka, c);
                    if (has_b) bb = rebin(kb, c);
                }
            }
            v[b * RF + j] = make_float2(a, bb);
        }
        dft<RF, false>(v + b * RF);
#pragma unroll
        for (int m = 0; m < RF; ++m) X[fft_swz((t + T * b) * RF + m)] = v[b * RF + m];
    }
    __syncthreads();
    // forward radix-16 passes, span L = RF, 16 RF, ...; the last keeps X[t + m T]
    int L = RF;
#pragma unroll
    for (int q = 0; q < S::NP16; ++q) {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = X[fft_swz(t + j * T)];
        pass16<LOG2N, false>(v, t, L, tw);
        if (q + 1 < S::NP16) {
            __syncthreads();
            const int k = t % L;
#pragma unroll
            for (int m = 0; m < 16; ++m) X[fft_swz((t - k) * 16 + k + m * L)] = v[m];
            __syncthreads();
        }
        L *= 16;
    }
    // spectrum: i * Im[K^](f) / N (negated for the adjoint), f = t + m T
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const float kim = ADJ ? -p.hil_im[t + m * T] : p.hil_im[t + m * T];
        v[m] = make_float2(-v[m].y * kim, v[m].x * kim);
    }
    // inverse radix-16 passes, span 1, 16, ...; the first starts from registers
    L = 1;
#pragma unroll
    for (int q = 0; q < S::NP16; ++q) {
        if (q > 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = X[fft_swz(t + j * T)];
            pass16<LOG2N, true>(v, t, L, tw);
        } else {
            dft<16, true>(v);
        }
        __syncthreads();
        const int k = t % L;
#pragma unroll
        for (int m = 0; m < 16; ++m) X[fft_swz((t - k) * 16 + k + m * L)] = v[m];
        __syncthreads();
        L *= 16;
    }
    // inverse edge pass, span N / RF: butterfly i = t + T b writes y[i + m N/RF]
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int ib = t + T * b;
        float2 w[RF];
        twiddles<RF, true>(tw, ib * (N / (RF * L)), w);
#pragma unroll
        for (int j = 0; j < RF; ++j) {
            const float2 x = X[fft_swz(ib + j * (N / RF))];
            v[b * RF + j] = j > 0 ? cmul(x, w[j]) : x;
        }
        dft<RF, true>(v + b * RF);
        if (live) {
#pragma unroll
            for (int m = 0; m < RF; ++m) {
                const int c = ib + m * (N / RF);
                if (m < RF / 2 && c < cols) {
                    row[ka * cols + c] = v[b * RF + m].x;
                    if (has_b) row[kb * cols + c] = v[b * RF + m].y;
                }
            }
        }
    }
}

template <bool ADJ>
void launch_hilbert(const KParams &k, const float *g2, float *g4, hipStream_t s) {
    const int n_pairs = (k.n_psi + 1) / 2;
    const long long nt = (long long)k.n_filt * n_pairs;
    auto blocks = [&](int log2n) {
        const int f = kFftThreads / ((1 << log2n) / 16);
        return dim3((unsigned)((nt + f - 1) / f));
    };
    switch (k.log2n) {
        case 6: hipLaunchKernelGGL((k_hilbert_fft<6, ADJ>), blocks(6), dim3(kFftThreads), 0, s, k, g2, g4); break;
        case 7: hipLaunchKernelGGL((k_hilbert_fft<7, ADJ>), blocks(7), dim3(kFftThreads), 0, s, k, g2, g4); break;
        case 8: hipLaunchKernelGGL((k_hilbert_fft<8, ADJ>), blocks(8), dim3(kFftThreads), 0, s, k, g2, g4); break;
        case 9: hipLaunchKernelGGL((k_hilbert_fft<9, ADJ>), blocks(9), dim3(kFftThreads), 0, s, k, g2, g4); break;
        case 10: hipLaunchKernelGGL((k_hilbert_fft<10, ADJ>), blocks(10), dim3(kFftThreads), 0, s, k, g2, g4); break;
        default: hipLaunchKernelGGL((k_hilbert_fft<11, ADJ>), blocks(11), dim3(kFftThreads), 0, s, k, g2, g4); break;
    }
}

// Forward height rebinning alone (eq. FR), for the matrix-core Hilbert: one thread per
// (column, group of kRebinLines kappa lines, 4 consecutive views) loads the lines' rebinning
// entries once and forms g3[i][k][c] = (1 - t) g2[i][r0][c] + t g2[i][r0+1][c] view after view,
// each view's loads issued before their first use (coalesced over the block's columns; the
// view's g2 stays in the cache); the block's max |g3| goes to vmax[view / 4][group][column
// block], the Hilbert's range scale (one thread per view and 16 lines: 88 against 80 us per
// 512-view chunk of the clinical workload; 8 or 32 lines per thread were slower).
__global__ __launch_bounds__(kDRThreads) void k_rebin(KParams p, const float *__restrict__ g2,
                                                      float *__restrict__ g3, float *__restrict__ vmax) {
    const long long i0 = (long long)blockIdx.x * kRebinViews;   // first filtered view of the block
    const int c = blockIdx.y * kDRThreads + threadIdx.x;
    const int k0 = blockIdx.z * kRebinLines;
    const int rows = p.rows, cols = p.cols;
    float mx = 0.0f;
    if (c < cols) {
        const FrEntry *fr = p.fr + c;
        FrEntry e[kRebinLines];
#pragma unroll
        for (int j = 0; j < kRebinLines; ++j)
            e[j] = k0 + j < p.n_psi ? fr[(k0 + j) * cols] : FrEntry{-2, 0.0f};
#pragma unroll
        for (int vv = 0; vv < kRebinViews; ++vv) {
            const long long i = i0 + vv;
            if (i >= p.n_filt) break;
            const float *v2 = g2 + (size_t)i * rows * cols + c;
            float *out = g3 + (size_t)i * p.n_psi * cols + c;
            float x0[kRebinLines], x1[kRebinLines];
#pragma unroll
            for (int j = 0; j < kRebinLines; ++j) {
                x0[j] = (e[j].r0 >= 0 && e[j].r0 < rows) ? v2[e[j].r0 * cols] : 0.0f;
                x1[j] = (e[j].r0 + 1 >= 0 && e[j].r0 + 1 < rows) ? v2[(e[j].r0 + 1) * cols] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < kRebinLines; ++j) {
                if (k0 + j < p.n_psi) {
                    const float v = (1.0f - e[j].w) * x0[j] + e[j].w * x1[j];
                    out[(size_t)(k0 + j) * cols] = v;
                    mx = fmaxf(mx, fabsf(v));
                }
            }
        }
    }
    __shared__ float red[kDRThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kDRThreads / 64; ++w) mx = fmaxf(mx, red[w]);
        vmax[((long long)blockIdx.x * gridDim.z + blockIdx.z) * gridDim.y + blockIdx.y] = mx;
    }
}

// Writes the zero-padded view [gf_rows][gf_cols] (border = 0).  One thread per (view,
// padded column, block of rows) takes its rows: successive rows use neighbouring
// kappa-lines of the same column (psi_hat rises with w), which the cache keeps, so g4 is
// read about once.  Views run along x (no 65535 limit), row blocks along z: eight blocks
// of a view's rows keep more short walks in flight than one walk over every row (clinical
// filter 2.32 -> 2.23 ms with the shorter derivative runs), and a block of up to kBrUnroll
// rows issues all its table and tap loads before the first use (1.87 -> 1.79 ms).
__global__ __launch_bounds__(kElemThreads) void k_br_cos(KParams p, const float *__restrict__ g4,
                                                         float *__restrict__ gF) {
    const long long i = blockIdx.x;
    const int cp = blockIdx.y * kElemThreads + threadIdx.x;
    const int pitch = p.gf_cols;
    if (cp >= pitch) return;
    const int rpb = (p.gf_rows + kBrBlocks - 1) / kBrBlocks;
    const int rp0 = blockIdx.z * rpb, rp1 = min(rp0 + rpb, p.gf_rows);
    const int c = cp - kPad;
    const bool incol = (unsigned)c < (unsigned)p.cols;
    float *out = gF + (size_t)i * p.gf_rows * pitch + cp;
    const float *v4 = g4 + (size_t)i * p.n_psi * p.cols + c;
    const float ca = incol ? p.cos_alpha[c] : 0.0f;
    if (rp1 - rp0 <= kBrUnroll) {
        // all table entries, then all taps, in flight before the first use
        int kk[kBrUnroll];
        float tt[kBrUnroll], xa[kBrUnroll], xb[kBrUnroll];
#pragma unroll
        for (int j = 0; j < kBrUnroll; ++j) {
            const int r = rp0 + j - kPad;
            kk[j] = -1;
            tt[j] = 0.0f;
            if (rp0 + j < rp1 && incol && (unsigned)r < (unsigned)p.rows) {
                kk[j] = p.br_k[r * p.cols + c];
                tt[j] = p.br_w[r * p.cols + c];
            }
        }
#pragma unroll
        for (int j = 0; j < kBrUnroll; ++j) {
            xa[j] = kk[j] >= 0 ? v4[kk[j] * p.cols] : 0.0f;
            xb[j] = kk[j] >= 0 ? v4[(kk[j] + 1) * p.cols] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < kBrUnroll; ++j)
            if (rp0 + j < rp1) out[(size_t)(rp0 + j) * pitch] = ca * ((1.0f - tt[j]) * xa[j] + tt[j] * xb[j]);
        return;
    }
    for (int rp = rp0; rp < rp1; ++rp) {
        const int r = rp - kPad;
        float o = 0.0f;
        if (incol && (unsigned)r < (unsigned)p.rows) {
            const int e = r * p.cols + c;
            const int k0 = p.br_k[e];
            const float t = p.br_w[e];
            o = ca * ((1.0f - t) * v4[k0 * p.cols] + t * v4[(k0 + 1) * p.cols]);
        }
        out[(size_t)rp * pitch] = o;
    }
}

// ----------------------------------------------------------------------------- adjoint
// Transposes of the three kernels above, in reverse order.

// BR^T and cos: g4bar[k, c] = sum over rows r with k0[r,c] in {k-1, k} of the weights times
// cos(alpha_c) gFbar[r, c].  One thread per (view, column) walks all rows (deterministic).
// k0 does not decrease along a column (psi_hat rises with w on the monotone branch), so the
// walk keeps the two kappa-lines it is filling (K, K + 1) in registers and writes every line
// once (the lines no row touches as zeros), the rows' table entries and samples loaded
// kBrTRows at a time before their use.  (A version accumulating in LDS needs three passes
// over the rows for 129 kappa-lines and measured 1.31 ms against 0.92 ms for a walk adding
// into HBM on the clinical workload.)
constexpr int kBrTRows = 16;
__global__ __launch_bounds__(kElemThreads) void k_br_cos_T(KParams p, const float *__restrict__ gFbar,
                                                           float *__restrict__ g4bar) {
    const long long i = blockIdx.x;
    const int c = blockIdx.y * kElemThreads + threadIdx.x;
    if (c >= p.cols) return;
    const float *src = gFbar + (size_t)i * p.rows * p.cols;
    float *dst = g4bar + (size_t)i * p.n_psi * p.cols + c;
    const float ca = p.cos_alpha[c];
    int K = 0;                 // lines below K are written
    int nxt = 0;               // first line not yet written (K, or K + 2 once P, Q hold K, K + 1)
    float P = 0.0f, Q = 0.0f;  // pending sums of lines K and K + 1 (valid when nxt == K + 2)
    for (int r0 = 0; r0 < p.rows; r0 += kBrTRows) {
        int kk[kBrTRows];
        float tt[kBrTRows], vv[kBrTRows];
#pragma unroll
        for (int j = 0; j < kBrTRows; ++j) {
            const int r = r0 + j;
            const bool ok = r < p.rows;
            const int e = (ok ? r : 0) * p.cols + c;
            kk[j] = ok ? p.br_k[e] : -1;
            tt[j] = ok ? p.br_w[e] : 0.0f;
            vv[j] = ok ? src[e] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < kBrTRows; ++j) {
            const int k0 = kk[j];
            if (k0 < 0) break;
            const float v = ca * vv[j];
            const float t = tt[j];
            if (nxt == K + 2 && k0 == K) {
                P += (1.0f - t) * v;
                Q += t * v;
                continue;
            }
            if (nxt == K + 2) {                           // lines K, K + 1 are complete or move on
                dst[(size_t)K * p.cols] = P;
                if (k0 == K + 1) {
                    P = Q + (1.0f - t) * v;
                    Q = t * v;
                    K = k0;
                    nxt = K + 2;
                    continue;
                }
                dst[(size_t)(K + 1) * p.cols] = Q;
            }
            for (int k = nxt; k < k0; ++k) dst[(size_t)k * p.cols] = 0.0f;   // untouched lines
            P = (1.0f - t) * v;
            Q = t * v;
            K = k0;
            nxt = K + 2;
        }
    }
    if (nxt == K + 2) {
        dst[(size_t)K * p.cols] = P;
        dst[(size_t)(K + 1) * p.cols] = Q;
    }
    for (int k = nxt; k < p.n_psi; ++k) dst[(size_t)k * p.cols] = 0.0f;
}

// FR^T + LW scatters along a detector column: one wave takes 64 columns of one view and each
// lane accumulates its own column in LDS (no sharing, no atomics), in chunks of kAccRows
// detector rows, then writes every output element once (1.12 ms against 1.50 ms for a
// read-modify-write walk in HBM on the clinical workload); the kappa-lines' table entries and
// samples are loaded 16 at a time before their use (whole clinical adjoint 44.5 -> 43.9 ms).
constexpr int kColWave = 64;
constexpr int kAccRows = 64;
constexpr int kFrTLines = 16;

// FR^T + LW: g2bar[r, c] = lw[r] * sum over kappa-lines k whose row pair (r0, r0+1) touches r
// of the weight times g3bar[k, c].
__global__ __launch_bounds__(kColWave) void k_fr_lw_T(KParams p, const float *__restrict__ g3bar,
                                                      float *__restrict__ g2bar) {
    __shared__ float acc[kAccRows * kColWave];
    const long long i = blockIdx.x;
    const int lane = threadIdx.x;
    const int c = blockIdx.y * kColWave + lane;
    if (c >= p.cols) return;
    const float *src = g3bar + (size_t)i * p.n_psi * p.cols + c;
    float *dst = g2bar + (size_t)i * p.rows * p.cols + c;
    for (int r0c = 0; r0c < p.rows; r0c += kAccRows) {
        for (int r = 0; r < kAccRows; ++r) acc[r * kColWave + lane] = 0.0f;
        // groups of kFrTLines kappa-lines: their table entries and samples loaded before use
        for (int k0 = 0; k0 < p.n_psi; k0 += kFrTLines) {
            FrEntry e[kFrTLines];
            float v[kFrTLines];
#pragma unroll
            for (int u = 0; u < kFrTLines; ++u) {
                const int k = k0 + u;
                const bool ok = k < p.n_psi;
                e[u] = ok ? p.fr[k * p.cols + c] : FrEntry{-(kAccRows + 2), 0.0f};
                v[u] = ok ? src[(size_t)k * p.cols] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kFrTLines; ++u) {
                const int r0 = e[u].r0 - r0c;
                const float t = e[u].w;
                if ((unsigned)r0 < (unsigned)kAccRows) acc[r0 * kColWave + lane] += (1.0f - t) * v[u];
                if ((unsigned)(r0 + 1) < (unsigned)kAccRows) acc[(r0 + 1) * kColWave + lane] += t * v[u];
            }
        }
        const int rn = min(kAccRows, p.rows - r0c);
        for (int r = 0; r < rn; ++r)
            dst[(size_t)(r0c + r) * p.cols] = acc[r * kColWave + lane] * p.lw[r0c + r];
    }
}

// Deriv^T gathered per sinogram sample: gsino[n, r, c] =
//   (g2bar[n-1] - g2bar[n+1]) / (2 dlambda) + (g2bar[c-1] - g2bar[c+1]) / (2 dalpha)
// over the filtered views (views outside contribute 0).  Every sinogram sample is written.
__global__ __launch_bounds__(kElemThreads) void k_deriv_T(KParams p, const float *__restrict__ g2bar,
                                                          float *__restrict__ gsino, long long n0, long long count) {
    // one thread per (row, column, run of kDerivRun sinogram views): the run's samples of
    // g2-bar (one view each side more) loaded first, the neighbouring columns from the
    // neighbouring lanes (a wave loads 64 columns and writes the 62 inner ones)
    const int lane = threadIdx.x & 63;
    const int c = (blockIdx.z * (kElemThreads / 64) + (threadIdx.x >> 6)) * kDerivColsPerWave + lane - 1;
    const bool inc = c >= 0 && c < p.cols;
    const bool out = inc && lane > 0 && lane < 63;
    const int r = blockIdx.y;
    const long long m0 = (long long)blockIdx.x * kDerivRun;    // first view of the run within the call
    const int nr = (int)(count - m0 < kDerivRun ? count - m0 : kDerivRun);
    const size_t rc = (size_t)p.rows * p.cols;
    const float *col = g2bar + (size_t)r * p.cols + (inc ? c : 0);
    float x[kDerivRun + 2];                     // filtered views n - 1 .. n + kDerivRun, n = n0 + m0
#pragma unroll
    for (int j = 0; j < kDerivRun + 2; ++j) {
        const long long i = n0 + m0 - 1 + j - p.first_view;
        x[j] = (inc && j < nr + 2 && i >= 0 && i < p.n_filt) ? col[(size_t)i * rc] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kDerivRun; ++j) {
        const float lf = __shfl_up(x[j + 1], 1, 64), rt = __shfl_down(x[j + 1], 1, 64);
        if (out && j < nr)
            gsino[(size_t)(n0 + m0 + j) * rc + (size_t)r * p.cols + c] =
                (x[j] - x[j + 2]) * p.inv_2dlam + (lf - rt) * p.inv_2dalpha;
    }
}

// Transpose of the half-sample derivative (LW^T is applied by k_fr_lw_T): sinogram
// sample (n, r, c) belongs to the cells (n-1 .. n) x (c-1 .. c) of the filtered grid.
__global__ __launch_bounds__(kElemThreads) void k_deriv_T_half(KParams p, const float *__restrict__ g2bar,
                                                               float *__restrict__ gsino, long long n0) {
    const long long n = n0 + blockIdx.x;            // sinogram view
    const int r = blockIdx.y;
    const int c = blockIdx.z * kElemThreads + threadIdx.x;
    if (c >= p.sino_cols) return;
    const size_t rc = (size_t)p.rows * p.cols;
    auto at = [&](long long view, int col) -> float {
        const long long i = view - p.first_view;
        if (i < 0 || i >= p.n_filt || col < 0 || col >= p.cols) return 0.0f;
        return g2bar[(size_t)i * rc + (size_t)r * p.cols + col];
    };
    const float a = p.inv_2dlam, b = p.inv_2dalpha;
    const float v = (b - a) * at(n, c - 1) - (a + b) * at(n, c) + (a + b) * at(n - 1, c - 1) +
                    (a - b) * at(n - 1, c);
    gsino[((size_t)n * p.rows + r) * p.sino_cols + c] = v;
}

}  // namespace

hipError_t launch_filter(const KParams &k, const float *sino, float *g2, float *g4, float *gF,
                         float *vmax, hipStream_t s) {
    if (k.n_filt <= 0) return hipSuccess;
    const unsigned runs = (unsigned)((k.n_filt + kDerivRun - 1) / kDerivRun);
    if (k.half) {
        const int per_block = (kDerivColsPerWave + 1) * (kElemThreads / 64);
        hipLaunchKernelGGL(k_deriv_lw_half, dim3((k.cols + per_block - 1) / per_block, k.rows, runs),
                           dim3(kElemThreads), 0, s, k, sino, g2);
    } else {
        const int per_block = kDerivColsPerWave * (kElemThreads / 64);
        hipLaunchKernelGGL(k_deriv_lw, dim3((k.cols + per_block - 1) / per_block, k.rows, runs),
                           dim3(kElemThreads), 0, s, k, sino, g2);
    }
    if (k.hil_mode == KATS_HILBERT_MFMA) {
        const dim3 grid((unsigned)((k.n_filt + kRebinViews - 1) / kRebinViews), (unsigned)((k.cols + kDRThreads - 1) / kDRThreads),
                        (unsigned)((k.n_psi + kRebinLines - 1) / kRebinLines));
        hipLaunchKernelGGL(k_rebin, grid, dim3(kDRThreads), 0, s, k, g2, g4, vmax);
        const hipError_t e = launch_hilbert_mfma(k, g4, vmax, s);
        if (e != hipSuccess) return e;
    } else {
        launch_hilbert<false>(k, g2, g4, s);
    }
    const int cbp = (k.gf_cols + kElemThreads - 1) / kElemThreads;
    hipLaunchKernelGGL(k_br_cos, dim3((unsigned)k.n_filt, cbp, kBrBlocks), dim3(kElemThreads), 0, s, k, g4, gF);
    return hipGetLastError();
}

hipError_t launch_filter_T_views(const KParams &k, const float *gFbar, float *g4bar, float *g2bar,
                                 hipStream_t s) {
    if (k.n_filt <= 0) return hipSuccess;
    const int cb = (k.cols + kElemThreads - 1) / kElemThreads;
    const unsigned cw = (unsigned)((k.cols + kColWave - 1) / kColWave);
    hipLaunchKernelGGL(k_br_cos_T, dim3((unsigned)k.n_filt, cb), dim3(kElemThreads), 0, s, k, gFbar, g4bar);
    launch_hilbert<true>(k, nullptr, g4bar, s);
    hipLaunchKernelGGL(k_fr_lw_T, dim3((unsigned)k.n_filt, cw), dim3(kColWave), 0, s, k, g4bar, g2bar);
    return hipGetLastError();
}

hipError_t launch_deriv_T(const KParams &k, const float *g2bar, float *gsino, long long n0,
                          long long count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (k.half) {
        const int cbs = (k.sino_cols + kElemThreads - 1) / kElemThreads;
        hipLaunchKernelGGL(k_deriv_T_half, dim3((unsigned)count, k.rows, cbs), dim3(kElemThreads), 0, s, k,
                           g2bar, gsino, n0);
    } else {
        const int per_block = kDerivColsPerWave * (kElemThreads / 64);
        hipLaunchKernelGGL(k_deriv_T, dim3((unsigned)((count + kDerivRun - 1) / kDerivRun), k.rows,
                                           (unsigned)((k.cols + per_block - 1) / per_block)),
                           dim3(kElemThreads), 0, s, k, g2bar, gsino, n0, count);
    }
    return hipGetLastError();
}

hipError_t launch_filter_T(const KParams &k, const float *gFbar, float *g4bar, float *g2bar,
                           float *gsino, hipStream_t s) {
    hipError_t e = launch_filter_T_views(k, gFbar, g4bar, g2bar, s);
    if (e != hipSuccess) return e;
    return launch_deriv_T(k, g2bar, gsino, 0, k.half ? k.sino_views : k.n_views, s);
}

}  // namespace kats

namespace kats {

namespace {
__global__ __launch_bounds__(256) void k_zero(float4 *__restrict__ p, size_t n4) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}
}  // namespace

// Fill kernel (used instead of hipMemsetAsync so that callers may capture the stream).
hipError_t launch_zero(void *ptr, uint64_t bytes, hipStream_t s) {
    const size_t n4 = bytes / 16;                    // buffers are 256-byte multiples
    if (n4 == 0) return hipSuccess;
    size_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<float4 *>(ptr), n4);
    return hipGetLastError();
}

}  // namespace kats
