// Filtering kernels of the Katsevich reconstruction for gfx950 (Sec. II steps 1-6):
//   k_deriv_lw    derivative at constant direction (eq. Deriv) + length weighting (eq. LW)
//   k_fr_hilbert  forward height rebinning onto two kappa-lines (eqs. FR, w_k) packed as one
//                 complex row, then the Hilbert transform in alpha (eq. HF, kernel of e4) as a
//                 zero-padded linear convolution by LDS Stockham FFTs
//   k_br_cos      backward height rebinning (eq. BR) + post-cosine weighting (eq. PW)
// All kernels are HBM-streaming: one pass over their input and output, coalesced along
// detector columns.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kats {

namespace {

constexpr int kElemThreads = 256;
constexpr int kFftThreads = 256;

__global__ __launch_bounds__(kElemThreads) void k_deriv_lw(KParams p, const float *__restrict__ sino,
                                                           float *__restrict__ g2) {
    const long long i = blockIdx.x;                 // filtered view index
    const int r = blockIdx.y;
    const int c = blockIdx.z * kElemThreads + threadIdx.x;
    if (c >= p.cols) return;
    const long long n = p.first_view + i;           // 1 <= n <= n_views-2 by construction
    const size_t rc = (size_t)p.rows * p.cols;
    const float *gm = sino + (size_t)(n - 1) * rc + (size_t)r * p.cols;
    const float *g0 = gm + rc;
    const float *gp = g0 + rc;
    const float dl = (gp[c] - gm[c]) * p.inv_2dlam;
    const float left = c > 0 ? g0[c - 1] : 0.0f;
    const float right = c + 1 < p.cols ? g0[c + 1] : 0.0f;
    const float da = (right - left) * p.inv_2dalpha;
    g2[(size_t)i * rc + (size_t)r * p.cols + c] = p.lw[r] * (dl + da);
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Stockham autosort FFT of length N = 2^log2n in LDS (radix-2 first pass when log2n is
// odd, then radix-4).  X holds the input; returns the buffer holding the output.
// tw[k] = exp(-2 pi i k / N); the inverse uses conjugate twiddles and +i rotations
// (no 1/N: that factor is folded into the Hilbert spectrum).
template <bool kInverse>
__device__ float2 *fft_lds(float2 *X, float2 *Y, const float2 *tw, int N, int log2n) {
    const int tid = threadIdx.x;
    int p = 1;
    if (log2n & 1) {
        const int half = N >> 1;
        for (int i = tid; i < half; i += kFftThreads) {
            const int k = i & (p - 1);
            float2 w = tw[k * (N / (2 * p))];
            if (kInverse) w.y = -w.y;
            const float2 u0 = X[i];
            const float2 u1 = cmul(X[i + half], w);
            const int j = ((i - k) << 1) + k;
            Y[j] = make_float2(u0.x + u1.x, u0.y + u1.y);
            Y[j + p] = make_float2(u0.x - u1.x, u0.y - u1.y);
        }
        __syncthreads();
        float2 *t = X; X = Y; Y = t;
        p = 2;
    }
    const int q = N >> 2;
    while (p < N) {
        const int s = N / (4 * p);
        for (int i = tid; i < q; i += kFftThreads) {
            const int k = i & (p - 1);
            float2 w1 = tw[k * s], w2 = tw[2 * k * s], w3 = tw[3 * k * s];
            if (kInverse) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
            const float2 u0 = X[i];
            const float2 u1 = cmul(X[i + q], w1);
            const float2 u2 = cmul(X[i + 2 * q], w2);
            const float2 u3 = cmul(X[i + 3 * q], w3);
            const float2 a0 = make_float2(u0.x + u2.x, u0.y + u2.y);
            const float2 a1 = make_float2(u0.x - u2.x, u0.y - u2.y);
            const float2 a2 = make_float2(u1.x + u3.x, u1.y + u3.y);
            const float2 d = make_float2(u1.x - u3.x, u1.y - u3.y);
            const float2 a3 = kInverse ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
            const int j = ((i - k) << 2) + k;
            Y[j] = make_float2(a0.x + a2.x, a0.y + a2.y);
            Y[j + p] = make_float2(a1.x + a3.x, a1.y + a3.y);
            Y[j + 2 * p] = make_float2(a0.x - a2.x, a0.y - a2.y);
            Y[j + 3 * p] = make_float2(a1.x - a3.x, a1.y - a3.y);
        }
        __syncthreads();
        float2 *t = X; X = Y; Y = t;
        p <<= 2;
    }
    return X;
}

// One block = one filtered view x one pair of kappa-lines (k_a = 2*pair, k_b = k_a + 1).
__global__ __launch_bounds__(kFftThreads) void k_fr_hilbert(KParams p, const float *__restrict__ g2,
                                                            float *__restrict__ g4) {
    extern __shared__ float2 lds[];
    const int N = p.fft_len;
    float2 *bufA = lds;
    float2 *bufB = lds + N;
    float2 *tw = lds + 2 * N;
    const int n_pairs = (p.n_psi + 1) >> 1;
    const long long i = blockIdx.x / n_pairs;
    const int ka = 2 * (int)(blockIdx.x % n_pairs);
    const int kb = ka + 1;
    const bool has_b = kb < p.n_psi;
    const int tid = threadIdx.x;
    for (int k = tid; k < N; k += kFftThreads) tw[k] = p.twiddle[k];
    const float *v2 = g2 + (size_t)i * p.rows * p.cols;
    for (int c = tid; c < N; c += kFftThreads) {
        float a = 0.0f, b = 0.0f;
        if (c < p.cols) {
            {
                const int r0 = p.fr_row[ka * p.cols + c];
                const float t = p.fr_w[ka * p.cols + c];
                const float x0 = (r0 >= 0 && r0 < p.rows) ? v2[r0 * p.cols + c] : 0.0f;
                const float x1 = (r0 + 1 >= 0 && r0 + 1 < p.rows) ? v2[(r0 + 1) * p.cols + c] : 0.0f;
                a = (1.0f - t) * x0 + t * x1;
            }
            if (has_b) {
                const int r0 = p.fr_row[kb * p.cols + c];
                const float t = p.fr_w[kb * p.cols + c];
                const float x0 = (r0 >= 0 && r0 < p.rows) ? v2[r0 * p.cols + c] : 0.0f;
                const float x1 = (r0 + 1 >= 0 && r0 + 1 < p.rows) ? v2[(r0 + 1) * p.cols + c] : 0.0f;
                b = (1.0f - t) * x0 + t * x1;
            }
        }
        bufA[c] = make_float2(a, b);
    }
    __syncthreads();
    float2 *Z = fft_lds<false>(bufA, bufB, tw, N, p.log2n);
    float2 *other = (Z == bufA) ? bufB : bufA;
    // multiply by the purely imaginary kernel spectrum i * Im[f] (1/N folded in)
    for (int f = tid; f < N; f += kFftThreads) {
        const float kim = p.hil_im[f];
        const float2 z = Z[f];
        Z[f] = make_float2(-z.y * kim, z.x * kim);
    }
    __syncthreads();
    float2 *Y = fft_lds<true>(Z, other, tw, N, p.log2n);
    float *out = g4 + (size_t)i * p.n_psi * p.cols;
    for (int c = tid; c < p.cols; c += kFftThreads) {
        const float2 y = Y[c];
        out[ka * p.cols + c] = y.x;
        if (has_b) out[kb * p.cols + c] = y.y;
    }
}

// Writes the zero-padded view [gf_rows][gf_cols] (border = 0).
__global__ __launch_bounds__(kElemThreads) void k_br_cos(KParams p, const float *__restrict__ g4,
                                                         float *__restrict__ gF) {
    const long long i = blockIdx.x;
    const int rp = blockIdx.y;
    const int cp = blockIdx.z * kElemThreads + threadIdx.x;
    const int pitch = p.gf_cols;
    if (cp >= pitch) return;
    const int r = rp - kPad, c = cp - kPad;
    float out = 0.0f;
    if ((unsigned)r < (unsigned)p.rows && (unsigned)c < (unsigned)p.cols) {
        const int e = r * p.cols + c;
        const int k0 = p.br_k[e];
        const float t = p.br_w[e];
        const float *v4 = g4 + (size_t)i * p.n_psi * p.cols;
        const float a = v4[k0 * p.cols + c];
        const float b = v4[(k0 + 1) * p.cols + c];
        out = p.cos_alpha[c] * ((1.0f - t) * a + t * b);
    }
    gF[((size_t)i * p.gf_rows + rp) * pitch + cp] = out;
}

// ----------------------------------------------------------------------------- adjoint
// Transposes of the three kernels above, in reverse order.

// BR^T and cos: g4bar[k, c] = sum over rows r with k0[r,c] in {k-1, k} of the weights times
// cos(alpha_c) gFbar[r, c].  One thread per (view, column) walks all rows (deterministic).
__global__ __launch_bounds__(kElemThreads) void k_br_cos_T(KParams p, const float *__restrict__ gFbar,
                                                           float *__restrict__ g4bar) {
    const long long i = blockIdx.x;
    const int c = blockIdx.y * kElemThreads + threadIdx.x;
    if (c >= p.cols) return;
    const float *src = gFbar + (size_t)i * p.rows * p.cols;
    float *dst = g4bar + (size_t)i * p.n_psi * p.cols;
    for (int k = 0; k < p.n_psi; ++k) dst[k * p.cols + c] = 0.0f;
    const float ca = p.cos_alpha[c];
    for (int r = 0; r < p.rows; ++r) {
        const int e = r * p.cols + c;
        const int k0 = p.br_k[e];
        const float t = p.br_w[e];
        const float v = ca * src[e];
        dst[k0 * p.cols + c] += (1.0f - t) * v;
        dst[(k0 + 1) * p.cols + c] += t * v;
    }
}

// H^T = -H: the same FFT convolution with the negated spectrum, then FR^T (scatter of the
// two kappa rows into detector rows is done by k_fr_T below, so this kernel only writes
// g3bar in place of g4bar).
__global__ __launch_bounds__(kFftThreads) void k_hilbert_T(KParams p, float *__restrict__ g4bar) {
    extern __shared__ float2 lds[];
    const int N = p.fft_len;
    float2 *bufA = lds;
    float2 *bufB = lds + N;
    float2 *tw = lds + 2 * N;
    const int n_pairs = (p.n_psi + 1) >> 1;
    const long long i = blockIdx.x / n_pairs;
    const int ka = 2 * (int)(blockIdx.x % n_pairs);
    const int kb = ka + 1;
    const bool has_b = kb < p.n_psi;
    const int tid = threadIdx.x;
    for (int k = tid; k < N; k += kFftThreads) tw[k] = p.twiddle[k];
    float *row = g4bar + (size_t)i * p.n_psi * p.cols;
    for (int c = tid; c < N; c += kFftThreads) {
        float a = 0.0f, b = 0.0f;
        if (c < p.cols) {
            a = row[ka * p.cols + c];
            if (has_b) b = row[kb * p.cols + c];
        }
        bufA[c] = make_float2(a, b);
    }
    __syncthreads();
    float2 *Z = fft_lds<false>(bufA, bufB, tw, N, p.log2n);
    float2 *other = (Z == bufA) ? bufB : bufA;
    for (int f = tid; f < N; f += kFftThreads) {
        const float kim = -p.hil_im[f];
        const float2 z = Z[f];
        Z[f] = make_float2(-z.y * kim, z.x * kim);
    }
    __syncthreads();
    float2 *Y = fft_lds<true>(Z, other, tw, N, p.log2n);
    for (int c = tid; c < p.cols; c += kFftThreads) {
        const float2 y = Y[c];
        row[ka * p.cols + c] = y.x;
        if (has_b) row[kb * p.cols + c] = y.y;
    }
}

// FR^T + LW: g2bar[r, c] = lw[r] * sum over kappa-lines k whose row pair (r0, r0+1) touches r
// of the weight times g3bar[k, c].  One thread per (view, column) walks all kappa-lines.
__global__ __launch_bounds__(kElemThreads) void k_fr_lw_T(KParams p, const float *__restrict__ g3bar,
                                                          float *__restrict__ g2bar) {
    const long long i = blockIdx.x;
    const int c = blockIdx.y * kElemThreads + threadIdx.x;
    if (c >= p.cols) return;
    const float *src = g3bar + (size_t)i * p.n_psi * p.cols;
    float *dst = g2bar + (size_t)i * p.rows * p.cols;
    for (int r = 0; r < p.rows; ++r) dst[r * p.cols + c] = 0.0f;
    for (int k = 0; k < p.n_psi; ++k) {
        const int r0 = p.fr_row[k * p.cols + c];
        const float t = p.fr_w[k * p.cols + c];
        const float v = src[k * p.cols + c];
        if (r0 >= 0 && r0 < p.rows) dst[r0 * p.cols + c] += (1.0f - t) * v;
        if (r0 + 1 >= 0 && r0 + 1 < p.rows) dst[(r0 + 1) * p.cols + c] += t * v;
    }
    for (int r = 0; r < p.rows; ++r) dst[r * p.cols + c] *= p.lw[r];
}

// Deriv^T gathered per sinogram sample: gsino[n, r, c] =
//   (g2bar[n-1] - g2bar[n+1]) / (2 dlambda) + (g2bar[c-1] - g2bar[c+1]) / (2 dalpha)
// over the filtered views (views outside contribute 0).  Every sinogram sample is written.
__global__ __launch_bounds__(kElemThreads) void k_deriv_T(KParams p, const float *__restrict__ g2bar,
                                                          float *__restrict__ gsino) {
    const long long n = blockIdx.x;                 // every sinogram view
    const int r = blockIdx.y;
    const int c = blockIdx.z * kElemThreads + threadIdx.x;
    if (c >= p.cols) return;
    const size_t rc = (size_t)p.rows * p.cols;
    auto at = [&](long long view, int col) -> float {
        const long long i = view - p.first_view;
        if (i < 0 || i >= p.n_filt || col < 0 || col >= p.cols) return 0.0f;
        return g2bar[(size_t)i * rc + (size_t)r * p.cols + col];
    };
    const float vl = (at(n - 1, c) - at(n + 1, c)) * p.inv_2dlam;
    const float va = (at(n, c - 1) - at(n, c + 1)) * p.inv_2dalpha;
    gsino[(size_t)n * rc + (size_t)r * p.cols + c] = vl + va;
}

}  // namespace

hipError_t launch_filter(const KParams &k, const float *sino, float *g2, float *g4, float *gF,
                         hipStream_t s) {
    if (k.n_filt <= 0) return hipSuccess;
    const int cb = (k.cols + kElemThreads - 1) / kElemThreads;
    hipLaunchKernelGGL(k_deriv_lw, dim3((unsigned)k.n_filt, k.rows, cb), dim3(kElemThreads), 0, s,
                       k, sino, g2);
    const int n_pairs = (k.n_psi + 1) / 2;
    const size_t lds = (size_t)3 * k.fft_len * sizeof(float2);
    hipLaunchKernelGGL(k_fr_hilbert, dim3((unsigned)(k.n_filt * n_pairs)), dim3(kFftThreads), lds, s,
                       k, g2, g4);
    const int cbp = (k.gf_cols + kElemThreads - 1) / kElemThreads;
    hipLaunchKernelGGL(k_br_cos, dim3((unsigned)k.n_filt, k.gf_rows, cbp), dim3(kElemThreads),
                       0, s, k, g4, gF);
    return hipGetLastError();
}

hipError_t launch_filter_T(const KParams &k, const float *gFbar, float *g4bar, float *g2bar,
                           float *gsino, hipStream_t s) {
    const int cb = (k.cols + kElemThreads - 1) / kElemThreads;
    if (k.n_filt > 0) {
        hipLaunchKernelGGL(k_br_cos_T, dim3((unsigned)k.n_filt, cb), dim3(kElemThreads), 0, s, k,
                           gFbar, g4bar);
        const int n_pairs = (k.n_psi + 1) / 2;
        const size_t lds = (size_t)3 * k.fft_len * sizeof(float2);
        hipLaunchKernelGGL(k_hilbert_T, dim3((unsigned)(k.n_filt * n_pairs)), dim3(kFftThreads), lds,
                           s, k, g4bar);
        hipLaunchKernelGGL(k_fr_lw_T, dim3((unsigned)k.n_filt, cb), dim3(kElemThreads), 0, s, k,
                           g4bar, g2bar);
    }
    hipLaunchKernelGGL(k_deriv_T, dim3((unsigned)k.n_views, k.rows, cb), dim3(kElemThreads), 0, s,
                       k, g2bar, gsino);
    return hipGetLastError();
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
