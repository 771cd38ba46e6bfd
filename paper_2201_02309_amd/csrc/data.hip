// Data path of the paper's sparse-detector experiments (Sec. III-C) and its image metrics
// (Sec. IV): keep every step-th detector column, interpolate the sinogram back to the full
// column grid, simulate photon and electronic noise, and compare a reconstruction with a
// reference by RMSE and SSIM.
//
//   k_upsample   linear interpolation in alpha between the kept columns (the last kept
//                column is held beyond its position)
//   k_noise      counts = I0 exp(-g/M) + sqrt(.) z1 + sqrt(var) z2 (Poisson counts by their
//                normal limit, Gaussian electronic noise), g_in = M log(I0 / counts);
//                z1, z2 through the Box-Muller transform from one Philox4x64-10 block per
//                pair of elements (counter = pair index, key = (seed, 0)): words 0, 1 for
//                the even element, 2, 3 for the odd one
//   k_max_*, k_moments_*  deterministic two-level reductions (block partials in caller
//                scratch, then one block in a fixed order), float64 accumulation
// All kernels are elementwise or reductions that stream their inputs once.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.hpp"

// Bytes of reduction scratch: 4096 block partials of 5 doubles, then 5 doubles of moments,
// rounded up to 256 bytes.
constexpr unsigned long long kDataScratchBytes = 4096ull * 5 * sizeof(double) + 256;

// Library-owned reduction scratch for callers that cannot allocate device memory: one
// copy per GPU (each device's code object holds its own), held until the process ends.
// In host code this name is only a shadow of the device array, never its address:
// kats::static_scratch() looks the address up once per device and returns it.
static __device__ __align__(256) unsigned char scratch[kDataScratchBytes];
static_assert(kDataScratchBytes == KATS_STATIC_SCRATCH_BYTES, "header size of the static scratch");

namespace kats {

namespace {

constexpr int kThreads = 256;
typedef float F4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- upsampling
// Thread q takes output columns 4p .. 4p+3 (p = q mod slots) of line q / slots: one 32-bit
// division per thread, the kept-column index advanced incrementally, one 16-byte store
// (non-temporal) when rows of the output are 16-byte aligned (cols a multiple of 4).  With
// step 4 (the paper's decimation) the four columns lie between kept columns p and p + 1, so
// two loads serve them; the arithmetic is the general path's.
__global__ __launch_bounds__(kThreads) void k_upsample(const float *__restrict__ sp, float *__restrict__ full,
                                                       unsigned lines, int cols, int ns, int step) {
    const unsigned slots = ((unsigned)cols + 3u) / 4u;
    const unsigned long long total = (unsigned long long)lines * slots;   // < 2^32 (host check)
    const bool vec = (cols & 3) == 0 && ((uintptr_t)full & 15) == 0;
    const float inv_step = 1.0f / (float)step;
    // the loop index is 64-bit: with a total just below 2^32 a 32-bit index would wrap on
    // its last stride and never reach the bound; inside the loop it is below 2^32, so the
    // line / slot split stays a 32-bit division
    const unsigned long long stride = (unsigned long long)gridDim.x * kThreads;
    for (unsigned long long qq = (unsigned long long)blockIdx.x * kThreads + threadIdx.x; qq < total;
         qq += stride) {
        const unsigned q = (unsigned)qq;
        const unsigned line = q / slots;
        const int c0 = (int)(q - line * slots) * 4;
        const float *s = sp + (size_t)line * ns;
        float v[4];
        if (step == 4) {
            const int j = c0 >> 2;
            if (j + 1 < ns) {
                const float a = s[j], d = s[j + 1] - a;
#pragma unroll
                for (int t = 0; t < 4; ++t) v[t] = fmaf((float)t * inv_step, d, a);
            } else {
                const float h = s[ns - 1];
#pragma unroll
                for (int t = 0; t < 4; ++t) v[t] = h;
            }
        } else {
            int j = c0 / step, k = c0 - j * step;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (j + 1 < ns) {
                    const float a = s[j], b = s[j + 1];
                    v[t] = fmaf((float)k * inv_step, b - a, a);
                } else {
                    v[t] = s[ns - 1];
                }
                if (++k == step) {
                    k = 0;
                    ++j;
                }
            }
        }
        float *o = full + (size_t)line * cols + c0;
        if (vec) {      // streaming store: the output is not read again here
            const F4 w = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(w, reinterpret_cast<F4 *>(o));
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (c0 + t < cols) o[t] = v[t];
        }
    }
}

// ---------------------------------------------------------------- Philox4x64-10
struct U64x4 {
    uint64_t v[4];
};

// Full 128-bit product hi:lo of two 64-bit words from four 32 x 32 -> 64 products, each
// carry folded into the next product's addend (one v_mad_u64_u32 apiece): with t = a0 b1 +
// hi(a0 b0) and u = a1 b0 + lo(t), a b = lo(a0 b0) + 2^32 u + 2^64 (a1 b1 + hi(t)).
__device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;
    lo = (u << 32) | (uint32_t)p00;
    hi = (uint64_t)a1 * b1 + ((t >> 32) + (u >> 32));
}

// Philox4x64 with 10 rounds (Salmon et al., SC'11): round multipliers 0xD2E7470EE14C6C93 and
// 0xCA5A826395121157, key increments (Weyl) 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B.
__device__ inline U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ull, c.v[0], hi0, lo0);
        mulhilo64(0xCA5A826395121157ull, c.v[2], hi1, lo1);
        U64x4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    return c;
}

// One pair of elements per thread.  Transcendentals are the hardware's: v_log_f32 (log2),
// v_exp_f32 (2^x), v_sin_f32 / v_cos_f32 (argument in turns), v_rcp_f32, v_sqrt_f32 (its
// arguments here are 0 or normal: -2 ln u1 in [0, 33.3], lambda >= I0 / e).
__device__ inline float noisy_value(float g, uint64_t w0, uint64_t w1, float M, float inv_M_log2e, float I0,
                                    float sd_e) {
    const float u1 = (float)((w0 >> 40) + 1) * 5.9604644775390625e-8f;     // (0, 1]
    const float u2 = (float)(w1 >> 40) * 5.9604644775390625e-8f;           // [0, 1)
    const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));   // sqrt(-2 ln u1)
    const float z1 = rho * __builtin_amdgcn_cosf(u2), z2 = rho * __builtin_amdgcn_sinf(u2);
    const float lam = I0 * __builtin_amdgcn_exp2f(-g * inv_M_log2e);
    float counts = fmaf(__builtin_amdgcn_sqrtf(lam), z1, lam) + sd_e * z2;
    counts = fmaxf(counts, 1.0f);
    return M * 0.69314718055994531f * __builtin_amdgcn_logf(I0 * __builtin_amdgcn_rcpf(counts));
}

__global__ __launch_bounds__(kThreads) void k_noise(const float *__restrict__ in, float *__restrict__ out,
                                                    unsigned long long n, const float *__restrict__ d_max,
                                                    float I0, float sd_e, uint64_t seed) {
    const unsigned long long pr = (unsigned long long)blockIdx.x * kThreads + threadIdx.x;
    const unsigned long long e = 2 * pr;
    if (e >= n) return;
    const float M = *d_max;
    const float inv_M_log2e = 1.4426950408889634f / M;
    U64x4 ctr;
    ctr.v[0] = pr;
    ctr.v[1] = 0;
    ctr.v[2] = 0;
    ctr.v[3] = 0;
    const U64x4 x = philox4x64_10(ctr, seed, 0);
    if (e + 1 < n && ((uintptr_t)(in + e) & 7) == 0 && ((uintptr_t)(out + e) & 7) == 0) {
        const float2 g = *reinterpret_cast<const float2 *>(in + e);
        *reinterpret_cast<float2 *>(out + e) =
            make_float2(noisy_value(g.x, x.v[0], x.v[1], M, inv_M_log2e, I0, sd_e),
                        noisy_value(g.y, x.v[2], x.v[3], M, inv_M_log2e, I0, sd_e));
    } else {
        out[e] = noisy_value(in[e], x.v[0], x.v[1], M, inv_M_log2e, I0, sd_e);
        if (e + 1 < n) out[e + 1] = noisy_value(in[e + 1], x.v[2], x.v[3], M, inv_M_log2e, I0, sd_e);
    }
}

// ---------------------------------------------------------------- reductions
constexpr int kRedBlocks = 4096;     // partials per reduction (5 doubles each in scratch)
static_assert((unsigned long long)kRedBlocks * 5 * sizeof(double) + 5 * sizeof(double) <= kDataScratchBytes,
              "reduction scratch too small");

__device__ inline double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

__device__ inline float block_max(float v, float *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__global__ __launch_bounds__(kThreads) void k_max_partial(const float *__restrict__ x, unsigned long long n,
                                                          float *__restrict__ part) {
    __shared__ float sh[4];
    float m = -INFINITY;
    const unsigned long long stride = (unsigned long long)gridDim.x * kThreads;
    const unsigned long long t0 = (unsigned long long)blockIdx.x * kThreads + threadIdx.x;
    if (((uintptr_t)x & 15) == 0) {                 // 16-byte loads, then the tail
        const unsigned long long n4 = n / 4;
        for (unsigned long long q = t0; q < n4; q += stride) {
            const float4 v = reinterpret_cast<const float4 *>(x)[q];
            m = fmaxf(m, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
        }
        for (unsigned long long i = n4 * 4 + t0; i < n; i += stride) m = fmaxf(m, x[i]);
    } else {
        for (unsigned long long i = t0; i < n; i += stride) m = fmaxf(m, x[i]);
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(kThreads) void k_max_final(const float *__restrict__ part, int np,
                                                        float *__restrict__ out) {
    __shared__ float sh[4];
    float m = -INFINITY;
    for (int i = threadIdx.x; i < np; i += kThreads) m = fmaxf(m, part[i]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) *out = m;
}

// pass 1 (mu == nullptr): sum f, sum g, sum (f-g)^2, min g, max g
// pass 2: sum (f-mu_f)^2, sum (g-mu_g)^2, sum (f-mu_f)(g-mu_g)
__global__ __launch_bounds__(kThreads) void k_moments_partial(const float *__restrict__ f,
                                                              const float *__restrict__ g,
                                                              unsigned long long n,
                                                              const double *__restrict__ mu,
                                                              double *__restrict__ part) {
    __shared__ double sh[4];
    __shared__ float shf[4];
    double a = 0.0, b = 0.0, c = 0.0;
    float lo = INFINITY, hi = -INFINITY;
    const double mf = mu ? mu[0] : 0.0, mg = mu ? mu[1] : 0.0;
    for (unsigned long long i = (unsigned long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * kThreads) {
        const double x = f[i], y = g[i];
        if (!mu) {
            a += x;
            b += y;
            c += (x - y) * (x - y);
            lo = fminf(lo, g[i]);
            hi = fmaxf(hi, g[i]);
        } else {
            a += (x - mf) * (x - mf);
            b += (y - mg) * (y - mg);
            c += (x - mf) * (y - mg);
        }
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    c = block_sum(c, sh);
    lo = -block_max(-lo, shf);
    hi = block_max(hi, shf);
    if (threadIdx.x == 0) {
        double *p = part + (size_t)blockIdx.x * 5;
        p[0] = a;
        p[1] = b;
        p[2] = c;
        p[3] = lo;
        p[4] = hi;
    }
}

// out: pass 1 -> mu[0..1] = means, stats[0] = sum (f-g)^2, stats[1..2] = min/max g;
//      pass 2 -> RMSE and SSIM into result[0..1]
__global__ __launch_bounds__(kThreads) void k_moments_final(const double *__restrict__ part, int np,
                                                            unsigned long long n, int pass,
                                                            double *__restrict__ mu,
                                                            double *__restrict__ result) {
    __shared__ double sh[4];
    __shared__ float shf[4];
    double a = 0.0, b = 0.0, c = 0.0;
    float lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < np; i += kThreads) {
        const double *p = part + (size_t)i * 5;
        a += p[0];
        b += p[1];
        c += p[2];
        lo = fminf(lo, (float)p[3]);
        hi = fmaxf(hi, (float)p[4]);
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    c = block_sum(c, sh);
    lo = -block_max(-lo, shf);
    hi = block_max(hi, shf);
    if (threadIdx.x != 0) return;
    const double dn = (double)n;
    if (pass == 1) {
        mu[0] = a / dn;
        mu[1] = b / dn;
        mu[2] = c;            // sum of squared differences
        mu[3] = lo;
        mu[4] = hi;
        return;
    }
    const double vf = a / dn, vg = b / dn, cov = c / dn;
    const double range = mu[4] - mu[3];
    const double c1 = (0.01 * range) * (0.01 * range), c2 = (0.03 * range) * (0.03 * range);
    result[0] = sqrt(mu[2] / dn);
    result[1] = (2.0 * mu[0] * mu[1] + c1) * (2.0 * cov + c2) /
                ((mu[0] * mu[0] + mu[1] * mu[1] + c1) * (vf + vg + c2));
}

int red_blocks(unsigned long long n) {
    const unsigned long long b = (n + kThreads * 16ull - 1) / (kThreads * 16ull);
    return (int)(b < 1 ? 1 : (b > (unsigned long long)kRedBlocks ? kRedBlocks : b));
}

}  // namespace

uint64_t data_scratch_bytes() { return kDataScratchBytes; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void **out, uint64_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {                      // first call on this device, device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_upsample(const float *sp, float *full, long long lines, int cols, int ns, int step,
                           hipStream_t s) {
    if (lines <= 0 || cols <= 0) return hipSuccess;
    const unsigned long long slots = ((unsigned long long)cols + 3) / 4;
    if ((unsigned long long)lines * slots >= (1ull << 32)) return hipErrorInvalidValue;
    const unsigned long long q = ((unsigned long long)lines * slots + kThreads - 1) / kThreads;
    const unsigned blocks = (unsigned)(q > 16384 ? 16384 : q);
    hipLaunchKernelGGL(k_upsample, dim3(blocks), dim3(kThreads), 0, s, sp, full, (unsigned)lines, cols, ns,
                       step);
    return hipGetLastError();
}

hipError_t launch_max(const float *x, unsigned long long n, float *out, void *scratch, hipStream_t s) {
    const int nb = red_blocks(n);
    float *part = static_cast<float *>(scratch);
    hipLaunchKernelGGL(k_max_partial, dim3(nb), dim3(kThreads), 0, s, x, n, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kThreads), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_noise(const float *in, float *out, unsigned long long n, const float *d_max, float I0,
                        float sd_e, uint64_t seed, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned long long pairs = (n + 1) / 2;
    hipLaunchKernelGGL(k_noise, dim3((unsigned)((pairs + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       in, out, n, d_max, I0, sd_e, seed);
    return hipGetLastError();
}

hipError_t launch_rmse_ssim(const float *f, const float *g, unsigned long long n, double *result,
                            void *scratch, hipStream_t s) {
    const int nb = red_blocks(n);
    double *part = static_cast<double *>(scratch);
    double *mu = part + (size_t)kRedBlocks * 5;           // 5 doubles after the partials
    hipLaunchKernelGGL(k_moments_partial, dim3(nb), dim3(kThreads), 0, s, f, g, n, (const double *)nullptr, part);
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(kThreads), 0, s, (const double *)part, nb, n, 1, mu,
                       result);
    hipLaunchKernelGGL(k_moments_partial, dim3(nb), dim3(kThreads), 0, s, f, g, n, (const double *)mu, part);
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(kThreads), 0, s, (const double *)part, nb, n, 2, mu,
                       result);
    return hipGetLastError();
}

}  // namespace kats
