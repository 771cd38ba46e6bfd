// Hilbert filtering along detector columns (eq. HF with the kernel of e4) as a dense Toeplitz
// product on the matrix cores: the alternative to the register FFT of filter.hip, selected by
// the plan's hilbert_mode.
//
// The kernel's taps K[m] vanish for even m, so outputs at even columns depend only on inputs
// at odd columns and the reverse.  With u[d] = K[2d + 1], x_e[j] = x[2j], x_o[j] = x[2j + 1]:
//     y[2j]     = sum_j' u[j - j' - 1] x_o[j'],      y[2j + 1] = sum_j' u[j - j'] x_e[j'],
// two Toeplitz products of half the width (half the multiply-adds of the full Toeplitz
// matrix).  Every kappa row of a chunk is one row of the GEMM operand A; the Toeplitz
// matrices are the operand B.
//
// Precision.  Float32 operands are split into float16 pairs, v = hi + lo with
// hi = fp16(v), lo = fp16(v - hi) (22 significant bits), and each product is
// hi_x hi_u + hi_x lo_u + lo_x hi_u with float32 accumulation (the dropped lo_x lo_u is 2^-22
// of the product).  Ranges: each group of kappa rows (16 lines of 4 views) is scaled by a
// power of two 2^-E with max |x| < 2^E over the group, so |x 2^-E| < 1; the taps come from
// the plan scaled by 2^14 (|K| <= 2/pi, so no float16 overflow and the smallest taps keep
// normal low halves).  The outputs are scaled back by exact powers of two.
//
// Layout.  A workgroup of 8 waves takes tiles of kMT = 32 kappa rows (persistent over the
// chunk's tiles, two workgroups per CU).  Waves 0-3 form the even outputs (A = x_o), waves 4-7
// the odd ones (A = x_e); each wave owns a quarter of the NP = 128 F padded outputs, F
// fragments of 32 columns of the tile's rows: F 32 x 32 float32 accumulators.  K runs in
// chunks of 64 (four v_mfma_f32_32x32x16_f16 steps) through double-buffered LDS tiles of the
// split rows.  Measured on the clinical filter: chunks of 32 were 0.04 ms slower (twice the
// barriers); tiles of 64 rows (two 32-row fragments per wave, B fragments read once for
// both, but 254 VGPRs and one workgroup per CU) 0.06 ms slower.
// The B fragments are read from the reversed tap sequence in LDS: a lane's 8 consecutive K
// entries of one column are 8 consecutive reversed taps, and 8 copies of that sequence
// shifted by 0..7 make every such read one aligned 16-byte load.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kats {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef _Float16 half4v __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMT = kHilTileRows; // kappa rows per tile
constexpr int kMF = kMT / 32;     // 32-row fragments per wave
constexpr int kRPT = kMT / 32;    // staging rows per thread (16 threads per row)
constexpr int kHT = 512;         // threads per workgroup (8 waves)
constexpr int kKC = 64;          // K chunk (four 16-deep MFMA steps)
constexpr int kAP = 72;          // LDS row pitch of the A tiles in halves: 144 bytes, so the
                                 // 16-byte fragment reads of 8 consecutive rows cover all banks

template <int F>
struct HilShape {
    static constexpr int NP = 128 * F;            // padded outputs per parity = padded K
    static constexpr int LQ = 2 * NP + 32;        // reversed taps: q = Q0 - d for u[d]
    static constexpr int Q0 = NP + 7;
    static constexpr int NCH = NP / kKC;          // K chunks
    // copy stride in halves; in bytes 16 (mod 128), so the 8 copies start 4 banks apart
    static constexpr int US = (((2 * LQ - 16) + 127) / 128 * 128 + 16) / 2;
};

template <int F>
struct HilShared {
    __attribute__((aligned(16))) _Float16 a[2][4][kMT * kAP];   // stage x {x_e hi, lo, x_o hi, lo}
    __attribute__((aligned(16))) _Float16 u[2][8][HilShape<F>::US];
    float iscale[kMT], oscale[kMT];
};

// 2^E with max |x| < 2^E from the bits of a non-negative float maximum, E in [-125, 127]
__device__ inline int scale_exponent(unsigned bits) {
    const int e = (int)((bits >> 23) & 0xffu) - 126;
    return e < -125 ? -125 : (e > 127 ? 127 : e);
}

// In place on the rebinned kappa rows g4 [rows of the chunk][cols]; rmax: max |g3| per (4
// views, group of kRebinLines lines, block of kDRThreads columns).  A tile's rows are read
// completely (through LDS) before any of them is written.
template <int F>
__global__ __launch_bounds__(kHT, 4) void k_hilbert_mfma(KParams p, float *__restrict__ g4,
                                                      const float *__restrict__ rmax) {
    using H = HilShape<F>;
    __shared__ HilShared<F> S;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int cols = p.cols;
    const long long nrows = p.n_filt * (long long)p.n_psi;
    const long long ntiles = (nrows + kMT - 1) / kMT;
    const int nvb = (cols + kDRThreads - 1) / kDRThreads;   // maxima per (view, line group)
    const int ngr = (p.n_psi + kRebinLines - 1) / kRebinLines;

    // taps: 8 shifted copies of the reversed sequence, split into halves
    for (int e = tid; e < 8 * H::LQ; e += kHT) {
        const int s = e / H::LQ, q = e - s * H::LQ;
        const float v = q + s < H::LQ ? p.hil_u[q + s] : 0.0f;
        const _Float16 h = (_Float16)v;
        S.u[0][s][q] = h;
        S.u[1][s][q] = (_Float16)(v - (float)h);
    }

    // staging role: 8 consecutive columns (four of each parity) of rows rg + 32 rr, rr < kRPT
    const int sq = tid & 15, rg = tid >> 4;
    const bool vec = (cols & 3) == 0;             // rows 16-byte aligned: float4 loads
    // compute role
    const int par = wave >> 2;                    // 0: even outputs from x_o; 1: odd from x_e
    const int quarter = wave & 3;
    const int ab = par == 0 ? 2 : 0;              // A arrays
    const int delta = par == 0 ? 1 : 0;
    const int kl0 = 8 * (lane >> 5);              // the lane's first K within a 16-step
    const int nl = lane & 31;

    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long R0 = tile * kMT;
        if (tid < kMT) {
            const long long R = R0 + tid;
            float is = 0.0f, os = 0.0f;
            if (R < nrows) {
                const long long i = R / p.n_psi;
                const long long grp = (i / kRebinViews) * ngr + (R - i * p.n_psi) / kRebinLines;
                float m = 0.0f;
                for (int j = 0; j < nvb; ++j) m = fmaxf(m, rmax[grp * nvb + j]);
                const int E = scale_exponent(__float_as_uint(m));
                is = ldexpf(1.0f, -E);
                os = ldexpf(p.hil_uinv, E);
            }
            S.iscale[tid] = is;
            S.oscale[tid] = os;
        }
        const float *srow[kRPT];
        bool rok[kRPT];
#pragma unroll
        for (int rr = 0; rr < kRPT; ++rr) {
            const long long R = R0 + rg + 32 * rr;
            rok[rr] = R < nrows;
            srow[rr] = g4 + (rok[rr] ? R : 0) * cols;
        }
        __syncthreads();
        float isc[kRPT];
#pragma unroll
        for (int rr = 0; rr < kRPT; ++rr) isc[rr] = S.iscale[rg + 32 * rr];

        // staging, pipelined over the K chunks: chunk ch + 1 is loaded before chunk ch's
        // products and scaled, split and stored into the other LDS buffer after them
        float x[kRPT][8];
        auto load = [&](int ch) {
            const int c0 = ch * 2 * kKC + 8 * sq;
#pragma unroll
            for (int rr = 0; rr < kRPT; ++rr) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c1 = c0 + 4 * h;
                    if (vec && rok[rr] && c1 + 3 < cols) {
                        const float4 v = *reinterpret_cast<const float4 *>(srow[rr] + c1);
                        x[rr][4 * h + 0] = v.x; x[rr][4 * h + 1] = v.y; x[rr][4 * h + 2] = v.z; x[rr][4 * h + 3] = v.w;
                    } else {
#pragma unroll
                        for (int cc = 0; cc < 4; ++cc)
                            x[rr][4 * h + cc] = (rok[rr] && c1 + cc < cols) ? srow[rr][c1 + cc] : 0.0f;
                    }
                }
            }
        };
        auto store = [&](int b) {
#pragma unroll
            for (int rr = 0; rr < kRPT; ++rr) {
                float v[8];
#pragma unroll
                for (int cc = 0; cc < 8; ++cc) v[cc] = x[rr][cc] * isc[rr];
                half4v hi_e, lo_e, hi_o, lo_o;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const _Float16 he = (_Float16)v[2 * j], ho = (_Float16)v[2 * j + 1];
                    hi_e[j] = he;
                    lo_e[j] = (_Float16)(v[2 * j] - (float)he);
                    hi_o[j] = ho;
                    lo_o[j] = (_Float16)(v[2 * j + 1] - (float)ho);
                }
                const int o = (rg + 32 * rr) * kAP + 4 * sq;
                *reinterpret_cast<half4v *>(&S.a[b][0][o]) = hi_e;
                *reinterpret_cast<half4v *>(&S.a[b][1][o]) = lo_e;
                *reinterpret_cast<half4v *>(&S.a[b][2][o]) = hi_o;
                *reinterpret_cast<half4v *>(&S.a[b][3][o]) = lo_o;
            }
        };

        f32x16 acc[kMF][F];
#pragma unroll
        for (int mf = 0; mf < kMF; ++mf)
#pragma unroll
            for (int nf = 0; nf < F; ++nf) acc[mf][nf] = (f32x16){};

        // one 16-deep K step from buffer b
        auto kstep = [&](int b, int ch, int ks) {
            const int kl = ks * 16 + kl0;
            half8 ah[kMF], al[kMF];
#pragma unroll
            for (int mf = 0; mf < kMF; ++mf) {
                const int o = (mf * 32 + nl) * kAP + kl;
                ah[mf] = *reinterpret_cast<const half8 *>(&S.a[b][ab][o]);
                al[mf] = *reinterpret_cast<const half8 *>(&S.a[b][ab + 1][o]);
            }
            const int kg = ch * kKC + kl;
#pragma unroll
            for (int nf = 0; nf < F; ++nf) {
                const int qs = H::Q0 - ((quarter * F + nf) * 32 + nl) + kg + delta;
                const int s = qs & 7, qq = qs - s;
                const half8 bh = *reinterpret_cast<const half8 *>(&S.u[0][s][qq]);
                const half8 bl = *reinterpret_cast<const half8 *>(&S.u[1][s][qq]);
#pragma unroll
                for (int mf = 0; mf < kMF; ++mf)
                    acc[mf][nf] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mf], bh, acc[mf][nf], 0, 0, 0);
#pragma unroll
                for (int mf = 0; mf < kMF; ++mf)
                    acc[mf][nf] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mf], bl, acc[mf][nf], 0, 0, 0);
#pragma unroll
                for (int mf = 0; mf < kMF; ++mf)
                    acc[mf][nf] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[mf], bh, acc[mf][nf], 0, 0, 0);
            }
        };

        load(0);
        store(0);
        __syncthreads();
#pragma unroll 1
        for (int ch = 0; ch < H::NCH; ++ch) {
            const int b = ch & 1;
            const bool more = ch + 1 < H::NCH;
            if (more) load(ch + 1);
            kstep(b, ch, 0);
            kstep(b, ch, 1);
            kstep(b, ch, 2);
            kstep(b, ch, 3);
            if (more) store(b ^ 1);
            __syncthreads();
        }

        // accumulator element i of a lane: row 8 (i / 4) + 4 (lane / 32) + i % 4, column lane % 32
        // (staging the results through LDS for 16-byte stores measured no faster)
#pragma unroll
        for (int mf = 0; mf < kMF; ++mf)
#pragma unroll
            for (int nf = 0; nf < F; ++nf) {
                const int c = 2 * ((quarter * F + nf) * 32 + nl) + par;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int m = mf * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                    const long long R = R0 + m;
                    if (R < nrows && c < cols) g4[R * cols + c] = acc[mf][nf][i] * S.oscale[m];
                }
            }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_hilbert_mfma(const KParams &k, float *g4, const float *rmax, hipStream_t s) {
    const long long ntiles = (k.n_filt * (long long)k.n_psi + kMT - 1) / kMT;
    if (ntiles <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)(ntiles < kHilBlocks ? ntiles : kHilBlocks);
    switch (k.hil_f) {
        case 1: hipLaunchKernelGGL(k_hilbert_mfma<1>, dim3(blocks), dim3(kHT), 0, s, k, g4, rmax); break;
        case 2: hipLaunchKernelGGL(k_hilbert_mfma<2>, dim3(blocks), dim3(kHT), 0, s, k, g4, rmax); break;
        case 3: hipLaunchKernelGGL(k_hilbert_mfma<3>, dim3(blocks), dim3(kHT), 0, s, k, g4, rmax); break;
        case 4: hipLaunchKernelGGL(k_hilbert_mfma<4>, dim3(blocks), dim3(kHT), 0, s, k, g4, rmax); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kats
