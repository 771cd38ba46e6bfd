// Device helpers and the launch arguments shared by the backprojector (bp.hip) and its
// adjoint (bp_adjoint.hip): both walk the same 16 x 16 voxel tiles, slice runs, PI-window
// hulls and footprint boxes of the plan.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace kats {
namespace bpdev {

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

constexpr int kT = kBpTile;       // 16
constexpr int kNT = kT * kT;      // 256 lanes
constexpr int kLP = kBpBoxCols;   // LDS tile row pitch (floats) = max box columns
// LDS tile depth (max box rows) of a slice run: runs of 32 slices span up to ~60 detector
// rows, shorter runs fit 32.
template <int KZ>
constexpr int lds_rows() { return KZ >= 32 ? 2 * kBpBoxRows : kBpBoxRows; }
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

inline BpArgs bp_args(const KParams &k) {
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

// A footprint box as stored by the plan: two dwords {r0 | nr << 16, c0 | nc << 16}.
__device__ inline BpBox unpack_box(uint2 w) {
    BpBox b;
    b.r0 = (int16_t)(w.x & 0xffffu);
    b.nr = (int16_t)(w.x >> 16);
    b.c0 = (int16_t)(w.y & 0xffffu);
    b.nc = (int16_t)(w.y >> 16);
    return b;
}

}  // namespace bpdev
}  // namespace kats
