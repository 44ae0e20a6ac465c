// Device helpers shared by the kernel files of the library: complex FP64
// arithmetic with every fused multiply-add written out (the library is
// compiled with -ffp-contract=off, so all launch shapes round identically),
// the work-group reduction of inner products, vector-plane offsets, DPP
// wavefront shifts, per-row buffer resources and the constants of the
// marching strips.
#pragma once

#include "kpm_internal.h"

namespace kpm {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// The library is compiled with -ffp-contract=off: every fused multiply-add
// below is written out, so all launch shapes round identically.
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
// s + a * b
__device__ __forceinline__ double2 cmla(double2 s, double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, s.x)), fma(a.x, b.y, fma(a.y, b.x, s.y)));
}
// a * b
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return cmla(make_double2(0.0, 0.0), a, b);
}
// s + conj(a) * b
__device__ __forceinline__ double2 cdot_acc(double2 s, double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, s.x)), fma(a.x, b.y, fma(-a.y, b.x, s.y)));
}
// s + h * x  (real h)
__device__ __forceinline__ double2 raxpy(double2 s, double h, double2 x) {
    return make_double2(fma(h, x.x, s.x), fma(h, x.y, s.y));
}
// 2 a - b
__device__ __forceinline__ double2 two_minus(double2 a, double2 b) {
    return make_double2(fma(2.0, a.x, -b.x), fma(2.0, a.y, -b.y));
}

// Block-wide segmented sum: lane l holds a value for vector l % R; the R
// sums of the work-group go to dst[0 .. R-1].  Fixed order.
__device__ __forceinline__ void block_sum(double2 s, int vshift, double2 *dst) {
    __shared__ double2 red[kBlock / kWave][kWave];
    const int r = 1 << vshift;
    for (int off = kWave / 2; off >= r; off >>= 1) {
        s.x += __shfl_down(s.x, off, kWave);
        s.y += __shfl_down(s.y, off, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    __syncthreads();                        // red may still be read by a previous call
    if (lane < r) red[wv][lane] = s;
    __syncthreads();
    if ((int)threadIdx.x < r) {
        double2 t = red[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < kBlock / kWave; ++q) t = cadd(t, red[q][threadIdx.x]);
        dst[threadIdx.x] = t;
    }
}

// The sum over the work-group of one value per lane (any number of
// wavefronts up to kMaxStripBlock / kWave) into dst[0].  Fixed order.
__device__ __forceinline__ void block_sum_waves(double2 s, double2 *dst) {
    __shared__ double2 red[kMaxStripBlock / kWave];
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        s.x += __shfl_down(s.x, off, kWave);
        s.y += __shfl_down(s.y, off, kWave);
    }
    const int nw = (int)blockDim.x / kWave;
    __syncthreads();                        // red may still be read by a previous call
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t = red[0];
        for (int q = 1; q < nw; ++q) t = cadd(t, red[q]);
        dst[0] = t;
    }
}

// Vector-major states: the element offset of this group's plane, a state
// pointer moved to it (null stays null), and the index of the group's
// partial of `slot` in [slot][nwg][planes] (times the vectors per row).
__device__ __forceinline__ int64_t plane_off(const Sweep &sw) {
    return (int64_t)blockIdx.y * sw.pstride;
}
template <typename T>
__device__ __forceinline__ T *on_plane(T *p, int64_t off) {
    return p ? p + off : p;
}
__device__ __forceinline__ int64_t part_index(const Sweep &sw, int slot) {
    return ((int64_t)slot * sw.nwg + blockIdx.x) * gridDim.y + blockIdx.y;
}

__device__ __forceinline__ int wrap_index(int x, int n) {
    return x < 0 ? x + n : (x >= n ? x - n : x);
}

// Cross-lane moves by one lane as DPP wavefront shifts (one VALU move per
// 32-bit half, no LDS): wave_shr:1 gives lane l the value of lane l - 1,
// wave_shl:1 that of lane l + 1; the end lane, which has no source, reads 0
// (bound_ctrl), so the move needs no copy of its old value.  End lanes are
// halo lanes of every tile: their values are never used.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true),
                            __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ double2 lane_prev(double2 v) {     // value of lane l - 1
    return make_double2(dpp_move<kDppWaveShr1>(v.x), dpp_move<kDppWaveShr1>(v.y));
}
__device__ __forceinline__ double2 lane_next(double2 v) {     // value of lane l + 1
    return make_double2(dpp_move<kDppWaveShl1>(v.x), dpp_move<kDppWaveShl1>(v.y));
}

// Row accesses of the register tiles: one buffer resource per row (a
// wave-uniform base and the row's byte size, so out-of-row offsets read 0 and
// drop stores) and the lane's byte offset in the row, shared by all rows.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufWord3 = 0x00020000;     // raw 32-bit access, gfx9 buffer resource
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ double2 buf_ld(const double2 *row, uint32_t bytes, uint32_t off) {
    const d2v v = __builtin_bit_cast(
        d2v, __builtin_amdgcn_raw_buffer_load_b128(row_rsrc(row, bytes), (int)off, 0, 0));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 buf_ld(const float2 *row, uint32_t bytes, uint32_t off) {
    const f2v v = __builtin_bit_cast(
        f2v, __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row, bytes), (int)off, 0, 0));
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void buf_st(double2 *row, uint32_t bytes, uint32_t off, double2 x) {
    d2v v;
    v.x = x.x;
    v.y = x.y;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), row_rsrc(row, bytes),
                                           (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(float2 *row, uint32_t bytes, uint32_t off, double2 x) {
    f2v v;
    v.x = (float)x.x;
    v.y = (float)x.y;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), row_rsrc(row, bytes),
                                          (int)off, 0, 0);
}

constexpr int kStateRing = 6;
constexpr int kRowRing = kMarchRows;
constexpr int kDs = 3;
constexpr uint32_t kOffNone = 0x80000000u;   // past the end of every row

// MODE: kMarchDirect (moments <phi_L|phi_{n+s}>), kMarchDirectRe (their real
// parts only, for callers that use no more: the same real parts, bit for
// bit), kMarchDoubled (the two doubling sums per level, phi_L unused) or
// kMarchBessel (the propagator's accumulator: lacc holds acc, updated acc +=
// c_{n+s} phi_{n+s} at each level in step order and stored after level K; no
// inner products).
constexpr int kMarchDirect = 0, kMarchDoubled = 1, kMarchBessel = 2, kMarchDirectRe = 3;

// The sample a work-group of the marching strips sweeps: its first row, chain
// length nx, chains ny, chains per strip J, the group's index among the
// sample's nwg groups, and the sample's t / E_s and 1 / E_s (one-sample
// systems: the lattice geometry and the sweep's single segment; batches: the
// group's segment, whose strips take one vector per row).
struct StripGeo {
    int64_t e0;
    int nx, ny, J, lb, nwg;
    double t, inv_es;
};
__device__ __forceinline__ StripGeo strip_geo(const Sweep &sw, const Lat2 &lat) {
    if (!sw.seg)
        return StripGeo{0, lat.nx, lat.ny, lat.tj, (int)blockIdx.x, sw.nwg, sw.one.t,
                        sw.one.inv_es};
    const Seg g = sw.seg[sw.wg_seg[blockIdx.x]];
    return StripGeo{g.e0, g.snx, (int)((g.e1 - g.e0) / g.snx), g.sj, (int)blockIdx.x - g.g0,
                    g.nwg, g.t, g.inv_es};
}

}  // namespace kpm
