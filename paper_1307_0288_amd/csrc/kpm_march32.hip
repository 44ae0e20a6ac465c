// Marching strips with the recursion in FP32 registers (precision KPM_FP32:
// FP32 states and FP32 recursion arithmetic; inner products and moments in
// FP64).
//
// The walk is that of march_sweep in kpm_kernels.hip: a wavefront walks a
// strip of (64 - 2K) columns chain by chain, level s = 1 .. K of the
// recursion on row t - s at iteration t, each level keeping its last three
// rows in registers, and the branch-free loop body loads rows past the window
// as zeros.  What differs is the arithmetic of a level: phi_{n+s} = 2 H~
// phi_{n+s-1} - phi_{n+s-2} in single precision, in the slot order of the
// FP64 form (on-site term, previous column, next column, previous chain, next
// chain), from float weights t / E_s and on-site terms eps / E_s.  A state
// value is then two 32-bit registers instead of four, the horizontal
// neighbours take two DPP moves instead of four, and the new state needs no
// rounding back from double.  Inner products take the exact FP64 product of
// two floats (phi_L is widened where it is used) and accumulate in FP64; the
// propagator's accumulator acc +=
// c_m phi_m is FP32 (the state it becomes is stored in FP32 either way).
#include "kpm_device.h"

namespace kpm {
namespace {

// s + h * x (real h), written as fused multiply-adds
__device__ __forceinline__ float2 fraxpy(float2 s, float h, float2 x) {
    return make_float2(fmaf(h, x.x, s.x), fmaf(h, x.y, s.y));
}
// s + x * h with the lane-shifted operand x first: the DPP move that
// produces it can then become the FMA's own DPP operand
__device__ __forceinline__ float2 fraxpy_shifted(float2 s, float2 x, float h) {
    return make_float2(fmaf(x.x, h, s.x), fmaf(x.y, h, s.y));
}
// 2 a - b
__device__ __forceinline__ float2 ftwo_minus(float2 a, float2 b) {
    return make_float2(fmaf(2.0f, a.x, -b.x), fmaf(2.0f, a.y, -b.y));
}
// s + a * b (complex)
__device__ __forceinline__ float2 fcmla(float2 s, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, s.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, s.y)));
}

template <int CTRL>
__device__ __forceinline__ float dpp_movef(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float2 lane_prevf(float2 v) {      // value of lane l - 1
    return make_float2(dpp_movef<kDppWaveShr1>(v.x), dpp_movef<kDppWaveShr1>(v.y));
}
__device__ __forceinline__ float2 lane_nextf(float2 v) {      // value of lane l + 1
    return make_float2(dpp_movef<kDppWaveShl1>(v.x), dpp_movef<kDppWaveShl1>(v.y));
}

__device__ __forceinline__ float2 buf_ldf(const float2 *row, uint32_t bytes, uint32_t off) {
    const f2v v = __builtin_bit_cast(
        f2v, __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row, bytes), (int)off, 0, 0));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void buf_stf(float2 *row, uint32_t bytes, uint32_t off, float2 x) {
    f2v v;
    v.x = x.x;
    v.y = x.y;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), row_rsrc(row, bytes),
                                          (int)off, 0, 0);
}

template <bool ONSF, int MODE, int K>
__device__ __forceinline__ void march_sweep_f32(const Ell &h, const Sweep &sw, const Lat2 &lat,
                                                const float2 *p1, const float2 *p0,
                                                float2 *__restrict__ out1,
                                                float2 *__restrict__ out2,
                                                float2 *__restrict__ lacc,
                                                double2 *__restrict__ partial, int slot,
                                                const CoefK &ck) {
    constexpr bool DBL = MODE == kMarchDoubled, BES = MODE == kMarchBessel,
                   RE = MODE == kMarchDirectRe;
    // the group's sample (the whole system, or its segment of a batch); row
    // pointers start at the sample's first row of this group's plane
    const StripGeo geo = strip_geo(sw, lat);
    const int64_t po = plane_off(sw) + geo.e0;
    p1 = on_plane(p1, po);
    p0 = on_plane(p0, po);
    out1 = on_plane(out1, po);
    out2 = on_plane(out2, po);
    lacc = on_plane(lacc, po);
    // the per-row structure (the strips' pattern ids, on-site terms) is
    // addressed from the kernel arguments plus the sample's first row, which
    // keeps no further pointers live in scalar registers
    const int64_t e0 = geo.e0;
    constexpr int TC = kWave - 2 * K;                  // columns per strip
    // states are prefetched 6 rows ahead (a ring of 12 rows: two 32-bit
    // registers per row, where the FP64 form affords 3 ahead in 6)
    constexpr int P = kRowRing, PS = 12, DS = 6, DR = kRowRing - 1 - K;
    constexpr int DL = DS < DR ? DS : DR;              // rows of phi_L loaded ahead
    constexpr int NA = BES ? 1 : (DBL ? 2 * K : K);
    static_assert(DR >= 1 && DS + 3 <= PS && P % PS == 0 && PS % 3 == 0 && DL + K < P,
                  "ring sizes");
    static_assert(K >= 2 && K <= 8, "steps per pass");
    const float tf = (float)geo.t, inv_esf = (float)geo.inv_es;
    // per pattern: (previous column, next column, next chain, previous chain)
    __shared__ float4 lwt[kMaxPatterns];
    for (int j = threadIdx.x; j < lat.nsp; j += (int)blockDim.x) {
        const uint32_t f = lat.flags[j];
        const float tv = (f & 4u) ? tf : 0.0f;
        lwt[j] = make_float4((f & 1u) ? tf : 0.0f, (f & 2u) ? tf : 0.0f, (f & 8u) ? tv : 0.0f,
                             (f & 8u) ? 0.0f : tv);
    }
    __syncthreads();
    // the K coefficients of a propagator pass in single precision
    float2 cf[K];
#pragma unroll
    for (int s = 0; s < K; ++s) cf[s] = make_float2((float)ck.c[s].x, (float)ck.c[s].y);
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = geo.nx, ny = geo.ny, J = geo.J;
    const int nst = (nx + TC - 1) / TC, nsg = (ny + J - 1) / J;
    const int ntile = nst * nsg;
    const int lb = geo.lb;
    const int per = (ntile + kXcds - 1) / kXcds;
    const int b0 = (lb % kXcds) * per, b1 = min(b0 + per, ntile);
    const int nwv = (int)blockDim.x / kWave;          // wavefronts per group
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int wloc = (lb / kXcds) * nwv + wv;
    const int wn = (geo.nwg / kXcds) * nwv;
    double2 acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int b = b0 + wloc; b < b1; b += wn) {
        const int strip = b % nst;                     // across the strips first
        const int j0 = (b / nst) * J, c0 = strip * TC;
        const int gi = wrap_index(c0 - K + lane, nx);
        const bool colok = lane >= K && lane < K + TC && c0 - K + lane < nx;
        const int Jt = min(J, ny - j0), T = Jt + 2 * K;
        const uint32_t ov = (uint32_t)gi * sizeof(float2), rb = (uint32_t)nx * sizeof(float2);
        const uint32_t ovo = colok ? ov : kOffNone;   // offset of the strip's own columns
        const double mcol = colok ? 1.0 : 0.0;
        // every band walks down the chains (alternating directions, as the
        // FP64 strips take them, cost these kernels their scalar registers)
        auto base = [&](int rho) { return (int64_t)wrap_index(j0 - K + rho, ny) * nx; };
        auto owned = [&](int rho) { return rho >= K && rho < K + Jt; };
        float2 X0[PS], Xm[PS];                         // phi_n, phi_{n-1} rings
        float2 LL[P];                                  // phi_L (or the accumulator) ring
        int PI[P];                                     // pattern ids
        float OO[P];                                   // scaled on-site terms
        float2 LV[K][3];                               // levels 1 .. K, last three rows
#pragma unroll
        for (int q = 0; q < PS; ++q) X0[q] = Xm[q] = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            LL[q] = make_float2(0.0f, 0.0f);
            PI[q] = 0;
            OO[q] = 0.0f;
        }
#pragma unroll
        for (int s = 0; s < K; ++s) LV[s][0] = LV[s][1] = LV[s][2] = make_float2(0.0f, 0.0f);
        auto load_state = [&](int rho, int q) {
            const int64_t rbase = base(rho);
            const uint32_t nb = rho < T ? rb : 0u;
            X0[q] = buf_ldf(p1 + rbase, nb, ov);
            Xm[q] = buf_ldf(p0 + rbase, nb, ov);
        };
        auto load_left = [&](int rho, int q) {
            if constexpr (DBL) return;
            LL[q] = buf_ldf(lacc + base(rho), owned(rho) ? rb : 0u, ovo);
        };
        auto load_row = [&](int rho, int q) {
            const int64_t rbase = base(rho) + e0;
            const bool in = rho < T;
            PI[q] = __builtin_amdgcn_raw_buffer_load_b8(
                row_rsrc(lat.sid + rbase, in ? (uint32_t)nx : 0u), gi, 0, 0);
            if (ONSF)
                OO[q] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(
                                       row_rsrc(h.onsf + rbase, in ? (uint32_t)nx * 4u : 0u),
                                       gi * 4, 0, 0)) *
                        inv_esf;
            else
                OO[q] = (float)__builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(
                                row_rsrc(h.ons + rbase, in ? (uint32_t)nx * 8u : 0u), gi * 8, 0,
                                0));
        };
#pragma unroll
        for (int r = 0; r < DS; ++r) load_state(r, r % PS);
#pragma unroll
        for (int r = 0; r < DL; ++r) load_left(r, r);
#pragma unroll
        for (int r = 0; r < DR; ++r) load_row(r, r);
        for (int t0 = 0; t0 < T; t0 += P) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const int tt = t0 + u;
                load_state(tt + DS, (u + DS) % PS);
                load_left(tt + DL, (u + DL) % P);
                load_row(tt + DR, (u + DR) % P);
#pragma unroll
                for (int s = 1; s <= K; ++s) {
                    const int rho = tt - s;
                    const int qp = ((u - s) % P + P) % P;               // per-row ring, row rho
                    const int qs = ((u - s) % PS + PS) % PS;            // state rings, row rho
                    const int q3 = ((u - s) % 3 + 3) % 3;               // level rings, row rho
                    const int q3m = (q3 + 2) % 3, q3p = (q3 + 1) % 3;   // rows rho - 1, rho + 1
                    const int qm = (qs + PS - 1) % PS, qq = (qs + 1) % PS;
                    float2 xm1, x0, xp1, old;
                    if (s == 1) {
                        xm1 = X0[qm];
                        x0 = X0[qs];
                        xp1 = X0[qq];
                        old = Xm[qs];
                    } else {
                        xm1 = LV[s - 2][q3m];
                        x0 = LV[s - 2][q3];
                        xp1 = LV[s - 2][q3p];
                        old = s == 2 ? X0[qs] : LV[s - 3 < 0 ? 0 : s - 3][q3];
                    }
                    const float4 w = lwt[PI[qp]];
                    const float o = OO[qp];
                    float2 a = make_float2(o * x0.x, o * x0.y);
                    a = fraxpy_shifted(a, lane_prevf(x0), w.x);
                    a = fraxpy_shifted(a, lane_nextf(x0), w.y);
                    a = fraxpy(a, w.w, xm1);
                    a = fraxpy(a, w.z, xp1);
                    const float2 c = ftwo_minus(a, old);
                    LV[s - 1][q3] = c;
                    if constexpr (BES) {
                        LL[qp] = fcmla(LL[qp], cf[s - 1], c);
                        if (s == K) {
                            const bool own = owned(rho);
                            const int64_t row = (int64_t)(own ? j0 + rho - K : 0) * nx;
                            buf_stf(lacc + row, own ? rb : 0u, ovo, LL[qp]);
                        }
                    } else if constexpr (DBL) {
                        const double m = owned(rho) ? mcol : 0.0;
                        const double xr = (double)x0.x, xi = (double)x0.y;
                        const double wr = xr * m, wi = xi * m;
                        // <phi_m|phi_n> is real for Hermitian H~: real parts only
                        acc[2 * (s - 1)].x = fma(wr, xr, fma(wi, xi, acc[2 * (s - 1)].x));
                        acc[2 * (s - 1) + 1].x =
                            fma(wr, (double)c.x, fma(wi, (double)c.y, acc[2 * (s - 1) + 1].x));
                    } else if constexpr (RE) {
                        acc[s - 1].x = fma((double)LL[qp].x, (double)c.x,
                                           fma((double)LL[qp].y, (double)c.y, acc[s - 1].x));
                    } else {
                        acc[s - 1] = cdot_acc(acc[s - 1],
                                              make_double2((double)LL[qp].x, (double)LL[qp].y),
                                              make_double2((double)c.x, (double)c.y));
                    }
                    if (s >= K - 1) {
                        const bool own = owned(rho);
                        const int64_t row = (int64_t)(own ? j0 + rho - K : 0) * nx;
                        buf_stf((s == K ? out2 : out1) + row, own ? rb : 0u, ovo, c);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if constexpr (BES) return;
#pragma unroll
    for (int k = 0; k < NA; ++k) block_sum_waves(acc[k], partial + part_index(sw, slot + k));
}

}  // namespace

template <bool ONSF, bool DBL, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_moment_march_f32(
    Ell h, Sweep sw, Lat2 lat, const float2 *p1, const float2 *p0, float2 *__restrict__ out1,
    float2 *__restrict__ out2, const float2 *__restrict__ phil, double2 *__restrict__ partial,
    int slot) {
    march_sweep_f32<ONSF, DBL ? kMarchDoubled : kMarchDirect, K>(
        h, sw, lat, p1, p0, out1, out2, const_cast<float2 *>(phil), partial, slot, CoefK{});
}

template <bool ONSF, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_moment_march_re_f32(
    Ell h, Sweep sw, Lat2 lat, const float2 *p1, const float2 *p0, float2 *__restrict__ out1,
    float2 *__restrict__ out2, const float2 *__restrict__ phil, double2 *__restrict__ partial,
    int slot) {
    march_sweep_f32<ONSF, kMarchDirectRe, K>(h, sw, lat, p1, p0, out1, out2,
                                             const_cast<float2 *>(phil), partial, slot, CoefK{});
}

template <bool ONSF, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_evolve_march_f32(
    Ell h, Sweep sw, Lat2 lat, const float2 *p1, const float2 *p0, float2 *__restrict__ out1,
    float2 *__restrict__ out2, float2 *__restrict__ acc, CoefK ck) {
    march_sweep_f32<ONSF, kMarchBessel, K>(h, sw, lat, p1, p0, out1, out2, acc, nullptr, 0, ck);
}

bool launch_moment_multi_f32(const Ell &h, const Sweep &sw, const Lat2 &lat, const float2 *p1,
                             const float2 *p0, float2 *out1, float2 *out2, const float2 *phil,
                             double2 *partial, int slot, bool dbl, bool re, hipStream_t s) {
    if (lat.reg != 2 || lat.k < 2 || lat.k > kMaxMarchSteps) return false;
#define KPM_M32(ONSF_, DBL_, K_)                                                              \
    do {                                                                                      \
        if (!(DBL_) && re)                                                                    \
            hipLaunchKernelGGL((k_moment_march_re_f32<ONSF_, K_>), dim3(sw.nwg, sw.nplanes),   \
                               dim3(sw.wpg * kWave), 0, s, h, sw, lat, p1, p0, out1, out2, phil,      \
                               partial, slot);                                                \
        else                                                                                  \
            hipLaunchKernelGGL((k_moment_march_f32<ONSF_, DBL_, K_>),                         \
                               dim3(sw.nwg, sw.nplanes), dim3(sw.wpg * kWave), 0, s, h, sw, lat, p1,  \
                               p0, out1, out2, phil, partial, slot);                          \
    } while (0)
#define KPM_M32K(ONSF_, DBL_)                                                                 \
    switch (lat.k) {                                                                          \
        case 8: KPM_M32(ONSF_, DBL_, 8); break;                                               \
        case 7: KPM_M32(ONSF_, DBL_, 7); break;                                               \
        case 6: KPM_M32(ONSF_, DBL_, 6); break;                                               \
        case 5: KPM_M32(ONSF_, DBL_, 5); break;                                               \
        case 4: KPM_M32(ONSF_, DBL_, 4); break;                                               \
        case 3: KPM_M32(ONSF_, DBL_, 3); break;                                               \
        default: KPM_M32(ONSF_, DBL_, 2); break;                                              \
    }
    if (h.onsf) {
        if (dbl) { KPM_M32K(true, true) } else { KPM_M32K(true, false) }
    } else {
        if (dbl) { KPM_M32K(false, true) } else { KPM_M32K(false, false) }
    }
#undef KPM_M32K
#undef KPM_M32
    return true;
}

bool launch_evolve_multi_f32(const Ell &h, const Sweep &sw, const Lat2 &lat, const float2 *p1,
                             const float2 *p0, float2 *out1, float2 *out2, float2 *acc,
                             const CoefK &ck, hipStream_t s) {
    if (lat.reg != 2 || lat.k < 2 || lat.k > kMaxMarchSteps) return false;
#define KPM_E32(ONSF_, K_)                                                                    \
    hipLaunchKernelGGL((k_evolve_march_f32<ONSF_, K_>), dim3(sw.nwg, sw.nplanes),              \
                       dim3(sw.wpg * kWave), 0, s, h, sw, lat, p1, p0, out1, out2, acc, ck)
#define KPM_E32K(ONSF_)                                                                       \
    switch (lat.k) {                                                                          \
        case 8: KPM_E32(ONSF_, 8); break;                                                     \
        case 7: KPM_E32(ONSF_, 7); break;                                                     \
        case 6: KPM_E32(ONSF_, 6); break;                                                     \
        case 5: KPM_E32(ONSF_, 5); break;                                                     \
        case 4: KPM_E32(ONSF_, 4); break;                                                     \
        case 3: KPM_E32(ONSF_, 3); break;                                                     \
        default: KPM_E32(ONSF_, 2); break;                                                    \
    }
    if (h.onsf) { KPM_E32K(true) }
    else { KPM_E32K(false) }
#undef KPM_E32K
#undef KPM_E32
    return true;
}

}  // namespace kpm
