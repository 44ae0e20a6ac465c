// The marching strips: the K-step sweeps of the Chebyshev recursion (Alg. 5)
// and of the Chebyshev-Bessel propagator (Alg. 6) that walk strips of chains
// row by row with each level's last rows in registers.  Shared by the
// library's kernel file (2 .. 8 steps per pass) and the file of the
// real-part passes of 9 and 10 steps, which is compiled with another
// instruction schedule.
#pragma once

#include "kpm_internal.h"
#include "kpm_device.h"

#include <type_traits>

namespace kpm {

// The value a store of v into storage type V will hold, back in double.
template <typename V> __device__ __forceinline__ double2 rounded(double2 v);
template <> __device__ __forceinline__ double2 rounded<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 rounded<float2>(double2 v) {
    return make_double2((double)(float)v.x, (double)(float)v.y);
}

// Marching form of the register-tiled K-step sweep (K = 2 .. 8, and 9 or 10
// for the real parts with FP64 states; each level costs only its three-row
// ring of registers): a wavefront takes a strip
// of (kWave - 2K) columns (lanes as in k_moment_stepk) and J chains, and walks
// down the chains.  Iteration t brings in chain row t of phi_n (window rows
// j0 - K .. j0 + J + K - 1) and computes level s = 1 .. K (phi_{n+s}) on row
// t - s, from level s - 1 on rows t - s - 1 .. t - s + 1 and level s - 2 on
// row t - s.  Each level keeps its last three rows in registers, so rows are
// computed once per level except the K - 1 boundary rows at each end of the
// strip, instead of once per tile as in k_moment_stepk.  phi_n, phi_{n-1} and
// phi_L are loaded kDs rows ahead (phi_L fewer at K = 8), the pattern id and
// on-site term kRowRing - 1 - K rows ahead; a row's slot weights (from a
// per-pattern table in LDS: t or 0 for the previous column, the next column,
// the next chain and the previous chain) and scaled on-site term are formed
// one iteration before their first use up to K = 5, and at each level above
// (their registers then go to the level rings).  The loop is unrolled by
// kRowRing (a multiple of kStateRing and of 3) so every ring index is a
// compile-time constant.  The same walk serves the moments (direct, real
// parts only, doubling) and the propagator (MODE below).
// The loop body has no branch: a strip runs whole passes of kRowRing rows,
// rows past the window load as zeros (buffer resources of size 0), levels are
// computed on every row (a value of a row outside a level's range is finite
// and feeds only other such rows), and rows or lanes that own no output read
// phi_L as 0 and store through an empty resource or an offset past the row.
// Every load is then issued on every path and stays where it is written, so
// the wait before each use leaves the later rows' loads in flight.  A zero
// weight adds an exact zero, so each state value is the one k_moment_step
// computes.


template <typename V, bool ONSF, int MODE, int K>
__device__ __forceinline__ void march_sweep(const Ell &h, const Sweep &sw, const Lat2 &lat,
                                            const V *p1, const V *p0, V *__restrict__ out1,
                                            V *__restrict__ out2, V *__restrict__ lacc,
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
    // the states are prefetched DS rows ahead (two at nine steps, which frees
    // the registers of the ninth level ring)
    constexpr int P = kRowRing, PS = kStateRing, DS = K >= 9 ? 2 : kDs,
                  DR = kRowRing - 1 - K;
    // phi_L rows are loaded DL ahead and used through K iterations after their
    // own (fewer rows ahead from K = 8 on keep those kernels within their
    // registers)
    constexpr int DL = K >= 9 ? 1
                              : (K >= 8 ? (sizeof(V) == sizeof(double2) ? 2 : 1) : (DS < DR ? DS : DR));
    constexpr int NA = BES ? 1 : (DBL ? 2 * K : K);
    static_assert(DR >= 1 && DS + 3 <= PS && P % PS == 0 && PS % 3 == 0 && DL + K < P,
                  "ring sizes");
    // up to 5 steps the row terms are formed once per row, ahead of their first
    // use; with more levels their registers are needed for the level rings
    // (nine and ten steps: the real-part pass with FP64 states only)
    static_assert(K >= 2 && (K <= kMaxMarchSteps || (K <= kReMarchSteps && RE &&
                                                      std::is_same<V, double2>::value)),
                  "steps per pass");
    // from ten steps on, each lane's real-part sums live in LDS (one slot per
    // level and thread, updated with the same fused multiply-adds), which
    // frees their registers for the level rings
    constexpr bool kAccLds = RE && K >= 10;
    __shared__ double lsum[kAccLds ? K : 1][kAccLds ? kMaxStripBlock : 1];
    constexpr bool kAhead = K <= 5;
    const double t = geo.t, inv_es = geo.inv_es;
    // per pattern and marching direction d: (previous column, next column),
    // then the weights of the rows after and before in marching order: (next
    // chain, previous chain) marching down the chains (d = 0), swapped
    // marching up (d = 1)
    __shared__ double2 lwt[4 * kMaxPatterns];
    for (int j = threadIdx.x; j < lat.nsp; j += (int)blockDim.x) {
        const uint32_t f = lat.flags[j];
        const double tv = (f & 4u) ? t : 0.0;
        const double wn = (f & 8u) ? tv : 0.0, wp = (f & 8u) ? 0.0 : tv;
        const double2 wh = make_double2((f & 1u) ? t : 0.0, (f & 2u) ? t : 0.0);
        lwt[4 * j] = lwt[4 * j + 2] = wh;
        lwt[4 * j + 1] = make_double2(wn, wp);
        lwt[4 * j + 3] = make_double2(wp, wn);
    }
    __syncthreads();
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
    if constexpr (kAccLds)
#pragma unroll
        for (int k = 0; k < K; ++k) lsum[k][threadIdx.x] = 0.0;
    for (int b = b0 + wloc; b < b1; b += wn) {
        const int strip = b % nst;                     // across the strips first
        const int j0 = (b / nst) * J, c0 = strip * TC;
        // odd bands of strips march up the chains: two neighbouring bands then
        // reach their shared boundary chains at the same time (both first or
        // both last), and the second reads of those rows hit the cache.  FP64
        // states only: with FP32 states (converted at every load and store)
        // the direction's scalar registers cost the pass its load pipelining
        const int dir = std::is_same<V, double2>::value ? (b / nst) & 1 : 0;
        const int gi = wrap_index(c0 - K + lane, nx);
        const bool colok = lane >= K && lane < K + TC && c0 - K + lane < nx;
        const int Jt = min(J, ny - j0), T = Jt + 2 * K;
        const uint32_t ov = (uint32_t)gi * sizeof(V), rb = (uint32_t)nx * sizeof(V);
        const uint32_t ovo = colok ? ov : kOffNone;   // offset of the strip's own columns
        const double mcol = colok ? 1.0 : 0.0;
        // chain of walked row rho (rows K .. K + Jt - 1 are the band's own)
        const int cst = dir ? j0 + Jt + K - 1 : j0 - K, sgn = dir ? -1 : 1;
        auto base = [&](int rho) { return (int64_t)wrap_index(cst + sgn * rho, ny) * nx; };
        auto owned = [&](int rho) { return rho >= K && rho < K + Jt; };
        const int wo = 2 * dir;                        // this direction's weights
        double2 X0[PS], Xm[PS], LL[P];                 // phi_n, phi_{n-1}, phi_L rings
        int PI[P];                                     // pattern ids
        float OF[P];
        double OD[P];
        double2 LV[K][3];                              // levels 1 .. K, last three rows
        // rows ahead of the first loads and the levels' first rows start as 0
#pragma unroll
        for (int q = 0; q < PS; ++q) X0[q] = Xm[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            LL[q] = make_double2(0.0, 0.0);
            PI[q] = 0;
            OF[q] = 0.0f;
            OD[q] = 0.0;
        }
#pragma unroll
        for (int s = 0; s < K; ++s) LV[s][0] = LV[s][1] = LV[s][2] = make_double2(0.0, 0.0);
        // per row: slot weights and on-site term, taken from the pattern table
        // and the loaded on-site value one iteration before their first use
        double2 WH[P], WV[P];
        double OO[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            WH[q] = WV[q] = make_double2(0.0, 0.0);
            OO[q] = 0.0;
        }
        auto row_terms = [&](int q) {
            if (!kAhead) return;
            WH[q] = lwt[4 * PI[q] + wo];
            WV[q] = lwt[4 * PI[q] + wo + 1];
            OO[q] = ONSF ? (double)OF[q] * inv_es : OD[q];
        };
        auto load_state = [&](int rho, int q) {
            const int64_t rbase = base(rho);
            const uint32_t nb = rho < T ? rb : 0u;
            X0[q] = buf_ld(p1 + rbase, nb, ov);
            Xm[q] = buf_ld(p0 + rbase, nb, ov);
        };
        auto load_left = [&](int rho, int q) {
            if (!DBL) LL[q] = buf_ld(lacc + base(rho), owned(rho) ? rb : 0u, ovo);
        };

        auto load_row = [&](int rho, int q) {
            const int64_t rbase = base(rho) + e0;
            const bool in = rho < T;
            PI[q] = __builtin_amdgcn_raw_buffer_load_b8(
                row_rsrc(lat.sid + rbase, in ? (uint32_t)nx : 0u), gi, 0, 0);
            if (ONSF)
                OF[q] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(
                               row_rsrc(h.onsf + rbase, in ? (uint32_t)nx * 4u : 0u), gi * 4, 0,
                               0));
            else
                OD[q] = __builtin_bit_cast(
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
                row_terms(u);
#pragma unroll
                for (int s = 1; s <= K; ++s) {
                    const int rho = tt - s;
                    // ring slots of rows rho - 1, rho, rho + 1 (rho = t0 + u - s)
                    const int qp = ((u - s) % P + P) % P;               // per-row ring, row rho
                    const int qs = ((u - s) % PS + PS) % PS;            // state rings, row rho
                    const int q3 = ((u - s) % 3 + 3) % 3;               // level rings, row rho
                    const int q3m = (q3 + 2) % 3, q3p = (q3 + 1) % 3;   // rows rho - 1, rho + 1
                    const int qm = (qs + PS - 1) % PS, qq = (qs + 1) % PS;
                    double2 xm1, x0, xp1, old;
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
                    // 2 H~ x - q in the slot order of k_moment_step (of the two
                    // vertical terms one has weight 0, so their order, the row
                    // before in marching order first, leaves the sum unchanged)
                    if (!kAhead) {                 // the row's terms, read at each level
                        WH[qp] = lwt[4 * PI[qp] + wo];
                        WV[qp] = lwt[4 * PI[qp] + wo + 1];
                        OO[qp] = ONSF ? (double)OF[qp] * inv_es : OD[qp];
                    }
                    double2 a = make_double2(OO[qp] * x0.x, OO[qp] * x0.y);
                    a = raxpy(a, WH[qp].x, lane_prev(x0));
                    a = raxpy(a, WH[qp].y, lane_next(x0));
                    a = raxpy(a, WV[qp].y, xm1);
                    a = raxpy(a, WV[qp].x, xp1);
                    const double2 c = rounded<V>(two_minus(a, old));
                    LV[s - 1][q3] = c;
                    if (BES) {
                        LL[qp] = rounded<V>(cmla(LL[qp], ck.c[s - 1], c));
                        if (s == K) {
                            const bool own = owned(rho);
                            const int64_t row = (int64_t)(own ? cst + sgn * rho : 0) * nx;
                            buf_st(lacc + row, own ? rb : 0u, ovo, LL[qp]);
                        }
                    } else if (DBL) {
                        const double m = owned(rho) ? mcol : 0.0;
                        const double2 xw = make_double2(x0.x * m, x0.y * m);
                        // <phi_m|phi_n> = <phi_0|T_m(H~) T_n(H~)|phi_0> is real (H~
                        // Hermitian): only the real parts are accumulated
                        acc[2 * (s - 1)].x = fma(xw.x, x0.x, fma(xw.y, x0.y, acc[2 * (s - 1)].x));
                        acc[2 * (s - 1) + 1].x =
                            fma(xw.x, c.x, fma(xw.y, c.y, acc[2 * (s - 1) + 1].x));
                    } else if (RE) {
                        if constexpr (kAccLds)
                            lsum[s - 1][threadIdx.x] = fma(
                                LL[qp].x, c.x, fma(LL[qp].y, c.y, lsum[s - 1][threadIdx.x]));
                        else
                            acc[s - 1].x = fma(LL[qp].x, c.x, fma(LL[qp].y, c.y, acc[s - 1].x));
                    } else {
                        acc[s - 1] = cdot_acc(acc[s - 1], LL[qp], c);
                    }
                    if (s >= K - 1) {
                        const bool own = owned(rho);
                        const int64_t row = (int64_t)(own ? cst + sgn * rho : 0) * nx;
                        buf_st((s == K ? out2 : out1) + row, own ? rb : 0u, ovo, c);
                    }
                }
                // each iteration is scheduled on its own: the live values stay
                // those of the rings
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (BES) return;
    if constexpr (kAccLds)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k].x = lsum[k][threadIdx.x];
    const int nw = sw.nwg;
#pragma unroll
    for (int k = 0; k < NA; ++k) block_sum_waves(acc[k], partial + part_index(sw, slot + k));
    (void)nw;
}

template <typename V, bool ONSF, bool DBL, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_moment_march(Ell h, Sweep sw, Lat2 lat,
                                                         const V *p1, const V *p0,
                                                         V *__restrict__ out1,
                                                         V *__restrict__ out2,
                                                         const V *__restrict__ phil,
                                                         double2 *__restrict__ partial,
                                                         int slot) {
    march_sweep<V, ONSF, DBL ? kMarchDoubled : kMarchDirect, K>(
        h, sw, lat, p1, p0, out1, out2, const_cast<V *>(phil), partial, slot, CoefK{});
}

// k_moment_march's direct form accumulating only Re <phi_L|phi_{n+s}>.
template <typename V, bool ONSF, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_moment_march_re(Ell h, Sweep sw, Lat2 lat,
                                                            const V *p1, const V *p0,
                                                            V *__restrict__ out1,
                                                            V *__restrict__ out2,
                                                            const V *__restrict__ phil,
                                                            double2 *__restrict__ partial,
                                                            int slot) {
    march_sweep<V, ONSF, kMarchDirectRe, K>(h, sw, lat, p1, p0, out1, out2, const_cast<V *>(phil),
                                            partial, slot, CoefK{});
}

// K steps of the Chebyshev-Bessel propagator (Alg. 6) per pass: the states as
// in k_moment_march, and acc += c_m phi_m for the K new states, c_m = ck.c[m - n - 1].
template <typename V, bool ONSF, int K>
__global__ __launch_bounds__(kMaxStripBlock, 1) void k_evolve_march(Ell h, Sweep sw, Lat2 lat,
                                                         const V *p1, const V *p0,
                                                         V *__restrict__ out1,
                                                         V *__restrict__ out2,
                                                         V *__restrict__ acc, CoefK ck) {
    march_sweep<V, ONSF, kMarchBessel, K>(h, sw, lat, p1, p0, out1, out2, acc, nullptr, 0, ck);
}

}  // namespace kpm
