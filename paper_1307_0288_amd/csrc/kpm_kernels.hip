// gfx950 kernels of the Chebyshev hot path.
//
// Every kernel is a sweep over the rows of the neighbour-list Hamiltonian
// (Alg. 8): one element = one (row, vector) pair, vectors fastest, so a row
// with R vectors is handled by R adjacent lanes that share its neighbour
// indices and each stream their own vector.  The paper's kernels -- the
// sparse product, the linear combinations and the inner product (Alg. 5-8)
// -- are fused: each recursion step reads every operand once and writes its
// result once, and the inner product is reduced in registers, across the
// wavefront with shuffles and across the work-group in LDS, leaving one
// partial per work-group that a second small kernel sums in a fixed order.
// The path is bound by HBM bandwidth (about 0.3 flop per byte), so there is
// no matrix-core work here.
//
// A system may hold several independent samples (segments) side by side;
// every work-group belongs to exactly one segment (see Seg in
// kpm_internal.h), so per-sample inner products need no atomics.
#include "kpm_internal.h"
#include "kpm_device.h"
#include "kpm_march.h"

#include <type_traits>

namespace kpm {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double2 ld(const double2 *p) { return *p; }
__device__ __forceinline__ double2 ld(const float2 *p) {
    float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void st(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void st(float2 *p, double2 v) {
    *p = make_float2((float)v.x, (float)v.y);
}

// Streaming (non-temporal) accesses for operands read or written once per
// step, so that L2 keeps the gathered vector for the neighbour reads.
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_nt(const float2 *p) {
    f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v) {
    d2v w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<d2v *>(p));
}
__device__ __forceinline__ void st_nt(float2 *p, double2 v) {
    f2v w;
    w.x = (float)v.x;
    w.y = (float)v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<f2v *>(p));
}

__device__ __forceinline__ double2 coef(const Coef &c, int sg) {
    return c.tab ? c.tab[sg * c.stride + c.idx] : c.val;
}

// The element blocks this work-group visits: blocks b0 + loc, b0 + loc +
// nloc, ... below b1 of its segment, elements e0 + b * kBlock + tid below e1;
// t and inv_es are the segment's uniform hopping / E_s and 1 / E_s.
struct Walk {
    int sg;
    int loc, nloc;
    int64_t b0, b1, e0, e1;
    double t, inv_es;
    // tiled traversal (tnx > 0): blocks per tile = 1 << lbps, nch chains,
    // division by nch as a multiply and shift
    int32_t tnx, tw, lbps, nch;
    uint64_t div_m;
    int32_t div_l;
};

// Element of thread `tid` in logical block b of the walk's segment, and
// whether it exists.  Row order: consecutive blocks.  Tiled: block b is part
// k of tile t = b >> lbps, the tile of chain j = t % nch in strip s = t / nch.
__device__ __forceinline__ bool block_elem(const Walk &w, int64_t b, int tid, int vshift,
                                           int64_t &e) {
    if (w.tnx == 0) {
        e = w.e0 + b * kBlock + tid;
        return e < w.e1;
    }
    const uint32_t t = (uint32_t)(b >> w.lbps);
    const uint32_t s = (uint32_t)(((uint64_t)t * w.div_m) >> (32 + w.div_l));
    const uint32_t j = t - s * (uint32_t)w.nch;
    const int64_t loc = ((b & ((1 << w.lbps) - 1)) * kBlock) + tid;
    const int64_t width = min((int64_t)w.tw, (int64_t)w.tnx - (int64_t)s * w.tw);
    e = w.e0 + (((int64_t)j * w.tnx + (int64_t)s * w.tw) << vshift) + loc;
    return loc < (width << vshift);
}

// Neighbour-offset patterns of the compact form, staged in LDS by every
// work-group (at most kMaxPatterns x kMaxWidth words).
#define KPM_PATTERNS(h)                                                          \
    __shared__ int32_t lpat[kMaxPatterns * kMaxWidth];                           \
    if ((h).pid) {                                                               \
        for (int j_ = threadIdx.x; j_ < (h).npat * kMaxWidth; j_ += kBlock)      \
            lpat[j_] = (h).pat[j_];                                              \
        __syncthreads();                                                         \
    }

// Pattern id of row i (0 for the explicit form).
__device__ __forceinline__ int row_pid(const Ell &h, int64_t i) {
    return h.pid ? (int)h.pid[i] : 0;
}

// Row held by slot k of row i, or -1.
__device__ __forceinline__ int32_t slot_row(const Ell &h, const int32_t *lpat, int pid,
                                            int64_t i, int k) {
    if (h.pid) {
        const int32_t d = lpat[pid * kMaxWidth + k];
        return d == kEmptySlot ? -1 : (int32_t)(i + d);
    }
    return h.nbr[k * h.n + i];
}

// H_ii / E_s of row i.
__device__ __forceinline__ double row_ons(const Ell &h, const Walk &wk, int64_t i) {
    return h.onsf ? (double)h.onsf[i] * wk.inv_es : h.ons[i];
}

// Sum of H~_im x_m over the filled slots of row i, plus the diagonal term.
template <typename V>
__device__ __forceinline__ double2 row_h(const Ell &h, const Walk &wk, const int32_t *lpat,
                                         const V *x, int64_t i, int64_t v, int vshift,
                                         double2 xi) {
    const double o = row_ons(h, wk, i);
    const int pid = row_pid(h, i);
    double2 acc = make_double2(o * xi.x, o * xi.y);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            const int32_t m = slot_row(h, lpat, pid, i, k);
            double hk = h.hop ? h.hop[k * h.n + i] : wk.t;
            const double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            hk = m < 0 ? 0.0 : hk;
            acc = raxpy(acc, hk, xm);
        }
    }
    return acc;
}

// H~ x and D x of row i together, sharing the gathered x_m.
template <typename V>
__device__ __forceinline__ void row_hd(const Ell &h, const Walk &wk, const int32_t *lpat,
                                       const V *x, int64_t i, int64_t v, int vshift,
                                       double2 xi, double2 &hx, double2 &dx) {
    const double o = row_ons(h, wk, i);
    const int pid = row_pid(h, i);
    hx = make_double2(o * xi.x, o * xi.y);
    dx = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            const int32_t m = slot_row(h, lpat, pid, i, k);
            double hk = h.hop ? h.hop[k * h.n + i] : wk.t;
            double xk = h.xw[k * h.n + i];
            const double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            hk = m < 0 ? 0.0 : hk;
            xk = m < 0 ? 0.0 : xk;
            hx = raxpy(hx, hk, xm);
            dx = raxpy(dx, xk, xm);
        }
    }
}

// D x of row i.
template <typename V>
__device__ __forceinline__ double2 row_d(const Ell &h, const int32_t *lpat, const V *x,
                                         int64_t i, int64_t v, int vshift) {
    const int pid = row_pid(h, i);
    double2 dx = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            const int32_t m = slot_row(h, lpat, pid, i, k);
            double xk = h.xw[k * h.n + i];
            const double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            xk = m < 0 ? 0.0 : xk;
            dx = raxpy(dx, xk, xm);
        }
    }
    return dx;
}



__device__ __forceinline__ Walk walk_of(const Sweep &sw) {
    Walk w;
    Seg s;
    if (sw.seg) {
        w.sg = sw.wg_seg[blockIdx.x];
        s = sw.seg[w.sg];
    } else {
        w.sg = 0;
        s = sw.one;
    }
    const int lb = (int)blockIdx.x - s.g0;      // g0 % 8 == 0: lb % 8 is the XCD
    w.loc = lb / kXcds;
    w.nloc = s.nwg / kXcds;
    w.tnx = s.tnx;
    w.tw = s.tw;
    w.div_m = s.div_m;
    w.div_l = s.div_l;
    int64_t nblk;
    if (s.tnx > 0) {
        const int64_t rows = (s.e1 - s.e0) >> sw.vshift;
        w.nch = (int32_t)(rows / s.tnx);
        w.lbps = 31 - __builtin_clz((uint32_t)((s.tw << sw.vshift) / kBlock));
        nblk = ((int64_t)(s.tnx + s.tw - 1) / s.tw) * w.nch << w.lbps;
    } else {
        w.nch = 0;
        w.lbps = 0;
        nblk = (s.e1 - s.e0 + kBlock - 1) / kBlock;
    }
    const int64_t per = (nblk + kXcds - 1) / kXcds;
    w.b0 = (int64_t)(lb % kXcds) * per;
    w.b1 = min(w.b0 + per, nblk);
    w.e0 = s.e0;
    w.e1 = s.e1;
    w.t = s.t;
    w.inv_es = s.inv_es;
    return w;
}

#define KPM_SWEEP_BEGIN(sw, h)                                                      \
    KPM_PATTERNS(h)                                                                 \
    const Walk wk_ = walk_of(sw);                                                   \
    const int sg = wk_.sg;                                                          \
    (void)sg;                                                                       \
    for (int64_t b_ = wk_.b0 + wk_.loc; b_ < wk_.b1; b_ += wk_.nloc) {              \
        int64_t e;                                                                  \
        if (block_elem(wk_, b_, threadIdx.x, (sw).vshift, e)) {                     \
            const int64_t i = e >> (sw).vshift;                                     \
            const int64_t v = e & ((1 << (sw).vshift) - 1);
#define KPM_SWEEP_END \
        }             \
    }

// ---------------------------------------------------------------- kernels
// First step of the moments: out = H~ in, <L|in> and <L|out>.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_moment_first(Ell h, Sweep sw, const V *in, V *out,
                                                         const V *__restrict__ phil,
                                                         double2 *__restrict__ partial,
                                                         int slot) {
    const int64_t po = plane_off(sw);
    in = on_plane(in, po);
    out = on_plane(out, po);
    phil = on_plane(phil, po);
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    KPM_SWEEP_BEGIN(sw, h)
    const double2 xi = ld(in + e);
    const double2 l = ld(phil + e);
    const double2 o = rounded<V>(row_h(h, wk_, lpat, in, i, v, sw.vshift, xi));
    st(out + e, o);
    s0 = cdot_acc(s0, l, xi);
    s1 = cdot_acc(s1, l, o);
    KPM_SWEEP_END
    const int64_t r = (int64_t)1 << sw.vshift;
    block_sum(s0, sw.vshift, partial + part_index(sw, slot) * r);
    block_sum(s1, sw.vshift, partial + part_index(sw, slot + 1) * r);
}

// Structure forms of the moment step.  kFormGeneric reads everything the
// Ell may hold and checks it at run time (any width <= kMaxWidth, explicit or
// compact neighbours, per-slot or uniform hopping, float or double on-site
// terms).  The other forms fix, at compile time, width 3 and uniform hopping
// (every graphene sample) and the neighbour and on-site storage, so the loop
// body is straight-line code whose loads the compiler can issue together.
enum { kFormGeneric = 0, kFormC3F = 1, kFormC3D = 2, kFormL3F = 3, kFormL3D = 4 };

template <int FORM> struct FormTraits {
    static constexpr bool generic = FORM == kFormGeneric;
    static constexpr int width = generic ? kMaxWidth : 3;
    static constexpr bool compact = FORM == kFormC3F || FORM == kFormC3D;
    static constexpr bool ons_float = FORM == kFormC3F || FORM == kFormL3F;
};

// Structure form of a system (see launch_step_shape).
inline int form_of(const Ell &h) {
    const bool fixed = h.w == 3 && !h.hop;
    if (fixed && h.pid) return h.onsf ? kFormC3F : kFormC3D;
    if (fixed) return h.onsf ? kFormL3F : kFormL3D;
    return kFormGeneric;
}

// Neighbours of row i in a fixed (width 3, uniform hopping) form.
template <int FORM>
__device__ __forceinline__ void row_nbrs(const Ell &h, const int32_t *lpat, int64_t i,
                                         int32_t m[3]) {
    if constexpr (FormTraits<FORM>::compact) {
        const int pid = h.pid[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int32_t d = lpat[pid * kMaxWidth + k];
            m[k] = d == kEmptySlot ? -1 : (int32_t)(i + d);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) m[k] = h.nbr[k * h.n + i];
    }
}

template <int FORM>
__device__ __forceinline__ double row_ons_f(const Ell &h, const Walk &wk, int64_t i) {
    if constexpr (FormTraits<FORM>::ons_float)
        return (double)h.onsf[i] * wk.inv_es;
    else
        return h.ons[i];
}

// row_h with the structure form fixed at compile time (same operations, in
// the same order, as row_h).
template <int FORM, typename V>
__device__ __forceinline__ double2 row_h_f(const Ell &h, const Walk &wk, const int32_t *lpat,
                                           const V *x, int64_t i, int64_t v, int vshift,
                                           double2 xi) {
    if constexpr (FormTraits<FORM>::generic) {
        return row_h(h, wk, lpat, x, i, v, vshift, xi);
    } else {
        int32_t m[3];
        row_nbrs<FORM>(h, lpat, i, m);
        const double o = row_ons_f<FORM>(h, wk, i);
        double2 xm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) xm[k] = ld(x + ((int64_t)(m[k] < 0 ? 0 : m[k]) << vshift) + v);
        double2 acc = make_double2(o * xi.x, o * xi.y);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc = raxpy(acc, m[k] < 0 ? 0.0 : wk.t, xm[k]);
        return acc;
    }
}

// row_hd with the structure form fixed at compile time.
template <int FORM, typename V>
__device__ __forceinline__ void row_hd_f(const Ell &h, const Walk &wk, const int32_t *lpat,
                                         const V *x, int64_t i, int64_t v, int vshift,
                                         double2 xi, double2 &hx, double2 &dx) {
    if constexpr (FormTraits<FORM>::generic) {
        row_hd(h, wk, lpat, x, i, v, vshift, xi, hx, dx);
    } else {
        int32_t m[3];
        row_nbrs<FORM>(h, lpat, i, m);
        const double o = row_ons_f<FORM>(h, wk, i);
        double2 xm[3];
        double xk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xm[k] = ld(x + ((int64_t)(m[k] < 0 ? 0 : m[k]) << vshift) + v);
            xk[k] = h.xw[k * h.n + i];
        }
        hx = make_double2(o * xi.x, o * xi.y);
        dx = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            hx = raxpy(hx, m[k] < 0 ? 0.0 : wk.t, xm[k]);
            dx = raxpy(dx, m[k] < 0 ? 0.0 : xk[k], xm[k]);
        }
    }
}

// Recursion step of the moments, out = 2 H~ p1 - p0 and <L|out>, with ILP
// elements per thread per pass: all loads of the ILP elements are issued
// before any arithmetic, so a wavefront keeps ILP times more bytes in flight
// (the gathers depend on the index loads, which would otherwise serialise
// two memory latencies per element).  Elements are visited in the same order,
// and every form performs the same floating-point operations, so all ILP,
// streaming and form choices give bit-identical results.
//
// DBL is the doubling form for phi_L = phi_R (the product identities
// T_{2n} = 2 T_n T_n - T_0 and T_{2n+1} = 2 T_{n+1} T_n - T_1): with
// p1 = phi_n it accumulates <phi_n|phi_n> into slot and <phi_n|phi_{n+1}>
// into slot + 1, from values the step holds anyway, so phi_L is not read.
template <typename V, int ILP, bool NT, int FORM, bool DBL>
__global__ __launch_bounds__(kBlock) void k_moment_step(Ell h, Sweep sw, const V *p1,
                                                        const V *p0, V *out,
                                                        const V *__restrict__ phil,
                                                        double2 *__restrict__ partial,
                                                        int slot) {
    using F = FormTraits<FORM>;
    const int64_t po = plane_off(sw);
    p1 = on_plane(p1, po);
    p0 = on_plane(p0, po);
    out = on_plane(out, po);
    phil = on_plane(phil, po);
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    __shared__ int32_t lpat[kMaxPatterns * kMaxWidth];
    if (F::compact || (F::generic && h.pid)) {
        for (int j = threadIdx.x; j < h.npat * kMaxWidth; j += kBlock) lpat[j] = h.pat[j];
        __syncthreads();
    }
    const Walk wk = walk_of(sw);
    const int64_t vmask = ((int64_t)1 << sw.vshift) - 1;
    for (int64_t b = wk.b0 + wk.loc; b < wk.b1; b += (int64_t)wk.nloc * ILP) {
        int64_t e[ILP];
        bool ok[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            const int64_t bu = b + (int64_t)u * wk.nloc;
            ok[u] = bu < wk.b1 && block_elem(wk, bu, threadIdx.x, sw.vshift, e[u]);
            e[u] = ok[u] ? e[u] : 0;          // a safe element; its result is dropped
        }
        int32_t m[ILP][F::width];
        double hk[ILP][F::width];
        double on[ILP];
        double2 xi[ILP], l[ILP], q[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            const int64_t i = e[u] >> sw.vshift;
            if constexpr (F::generic) {
                const int pid = row_pid(h, i);
#pragma unroll
                for (int k = 0; k < F::width; ++k) {
                    m[u][k] = k < h.w ? slot_row(h, lpat, pid, i, k) : -1;
                    hk[u][k] = (k < h.w && h.hop) ? h.hop[k * h.n + i] : wk.t;
                }
                on[u] = row_ons(h, wk, i);
            } else {
                if constexpr (F::compact) {
                    const int pid = h.pid[i];
#pragma unroll
                    for (int k = 0; k < F::width; ++k) {
                        const int32_t d = lpat[pid * kMaxWidth + k];
                        m[u][k] = d == kEmptySlot ? -1 : (int32_t)(i + d);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < F::width; ++k) m[u][k] = h.nbr[k * h.n + i];
                }
#pragma unroll
                for (int k = 0; k < F::width; ++k) hk[u][k] = wk.t;
                if constexpr (F::ons_float)
                    on[u] = (double)h.onsf[i] * wk.inv_es;
                else
                    on[u] = h.ons[i];
            }
            xi[u] = ld(p1 + e[u]);
            if constexpr (DBL)
                l[u] = xi[u];
            else
                l[u] = NT ? ld_nt(phil + e[u]) : ld(phil + e[u]);
            q[u] = NT ? ld_nt(p0 + e[u]) : ld(p0 + e[u]);
        }
        double2 acc[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            const int64_t v = e[u] & vmask;
            acc[u] = make_double2(on[u] * xi[u].x, on[u] * xi[u].y);
#pragma unroll
            for (int k = 0; k < F::width; ++k) {
                if (F::generic && k >= h.w) continue;
                const int32_t mm = m[u][k];
                const double2 xm = ld(p1 + ((int64_t)(mm < 0 ? 0 : mm) << sw.vshift) + v);
                const double hh = mm < 0 ? 0.0 : hk[u][k];
                acc[u] = raxpy(acc[u], hh, xm);
            }
        }
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            if (ok[u]) {
                const double2 o = rounded<V>(two_minus(acc[u], q[u]));
                if (NT)
                    st_nt(out + e[u], o);
                else
                    st(out + e[u], o);
                if constexpr (DBL) {
                    s0 = cdot_acc(s0, l[u], xi[u]);
                    s1 = cdot_acc(s1, l[u], o);
                } else {
                    s0 = cdot_acc(s0, l[u], o);
                }
            }
        }
    }
    const int64_t r = (int64_t)1 << sw.vshift;
    block_sum(s0, sw.vshift, partial + part_index(sw, slot) * r);
    if constexpr (DBL) block_sum(s1, sw.vshift, partial + part_index(sw, slot + 1) * r);
}

// Moments from the doubling sums, in place: row t of mom holds
// a_j = <phi_n|phi_n> (j = 2n) and <phi_n|phi_{n+1}> (j = 2n + 1) for j >= 2 and
// C_0, C_1 at j = 0, 1; C_j = 2 a_j - C_{j mod 2}.
__global__ __launch_bounds__(kBlock) void k_undouble(double2 *__restrict__ mom, int rows,
                                                     int64_t stride, int64_t offset, int nm) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t per = nm - 2;
    if (per <= 0 || id >= (int64_t)rows * per) return;
    const int64_t t = id / per;
    const int j = (int)(id % per) + 2;
    double2 *c = mom + t * stride + offset;
    const double2 a = c[j], b = c[j & 1];
    c[j] = make_double2(fma(2.0, a.x, -b.x), fma(2.0, a.y, -b.y));
}

// Loads and stores of the propagator kernels: non-temporal when NT, cached
// otherwise (with few vectors the written state, gathered again by the next
// step, then stays in cache).
template <bool NT, typename V>
__device__ __forceinline__ double2 ldx(const V *p) {
    return NT ? ld_nt(p) : ld(p);
}
template <bool NT, typename V>
__device__ __forceinline__ void stx(V *p, double2 v) {
    if (NT)
        st_nt(p, v);
    else
        st(p, v);
}

template <typename V, bool FIRST, int FORM, bool NT>
__global__ __launch_bounds__(kBlock) void k_evolve_step(Ell h, Sweep sw, const V *p1,
                                                        const V *p0, V *out, V *acc,
                                                        const V *add, Coef c0, Coef c) {
    const int64_t po = plane_off(sw);
    p1 = on_plane(p1, po);
    p0 = on_plane(p0, po);
    out = on_plane(out, po);
    acc = on_plane(acc, po);
    add = on_plane(add, po);
    KPM_SWEEP_BEGIN(sw, h)
    const double2 cm = coef(c, sg);
    const double2 xi = ld(p1 + e);
    const double2 hx = row_h_f<FORM>(h, wk_, lpat, p1, i, v, sw.vshift, xi);
    double2 o, a;
    if (FIRST) {
        o = rounded<V>(hx);
        a = cmla(cmul(coef(c0, sg), xi), cm, o);
        if (add) a = cadd(ldx<NT>(add + e), a);
    } else {
        o = rounded<V>(two_minus(hx, ldx<NT>(p0 + e)));
        a = cmla(ldx<NT>(acc + e), cm, o);
    }
    stx<NT>(out + e, o);
    stx<NT>(acc + e, a);
    KPM_SWEEP_END
}

template <typename V, bool FIRST, int FORM, bool NT>
__global__ __launch_bounds__(kBlock) void k_evolve_x_step(Ell h, Sweep sw, const V *p1,
                                                          const V *p0, V *pout,
                                                          const V *q1, const V *q0,
                                                          V *qout, V *accx, V *accu,
                                                          Coef c0, Coef c) {
    const int64_t po = plane_off(sw);
    p1 = on_plane(p1, po);
    p0 = on_plane(p0, po);
    pout = on_plane(pout, po);
    q1 = on_plane(q1, po);
    q0 = on_plane(q0, po);
    qout = on_plane(qout, po);
    accx = on_plane(accx, po);
    accu = on_plane(accu, po);
    KPM_SWEEP_BEGIN(sw, h)
    const double2 cm = coef(c, sg);
    const double2 xi = ld(p1 + e);
    double2 hp, dp;
    row_hd_f<FORM>(h, wk_, lpat, p1, i, v, sw.vshift, xi, hp, dp);
    if (FIRST) {
        hp = rounded<V>(hp);
        dp = rounded<V>(dp);
        stx<NT>(pout + e, hp);
        stx<NT>(qout + e, dp);
        stx<NT>(accx + e, cmul(cm, dp));
        stx<NT>(accu + e, cmla(cmul(coef(c0, sg), xi), cm, hp));
    } else {
        const double2 qi = ld(q1 + e);
        const double2 hq = row_h_f<FORM>(h, wk_, lpat, q1, i, v, sw.vshift, qi);
        const double2 pp = ldx<NT>(p0 + e);
        const double2 qq = q0 ? ldx<NT>(q0 + e) : make_double2(0.0, 0.0);
        const double2 po = rounded<V>(two_minus(hp, pp));
        const double2 qo = rounded<V>(two_minus(cadd(dp, hq), qq));
        stx<NT>(pout + e, po);
        stx<NT>(qout + e, qo);
        stx<NT>(accx + e, cmla(ldx<NT>(accx + e), cm, qo));
        stx<NT>(accu + e, cmla(ldx<NT>(accu + e), cm, po));
    }
    KPM_SWEEP_END
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_apply_d(Ell h, Sweep sw, const V *x, V *y,
                                                    Coef alpha) {
    const int64_t po = plane_off(sw);
    x = on_plane(x, po);
    y = on_plane(y, po);
    KPM_SWEEP_BEGIN(sw, h)
    st(y + e, cmul(coef(alpha, sg), row_d(h, lpat, x, i, v, sw.vshift)));
    KPM_SWEEP_END
}

// partial[slot] = <a|b> per work-group (and vector).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_dot(Sweep sw, const V *__restrict__ a,
                                                const V *__restrict__ b,
                                                double2 *__restrict__ partial, int slot) {
    const int64_t po = plane_off(sw);
    a = on_plane(a, po);
    b = on_plane(b, po);
    double2 s0 = make_double2(0.0, 0.0);
    const Walk wk = walk_of(sw);
    for (int64_t blk = wk.b0 + wk.loc; blk < wk.b1; blk += wk.nloc) {
        int64_t e;
        if (block_elem(wk, blk, threadIdx.x, sw.vshift, e))
            s0 = cdot_acc(s0, ld_nt(a + e), ld_nt(b + e));
    }
    const int64_t r = (int64_t)1 << sw.vshift;
    block_sum(s0, sw.vshift, partial + part_index(sw, slot) * r);
}

// Layout conversion of a state with R = 2^vshift vectors: rows-major [n][R]
// (to_planar: source) and vector-major [R][n].  A group moves a tile of
// kPlanarTile / R rows through LDS, so both sides are read and written in
// contiguous runs; the tile is padded by one element per 32 against bank
// conflicts.  Values are copied bit for bit.
constexpr int kPlanarTile = 2048;
__device__ __forceinline__ int planar_pad(int q) { return q + (q >> 5); }

template <typename V>
__global__ __launch_bounds__(kBlock) void k_planar(const V *__restrict__ src, V *__restrict__ dst,
                                                   int64_t n, int vshift, int to_planar) {
    __shared__ V tile[kPlanarTile + kPlanarTile / 32];
    const int r = 1 << vshift;
    const int tr = kPlanarTile >> vshift;                 // rows per tile
    const int64_t row0 = (int64_t)blockIdx.x * tr;
    const int rows = (int)min((int64_t)tr, n - row0);
    const int cnt = rows << vshift;
    if (to_planar) {
        for (int q = threadIdx.x; q < cnt; q += kBlock)
            tile[planar_pad((q & (r - 1)) * tr + (q >> vshift))] = src[(row0 << vshift) + q];
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            const int v = q / rows, i = q - v * rows;
            dst[(int64_t)v * n + row0 + i] = tile[planar_pad(v * tr + i)];
        }
    } else {
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            const int v = q / rows, i = q - v * rows;
            tile[planar_pad(v * tr + i)] = src[(int64_t)v * n + row0 + i];
        }
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock)
            dst[(row0 << vshift) + q] = tile[planar_pad((q & (r - 1)) * tr + (q >> vshift))];
    }
}

// One thread per (row, energy): Hanning-windowed Fourier sum (Eq. 22-24),
// sum_n w_n Re[exp(i theta_k n) F_n] with theta_k = E_k dtau / hbar.
__global__ __launch_bounds__(kBlock) void k_ftm_sum(const double2 *__restrict__ f, int rows,
                                                    int nm, const double *__restrict__ w,
                                                    const double *__restrict__ theta, int ne,
                                                    double pref, double *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= (int64_t)rows * ne) return;
    const int t = (int)(id / ne), k = (int)(id % ne);
    const double2 *c = f + (int64_t)t * (2 * nm + 1);
    double acc = 0.0;
    for (int j = 0; j <= 2 * nm; ++j) {
        double sn, cs;
        sincos(theta[k] * (double)(j - nm), &sn, &cs);
        acc = fma(w[j], fma(cs, c[j].x, -sn * c[j].y), acc);
    }
    out[id] = pref * acc;
}

// One block per (slot, vector, segment): sums the segment's group partials
// in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce(const double2 *__restrict__ partial,
                                                   Sweep sw, double2 *__restrict__ dst,
                                                   int64_t stride_r, int64_t offset) {
    const int slot = blockIdx.x;
    const int r = blockIdx.y;
    const int sgi = blockIdx.z;
    const Seg s = sw.seg ? sw.seg[sgi] : sw.one;
    const int64_t nr = (int64_t)1 << sw.vshift;
    const double2 *p = partial + ((int64_t)slot * sw.nwg + s.g0) * nr + r;
    double2 acc = make_double2(0.0, 0.0);
    for (int g = threadIdx.x; g < s.nwg; g += kBlock) acc = cadd(acc, p[(int64_t)g * nr]);
    __shared__ double2 red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[((int64_t)sgi * nr + r) * stride_r + offset + slot] = red[0];
}

// One thread per (row, energy): Chebyshev series by the three-term recurrence.
__global__ __launch_bounds__(kBlock) void k_kpm_sum(const double *__restrict__ mom, int rows,
                                                    int nm, const double *__restrict__ w,
                                                    const double *__restrict__ eps,
                                                    const double *__restrict__ pref, int ne,
                                                    double *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= (int64_t)rows * ne) return;
    const int t = (int)(id / ne), k = (int)(id % ne);
    const double x = eps[k];
    const double *c = mom + (int64_t)t * nm;
    double tm2 = 1.0, tm1 = x;
    double s = w[0] * c[0];
    if (nm > 1) s = fma(w[1] * x, c[1], s);
    for (int m = 2; m < nm; ++m) {
        const double tm = fma(2.0 * x, tm1, -tm2);
        s = fma(w[m] * tm, c[m], s);
        tm2 = tm1;
        tm1 = tm;
    }
    out[id] = pref[k] * s;
}

// ---------------------------------------------------------------- multi-step sweeps
// Two recursion steps of the moments per pass over a chain lattice (one
// vector per row, width-3 compact form): from phi_n (p1) and phi_{n-1} (p0)
// it writes phi_{n+1} (out1) and phi_{n+2} (out2), so each row's operands
// cross HBM once per two steps instead of once per step.
//
// A work-group takes a tile of TJ chains x kTileCols columns.  It
// stages phi_n on the tile widened by two columns and two chains in LDS
// (s0w), computes phi_{n+1} on the tile widened by one (s1w; the ring around
// the tile is recomputed by the neighbouring tiles too), writes the tile's
// phi_{n+1}, and then phi_{n+2} of the tile from s1w.  Neighbours are found
// in LDS from each pattern's (chain, column) steps in lat.code, which the host
// has checked against every row.  Periodic wrap is by index, so any tile of
// any sample size reads in bounds.  Every element goes through the same
// floating-point operations as k_moment_step (phi_{n+1} stored in s1w is the
// value a store into V holds), so the states are the single-step states;
// only the grouping of the inner-product partial sums differs.
//
// Inputs are never written: out1 and out2 must differ from p1, p0 and each
// other (a neighbouring tile may still read p0 and p1 at this tile's rows).
// Non-DBL: partial[slot] = <L|phi_{n+1}>, partial[slot+1] = <L|phi_{n+2}>.
// DBL (phi_L = phi_R): slots slot .. slot+3 get <phi_n|phi_n>,
// <phi_n|phi_{n+1}>, <phi_{n+1}|phi_{n+1}>, <phi_{n+1}|phi_{n+2}>.

// Row offset in a window of row width WW for slot code c (0xFF = empty: 0).
template <int WW>
__device__ __forceinline__ int code_offset(uint32_t c) {
    const int dj = (int)((c * 11u) >> 5) - 1;    // c / 3 - 1 for c < 9
    const int di = (int)c - 3 * (dj + 1) - 1;
    return c == 0xFFu ? 0 : dj * WW + di;
}

template <typename V, bool NT, bool ONSF, bool DBL, int TJ>
__global__ __launch_bounds__(kBlock) void k_moment_step2(Ell h, Sweep sw, Lat2 lat,
                                                         const V *p1, const V *p0,
                                                         V *__restrict__ out1,
                                                         V *__restrict__ out2,
                                                         const V *__restrict__ phil,
                                                         double2 *__restrict__ partial,
                                                         int slot) {
    constexpr int TI = kTileCols;
    constexpr int W0 = TI + 4, W1 = TI + 2;           // row widths of the two windows
    constexpr int N0 = (TJ + 4) * W0, N1 = (TJ + 2) * W1;
    constexpr int L0 = (N0 + kBlock - 1) / kBlock;     // window loads per thread
    constexpr int NI = TJ * TI / kBlock;               // tile elements per thread
    static_assert(TJ * TI % kBlock == 0 && 2 * W1 + 2 * TJ <= kBlock, "tile shape");
    __shared__ double2 s0w[N0];
    __shared__ double2 s1w[N1];
    __shared__ uint32_t lcode[kMaxPatterns];
    for (int j = threadIdx.x; j < h.npat; j += kBlock) lcode[j] = lat.code[j];
    __syncthreads();
    const int tid = threadIdx.x;
    const int nx = lat.nx, ny = lat.ny;
    const double t = sw.one.t, inv_es = sw.one.inv_es;
    const int lb = blockIdx.x;
    const int loc = lb / kXcds, nloc = sw.nwg / kXcds;
    const int ntile = lat.nti * lat.ntj;
    const int per = (ntile + kXcds - 1) / kXcds;
    const int b0 = (lb % kXcds) * per, b1 = min(b0 + per, ntile);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
    for (int b = b0 + loc; b < b1; b += nloc) {
        const int strip = b / lat.ntj;
        const int i0 = strip * TI, j0 = (b - strip * lat.ntj) * TJ;
        const int W = min(TI, nx - i0), H = min(TJ, ny - j0);
        const int n0 = (H + 4) * W0;
        // global loads of the whole tile first
        double2 win[L0];
#pragma unroll
        for (int u = 0; u < L0; ++u) {
            const int idx = tid + u * kBlock;
            const int wj = idx / W0, wi = idx - (idx / W0) * W0;
            const int gj = wrap_index(j0 - 2 + wj, ny), gi = wrap_index(i0 - 2 + wi, nx);
            win[u] = idx < n0 ? ld(p1 + (int64_t)gj * nx + gi) : make_double2(0.0, 0.0);
        }
        int rI[NI], pI[NI];
        bool okI[NI];
        double oI[NI];
        double2 qI[NI], lI[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int idx = tid + u * kBlock;
            const int wi = idx % TI, wj = idx / TI;
            okI[u] = wi < W && wj < H;
            rI[u] = okI[u] ? (j0 + wj) * nx + i0 + wi : 0;     // row 0: a safe row
            pI[u] = h.pid[rI[u]];
            oI[u] = ONSF ? (double)h.onsf[rI[u]] * inv_es : h.ons[rI[u]];
            qI[u] = ldx<NT>(p0 + rI[u]);
            lI[u] = DBL ? make_double2(0.0, 0.0) : ldx<NT>(phil + rI[u]);
        }
        // the ring of window 1 around the tile: one element per thread
        const int nh = 2 * (W + 2) + 2 * H;
        int hj, hi;
        if (tid < W + 2) {
            hj = 0;
            hi = tid;
        } else if (tid < 2 * (W + 2)) {
            hj = H + 1;
            hi = tid - (W + 2);
        } else {
            const int k = tid - 2 * (W + 2);
            hj = 1 + (k >> 1);
            hi = (k & 1) ? W + 1 : 0;
        }
        const bool okH = tid < nh;
        const int rH = okH ? wrap_index(j0 - 1 + hj, ny) * nx + wrap_index(i0 - 1 + hi, nx) : 0;
        const int pH = h.pid[rH];
        const double oH = ONSF ? (double)h.onsf[rH] * inv_es : h.ons[rH];
        const double2 qH = ldx<NT>(p0 + rH);

        __syncthreads();                 // the previous tile is done with s0w and s1w
#pragma unroll
        for (int u = 0; u < L0; ++u) {
            const int idx = tid + u * kBlock;
            if (idx < n0) s0w[idx] = win[u];
        }
        __syncthreads();
        // Pattern codes are looked up only now: an LDS lookup that depends on a
        // global load would wait for every load issued before it.
        uint32_t cI[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) cI[u] = lcode[pI[u]];
        const uint32_t cH = lcode[pH];
        // phase 1: phi_{n+1} on the tile (kept for phase 2) and on the ring
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int idx = tid + u * kBlock;
            const int wi = idx % TI, wj = idx / TI;
            const int pos = (wj + 2) * W0 + wi + 2;
            const double2 x = s0w[pos];
            double2 acc = make_double2(oI[u] * x.x, oI[u] * x.y);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t c = (cI[u] >> (8 * k)) & 0xFFu;
                acc = raxpy(acc, c == 0xFFu ? 0.0 : t, s0w[pos + code_offset<W0>(c)]);
            }
            const double2 y = rounded<V>(two_minus(acc, qI[u]));
            if (okI[u]) {
                s1w[(wj + 1) * W1 + wi + 1] = y;
                stx<NT>(out1 + rI[u], y);
                if (DBL) {
                    a0 = cdot_acc(a0, x, x);
                    a1 = cdot_acc(a1, x, y);
                } else {
                    a0 = cdot_acc(a0, lI[u], y);
                }
            }
        }
        if (okH) {
            const int pos = (hj + 1) * W0 + hi + 1;
            const double2 x = s0w[pos];
            double2 acc = make_double2(oH * x.x, oH * x.y);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t c = (cH >> (8 * k)) & 0xFFu;
                acc = raxpy(acc, c == 0xFFu ? 0.0 : t, s0w[pos + code_offset<W0>(c)]);
            }
            s1w[hj * W1 + hi] = rounded<V>(two_minus(acc, qH));
        }
        __syncthreads();
        // phase 2: phi_{n+2} on the tile
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (!okI[u]) continue;
            const int idx = tid + u * kBlock;
            const int wi = idx % TI, wj = idx / TI;
            const int pos = (wj + 1) * W1 + wi + 1;
            const double2 x = s1w[pos];
            double2 acc = make_double2(oI[u] * x.x, oI[u] * x.y);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t c = (cI[u] >> (8 * k)) & 0xFFu;
                acc = raxpy(acc, c == 0xFFu ? 0.0 : t, s1w[pos + code_offset<W1>(c)]);
            }
            const double2 z = rounded<V>(two_minus(acc, s0w[(wj + 2) * W0 + wi + 2]));
            stx<NT>(out2 + rI[u], z);
            if (DBL) {
                a2 = cdot_acc(a2, x, x);
                a3 = cdot_acc(a3, x, z);
            } else {
                a1 = cdot_acc(a1, lI[u], z);
            }
        }
    }
    const int nw = sw.nwg;
    block_sum(a0, 0, partial + (int64_t)slot * nw + blockIdx.x);
    block_sum(a1, 0, partial + (int64_t)(slot + 1) * nw + blockIdx.x);
    if (DBL) {
        block_sum(a2, 0, partial + (int64_t)(slot + 2) * nw + blockIdx.x);
        block_sum(a3, 0, partial + (int64_t)(slot + 3) * nw + blockIdx.x);
    }
}

// Register-tiled sweep of K = 2, 3 or 4 recursion steps per pass, for
// lattices whose slots are ordered like the graphene builder's (slot 0 the
// previous column, slot 1 the next column, slot 2 the previous or next chain,
// each possibly empty; lat.flags[p] bit k = slot k filled, bit 3 = slot 2 is
// the next chain).  A wavefront takes a tile of TJ chains x (kWave - 2K)
// columns on its own: lane l holds column c0 - K + l of every row, so a row's
// vertical neighbours sit in the lane's own registers and its horizontal ones
// in lanes l -+ 1 (DPP wavefront shifts).  phi_n is loaded on TJ + 2K chains and
// step s computes phi_{n+s} on TJ + 2 (K - s) of them, valid in lanes
// s .. kWave - 1 - s, so after K steps the tile (lanes K .. kWave - 1 - K)
// holds phi_{n+K}.  Only phi_{n+K-1} (out1) and phi_{n+K} (out2) are written,
// the two states the next pass starts from: per row, phi_n, phi_{n-1}, phi_L
// and the structure are read and two states written once per K steps.  No
// LDS tile and no barrier: every load of a tile is issued before its
// arithmetic.  Each state value goes through the operations of
// k_moment_step, in its slot order.
// Partials: non-DBL slot + s - 1 = <L|phi_{n+s}>, s = 1 .. K; DBL slots
// slot + 2 (s - 1) and + 1 = <phi_{n+s-1}|phi_{n+s-1}>, <phi_{n+s-1}|phi_{n+s}>.

// 2 H~ x - q at a row with flags f: own value x, horizontal neighbours from
// the adjacent lanes, vertical from xup (next chain) or xdn (previous chain).
__device__ __forceinline__ double2 reg_row_step(double o, double t, uint32_t f, double2 x,
                                                double2 xup, double2 xdn, double2 q) {
    const double2 xl = lane_prev(x), xr = lane_next(x);
    const double2 xv = (f & 8u) ? xup : xdn;
    double2 acc = make_double2(o * x.x, o * x.y);
    acc = raxpy(acc, (f & 1u) ? t : 0.0, xl);
    acc = raxpy(acc, (f & 2u) ? t : 0.0, xr);
    acc = raxpy(acc, (f & 4u) ? t : 0.0, xv);
    return two_minus(acc, q);
}

template <typename V, bool ONSF, bool DBL, int TJ, int K>
__global__ __launch_bounds__(kBlock) void k_moment_stepk(Ell h, Sweep sw, Lat2 lat,
                                                         const V *p1, const V *p0,
                                                         V *__restrict__ out1,
                                                         V *__restrict__ out2,
                                                         const V *__restrict__ phil,
                                                         double2 *__restrict__ partial,
                                                         int slot) {
    constexpr int TC = kWave - 2 * K;                  // columns per tile
    constexpr int R0 = TJ + 2 * K;                     // window: chains j0 - K .. j0 + TJ + K - 1
    constexpr int NA = DBL ? 2 * K : K;                // partial sums
    __shared__ uint32_t lflag[kMaxPatterns];
    for (int j = threadIdx.x; j < h.npat; j += kBlock) lflag[j] = lat.flags[j];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = lat.nx, ny = lat.ny;
    const double t = sw.one.t, inv_es = sw.one.inv_es;
    const int nst = (nx + TC - 1) / TC, nrb = (ny + TJ - 1) / TJ;
    const int ntile = nst * nrb;
    const int lb = blockIdx.x;
    const int per = (ntile + kXcds - 1) / kXcds;
    const int b0 = (lb % kXcds) * per, b1 = min(b0 + per, ntile);
    constexpr int kWaves = kBlock / kWave;
    // the wavefront's index as a scalar: tile coordinates and row bases are
    // then scalar, and each load takes the lane's column as its offset
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int wloc = (lb / kXcds) * kWaves + wv;
    const int wn = (sw.nwg / kXcds) * kWaves;
    double2 acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int b = b0 + wloc; b < b1; b += wn) {
        // tiles across the strips first: the column halos a tile shares with
        // its horizontal neighbours, like the chain halos it shares with its
        // vertical ones, are then read by wavefronts in flight together
        const int strip = b % nst;
        const int j0 = (b / nst) * TJ, c0 = strip * TC;
        const int gi = wrap_index(c0 - K + lane, nx);
        const bool colok = lane >= K && lane < K + TC && c0 - K + lane < nx;
        const int H = min(TJ, ny - j0);
        const uint32_t ov = (uint32_t)gi * sizeof(V), rb = (uint32_t)nx * sizeof(V);
        auto base = [&](int w) { return (int64_t)wrap_index(j0 - K + w, ny) * nx; };
        // every load of the tile first, pattern ids leading (their flag
        // lookups then wait for nothing else)
        int pf[R0];
#pragma unroll
        for (int w = 1; w < R0 - 1; ++w)
            pf[w] = __builtin_amdgcn_raw_buffer_load_b8(row_rsrc(h.pid + base(w), (uint32_t)nx),
                                                        gi, 0, 0);
        double2 B[R0];                                  // phi_n
#pragma unroll
        for (int w = 0; w < R0; ++w) B[w] = buf_ld(p1 + base(w), rb, ov);
        double2 A[R0];                                  // phi_{n-1}
        float of[R0];
        double od[R0];
#pragma unroll
        for (int w = 1; w < R0 - 1; ++w) {
            A[w] = buf_ld(p0 + base(w), rb, ov);
            if (ONSF)
                of[w] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(
                               row_rsrc(h.onsf + base(w), (uint32_t)nx * 4u), gi * 4, 0, 0));
            else
                od[w] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(
                                row_rsrc(h.ons + base(w), (uint32_t)nx * 8u), gi * 8, 0, 0));
        }
        double2 L[TJ];
#pragma unroll
        for (int r = 0; r < TJ; ++r)
            L[r] = DBL ? make_double2(0.0, 0.0) : buf_ld(phil + base(K + r), rb, ov);
        uint32_t fl[R0];
#pragma unroll
        for (int w = 1; w < R0 - 1; ++w) fl[w] = lflag[pf[w]];
#pragma unroll
        for (int s = 1; s <= K; ++s) {
            double2 C[R0];
#pragma unroll
            for (int w = s; w < R0 - s; ++w) {
                const double o = ONSF ? (double)of[w] * inv_es : od[w];
                C[w] = rounded<V>(reg_row_step(o, t, fl[w], B[w], B[w + 1], B[w - 1], A[w]));
            }
#pragma unroll
            for (int r = 0; r < TJ; ++r) {
                if (r < H && colok) {
                    if (DBL) {
                        acc[2 * (s - 1)] = cdot_acc(acc[2 * (s - 1)], B[K + r], B[K + r]);
                        acc[2 * (s - 1) + 1] = cdot_acc(acc[2 * (s - 1) + 1], B[K + r], C[K + r]);
                    } else {
                        acc[s - 1] = cdot_acc(acc[s - 1], L[r], C[K + r]);
                    }
                }
            }
#pragma unroll
            for (int w = s; w < R0 - s; ++w) {
                A[w] = B[w];
                B[w] = C[w];
            }
        }
#pragma unroll
        for (int r = 0; r < TJ; ++r) {
            if (r < H && colok) {
                const int64_t row = (int64_t)(j0 + r) * nx;
                buf_st(out1 + row, rb, ov, A[K + r]);
                buf_st(out2 + row, rb, ov, B[K + r]);
            }
        }
    }
    const int nw = sw.nwg;
#pragma unroll
    for (int k = 0; k < NA; ++k) block_sum(acc[k], 0, partial + (int64_t)(slot + k) * nw + blockIdx.x);
}

// Marching form of the register-tiled K-step sweep: kpm_march.h

// ---------------------------------------------------------------- launchers
template <typename V, int ILP, bool NT, bool DBL>
static void launch_step_shape(const Ell &h, const Sweep &sw, const V *p1, const V *p0, V *out,
                              const V *phil, double2 *partial, int slot, hipStream_t s) {
    switch (form_of(h)) {
#define KPM_FORM_CASE(F)                                                                       \
        case F:                                                                                \
            hipLaunchKernelGGL((k_moment_step<V, ILP, NT, F, DBL>), dim3(sw.nwg, sw.nplanes), dim3(kBlock), \
                               0, s, h, sw, p1, p0, out, phil, partial, slot);                 \
            break;
        KPM_FORM_CASE(kFormC3F)
        KPM_FORM_CASE(kFormC3D)
        KPM_FORM_CASE(kFormL3F)
        KPM_FORM_CASE(kFormL3D)
        default:
        KPM_FORM_CASE(kFormGeneric)
#undef KPM_FORM_CASE
    }
}

template <typename V, bool DBL>
static void launch_step_ilp(const Ell &h, const Sweep &sw, const V *p1, const V *p0, V *out,
                            const V *phil, double2 *partial, int slot, hipStream_t s) {
    const int ilp = sw.ilp >= 4 ? 4 : (sw.ilp == 2 ? 2 : 1);
    if (sw.nt) {
        if (ilp == 4) launch_step_shape<V, 4, true, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
        else if (ilp == 2) launch_step_shape<V, 2, true, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
        else launch_step_shape<V, 1, true, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
    } else {
        if (ilp == 4) launch_step_shape<V, 4, false, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
        else if (ilp == 2) launch_step_shape<V, 2, false, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
        else launch_step_shape<V, 1, false, DBL>(h, sw, p1, p0, out, phil, partial, slot, s);
    }
}

template <typename V>
void launch_moment_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                        const V *p0, V *out, const V *phil, double2 *partial, int slot,
                        hipStream_t s) {
    if (first) {
        hipLaunchKernelGGL((k_moment_first<V>), dim3(sw.nwg, sw.nplanes), dim3(kBlock), 0, s, h, sw, p1,
                           out, phil, partial, slot);
        return;
    }
    launch_step_ilp<V, false>(h, sw, p1, p0, out, phil, partial, slot, s);
}

template <typename V>
void launch_moment_step_doubled(const Ell &h, const Sweep &sw, const V *p1, const V *p0,
                                V *out, double2 *partial, int slot, hipStream_t s) {
    launch_step_ilp<V, true>(h, sw, p1, p0, out, nullptr, partial, slot, s);
}

void launch_undouble(double2 *mom, int rows, int64_t stride, int64_t offset, int nm,
                     hipStream_t s) {
    const int64_t total = (int64_t)rows * (nm - 2);
    if (total <= 0) return;
    const int blocks = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_undouble, dim3(blocks), dim3(kBlock), 0, s, mom, rows, stride, offset,
                       nm);
}

#define KPM_BY_FORM(form, CALL)                                                    \
    switch (form) {                                                                \
        case kFormC3F: { constexpr int F = kFormC3F; CALL; } break;                \
        case kFormC3D: { constexpr int F = kFormC3D; CALL; } break;                \
        case kFormL3F: { constexpr int F = kFormL3F; CALL; } break;                \
        case kFormL3D: { constexpr int F = kFormL3D; CALL; } break;                \
        default: { constexpr int F = kFormGeneric; CALL; } break;                  \
    }

template <typename V>
void launch_evolve_step(const Ell &h, const Sweep &sw, bool first, const V *p1, const V *p0,
                        V *out, V *acc, const V *add, Coef c0, Coef c, hipStream_t s) {
#define KPM_EVOLVE(FIRST_, NT_)                                                               \
    KPM_BY_FORM(form_of(h),                                                                   \
                hipLaunchKernelGGL((k_evolve_step<V, FIRST_, F, NT_>), dim3(sw.nwg, sw.nplanes),          \
                                   dim3(kBlock), 0, s, h, sw, p1, p0, out, acc, add, c0, c))
    if (first && sw.nt) { KPM_EVOLVE(true, true) }
    else if (first) { KPM_EVOLVE(true, false) }
    else if (sw.nt) { KPM_EVOLVE(false, true) }
    else { KPM_EVOLVE(false, false) }
#undef KPM_EVOLVE
}

template <typename V>
void launch_evolve_x_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                          const V *p0, V *pout, const V *q1, const V *q0, V *qout,
                          V *accx, V *accu, Coef c0, Coef c, hipStream_t s) {
#define KPM_EVOLVE_X(FIRST_, NT_)                                                             \
    KPM_BY_FORM(form_of(h),                                                                   \
                hipLaunchKernelGGL((k_evolve_x_step<V, FIRST_, F, NT_>), dim3(sw.nwg, sw.nplanes),        \
                                   dim3(kBlock), 0, s, h, sw, p1, p0, pout, q1, q0, qout,     \
                                   accx, accu, c0, c))
    // always non-temporal: with ten state streams per step, caching them evicts
    // the gathered state (measured slower with one vector as well)
    if (first) { KPM_EVOLVE_X(true, true) }
    else { KPM_EVOLVE_X(false, true) }
#undef KPM_EVOLVE_X
}

template <typename V>
void launch_apply_d(const Ell &h, const Sweep &sw, const V *x, V *y, Coef alpha,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_apply_d<V>), dim3(sw.nwg, sw.nplanes), dim3(kBlock), 0, s, h, sw, x, y, alpha);
}

void launch_reduce(const double2 *partial, const Sweep &sw, int slots, double2 *dst,
                   int64_t stride_r, int64_t offset, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(slots, 1 << sw.vshift, sw.nseg), dim3(kBlock), 0, s,
                       partial, sw, dst, stride_r, offset);
}

template <typename V>
void launch_dot(const Sweep &sw, const V *a, const V *b, double2 *partial, int slot,
                hipStream_t s) {
    hipLaunchKernelGGL((k_dot<V>), dim3(sw.nwg, sw.nplanes), dim3(kBlock), 0, s, sw, a, b, partial, slot);
}

template <typename V>
void launch_planar(const V *src, V *dst, int64_t n, int vshift, bool to_planar, hipStream_t s) {
    const int64_t tr = kPlanarTile >> vshift;
    const int64_t blocks = (n + tr - 1) / tr;
    if (blocks <= 0) return;
    hipLaunchKernelGGL((k_planar<V>), dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, n,
                       vshift, to_planar ? 1 : 0);
}

void launch_ftm_sum(const double2 *f, int rows, int nm, const double *w, const double *theta,
                    int ne, double pref, double *out, hipStream_t s) {
    const int64_t total = (int64_t)rows * ne;
    const int blocks = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ftm_sum, dim3(blocks), dim3(kBlock), 0, s, f, rows, nm, w, theta, ne,
                       pref, out);
}

void launch_kpm_sum(const double *mom, int rows, int nm, const double *w, const double *eps,
                    const double *pref, int ne, double *out, hipStream_t s) {
    const int64_t total = (int64_t)rows * ne;
    const int blocks = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_kpm_sum, dim3(blocks), dim3(kBlock), 0, s, mom, rows, nm, w, eps,
                       pref, ne, out);
}

template <typename V>
bool launch_moment_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const V *p1,
                         const V *p0, V *out1, V *out2, const V *phil, double2 *partial,
                         int slot, bool dbl, bool re, hipStream_t s) {
    const bool onsf = h.onsf != nullptr;
    // the step counts each form is built for: LDS tiles 2, register tiles
    // 2 .. 4, marching strips 2 .. 8
    // (the real-part strips with FP64 states also nine)
    const int kmax = lat.reg == 2 ? (re && !dbl && std::is_same<V, double2>::value ? kReMarchSteps
                                                                                 : kMaxMarchSteps)
                                  : (lat.reg == 1 ? 4 : 2);
    if (lat.k < 2 || lat.k > kmax) return false;
    // vector-major states and batches run only in the marching strips
    if ((sw.nplanes > 1 || sw.seg) && lat.reg != 2) return false;
    if constexpr (std::is_same<V, float2>::value)
        if (lat.arith32 && lat.reg == 2)
            return launch_moment_multi_f32(h, sw, lat, p1, p0, out1, out2, phil, partial, slot,
                                           dbl, re, s);
#define KPM_LDS2(NT_, ONSF_, DBL_)                                                            \
    hipLaunchKernelGGL((k_moment_step2<V, NT_, ONSF_, DBL_, 16>), dim3(sw.nwg), dim3(kBlock),  \
                       0, s, h, sw, lat, p1, p0, out1, out2, phil, partial, slot)
#define KPM_REGK(ONSF_, DBL_, TJ_, K_)                                                        \
    hipLaunchKernelGGL((k_moment_stepk<V, ONSF_, DBL_, TJ_, K_>), dim3(sw.nwg), dim3(kBlock),  \
                       0, s, h, sw, lat, p1, p0, out1, out2, phil, partial, slot)
#define KPM_REG_K(ONSF_, DBL_, TJ_)                                                           \
    do {                                                                                      \
        if (lat.k == 4) KPM_REGK(ONSF_, DBL_, TJ_, 4);                                        \
        else if (lat.k == 3) KPM_REGK(ONSF_, DBL_, TJ_, 3);                                   \
        else KPM_REGK(ONSF_, DBL_, TJ_, 2);                                                   \
    } while (0)
#define KPM_MARCHK(ONSF_, DBL_, K_)                                                          \
    do {                                                                                      \
        if (!(DBL_) && re)                                                                    \
            hipLaunchKernelGGL((k_moment_march_re<V, ONSF_, K_>), dim3(sw.nwg, sw.nplanes), dim3(sw.wpg * kWave),  \
                               0, s, h, sw, lat, p1, p0, out1, out2, phil, partial, slot);    \
        else                                                                                  \
            hipLaunchKernelGGL((k_moment_march<V, ONSF_, DBL_, K_>), dim3(sw.nwg, sw.nplanes),            \
                               dim3(sw.wpg * kWave), 0, s, h, sw, lat, p1, p0, out1, out2, phil,      \
                               partial, slot);                                                \
    } while (0)
#define KPM_REG(ONSF_, DBL_)                                                                  \
    do {                                                                                      \
        if (lat.reg == 2) {                                                                   \
            if (lat.k > kMaxMarchSteps) {                                                     \
                if constexpr (std::is_same<V, double2>::value && !(DBL_)) {                   \
                    if (!launch_moment_march_re_long(h, sw, lat, p1, p0, out1, out2, phil,    \
                                                     partial, slot, s))                       \
                        return false;                                                         \
                } else {                                                                      \
                    return false;           /* no such pass (excluded by kmax above) */       \
                }                                                                             \
            } else if (lat.k == 8) KPM_MARCHK(ONSF_, DBL_, 8);                                \
            else if (lat.k == 7) KPM_MARCHK(ONSF_, DBL_, 7);                                  \
            else if (lat.k == 6) KPM_MARCHK(ONSF_, DBL_, 6);                                  \
            else if (lat.k == 5) KPM_MARCHK(ONSF_, DBL_, 5);                                  \
            else if (lat.k == 4) KPM_MARCHK(ONSF_, DBL_, 4);                                  \
            else if (lat.k == 3) KPM_MARCHK(ONSF_, DBL_, 3);                                  \
            else KPM_MARCHK(ONSF_, DBL_, 2);                                                  \
        } else if (lat.tj == 4) {                                                             \
            KPM_REG_K(ONSF_, DBL_, 4);                                                        \
        } else {                                                                              \
            KPM_REG_K(ONSF_, DBL_, 8);                                                        \
        }                                                                                     \
    } while (0)
    if (lat.reg) {
        if (onsf) { if (dbl) KPM_REG(true, true); else KPM_REG(true, false); }
        else { if (dbl) KPM_REG(false, true); else KPM_REG(false, false); }
    } else if (sw.nt) {
        if (onsf) { if (dbl) KPM_LDS2(true, true, true); else KPM_LDS2(true, true, false); }
        else { if (dbl) KPM_LDS2(true, false, true); else KPM_LDS2(true, false, false); }
    } else {
        if (onsf) { if (dbl) KPM_LDS2(false, true, true); else KPM_LDS2(false, true, false); }
        else { if (dbl) KPM_LDS2(false, false, true); else KPM_LDS2(false, false, false); }
    }
#undef KPM_LDS2
#undef KPM_REGK
#undef KPM_REG_K
#undef KPM_REG
#undef KPM_MARCHK
    return true;
}

template <typename V>
bool launch_evolve_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const V *p1,
                         const V *p0, V *out1, V *out2, V *acc, const CoefK &ck,
                         hipStream_t s) {
    if (lat.reg != 2 || lat.k < 2 || lat.k > kMaxMarchSteps) return false;
    if constexpr (std::is_same<V, float2>::value)
        if (lat.arith32) return launch_evolve_multi_f32(h, sw, lat, p1, p0, out1, out2, acc, ck, s);
#define KPM_EVK(ONSF_, K_)                                                                    \
    hipLaunchKernelGGL((k_evolve_march<V, ONSF_, K_>), dim3(sw.nwg, sw.nplanes), dim3(sw.wpg * kWave), 0, s, h,   \
                       sw, lat, p1, p0, out1, out2, acc, ck)
#define KPM_EV(ONSF_)                                                                         \
    switch (lat.k) {                                                                          \
        case 8: KPM_EVK(ONSF_, 8); break;                                                     \
        case 7: KPM_EVK(ONSF_, 7); break;                                                     \
        case 6: KPM_EVK(ONSF_, 6); break;                                                     \
        case 5: KPM_EVK(ONSF_, 5); break;                                                     \
        case 4: KPM_EVK(ONSF_, 4); break;                                                     \
        case 3: KPM_EVK(ONSF_, 3); break;                                                     \
        default: KPM_EVK(ONSF_, 2); break;                                                    \
    }
    if (h.onsf) { KPM_EV(true) }
    else { KPM_EV(false) }
#undef KPM_EV
#undef KPM_EVK
    return true;
}

#define KPM_INSTANTIATE(V)                                                                  \
    template void launch_moment_step<V>(const Ell &, const Sweep &, bool, const V *,        \
                                        const V *, V *, const V *, double2 *, int,          \
                                        hipStream_t);                                       \
    template void launch_moment_step_doubled<V>(const Ell &, const Sweep &, const V *,      \
                                                const V *, V *, double2 *, int,             \
                                                hipStream_t);                               \
    template void launch_evolve_step<V>(const Ell &, const Sweep &, bool, const V *,        \
                                        const V *, V *, V *, const V *, Coef, Coef,         \
                                        hipStream_t);                                       \
    template void launch_evolve_x_step<V>(const Ell &, const Sweep &, bool, const V *,      \
                                          const V *, V *, const V *, const V *, V *, V *,   \
                                          V *, Coef, Coef, hipStream_t);                    \
    template void launch_apply_d<V>(const Ell &, const Sweep &, const V *, V *, Coef,       \
                                    hipStream_t);                                           \
    template void launch_dot<V>(const Sweep &, const V *, const V *, double2 *, int,        \
                                hipStream_t);                                               \
    template void launch_planar<V>(const V *, V *, int64_t, int, bool, hipStream_t);        \
    template bool launch_moment_multi<V>(const Ell &, const Sweep &, const Lat2 &, const V *, \
                                         const V *, V *, V *, const V *, double2 *, int,    \
                                         bool, bool, hipStream_t);                          \
    template bool launch_evolve_multi<V>(const Ell &, const Sweep &, const Lat2 &, const V *, \
                                         const V *, V *, V *, V *, const CoefK &,           \
                                         hipStream_t);

KPM_INSTANTIATE(double2)
KPM_INSTANTIATE(float2)

// ---------------------------------------------------------------- coupled propagator strips
// K coupled steps of Alg. 7 per pass (Eq. 37-41): the recursion of T_m(H~) psi
// (p) and of [X, T_m(H~)] psi (q), q_{m+1} = 2 ([X, H~] p_m + H~ q_m) - q_{m-1},
// walked in marching strips as k_moment_march walks one recursion: each level
// keeps three rows of p and of q in registers.  acc_u += c_m p_m and acc_x +=
// c_m q_m are loaded once per pass for the rows a strip owns, updated at each
// level in step order and stored after the last one.  q0 may be null (q_0 =
// 0).  The commutator weights come from a per-pattern table (xw[pattern][slot],
// the same for every row of a pattern).  Every value goes through the
// operations of k_evolve_x_step in its order.
template <typename V, bool ONSF, int K>
__global__ __launch_bounds__(kBlock, 2) void k_evolve_x_march(
    Ell h, Sweep sw, Lat2 lat, const double *pxw, const V *p1, const V *p0,
    V *__restrict__ pout1, V *__restrict__ pout2, const V *q1, const V *q0,
    V *__restrict__ qout1, V *__restrict__ qout2, V *__restrict__ accx, V *__restrict__ accu,
    CoefK ck) {
    constexpr int TC = kWave - 2 * K;
    constexpr int P = kRowRing, PS = kStateRing, DS = kDs, DR = kRowRing - 1 - K;
    constexpr int DL = DS < DR ? DS : DR;
    static_assert(K >= 2 && K <= 3, "coupled steps per pass");
    static_assert(DR >= 1 && DS + 3 <= PS && P % PS == 0 && PS % 3 == 0 && DL + K < P,
                  "ring sizes");
    const int64_t po = plane_off(sw);
    p1 = on_plane(p1, po);
    p0 = on_plane(p0, po);
    pout1 = on_plane(pout1, po);
    pout2 = on_plane(pout2, po);
    q1 = on_plane(q1, po);
    q0 = on_plane(q0, po);
    qout1 = on_plane(qout1, po);
    qout2 = on_plane(qout2, po);
    accx = on_plane(accx, po);
    accu = on_plane(accu, po);
    const double t = sw.one.t, inv_es = sw.one.inv_es;
    // per pattern: hopping (previous column, next column), (next chain, previous
    // chain), then commutator weights in the same order
    __shared__ double2 lwt[4 * kMaxPatterns];
    for (int j = threadIdx.x; j < h.npat; j += kBlock) {
        const uint32_t f = lat.flags[j];
        const double tv = (f & 4u) ? t : 0.0, xv = pxw[4 * j + 2];
        lwt[4 * j] = make_double2((f & 1u) ? t : 0.0, (f & 2u) ? t : 0.0);
        lwt[4 * j + 1] = make_double2((f & 8u) ? tv : 0.0, (f & 8u) ? 0.0 : tv);
        lwt[4 * j + 2] = make_double2(pxw[4 * j], pxw[4 * j + 1]);
        lwt[4 * j + 3] = make_double2((f & 8u) ? xv : 0.0, (f & 8u) ? 0.0 : xv);
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = lat.nx, ny = lat.ny, J = lat.tj;
    const int nst = (nx + TC - 1) / TC, nsg = (ny + J - 1) / J;
    const int ntile = nst * nsg;
    const int lb = blockIdx.x;
    const int per = (ntile + kXcds - 1) / kXcds;
    const int b0 = (lb % kXcds) * per, b1 = min(b0 + per, ntile);
    // work-groups of kBlock threads (a run-time group size costs this kernel,
    // at the edge of its registers, spills)
    constexpr int nwv = kBlock / kWave;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int wloc = (lb / kXcds) * nwv + wv;
    const int wn = (sw.nwg / kXcds) * nwv;
    for (int b = b0 + wloc; b < b1; b += wn) {
        const int strip = b % nst;
        const int j0 = (b / nst) * J, c0 = strip * TC;
        const int gi = wrap_index(c0 - K + lane, nx);
        const bool colok = lane >= K && lane < K + TC && c0 - K + lane < nx;
        const int Jt = min(J, ny - j0), T = Jt + 2 * K;
        const uint32_t ov = (uint32_t)gi * sizeof(V), rb = (uint32_t)nx * sizeof(V);
        const uint32_t ovo = colok ? ov : kOffNone;
        auto base = [&](int rho) { return (int64_t)wrap_index(j0 - K + rho, ny) * nx; };
        auto owned = [&](int rho) { return rho >= K && rho < K + Jt; };
        double2 X0[PS], Xm[PS], Y0[PS], Ym[PS];        // p_n, p_{n-1}, q_n, q_{n-1}
        double2 AU[P], AX[P];                          // accumulators of the owned rows
        int PI[P];
        float OF[P];
        double OD[P];
        double2 LP[K][3], LQ[K][3];                    // levels 1 .. K of p and q
#pragma unroll
        for (int q = 0; q < PS; ++q) X0[q] = Xm[q] = Y0[q] = Ym[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            AU[q] = AX[q] = make_double2(0.0, 0.0);
            PI[q] = 0;
            OF[q] = 0.0f;
            OD[q] = 0.0;
        }
#pragma unroll
        for (int s = 0; s < K; ++s)
            LP[s][0] = LP[s][1] = LP[s][2] = LQ[s][0] = LQ[s][1] = LQ[s][2] =
                make_double2(0.0, 0.0);
        auto load_state = [&](int rho, int q) {
            const int64_t rbase = base(rho);
            const uint32_t nb = rho < T ? rb : 0u;
            X0[q] = buf_ld(p1 + rbase, nb, ov);
            Xm[q] = buf_ld(p0 + rbase, nb, ov);
            Y0[q] = buf_ld(q1 + rbase, nb, ov);
            Ym[q] = buf_ld(q0 ? q0 + rbase : q1, q0 ? nb : 0u, ov);
        };
        auto load_acc = [&](int rho, int q) {
            const int64_t rbase = base(rho);
            const uint32_t nb = owned(rho) ? rb : 0u;
            AU[q] = buf_ld(accu + rbase, nb, ovo);
            AX[q] = buf_ld(accx + rbase, nb, ovo);
        };
        auto load_row = [&](int rho, int q) {
            const int64_t rbase = base(rho);
            const bool in = rho < T;
            PI[q] = __builtin_amdgcn_raw_buffer_load_b8(
                row_rsrc(h.pid + rbase, in ? (uint32_t)nx : 0u), gi, 0, 0);
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
        for (int r = 0; r < DL; ++r) load_acc(r, r);
#pragma unroll
        for (int r = 0; r < DR; ++r) load_row(r, r);
        for (int t0 = 0; t0 < T; t0 += P) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const int tt = t0 + u;
                load_state(tt + DS, (u + DS) % PS);
                load_acc(tt + DL, (u + DL) % P);
                load_row(tt + DR, (u + DR) % P);
#pragma unroll
                for (int s = 1; s <= K; ++s) {
                    const int rho = tt - s;
                    const int qp = ((u - s) % P + P) % P;
                    const int qs = ((u - s) % PS + PS) % PS;
                    const int q3 = ((u - s) % 3 + 3) % 3;
                    const int q3m = (q3 + 2) % 3, q3p = (q3 + 1) % 3;
                    const int qm = (qs + PS - 1) % PS, qq = (qs + 1) % PS;
                    double2 xm1, x0, xp1, xo, ym1, y0, yp1, yo;
                    if (s == 1) {
                        xm1 = X0[qm]; x0 = X0[qs]; xp1 = X0[qq]; xo = Xm[qs];
                        ym1 = Y0[qm]; y0 = Y0[qs]; yp1 = Y0[qq]; yo = Ym[qs];
                    } else {
                        xm1 = LP[s - 2][q3m]; x0 = LP[s - 2][q3]; xp1 = LP[s - 2][q3p];
                        ym1 = LQ[s - 2][q3m]; y0 = LQ[s - 2][q3]; yp1 = LQ[s - 2][q3p];
                        xo = s == 2 ? X0[qs] : LP[s - 3 < 0 ? 0 : s - 3][q3];
                        yo = s == 2 ? Y0[qs] : LQ[s - 3 < 0 ? 0 : s - 3][q3];
                    }
                    const double o = ONSF ? (double)OF[qp] * inv_es : OD[qp];
                    const double2 wh = lwt[4 * PI[qp]], wv2 = lwt[4 * PI[qp] + 1];
                    const double2 xh = lwt[4 * PI[qp] + 2], xv2 = lwt[4 * PI[qp] + 3];
                    // H~ p and [X, H~] p, then H~ q, each in slot order (one of
                    // the two vertical terms has weight 0)
                    const double2 xl = lane_prev(x0), xr = lane_next(x0);
                    double2 hp = make_double2(o * x0.x, o * x0.y);
                    double2 dp = make_double2(0.0, 0.0);
                    hp = raxpy(hp, wh.x, xl);
                    dp = raxpy(dp, xh.x, xl);
                    hp = raxpy(hp, wh.y, xr);
                    dp = raxpy(dp, xh.y, xr);
                    hp = raxpy(hp, wv2.y, xm1);
                    dp = raxpy(dp, xv2.y, xm1);
                    hp = raxpy(hp, wv2.x, xp1);
                    dp = raxpy(dp, xv2.x, xp1);
                    double2 hq = make_double2(o * y0.x, o * y0.y);
                    hq = raxpy(hq, wh.x, lane_prev(y0));
                    hq = raxpy(hq, wh.y, lane_next(y0));
                    hq = raxpy(hq, wv2.y, ym1);
                    hq = raxpy(hq, wv2.x, yp1);
                    const double2 po = rounded<V>(two_minus(hp, xo));
                    const double2 qo = rounded<V>(two_minus(cadd(dp, hq), yo));
                    LP[s - 1][q3] = po;
                    LQ[s - 1][q3] = qo;
                    AU[qp] = rounded<V>(cmla(AU[qp], ck.c[s - 1], po));
                    AX[qp] = rounded<V>(cmla(AX[qp], ck.c[s - 1], qo));
                    if (s >= K - 1) {
                        const bool own = owned(rho);
                        const int64_t row = (int64_t)(own ? j0 + rho - K : 0) * nx;
                        const uint32_t nb = own ? rb : 0u;
                        buf_st((s == K ? pout2 : pout1) + row, nb, ovo, po);
                        buf_st((s == K ? qout2 : qout1) + row, nb, ovo, qo);
                        if (s == K) {
                            buf_st(accu + row, nb, ovo, AU[qp]);
                            buf_st(accx + row, nb, ovo, AX[qp]);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

template <typename V>
bool launch_evolve_x_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const double *pxw,
                           const V *p1, const V *p0, V *pout1, V *pout2, const V *q1,
                           const V *q0, V *qout1, V *qout2, V *accx, V *accu, const CoefK &ck,
                           hipStream_t s) {
    if (lat.reg != 2 || lat.k < 2 || lat.k > 3) return false;
#define KPM_EXK(ONSF_, K_)                                                                    \
    hipLaunchKernelGGL((k_evolve_x_march<V, ONSF_, K_>), dim3(sw.nwg, sw.nplanes),            \
                       dim3(kBlock), 0, s, h, sw, lat, pxw, p1, p0, pout1, pout2, q1, q0,     \
                       qout1, qout2, accx, accu, ck)
#define KPM_EX(ONSF_)                                                                         \
    switch (lat.k) {                                                                          \
        case 3: KPM_EXK(ONSF_, 3); break;                                                     \
        default: KPM_EXK(ONSF_, 2); break;                                                    \
    }
    if (h.onsf) { KPM_EX(true) }
    else { KPM_EX(false) }
#undef KPM_EX
#undef KPM_EXK
    return true;
}

template bool launch_evolve_x_multi<double2>(const Ell &, const Sweep &, const Lat2 &,
                                             const double *, const double2 *, const double2 *,
                                             double2 *, double2 *, const double2 *,
                                             const double2 *, double2 *, double2 *, double2 *,
                                             double2 *, const CoefK &, hipStream_t);
template bool launch_evolve_x_multi<float2>(const Ell &, const Sweep &, const Lat2 &,
                                            const double *, const float2 *, const float2 *,
                                            float2 *, float2 *, const float2 *, const float2 *,
                                            float2 *, float2 *, float2 *, float2 *,
                                            const CoefK &, hipStream_t);

}  // namespace kpm
