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
#include "kpm_internal.h"

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

// The value a store of v into storage type V will hold, back in double.
template <typename V> __device__ __forceinline__ double2 rounded(double2 v);
template <> __device__ __forceinline__ double2 rounded<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 rounded<float2>(double2 v) {
    return make_double2((double)(float)v.x, (double)(float)v.y);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) {
    return make_double2(s * a.x, s * a.y);
}
// a * b
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cdot(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Sum of H~_im x_m over the filled slots of row i, plus the diagonal term.
template <typename V>
__device__ __forceinline__ double2 row_h(const Ell &h, const V *x, int64_t i,
                                         int64_t v, int vshift, double2 xi) {
    double o = h.ons[i];
    double2 acc = make_double2(o * xi.x, o * xi.y);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            int32_t m = h.nbr[k * h.n + i];
            double hk = h.hop ? h.hop[k * h.n + i] : h.t;
            double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            hk = m < 0 ? 0.0 : hk;
            acc.x += hk * xm.x;
            acc.y += hk * xm.y;
        }
    }
    return acc;
}

// H~ x and D x of row i together, sharing the gathered x_m.
template <typename V>
__device__ __forceinline__ void row_hd(const Ell &h, const V *x, int64_t i, int64_t v,
                                       int vshift, double2 xi, double2 &hx, double2 &dx) {
    double o = h.ons[i];
    hx = make_double2(o * xi.x, o * xi.y);
    dx = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            int32_t m = h.nbr[k * h.n + i];
            double hk = h.hop ? h.hop[k * h.n + i] : h.t;
            double xk = h.xw[k * h.n + i];
            double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            hk = m < 0 ? 0.0 : hk;
            xk = m < 0 ? 0.0 : xk;
            hx.x += hk * xm.x;
            hx.y += hk * xm.y;
            dx.x += xk * xm.x;
            dx.y += xk * xm.y;
        }
    }
}

// D x of row i.
template <typename V>
__device__ __forceinline__ double2 row_d(const Ell &h, const V *x, int64_t i, int64_t v,
                                         int vshift) {
    double2 dx = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < kMaxWidth; ++k) {
        if (k < h.w) {
            int32_t m = h.nbr[k * h.n + i];
            double xk = h.xw[k * h.n + i];
            double2 xm = ld(x + ((int64_t)(m < 0 ? 0 : m) << vshift) + v);
            xk = m < 0 ? 0.0 : xk;
            dx.x += xk * xm.x;
            dx.y += xk * xm.y;
        }
    }
    return dx;
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

// Iterates the element blocks assigned to this work-group (see Sweep).
#define KPM_SWEEP_BEGIN(sw)                                                         \
    const int xcd_ = blockIdx.x % kXcds;                                            \
    const int loc_ = blockIdx.x / kXcds;                                            \
    const int nloc_ = (sw).nwg / kXcds;                                             \
    const int64_t b0_ = (int64_t)xcd_ * (sw).per_xcd;                               \
    const int64_t b1_ = min(b0_ + (sw).per_xcd, (sw).nblk);                         \
    for (int64_t b_ = b0_ + loc_; b_ < b1_; b_ += nloc_) {                          \
        const int64_t e = b_ * kBlock + threadIdx.x;                                \
        if (e < (sw).total) {                                                       \
            const int64_t i = e >> (sw).vshift;                                     \
            const int64_t v = e & ((1 << (sw).vshift) - 1);
#define KPM_SWEEP_END \
        }             \
    }

// ---------------------------------------------------------------- kernels
template <typename V, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_moment_step(Ell h, Sweep sw, const V *p1,
                                                        const V *p0, V *out,
                                                        const V *__restrict__ phil,
                                                        double2 *__restrict__ partial,
                                                        int slot) {
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    KPM_SWEEP_BEGIN(sw)
    double2 xi = ld(p1 + e);
    double2 l = ld(phil + e);
    double2 hx = row_h(h, p1, i, v, sw.vshift, xi);
    double2 o;
    if (FIRST) {
        o = hx;
        double2 d0 = cdot(l, xi);
        s1 = cadd(s1, d0);
    } else {
        double2 q = ld(p0 + e);
        o = make_double2(2.0 * hx.x - q.x, 2.0 * hx.y - q.y);
    }
    // the dot uses the stored (rounded) value, which the next step reads
    o = rounded<V>(o);
    st(out + e, o);
    s0 = cadd(s0, cdot(l, o));
    KPM_SWEEP_END
    const int64_t r = (int64_t)1 << sw.vshift;
    if (FIRST) {
        block_sum(s1, sw.vshift, partial + ((int64_t)slot * sw.nwg + blockIdx.x) * r);
        block_sum(s0, sw.vshift, partial + ((int64_t)(slot + 1) * sw.nwg + blockIdx.x) * r);
    } else {
        block_sum(s0, sw.vshift, partial + ((int64_t)slot * sw.nwg + blockIdx.x) * r);
    }
}

template <typename V, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_evolve_step(Ell h, Sweep sw, const V *p1,
                                                        const V *p0, V *out, V *acc,
                                                        const V *add, double2 c0,
                                                        double2 c) {
    KPM_SWEEP_BEGIN(sw)
    double2 xi = ld(p1 + e);
    double2 hx = row_h(h, p1, i, v, sw.vshift, xi);
    double2 o, a;
    if (FIRST) {
        o = rounded<V>(hx);
        a = cadd(cmul(c0, xi), cmul(c, o));
        if (add) a = cadd(ld(add + e), a);
    } else {
        double2 q = ld(p0 + e);
        o = rounded<V>(make_double2(2.0 * hx.x - q.x, 2.0 * hx.y - q.y));
        a = cadd(ld(acc + e), cmul(c, o));
    }
    st(out + e, o);
    st(acc + e, a);
    KPM_SWEEP_END
}

template <typename V, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_evolve_x_step(Ell h, Sweep sw, const V *p1,
                                                          const V *p0, V *pout,
                                                          const V *q1, const V *q0,
                                                          V *qout, V *accx, V *accu,
                                                          double2 c0, double2 c) {
    KPM_SWEEP_BEGIN(sw)
    double2 xi = ld(p1 + e);
    double2 hp, dp;
    row_hd(h, p1, i, v, sw.vshift, xi, hp, dp);
    if (FIRST) {
        hp = rounded<V>(hp);
        dp = rounded<V>(dp);
        st(pout + e, hp);
        st(qout + e, dp);
        st(accx + e, cmul(c, dp));
        st(accu + e, cadd(cmul(c0, xi), cmul(c, hp)));
    } else {
        double2 qi = ld(q1 + e);
        double2 hq = row_h(h, q1, i, v, sw.vshift, qi);
        double2 pp = ld(p0 + e);
        double2 qq = q0 ? ld(q0 + e) : make_double2(0.0, 0.0);
        double2 po = rounded<V>(make_double2(2.0 * hp.x - pp.x, 2.0 * hp.y - pp.y));
        double2 qo = rounded<V>(make_double2(2.0 * dp.x + 2.0 * hq.x - qq.x,
                                             2.0 * dp.y + 2.0 * hq.y - qq.y));
        st(pout + e, po);
        st(qout + e, qo);
        st(accx + e, cadd(ld(accx + e), cmul(c, qo)));
        st(accu + e, cadd(ld(accu + e), cmul(c, po)));
    }
    KPM_SWEEP_END
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_apply_d(Ell h, Sweep sw, const V *x, V *y,
                                                    double2 alpha) {
    KPM_SWEEP_BEGIN(sw)
    st(y + e, cmul(alpha, row_d(h, x, i, v, sw.vshift)));
    KPM_SWEEP_END
}

// One block per (slot, vector): sums the nwg partials in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce(const double2 *__restrict__ partial,
                                                   int nwg, int vshift,
                                                   double2 *__restrict__ dst,
                                                   int64_t stride_r, int64_t offset) {
    const int slot = blockIdx.x;
    const int r = blockIdx.y;
    const int64_t nr = (int64_t)1 << vshift;
    const double2 *p = partial + (int64_t)slot * nwg * nr + r;
    double2 s = make_double2(0.0, 0.0);
    for (int g = threadIdx.x; g < nwg; g += kBlock) s = cadd(s, p[(int64_t)g * nr]);
    __shared__ double2 red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[(int64_t)r * stride_r + offset + slot] = red[0];
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
    if (nm > 1) s += w[1] * x * c[1];
    for (int m = 2; m < nm; ++m) {
        double tm = 2.0 * x * tm1 - tm2;
        s += w[m] * tm * c[m];
        tm2 = tm1;
        tm1 = tm;
    }
    out[id] = pref[k] * s;
}

// ---------------------------------------------------------------- launchers
Sweep make_sweep(int64_t rows, int vshift, int nwg) {
    Sweep sw;
    sw.total = rows << vshift;
    sw.nblk = (sw.total + kBlock - 1) / kBlock;
    sw.nwg = nwg;
    sw.per_xcd = (sw.nblk + kXcds - 1) / kXcds;
    sw.vshift = vshift;
    return sw;
}

template <typename V>
void launch_moment_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                        const V *p0, V *out, const V *phil, double2 *partial, int slot,
                        hipStream_t s) {
    if (first)
        hipLaunchKernelGGL((k_moment_step<V, true>), dim3(sw.nwg), dim3(kBlock), 0, s, h, sw,
                           p1, p0, out, phil, partial, slot);
    else
        hipLaunchKernelGGL((k_moment_step<V, false>), dim3(sw.nwg), dim3(kBlock), 0, s, h, sw,
                           p1, p0, out, phil, partial, slot);
}

template <typename V>
void launch_evolve_step(const Ell &h, const Sweep &sw, bool first, const V *p1, const V *p0,
                        V *out, V *acc, const V *add, double2 c0, double2 c, hipStream_t s) {
    if (first)
        hipLaunchKernelGGL((k_evolve_step<V, true>), dim3(sw.nwg), dim3(kBlock), 0, s, h, sw,
                           p1, p0, out, acc, add, c0, c);
    else
        hipLaunchKernelGGL((k_evolve_step<V, false>), dim3(sw.nwg), dim3(kBlock), 0, s, h, sw,
                           p1, p0, out, acc, add, c0, c);
}

template <typename V>
void launch_evolve_x_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                          const V *p0, V *pout, const V *q1, const V *q0, V *qout,
                          V *accx, V *accu, double2 c0, double2 c, hipStream_t s) {
    if (first)
        hipLaunchKernelGGL((k_evolve_x_step<V, true>), dim3(sw.nwg), dim3(kBlock), 0, s, h,
                           sw, p1, p0, pout, q1, q0, qout, accx, accu, c0, c);
    else
        hipLaunchKernelGGL((k_evolve_x_step<V, false>), dim3(sw.nwg), dim3(kBlock), 0, s, h,
                           sw, p1, p0, pout, q1, q0, qout, accx, accu, c0, c);
}

template <typename V>
void launch_apply_d(const Ell &h, const Sweep &sw, const V *x, V *y, double2 alpha,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_apply_d<V>), dim3(sw.nwg), dim3(kBlock), 0, s, h, sw, x, y, alpha);
}

void launch_reduce(const double2 *partial, int nwg, int vshift, int slots, double2 *dst,
                   int64_t stride_r, int64_t offset, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(slots, 1 << vshift), dim3(kBlock), 0, s, partial, nwg,
                       vshift, dst, stride_r, offset);
}

void launch_kpm_sum(const double *mom, int rows, int nm, const double *w, const double *eps,
                    const double *pref, int ne, double *out, hipStream_t s) {
    int64_t total = (int64_t)rows * ne;
    int blocks = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_kpm_sum, dim3(blocks), dim3(kBlock), 0, s, mom, rows, nm, w, eps,
                       pref, ne, out);
}

#define KPM_INSTANTIATE(V)                                                                  \
    template void launch_moment_step<V>(const Ell &, const Sweep &, bool, const V *,        \
                                        const V *, V *, const V *, double2 *, int,          \
                                        hipStream_t);                                       \
    template void launch_evolve_step<V>(const Ell &, const Sweep &, bool, const V *,        \
                                        const V *, V *, V *, const V *, double2, double2,   \
                                        hipStream_t);                                       \
    template void launch_evolve_x_step<V>(const Ell &, const Sweep &, bool, const V *,      \
                                          const V *, V *, const V *, const V *, V *, V *,   \
                                          V *, double2, double2, hipStream_t);              \
    template void launch_apply_d<V>(const Ell &, const Sweep &, const V *, V *, double2,    \
                                    hipStream_t);

KPM_INSTANTIATE(double2)
KPM_INSTANTIATE(float2)

}  // namespace kpm
