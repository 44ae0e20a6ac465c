// Fully connected network of the learned moment-to-spectrum reconstruction:
// FP32 forward pass, backpropagation of the mean squared error and Adam, on
// gfx950.  Dense products run on the matrix cores (v_mfma_f32_16x16x4_f32)
// with the bias, tanh and tanh-derivative epilogues fused into the product.
//
// Layout: weights W_l [d_{l+1}][d_l] row-major, biases b_l [d_{l+1}], packed
// as [W_0, b_0, W_1, b_1, ...]; activations and gradients [batch][width].
#include "kpm.h"
#include "kpm_error.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kTile = 64;     // block tile of C (rows and columns)
constexpr int kChunk = 32;    // K staged in LDS per pass
constexpr int kMaxSplit = 8;  // K ranges of a split product
constexpr int kLoads = kTile * kChunk / kThreads;   // values of A (and of B) per thread per pass

enum { kEpiNone = 0, kEpiBias = 1, kEpiBiasTanh = 2, kEpiTanhGrad = 3 };

template <int EPI>
__device__ __forceinline__ float epilogue(float v, int row, int col, int ldc,
                                          const float *__restrict__ bias,
                                          const float *__restrict__ aux) {
    if (EPI == kEpiBias) v += bias[col];
    if (EPI == kEpiBiasTanh) v = tanhf(v + bias[col]);
    if (EPI == kEpiTanhGrad) {
        const float t = aux[(size_t)row * ldc + col];
        v *= 1.f - t * t;
    }
    return v;
}

// C[M][N] = op(A) op(B) over k in [z Kc, (z + 1) Kc) for z = blockIdx.z, with
// A(m, k) = TA ? A[k lda + m] : A[m lda + k] and B(k, n) = TB ? B[n ldb + k] :
// B[k ldb + n].  One K range (gridDim.z = 1): the epilogue is applied and C
// written; several: the raw partial goes to ws[z][M][N] for k_split_sum.
//   kEpiBias:     + bias[n]
//   kEpiBiasTanh: tanh(. + bias[n])
//   kEpiTanhGrad: . * (1 - aux[m ldc + n]^2)
// Block: 4 waves, each a 32 x 32 quarter of the 64 x 64 tile as 2 x 2 MFMA
// 16 x 16 tiles.  For v_mfma_f32_16x16x4_f32 lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16) of its 16 x 4 and 4 x 16 operands and holds
// C(4 (l / 16) + r, l % 16) in accumulator element r.  The next K chunk is
// loaded into registers while the current one is multiplied out of LDS.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kThreads) void k_gemm(int M, int N, int K, int Kc,
                                                   const float *__restrict__ A, int lda,
                                                   const float *__restrict__ B, int ldb,
                                                   float *__restrict__ C, int ldc,
                                                   const float *__restrict__ bias,
                                                   const float *__restrict__ aux,
                                                   float *__restrict__ ws) {
    __shared__ float sa[kChunk][kTile + 4];
    __shared__ float sb[kChunk][kTile + 4];
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int kb = blockIdx.z * Kc, ke = min(K, kb + Kc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    float ra[kLoads], rb[kLoads];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
            const int idx = tid + q * kThreads;
            const int mm = TA ? idx % kTile : idx / kChunk;
            const int ka = TA ? idx / kTile : idx % kChunk;
            const int gm = m0 + mm, gka = k0 + ka;
            ra[q] = (gm < M && gka < ke) ? (TA ? A[(size_t)gka * lda + gm] : A[(size_t)gm * lda + gka])
                                         : 0.f;
            const int nn = TB ? idx / kChunk : idx % kTile;
            const int kbb = TB ? idx % kChunk : idx / kTile;
            const int gn = n0 + nn, gkb = k0 + kbb;
            rb[q] = (gn < N && gkb < ke) ? (TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn])
                                         : 0.f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
            const int idx = tid + q * kThreads;
            sa[TA ? idx / kTile : idx % kChunk][TA ? idx % kTile : idx / kChunk] = ra[q];
            sb[TB ? idx % kChunk : idx / kTile][TB ? idx / kChunk : idx % kTile] = rb[q];
        }
    };
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += kChunk) {
        __syncthreads();                 // the previous chunk is no longer read
        stash();
        __syncthreads();
        if (k0 + kChunk < ke) fetch(k0 + kChunk);
#pragma unroll
        for (int ks = 0; ks < kChunk; ks += 4) {
            const int kk = ks + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = sa[kk][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = sb[kk][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                if (split)
                    ws[((size_t)blockIdx.z * M + row) * N + col] = acc[i][j][r];
                else
                    C[(size_t)row * ldc + col] = epilogue<EPI>(acc[i][j][r], row, col, ldc, bias, aux);
            }
}

// C = epilogue(sum over z < S of ws[z]), summed in z order.
template <int EPI>
__global__ __launch_bounds__(kThreads) void k_split_sum(int M, int N, int S,
                                                        const float *__restrict__ ws,
                                                        float *__restrict__ C, int ldc,
                                                        const float *__restrict__ bias,
                                                        const float *__restrict__ aux) {
    const int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (id >= (int64_t)M * N) return;
    const int row = (int)(id / N), col = (int)(id % N);
    float v = 0.f;
    for (int z = 0; z < S; ++z) v += ws[(size_t)z * M * N + id];
    C[(size_t)row * ldc + col] = epilogue<EPI>(v, row, col, ldc, bias, aux);
}

// out[n] = sum_m G[m N + n], one thread per column, in row order (double sum).
__global__ __launch_bounds__(kThreads) void k_colsum(int M, int N, const float *__restrict__ G,
                                                     float *__restrict__ out) {
    const int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += G[(size_t)m * N + n];
    out[n] = (float)s;
}

// g = scale (p - y); part[block] = sum over the block's elements of (p - y)^2.
__global__ __launch_bounds__(kThreads) void k_mse(int64_t count, const float *__restrict__ p,
                                                  const float *__restrict__ y, float scale,
                                                  float *__restrict__ g, double *__restrict__ part) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kThreads) {
        const float d = p[i] - y[i];
        g[i] = scale * d;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (Kingma and Ba): m, v moving averages; c1 = 1 / (1 - beta1^t),
// c2 = 1 / (1 - beta2^t) bias corrections.
__global__ __launch_bounds__(kThreads) void k_adam(int64_t n, float *__restrict__ p,
                                                   const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// Products with few output tiles split K over up to kMaxSplit ranges (at
// least 64 deep each) so that about 256 blocks run; the partials go through
// `ws` (ws_elems floats) and are summed in a fixed order.
template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, float *ws, size_t ws_elems, int M, int N, int K, const float *A,
          int lda, const float *B, int ldb, float *C, int ldc, const float *bias = nullptr,
          const float *aux = nullptr) {
    const int mt = (M + kTile - 1) / kTile, nt = (N + kTile - 1) / kTile;
    int split = std::max(1, std::min({kMaxSplit, 256 / (mt * nt), (K + 63) / 64}));
    while (split > 1 && (size_t)split * M * N > ws_elems) --split;
    const int kc = ((K + split - 1) / split + kChunk - 1) / kChunk * kChunk;
    split = (K + kc - 1) / kc;
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), dim3(nt, mt, std::max(split, 1)), dim3(kThreads), 0,
                       s, M, N, K, kc, A, lda, B, ldb, C, ldc, bias, aux, ws);
    if (split > 1) {
        const int64_t total = (int64_t)M * N;
        hipLaunchKernelGGL((k_split_sum<EPI>), dim3((unsigned)((total + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, s, M, N, split, ws, C, ldc, bias, aux);
    }
}

constexpr int kLossBlocks = 64;

kpm_status err(kpm_status st, const char *msg) { return kpm_detail::set_error(st, msg); }

}  // namespace

struct kpm_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int layers = 0;                 // weight layers
    std::vector<int> d;             // widths d_0 .. d_L
    int max_batch = 0;
    std::vector<int64_t> w_off, b_off;
    int64_t np = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    std::vector<float *> act;       // act[l], l = 1 .. L: [max_batch][d_l]
    float *gbuf[2] = {nullptr, nullptr};
    float *ws = nullptr;            // partial products of split-K products
    size_t ws_elems = 0;
    double *lpart = nullptr;
    int64_t t = 0;                  // Adam steps taken

    ~kpm_mlp() {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        for (float *p : {params, grads, m, v, gbuf[0], gbuf[1], ws})
            if (p) (void)hipFree(p);
        for (float *p : act)
            if (p) (void)hipFree(p);
        if (lpart) (void)hipFree(lpart);
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

namespace {

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~Dev() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

#define MLP_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            char b_[256];                                                              \
            snprintf(b_, sizeof b_, "%s: %s", #call, hipGetErrorString(e_));           \
            return err(e_ == hipErrorOutOfMemory ? KPM_ERR_OOM : KPM_ERR_DEVICE, b_);  \
        }                                                                              \
    } while (0)

// Forward pass into net->act (the last layer into `out` when given).
kpm_status forward(kpm_mlp *net, int batch, const float *x, float *out) {
    hipStream_t s = net->stream;
    const float *a = x;
    for (int l = 0; l < net->layers; ++l) {
        const int di = net->d[l], dn = net->d[l + 1];
        const float *w = net->params + net->w_off[l], *b = net->params + net->b_off[l];
        const bool last = l == net->layers - 1;
        float *c = (last && out) ? out : net->act[l + 1];
        if (last)
            gemm<false, true, kEpiBias>(s, net->ws, net->ws_elems, batch, dn, di, a, di, w, di, c, dn, b);
        else
            gemm<false, true, kEpiBiasTanh>(s, net->ws, net->ws_elems, batch, dn, di, a, di, w, di, c, dn,
                                            b);
        a = c;
    }
    MLP_HIP(hipGetLastError());
    return KPM_OK;
}

// Loss and gradients of the mean squared error into net->grads.
kpm_status backward(kpm_mlp *net, int batch, const float *x, const float *y, double *loss) {
    hipStream_t s = net->stream;
    {
        kpm_status st = forward(net, batch, x, nullptr);
        if (st != KPM_OK) return st;
    }
    const int L = net->layers, dl = net->d[L];
    const int64_t count = (int64_t)batch * dl;
    float *g = net->gbuf[0];
    hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kThreads), 0, s, count, net->act[L], y,
                       (float)(2.0 / (double)count), g, net->lpart);
    for (int l = L - 1; l >= 0; --l) {
        const int di = net->d[l], dn = net->d[l + 1];
        const float *a = l == 0 ? x : net->act[l];
        const float *w = net->params + net->w_off[l];
        // dW_l = G^T a_l, db_l = column sums of G
        gemm<true, false, kEpiNone>(s, net->ws, net->ws_elems, dn, di, batch, g, dn, a, di,
                                    net->grads + net->w_off[l], di);
        hipLaunchKernelGGL(k_colsum, dim3((dn + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                           batch, dn, g, net->grads + net->b_off[l]);
        if (l > 0) {
            // G_{l-1} = (G W_l) * (1 - a_l^2)
            float *gn = g == net->gbuf[0] ? net->gbuf[1] : net->gbuf[0];
            gemm<false, false, kEpiTanhGrad>(s, net->ws, net->ws_elems, batch, di, dn, g, dn, w, di, gn,
                                             di, nullptr, a);
            g = gn;
        }
    }
    MLP_HIP(hipGetLastError());
    if (!loss) return KPM_OK;            // no host value asked for: stay asynchronous
    double part[kLossBlocks];
    MLP_HIP(hipMemcpyAsync(part, net->lpart, sizeof part, hipMemcpyDeviceToHost, s));
    MLP_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int b = 0; b < kLossBlocks; ++b) sum += part[b];
    *loss = sum / (double)count;
    return KPM_OK;
}

kpm_status check_batch(kpm_mlp *net, int batch, const void *x, const void *y) {
    if (!net) return err(KPM_ERR_INVALID, "null network");
    if (batch < 1 || batch > net->max_batch) return err(KPM_ERR_INVALID, "batch outside 1 .. max_batch");
    if (!x || !y) return err(KPM_ERR_INVALID, "null buffer");
    return KPM_OK;
}

}  // namespace

extern "C" {

kpm_status kpm_mlp_create(int n_layers, const int32_t *widths, int max_batch, int device,
                          void *hip_stream, kpm_mlp **out) {
    if (!out || !widths) return err(KPM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (n_layers < 1 || n_layers > 16) return err(KPM_ERR_INVALID, "n_layers outside 1 .. 16");
    if (max_batch < 1 || max_batch > 65536) return err(KPM_ERR_INVALID, "max_batch outside 1 .. 65536");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 65536) return err(KPM_ERR_INVALID, "width outside 1 .. 65536");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return err(KPM_ERR_DEVICE, "no such HIP device");
    kpm_mlp *net = new (std::nothrow) kpm_mlp();
    if (!net) return err(KPM_ERR_OOM, "host allocation");
    net->device = device;
    net->stream = (hipStream_t)hip_stream;
    net->layers = n_layers;
    net->d.assign(widths, widths + n_layers + 1);
    net->max_batch = max_batch;
    int64_t o = 0;
    int dmax = 0;
    for (int l = 0; l < n_layers; ++l) {
        net->w_off.push_back(o);
        o += (int64_t)widths[l] * widths[l + 1];
        net->b_off.push_back(o);
        o += widths[l + 1];
    }
    for (int l = 0; l <= n_layers; ++l) dmax = std::max(dmax, widths[l]);
    net->np = o;
    net->ws_elems = (size_t)kMaxSplit * max_batch * dmax;
    Dev g(device);
    auto alloc = [&](float **p, size_t n) -> bool {
        return hipMalloc(p, n * sizeof(float)) == hipSuccess;
    };
    bool ok = alloc(&net->params, o) && alloc(&net->grads, o) && alloc(&net->m, o) &&
              alloc(&net->v, o) && alloc(&net->gbuf[0], (size_t)max_batch * dmax) &&
              alloc(&net->gbuf[1], (size_t)max_batch * dmax) &&
              alloc(&net->ws, (size_t)kMaxSplit * max_batch * dmax) &&
              hipMalloc(&net->lpart, kLossBlocks * sizeof(double)) == hipSuccess;
    net->act.assign(n_layers + 1, nullptr);
    for (int l = 1; ok && l <= n_layers; ++l) ok = alloc(&net->act[l], (size_t)max_batch * widths[l]);
    if (ok) ok = hipMemsetAsync(net->params, 0, o * sizeof(float), net->stream) == hipSuccess &&
                 hipMemsetAsync(net->m, 0, o * sizeof(float), net->stream) == hipSuccess &&
                 hipMemsetAsync(net->v, 0, o * sizeof(float), net->stream) == hipSuccess &&
                 hipStreamSynchronize(net->stream) == hipSuccess;
    if (!ok) {
        delete net;
        return err(KPM_ERR_OOM, "device allocation for the network");
    }
    *out = net;
    return KPM_OK;
}

kpm_status kpm_mlp_destroy(kpm_mlp *net) {
    delete net;
    return KPM_OK;
}

int64_t kpm_mlp_n_params(const kpm_mlp *net) { return net ? net->np : -1; }

kpm_status kpm_mlp_set_params(kpm_mlp *net, const float *params) {
    if (!net || !params) return err(KPM_ERR_INVALID, "null argument");
    Dev g(net->device);
    const size_t bytes = (size_t)net->np * sizeof(float);
    MLP_HIP(hipMemcpyAsync(net->params, params, bytes, hipMemcpyHostToDevice, net->stream));
    MLP_HIP(hipMemsetAsync(net->m, 0, bytes, net->stream));
    MLP_HIP(hipMemsetAsync(net->v, 0, bytes, net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    net->t = 0;
    return KPM_OK;
}

kpm_status kpm_mlp_get_params(kpm_mlp *net, float *params) {
    if (!net || !params) return err(KPM_ERR_INVALID, "null argument");
    Dev g(net->device);
    MLP_HIP(hipMemcpyAsync(params, net->params, (size_t)net->np * sizeof(float),
                           hipMemcpyDeviceToHost, net->stream));
    MLP_HIP(hipStreamSynchronize(net->stream));
    return KPM_OK;
}

kpm_status kpm_mlp_forward(kpm_mlp *net, int batch, const float *x, float *y) {
    {
        kpm_status st = check_batch(net, batch, x, y);
        if (st != KPM_OK) return st;
    }
    Dev g(net->device);
    return forward(net, batch, x, y);
}

kpm_status kpm_mlp_gradients(kpm_mlp *net, int batch, const float *x, const float *y,
                             double *loss, float *grads) {
    {
        kpm_status st = check_batch(net, batch, x, y);
        if (st != KPM_OK) return st;
    }
    if (!loss) return err(KPM_ERR_INVALID, "null loss");
    Dev g(net->device);
    kpm_status st = backward(net, batch, x, y, loss);
    if (st != KPM_OK) return st;
    if (grads) {
        MLP_HIP(hipMemcpyAsync(grads, net->grads, (size_t)net->np * sizeof(float),
                               hipMemcpyDeviceToHost, net->stream));
        MLP_HIP(hipStreamSynchronize(net->stream));
    }
    return KPM_OK;
}

kpm_status kpm_mlp_train_step(kpm_mlp *net, int batch, const float *x, const float *y,
                              const kpm_adam *opt, double *loss) {
    {
        kpm_status st = check_batch(net, batch, x, y);
        if (st != KPM_OK) return st;
    }
    if (!opt) return err(KPM_ERR_INVALID, "null argument");
    if (!(opt->lr > 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) ||
        !(opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps > 0))
        return err(KPM_ERR_INVALID, "Adam parameters out of range");
    Dev g(net->device);
    kpm_status st = backward(net, batch, x, y, loss);
    if (st != KPM_OK) return st;
    net->t += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)opt->beta1, (double)net->t));
    const double c2 = 1.0 / (1.0 - std::pow((double)opt->beta2, (double)net->t));
    const int blocks = (int)std::min<int64_t>((net->np + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(kThreads), 0, net->stream, net->np,
                       net->params, net->grads, net->m, net->v, opt->lr, opt->beta1, opt->beta2,
                       opt->eps, (float)c1, (float)c2);
    MLP_HIP(hipGetLastError());
    return KPM_OK;
}

}  // extern "C"
