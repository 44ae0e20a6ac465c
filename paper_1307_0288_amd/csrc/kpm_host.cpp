// Host side of the C ABI declared in include/kpm.h: packing of validated
// descriptors, device residency of the scaled Hamiltonian (one sample, or many
// side by side), recursion scratch, and the drivers of Alg. 2, 3, 5, 6 and 7
// that sequence the gfx950 kernels.
#include "kpm.h"
#include "kpm_internal.h"
#include "kpm_error.h"
#include "kpm_lattice.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr double kHbar = 0.6582119569;   // eV fs
constexpr double kPi = 3.14159265358979323846;
constexpr int kPartialRing = 256;        // moment slots of group partials kept at once

using kpm_detail::fail;
using kpm_detail::Packed;
using kpm_detail::pack_desc;

#define KPM_HIP(call)                                                                \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(e_ == hipErrorOutOfMemory ? KPM_ERR_OOM : KPM_ERR_DEVICE,    \
                        "%s: %s", #call, hipGetErrorString(e_));                     \
    } while (0)

#define KPM_TRY(expr)                          \
    do {                                       \
        kpm_status s_ = (expr);                \
        if (s_ != KPM_OK) return s_;           \
    } while (0)

int vshift_of(int n_vec) {
    for (int s = 0; s <= 6; ++s)
        if ((1 << s) == n_vec) return s;
    return -1;
}

// Chebyshev-Bessel coefficients of Eq. 36: c_m = (2 - delta_m0) (-i s)^m J_m(x).
// J_m from the C++17 special functions (std::cyl_bessel_j).
void bessel_coeffs(int np, double x, int sign, double2 *c) {
    for (int m = 0; m < np; ++m) {
        const double f = (m == 0 ? 1.0 : 2.0) * std::cyl_bessel_j((double)m, x);
        // (-i s)^m cycles through 1, -i s, -1, i s
        double re = 0, im = 0;
        switch (m & 3) {
            case 0: re = f; break;
            case 1: im = -sign * f; break;
            case 2: re = -f; break;
            case 3: im = sign * f; break;
        }
        c[m] = make_double2(re, im);
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool valid_launch(const kpm_launch &l) {
    return l.groups_per_cu >= 1 && l.groups_per_cu <= 32 &&
           (l.ilp == 1 || l.ilp == 2 || l.ilp == 4) && (l.streaming == 0 || l.streaming == 1) &&
           (l.compact == 0 || l.compact == 1) && l.tiled >= 0 &&
           l.tiled <= (l.steps > 1 ? 5 : 3) && l.steps >= 1 &&
           l.steps <= (l.tiled >= 3 ? 8 : 4) &&
           (l.vectors_per_wave == 0 || l.vectors_per_wave == 1) &&
           (l.plane_groups == 0 ||
            (l.plane_groups >= kpm::kXcds && l.plane_groups <= 65536 &&
             l.plane_groups % kpm::kXcds == 0)) &&
           // vector-major states take several steps per pass only in the strips
           !(l.vectors_per_wave == 1 && l.steps > 1 && l.tiled < 3) &&
           (l.group_size == 0 || l.group_size == 64 || l.group_size == 128 ||
            l.group_size == 256 || l.group_size == 512);
}

// Wavefronts per work-group of the marching strips under shape l.
int strip_waves(const kpm_launch &l) {
    return (l.group_size > 0 ? l.group_size : kpm::kBlock) / kpm::kWave;
}

// Tile width (rows) of the tiled traversal for 2^vshift vectors per row: a
// power of two with tw << vshift a multiple of the block, at least 64 rows.
int tile_rows(int vshift) { return std::max(64, kpm::kBlock >> vshift); }

// Chain length of a lattice sample: the most common neighbour offset beyond 1
// when it divides the rows into at least two chains of at least 68 rows; 0
// otherwise.
int32_t chain_length(const std::vector<int32_t> &nbr, int w, int64_t n) {
    std::vector<std::pair<int64_t, int64_t>> counts;    // (offset, count), few distinct
    for (int64_t r = 0; r < n; ++r)
        for (int k = 0; k < w; ++k) {
            const int32_t m = nbr[(size_t)k * n + r];
            if (m < 0) continue;
            const int64_t d = m > r ? m - r : r - m;
            if (d <= 1) continue;
            bool found = false;
            for (auto &c : counts)
                if (c.first == d) {
                    ++c.second;
                    found = true;
                    break;
                }
            if (!found) {
                if (counts.size() >= 64) return 0;       // not a lattice
                counts.emplace_back(d, 1);
            }
        }
    int64_t best = 0, cnt = 0;
    for (const auto &c : counts)
        if (c.second > cnt) {
            best = c.first;
            cnt = c.second;
        }
    if (best < kpm::kTileCols + 4 || best >= ((int64_t)1 << 30) || n % best != 0 || n / best < 2)
        return 0;
    return (int32_t)best;
}

// (chain, column) step codes of the two-step sweep (see kpm::Lat2) for the
// sample in rows [r0, r1) of a system of n rows, with nx-row chains: for every
// row, the chain and column distance to each neighbour, -1, 0 or 1 under
// periodic wrap, must be the same for every row of its pattern, here and in
// the samples already seen (code and seen carry over from call to call; empty
// vectors start them).  False when some row breaks this or has a neighbour
// outside its sample.
bool lattice_codes(const std::vector<int32_t> &nbr, int w, int64_t n, int64_t r0, int64_t r1,
                   int64_t nx, const std::vector<uint8_t> &pid, int npat,
                   std::vector<uint32_t> &code, std::vector<uint8_t> &seen) {
    const int64_t ns = r1 - r0;
    if (nx < kpm::kTileCols + 4 || ns % nx != 0 || ns / nx < 4 || w > 4) return false;
    const int64_t ny = ns / nx;
    if (code.empty()) code.assign(npat, 0u);
    if (seen.empty()) seen.assign(npat, 0);
    for (int64_t r = 0; r < ns; ++r) {
        const int64_t j = r / nx, i = r % nx;
        uint32_t c = 0xFFFFFFFFu;
        for (int k = 0; k < w; ++k) {
            const int32_t mg = nbr[(size_t)k * n + r0 + r];
            if (mg < 0) continue;
            if (mg < r0 || mg >= r1) return false;
            const int64_t m = mg - r0;
            int64_t di = m % nx - i, dj = m / nx - j;
            if (di == nx - 1) di = -1;
            if (di == 1 - nx) di = 1;
            if (dj == ny - 1) dj = -1;
            if (dj == 1 - ny) dj = 1;
            if (di < -1 || di > 1 || dj < -1 || dj > 1) return false;
            const uint32_t b = (uint32_t)((dj + 1) * 3 + (di + 1));
            c = (c & ~(0xFFu << (8 * k))) | (b << (8 * k));
        }
        const int p = pid[r0 + r];
        if (!seen[p]) {
            seen[p] = 1;
            code[p] = c;
        } else if (code[p] != c) {
            return false;
        }
    }
    return true;
}

// (chain, column) step codes (as in lattice_codes) of every row of the sample
// in rows [r0, r1) of a system of n rows with nx-row chains, appended to rc.
// False when a row has a neighbour outside its sample or more than one chain
// or column away.
bool row_codes(const std::vector<int32_t> &nbr, int w, int64_t n, int64_t r0, int64_t r1,
               int64_t nx, std::vector<uint32_t> &rc) {
    const int64_t ns = r1 - r0;
    if (nx < kpm::kTileCols + 4 || ns % nx != 0 || ns / nx < 4 || w > 4) return false;
    const int64_t ny = ns / nx;
    for (int64_t r = 0; r < ns; ++r) {
        const int64_t j = r / nx, i = r % nx;
        uint32_t c = 0xFFFFFFFFu;
        for (int k = 0; k < w; ++k) {
            const int32_t mg = nbr[(size_t)k * n + r0 + r];
            if (mg < 0) continue;
            if (mg < r0 || mg >= r1) return false;
            const int64_t m = mg - r0;
            int64_t di = m % nx - i, dj = m / nx - j;
            if (di == nx - 1) di = -1;
            if (di == 1 - nx) di = 1;
            if (dj == ny - 1) dj = -1;
            if (dj == 1 - ny) dj = 1;
            if (di < -1 || di > 1 || dj < -1 || dj > 1) return false;
            const uint32_t b = (uint32_t)((dj + 1) * 3 + (di + 1));
            c = (c & ~(0xFFu << (8 * k))) | (b << (8 * k));
        }
        rc.push_back(c);
    }
    return true;
}

// Slot flags of the register-tiled two-step sweep from the lattice codes:
// slot 0 the previous column, slot 1 the next, slot 2 the previous or next
// chain, each possibly empty, and no fourth slot.  False otherwise.
bool graphene_flags(const std::vector<uint32_t> &code, std::vector<uint32_t> &flags) {
    flags.assign(code.size(), 0u);
    for (size_t p = 0; p < code.size(); ++p) {
        const uint32_t b0 = code[p] & 0xFFu, b1 = (code[p] >> 8) & 0xFFu,
                       b2 = (code[p] >> 16) & 0xFFu, b3 = code[p] >> 24;
        // byte = (dj + 1) * 3 + (di + 1): 3 = (0, -1), 5 = (0, +1), 7 = (+1, 0), 1 = (-1, 0)
        if ((b0 != 0xFFu && b0 != 3u) || (b1 != 0xFFu && b1 != 5u) ||
            (b2 != 0xFFu && b2 != 7u && b2 != 1u) || b3 != 0xFFu)
            return false;
        flags[p] = (b0 != 0xFFu ? 1u : 0u) | (b1 != 0xFFu ? 2u : 0u) | (b2 != 0xFFu ? 4u : 0u) |
                   (b2 == 7u ? 8u : 0u);
    }
    return true;
}

// Launch shape used until kpm_autotune or kpm_set_launch picks another.
kpm_launch default_launch(int vshift, kpm_precision prec) {
    kpm_launch l{};
    // measured on MI355X (paper-scale sheet): one vector favours 4 groups per
    // CU, many vectors 8; streaming helps every vector count
    // the compact neighbour form pays off while the per-row structure is a
    // noticeable share of the bytes (few vectors per row)
    l.groups_per_cu = vshift == 0 ? 4 : 8;
    l.ilp = (vshift >= 6 && prec != KPM_FP64) ? 4 : 1;
    l.streaming = vshift == 0 ? 0 : 1;
    l.compact = vshift <= 3 ? 1 : 0;
    // with 8+ vectors per row a row's vertical neighbour lies megabytes ahead in
    // row order, beyond an XCD's L2
    l.tiled = vshift >= 3 ? 1 : 0;
    l.steps = 1;
    // one vector: eight recursion steps per pass in marching strips sized for
    // the grid, where the sample allows (measured fastest on paper-scale
    // sheets, in both forms, with 2 groups per CU); elsewhere single steps in
    // row order
    if (vshift == 0) {
        l.groups_per_cu = 2;
        l.tiled = 5;
        l.steps = 8;
    }
    return l;
}

// The default shape for 2^vshift vectors with the KPM_* environment overrides
// applied (KPM_GROUPS_PER_CU, KPM_ILP, KPM_STREAMING, KPM_COMPACT_LAUNCH,
// KPM_TILED, KPM_STEPS; each value clamped to its range).  A shape must stay
// one the kernels exist for: more than 4 steps per pass run only in the
// marching strips (KPM_STEPS above 4 selects them), a traversal below the
// strips caps the steps at 4, and single steps take a traversal of at most 3
// (row order when the default was a strip shape).  KPM_ERR_INVALID when the
// result is still not a valid shape.
bool launch_env_set() {
    for (const char *v : {"KPM_GROUPS_PER_CU", "KPM_ILP", "KPM_STREAMING", "KPM_COMPACT_LAUNCH",
                          "KPM_TILED", "KPM_STEPS"})
        if (std::getenv(v)) return true;
    return false;
}

kpm_status env_launch(int vshift, kpm_precision prec, kpm_launch *out) {
    kpm_launch l = default_launch(vshift, prec);
    if (const char *env = std::getenv("KPM_GROUPS_PER_CU"))
        l.groups_per_cu = std::max(1, std::min(32, atoi(env)));
    if (const char *env = std::getenv("KPM_ILP"))
        l.ilp = atoi(env) >= 4 ? 4 : (atoi(env) == 2 ? 2 : 1);
    if (const char *env = std::getenv("KPM_STREAMING")) l.streaming = atoi(env) != 0;
    if (const char *env = std::getenv("KPM_COMPACT_LAUNCH")) l.compact = atoi(env) != 0;
    const char *env_tiled = std::getenv("KPM_TILED");
    const char *env_steps = std::getenv("KPM_STEPS");
    if (env_tiled) l.tiled = std::max(0, std::min(5, atoi(env_tiled)));
    if (env_steps) {
        l.steps = std::max(1, std::min(8, atoi(env_steps)));
        if (l.steps > 4 && l.tiled < 3) l.tiled = 5;
    }
    if (l.steps > 4 && l.tiled < 3) l.steps = 4;
    if (l.steps == 1 && l.tiled > 3) l.tiled = env_tiled ? 3 : 0;
    if (!valid_launch(l))
        return fail(KPM_ERR_INVALID,
                    "KPM_* launch overrides give an invalid shape (groups %d ilp %d streaming "
                    "%d compact %d tiled %d steps %d)",
                    l.groups_per_cu, l.ilp, l.streaming, l.compact, l.tiled, l.steps);
    *out = l;
    return KPM_OK;
}

}  // namespace

struct kpm_system {
    int device = 0;
    hipStream_t stream = nullptr;
    kpm_precision prec = KPM_FP64;
    int64_t n = 0;              // rows of all samples
    int w = 0;
    bool has_dx = false;
    int cus = 256;
    kpm_launch launch[7];       // launch shape of the moment step per log2(n_vec)
    kpm_launch launch_dbl[7];   // the same for moment sets in the doubling form

    const kpm_launch &shape(int vshift, bool dbl) const {
        return dbl ? launch_dbl[vshift] : launch[vshift];
    }
    // samples: rows [off[s], off[s+1]) hold sample s, whose scale is es[s]
    int nseg = 1;
    std::vector<int64_t> off;
    std::vector<double> es;
    std::vector<double> seg_t;   // uniform hopping / E_s of each sample
    std::vector<int32_t> chain;  // chain length of each sample (tiled traversal), 0 = none
    // two-step sweep (kpm_launch.steps = 2): lattice codes of a one-sample
    // chain lattice, or none; its two extra recursion states
    int32_t l2nx = 0, l2ny = 0;
    uint32_t *d_code = nullptr;
    uint32_t *d_flags = nullptr;   // graphene slot flags (register tiles), or none
    // a batch of chain lattices whose moment sets take the marching strips:
    // per-row strip pattern ids d_sid (nsp distinct (chain, column) step
    // codes over all samples), d_flags per id; d_code stays unset
    bool bstrips = false;
    uint8_t *d_sid = nullptr;
    int nsp = 0;
    void *xbuf[4] = {nullptr, nullptr, nullptr, nullptr};
    int xbuf_count = 0;
    size_t xbuf_bytes = 0;
    // device Hamiltonian
    int32_t *d_nbr = nullptr;   // explicit neighbour list, or
    uint8_t *d_pid = nullptr;   // compact form: pattern id per row
    int32_t *d_pat = nullptr;   //   and offset patterns [npat][kMaxWidth]
    int npat = 0;
    double *d_hop = nullptr;
    double *d_xw = nullptr;
    double *d_pxw = nullptr;    // [npat][4] commutator weights per slot (chain lattices)
    double *d_ons = nullptr;    // H_nn / E_s, or
    float *d_onsf = nullptr;    // H_nn (eV) when every value is a float
    bool uniform_hop = true;
    double2 *d_alpha = nullptr;  // [nseg] velocity prefactor -i E_s / hbar (batches)
    // segment tables per (vshift, requested groups); batches only
    struct SegTab {
        int vshift;
        int64_t want;          // groups asked for (all samples)
        int tiled, ksteps, wpg;// single-step traversal; strip steps and group size
        int nwg;
        kpm::Seg *seg;
        int32_t *wg;
    };
    std::vector<SegTab> segtabs;
    // Bessel coefficient tables [nseg][np] per (dt, sign, np); batches only
    struct CoefTab {
        double dt;
        int sign, np;
        double2 *d;
    };
    std::vector<CoefTab> coeftabs;
    // scratch
    std::vector<void *> vecs;
    size_t vec_bytes = 0;
    double2 *partial = nullptr;
    size_t partial_elems = 0;
    double2 *dmom = nullptr;
    size_t dmom_elems = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    std::vector<std::pair<int64_t, int64_t>> ev_runs;   // (rows x vectors, launches) per pair
    kpm_stats stats{};
    // captured moment sets (kpm_set_graphs): one executable graph per set of
    // buffers, sizes and launch shape; dropped whenever scratch is reallocated
    bool graphs = false;
    hipStream_t cap = nullptr;
    struct GraphKey {
        const void *phil, *phir, *a, *b, *partial, *dmom;
        // planes and groups of the sweep as run (layout and plane grid), strip group size
        int nm, vshift, groups, ilp, streaming, compact, tiled, steps, dbl, re, planes, nwg, gs;
        int64_t stride_r, offset;
        bool operator==(const GraphKey &o) const {
            return phil == o.phil && phir == o.phir && a == o.a && b == o.b &&
                   partial == o.partial && dmom == o.dmom && nm == o.nm && vshift == o.vshift &&
                   groups == o.groups && ilp == o.ilp && streaming == o.streaming &&
                   compact == o.compact && tiled == o.tiled && steps == o.steps &&
                   dbl == o.dbl && re == o.re && planes == o.planes && nwg == o.nwg &&
                   gs == o.gs &&
                   stride_r == o.stride_r &&
                   offset == o.offset;
        }
    };
    struct GraphEntry {
        GraphKey key;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graph_cache;

    hipGraphExec_t find_graph(const GraphKey &k) const {
        for (const GraphEntry &g : graph_cache)
            if (g.key == k) return g.exec;
        return nullptr;
    }

    void drop_graphs() {
        for (GraphEntry &g : graph_cache) (void)hipGraphExecDestroy(g.exec);
        graph_cache.clear();
    }

    kpm_status ensure_capture_stream() {
        // default priority, non-blocking: the library never changes priorities
        if (!cap) KPM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        return KPM_OK;
    }

    size_t elem_bytes() const { return prec == KPM_FP64 ? 16 : 8; }
    size_t state_bytes(int vshift) const { return (size_t)n * ((size_t)1 << vshift) * elem_bytes(); }

    // The device Hamiltonian as a launch with shape l reads it.
    kpm::Ell ell_for(const kpm_launch &l) const {
        kpm::Ell h = ell();
        if (!l.compact) h.pid = nullptr;
        return h;
    }

    // Recursion steps per pass of moment sets with 2^vshift vectors under
    // launch shape l: l.steps where a multi-step sweep applies (one vector,
    // chain lattice, compact form; 3 and 4 steps need the graphene slot order,
    // else 2), 1 otherwise.
    int multi_steps(int vshift, const kpm_launch &l) const {
        // batches: the marching strips only (their moment sets; the propagators
        // of a batch take single steps)
        if (nseg > 1)
            return bstrips && vshift == 0 && l.steps >= 2 && l.tiled >= 3 ? l.steps : 1;
        // the tiles address a row through a buffer resource of 32-bit byte size,
        // with offsets from 2^31 up as the "no access" offset
        if (!d_code || vshift != 0 || l.steps < 2 || !l.compact || l2ny < kpm::kMinChains ||
            (int64_t)l2nx * (int64_t)sizeof(double2) >= ((int64_t)1 << 31))
            return 1;
        return d_flags ? l.steps : 2;
    }

    // Chains per marching strip of k steps on an nx x ny chain lattice swept
    // by `waves` wavefronts: 16 or 32 (tiled = 3, 4), or sized for the grid
    // (tiled = 5): the fewest loop passes of the wavefront with the most
    // strips (passes of kMarchRows rows, tj + 2k rows per strip), then the
    // longest strips (fewer reloaded boundary chains); at least 8 chains, up
    // to the whole sample when there are few wavefronts per sample
    // (vector-major states with few groups per plane).
    static int strip_chains(const kpm_launch &l, int k, int64_t nx, int64_t ny, int64_t waves) {
        if (l.tiled < 5) return 16 << (l.tiled - 3);
        const int64_t nst = (nx + kpm::kWave - 2 * k - 1) / (kpm::kWave - 2 * k);
        int64_t best = -1;
        int tj = 8;
        const int jmax = (int)std::max<int64_t>(64, ny);
        for (int j = 8; j <= jmax; ++j) {
            const int64_t strips = nst * ((ny + j - 1) / j);
            const int64_t passes = (j + 2 * k + kpm::kMarchRows - 1) / kpm::kMarchRows;
            const int64_t cost = (strips + waves - 1) / waves * passes;
            if (best < 0 || cost <= best) {
                best = cost;
                tj = j;
            }
        }
        return tj;
    }

    // Multi-step tiles: two steps in LDS tiles of 16 chains x kTileCols
    // columns (tiled = 0, or no graphene slot order); register tiles of 8
    // chains (tiled = 1, or tiled = 0 with 3 or 4 steps) or 4 (tiled = 2);
    // marching strips of 16 or 32 chains (tiled = 3, 4), or as long as one
    // strip per wavefront of the grid allows (tiled = 5).
    kpm::Lat2 lat2(const kpm_launch &l, int k, int nwg) const {
        const int reg = !d_flags ? 0 : (l.tiled >= 3 ? 2 : ((l.tiled >= 1 || k > 2) ? 1 : 0));
        int tj = reg == 2 ? 16 << (l.tiled - 3) : (reg == 1 ? (l.tiled == 2 ? 4 : 8) : 16);
        if (reg == 2 && nseg == 1)
            tj = strip_chains(l, k, l2nx, l2ny, (int64_t)nwg * strip_waves(l));
        // (a batch's strips take their geometry from its segment table)
        return kpm::Lat2{l2nx, l2ny, k, reg, tj, (l2nx + kpm::kTileCols - 1) / kpm::kTileCols,
                         (l2ny + tj - 1) / tj, d_code, d_flags, prec == KPM_FP32 ? 1 : 0,
                         nseg == 1 ? d_pid : d_sid, nseg == 1 ? npat : nsp};
    }

    kpm::Ell ell() const {
        kpm::Ell h;
        h.nbr = d_nbr;
        h.pid = d_pid;
        h.pat = d_pat;
        h.npat = npat;
        h.hop = d_hop;
        h.xw = d_xw;
        h.ons = d_ons;
        h.onsf = d_onsf;
        h.n = n;
        h.w = w;
        return h;
    }

    // Algorithmic bytes of one moment-step launch: four state accesses per
    // element (read phi_1, phi_0, phi_L, write phi_0; three in the doubling
    // form, which reads no phi_L) and the row structure once per row
    // (neighbours, on-site term, per-slot hopping).
    int64_t step_bytes(int vshift, bool dbl = false) const {
        const bool compact = d_pid && shape(vshift, dbl).compact;
        const int64_t per_row = (compact ? 1 : 4 * w) + (d_onsf ? 4 : 8) + (d_hop ? 8 * w : 0);
        const int64_t acc = dbl ? 3 : 4;
        return n * ((acc * elem_bytes()) << vshift) + n * per_row;
    }

    // Algorithmic bytes of one multi-step launch (one vector, compact form):
    // read phi_n, phi_{n-1} (and phi_L), write the last two states, and the
    // row structure once.
    int64_t step2_bytes(bool dbl) const {
        const int64_t acc = dbl ? 4 : 5;
        return n * (acc * (int64_t)elem_bytes() + 1 + (d_onsf ? 4 : 8));
    }

    // The sweep of the moment step (and every other kernel) for n_vec =
    // 2^vshift under launch shape l.  Batches give each sample a contiguous
    // run of work-groups (a multiple of 8) in proportion to its rows; their
    // device segment table is built on first use (may_alloc), or must exist.
    kpm_status sweep_with(int vshift, const kpm_launch &l, kpm::Sweep *out,
                          bool may_alloc = true, int64_t want_groups = 0) {
        kpm::Sweep sw{};
        sw.nplanes = 1;
        sw.pstride = 0;
        sw.wpg = strip_waves(l);
        sw.total = n << vshift;
        sw.vshift = vshift;
        sw.ilp = l.ilp;
        sw.nt = l.streaming;
        const int64_t want = want_groups > 0 ? want_groups
                             : std::max<int64_t>(kpm::kXcds, ((int64_t)cus * l.groups_per_cu) /
                                                                 kpm::kXcds * kpm::kXcds);
        // the single-step traversal; under a multi-step shape, tiled selects
        // the multi-step tiles and single steps keep row order
        const int tiled = l.steps == 1 ? l.tiled : 0;
        const int tw = tiled > 0 ? tile_rows(vshift) << (tiled - 1) : tile_rows(vshift);
        auto tiling = [&](int s, int32_t *tnx) {
            *tnx = (tiled && chain[s] >= 2 * tw) ? chain[s] : 0;
        };
        // multiply-shift constants for t / nch (nch = rows / tnx chains)
        auto divider = [&](int s, int32_t tnx, kpm::Seg &g) {
            g.div_m = 0;
            g.div_l = 0;
            if (!tnx) return;
            const uint64_t d = (uint64_t)((off[s + 1] - off[s]) / tnx);
            int l = 0;
            while (((uint64_t)1 << l) < d) ++l;
            g.div_l = l;
            // ceil(2^(32 + l) / d) < 2^33
            const unsigned __int128 num = (unsigned __int128)1 << (32 + l);
            g.div_m = (uint64_t)((num + d - 1) / d);
        };
        if (nseg == 1) {
            const int64_t nblk = (sw.total + kpm::kBlock - 1) / kpm::kBlock;
            const int64_t cap = ((nblk + kpm::kXcds - 1) / kpm::kXcds) * kpm::kXcds;
            sw.nwg = (int)std::max<int64_t>(kpm::kXcds, std::min(want, cap));
            sw.nseg = 1;
            sw.seg = nullptr;
            sw.wg_seg = nullptr;
            int32_t tnx;
            tiling(0, &tnx);
            sw.one = kpm::Seg{0, sw.total, 0, sw.nwg, seg_t[0], 1.0 / es[0], tnx, tw, 0, 0};
            divider(0, tnx, sw.one);
            *out = sw;
            return KPM_OK;
        }
        // marching strips of a batch: each sample's chain length and strip
        // chains for its wavefronts
        const int ksteps = multi_steps(vshift, l) > 1 ? l.steps : 0;
        for (const SegTab &t : segtabs) {
            if (t.vshift == vshift && t.want == want && t.tiled == tiled && t.ksteps == ksteps &&
                t.wpg == (ksteps ? sw.wpg : 0)) {
                sw.nwg = t.nwg;
                sw.nseg = nseg;
                sw.seg = t.seg;
                sw.wg_seg = t.wg;
                *out = sw;
                return KPM_OK;
            }
        }
        if (!may_alloc)
            return fail(KPM_ERR_UNSUPPORTED, "no segment table for this launch shape");
        const int64_t units = want / kpm::kXcds;
        std::vector<kpm::Seg> seg(nseg);
        int64_t g0 = 0;
        for (int s = 0; s < nseg; ++s) {
            const int64_t rows = off[s + 1] - off[s];
            const int64_t nblk = ((rows << vshift) + kpm::kBlock - 1) / kpm::kBlock;
            int64_t u = (int64_t)std::llround((double)units * rows / (double)n);
            u = std::max<int64_t>(1, std::min(u, (nblk + kpm::kXcds - 1) / kpm::kXcds));
            int32_t tnx;
            tiling(s, &tnx);
            seg[s] = kpm::Seg{off[s] << vshift, off[s + 1] << vshift, (int32_t)g0,
                              (int32_t)(u * kpm::kXcds), seg_t[s], 1.0 / es[s], tnx, tw, 0, 0};
            divider(s, tnx, seg[s]);
            if (ksteps) {
                seg[s].snx = chain[s];
                seg[s].sj = strip_chains(l, ksteps, chain[s], rows / chain[s],
                                         u * kpm::kXcds * sw.wpg);
            }
            g0 += u * kpm::kXcds;
        }
        if (g0 > (1 << 30)) return fail(KPM_ERR_INVALID, "batch needs too many work-groups");
        std::vector<int32_t> wg(g0);
        for (int s = 0; s < nseg; ++s)
            for (int g = 0; g < seg[s].nwg; ++g) wg[seg[s].g0 + g] = s;
        SegTab t{vshift, want, tiled, ksteps, ksteps ? sw.wpg : 0, (int)g0, nullptr, nullptr};
        KPM_HIP(hipMalloc(&t.seg, seg.size() * sizeof(kpm::Seg)));
        KPM_HIP(hipMalloc(&t.wg, wg.size() * sizeof(int32_t)));
        KPM_HIP(hipMemcpy(t.seg, seg.data(), seg.size() * sizeof(kpm::Seg), hipMemcpyHostToDevice));
        KPM_HIP(hipMemcpy(t.wg, wg.data(), wg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        segtabs.push_back(t);
        sw.nwg = t.nwg;
        sw.nseg = nseg;
        sw.seg = t.seg;
        sw.wg_seg = t.wg;
        *out = sw;
        return KPM_OK;
    }

    // Whether calls with 2^vshift vectors keep their states vector-major (one
    // plane per vector; one-sample systems, or batches whose moment sets take
    // the marching strips, under a shape with one vector per wavefront).  The
    // direct form's shape decides for both forms.
    bool planar(int vshift) const {
        return vshift > 0 && (nseg == 1 || bstrips) && launch[vshift].vectors_per_wave == 1;
    }

    // The sweep of every kernel of a call with 2^vshift vectors under shape l:
    // sweep_with, or for vector-major states the one-vector sweep of each
    // plane (plane_groups work-groups, when set) over 2^vshift planes.
    kpm_status sweep_planes(int vshift, const kpm_launch &l, kpm::Sweep *out,
                            bool may_alloc = true) {
        // a batch shares plane_groups out among its samples
        KPM_TRY(sweep_with(0, l, out, may_alloc, nseg > 1 ? l.plane_groups : 0));
        if (l.plane_groups > 0 && nseg == 1) {
            out->nwg = l.plane_groups;
            out->one.nwg = l.plane_groups;
        }
        out->nplanes = 1 << vshift;
        out->pstride = n;
        return KPM_OK;
    }
    kpm_status sweep_for(int vshift, const kpm_launch &l, kpm::Sweep *out,
                         bool may_alloc = true) {
        return planar(vshift) ? sweep_planes(vshift, l, out, may_alloc)
                              : sweep_with(vshift, l, out, may_alloc);
    }
    kpm_status sweep(int vshift, kpm::Sweep *out) { return sweep_for(vshift, launch[vshift], out); }

    // Algorithmic bytes of one single-step moment launch of sweep sw under
    // shape l (step_bytes for any layout).
    int64_t sweep_step_bytes(const kpm::Sweep &sw, const kpm_launch &l, bool dbl) const {
        const bool compact = d_pid && l.compact;
        const int64_t per_row = (compact ? 1 : 4 * w) + (d_onsf ? 4 : 8) + (d_hop ? 8 * w : 0);
        const int64_t acc = dbl ? 3 : 4;
        return (int64_t)sw.nplanes * (n * ((acc * (int64_t)elem_bytes()) << sw.vshift) + n * per_row);
    }

    // Coefficients c_m of Eq. 36 for every sample: host values for a single
    // sample (kernel arguments), a cached device table [nseg][np] otherwise.
    kpm_status bessel(double dt, int sign, int np, std::vector<double2> &host,
                      const double2 **tab) {
        host.resize((size_t)np * nseg);
        for (int s = 0; s < nseg; ++s) bessel_coeffs(np, es[s] * dt / kHbar, sign, &host[(size_t)s * np]);
        *tab = nullptr;
        if (nseg == 1) return KPM_OK;
        for (const CoefTab &c : coeftabs)
            if (c.dt == dt && c.sign == sign && c.np == np) {
                *tab = c.d;
                return KPM_OK;
            }
        CoefTab c{dt, sign, np, nullptr};
        KPM_HIP(hipMalloc(&c.d, host.size() * sizeof(double2)));
        KPM_HIP(hipMemcpy(c.d, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice));
        coeftabs.push_back(c);
        *tab = c.d;
        return KPM_OK;
    }

    // Elements one launch of sweep sw updates (rows x vectors).
    static int64_t sweep_elems(const kpm::Sweep &sw) { return sw.total * sw.nplanes; }

    kpm::Coef alpha() const {
        const double2 v = make_double2(0.0, -es[0] / kHbar);   // V = -i (E_s/hbar) D
        return nseg == 1 ? kpm::coef_val(v) : kpm::coef_tab(d_alpha, 1, 0, v);
    }

    // This device's fixed scratch (kpm_moments_noalloc), looked up at creation.
    void *static_scratch = nullptr;

    // Scratch limit (KPM_SCRATCH_LIMIT_MB at creation; 0 = none): the recursion
    // buffers, partials and moments together may not exceed it.
    size_t scratch_limit = 0;
    // xbytes: all extra multi-step states together
    kpm_status check_scratch(size_t nvec, size_t vbytes, size_t pelems, size_t delems,
                             size_t xbytes) const {
        const size_t total = nvec * vbytes + xbytes + (pelems + delems) * sizeof(double2);
        if (scratch_limit && total > scratch_limit)
            return fail(KPM_ERR_OOM, "scratch of %zu bytes exceeds the limit of %zu bytes", total,
                        scratch_limit);
        return KPM_OK;
    }

    // Makes sure `count` state vectors of n_vec vectors each exist.
    kpm_status ensure_vecs(int count, int vshift) {
        const size_t bytes = state_bytes(vshift);
        KPM_TRY(check_scratch(std::max<size_t>(count, vecs.size()), std::max(bytes, vec_bytes),
                              partial_elems, dmom_elems, xbuf_bytes * xbuf_count));
        if (bytes > vec_bytes) {
            drop_graphs();
            KPM_HIP(hipStreamSynchronize(stream));
            for (void *p : vecs) (void)hipFree(p);
            vecs.clear();
            vec_bytes = bytes;
        }
        while ((int)vecs.size() < count) {
            void *p = nullptr;
            KPM_HIP(hipMalloc(&p, vec_bytes));
            KPM_HIP(hipMemsetAsync(p, 0, vec_bytes, stream));
            vecs.push_back(p);
        }
        return KPM_OK;
    }

    // The extra recursion states of the multi-step sweeps: two (one
    // recursion) or four (the coupled propagator).
    kpm_status ensure_xbuf(int vshift, int count = 2) {
        const size_t bytes = state_bytes(vshift);
        if (bytes <= xbuf_bytes && count <= xbuf_count) return KPM_OK;
        count = std::max(count, xbuf_count);
        KPM_TRY(check_scratch(vecs.size(), vec_bytes, partial_elems, dmom_elems,
                              std::max(bytes, xbuf_bytes) * (size_t)count));
        const size_t nb = std::max(bytes, xbuf_bytes);
        drop_graphs();
        KPM_HIP(hipStreamSynchronize(stream));
        for (void *&p : xbuf) {
            if (p) (void)hipFree(p);
            p = nullptr;
        }
        xbuf_bytes = 0;
        xbuf_count = 0;
        for (int i = 0; i < count; ++i) KPM_HIP(hipMalloc(&xbuf[i], nb));
        xbuf_bytes = nb;
        xbuf_count = count;
        return KPM_OK;
    }

    kpm_status ensure_partial(int slots, int nwg, int n_vec) {
        const size_t need = (size_t)slots * nwg * n_vec;
        if (need > partial_elems) {
            KPM_TRY(check_scratch(vecs.size(), vec_bytes, need, dmom_elems,
                                  xbuf_bytes * xbuf_count));
            drop_graphs();
            KPM_HIP(hipStreamSynchronize(stream));
            if (partial) (void)hipFree(partial);
            partial = nullptr;
            KPM_HIP(hipMalloc(&partial, need * sizeof(double2)));
            partial_elems = need;
        }
        return KPM_OK;
    }

    kpm_status ensure_dmom(size_t elems) {
        if (elems > dmom_elems) {
            KPM_TRY(check_scratch(vecs.size(), vec_bytes, partial_elems, elems,
                                  xbuf_bytes * xbuf_count));
            drop_graphs();
            KPM_HIP(hipStreamSynchronize(stream));
            if (dmom) (void)hipFree(dmom);
            dmom = nullptr;
            KPM_HIP(hipMalloc(&dmom, elems * sizeof(double2)));
            dmom_elems = elems;
        }
        return KPM_OK;
    }

    // An event pair for a run of `launches` moment-step launches of `rows`
    // rows x vectors each (the count may be set once the run is closed).
    kpm_status event_pair(hipEvent_t *a, hipEvent_t *b, int64_t rows, int64_t launches = 0) {
        while (events.size() < events_used + 2) {
            hipEvent_t e;
            KPM_HIP(hipEventCreate(&e));
            events.push_back(e);
        }
        *a = events[events_used];
        *b = events[events_used + 1];
        events_used += 2;
        ev_runs.resize(events_used / 2);
        ev_runs.back() = {rows, launches};
        return KPM_OK;
    }
    void close_run(int64_t launches) { ev_runs.back().second = launches; }

    // Adds the elapsed time of every recorded event pair to the stats (and to
    // the widest runs' figures).  The stream must have been synchronised.
    kpm_status harvest_events() {
        for (size_t k = 0; k + 1 < events_used; k += 2) {
            float ms = 0;
            KPM_HIP(hipEventElapsedTime(&ms, events[k], events[k + 1]));
            stats.step_ms += ms;
            const auto &run = ev_runs[k / 2];
            if (run.first > stats.wide_rows) {
                stats.wide_rows = run.first;
                stats.wide_ms = 0;
                stats.wide_launches = 0;
            }
            if (run.first == stats.wide_rows) {
                stats.wide_ms += ms;
                stats.wide_launches += run.second;
            }
        }
        events_used = 0;
        ev_runs.clear();
        return KPM_OK;
    }

    ~kpm_system() {
        DeviceGuard g(device);
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (void *p : vecs) (void)hipFree(p);
        for (void *p : xbuf)
            if (p) (void)hipFree(p);
        if (d_code) (void)hipFree(d_code);
        if (d_sid) (void)hipFree(d_sid);
        if (d_flags) (void)hipFree(d_flags);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (SegTab &t : segtabs) {
            (void)hipFree(t.seg);
            (void)hipFree(t.wg);
        }
        for (CoefTab &c : coeftabs) (void)hipFree(c.d);
        if (partial) (void)hipFree(partial);
        if (dmom) (void)hipFree(dmom);
        if (d_nbr) (void)hipFree(d_nbr);
        if (d_pid) (void)hipFree(d_pid);
        if (d_pat) (void)hipFree(d_pat);
        if (d_onsf) (void)hipFree(d_onsf);
        if (d_hop) (void)hipFree(d_hop);
        if (d_xw) (void)hipFree(d_xw);
        if (d_pxw) (void)hipFree(d_pxw);
        if (d_ons) (void)hipFree(d_ons);
        if (d_alpha) (void)hipFree(d_alpha);
    }
};

namespace {

kpm::Coef step_coef(const std::vector<double2> &host, const double2 *tab, int np, int m) {
    return tab ? kpm::coef_tab(tab, np, m, host[m]) : kpm::coef_val(host[m]);
}

// ---------------------------------------------------------------- drivers
// Number of moment slots of a set: one per moment, or in the doubling form
// (phi_L = phi_R) two per recursion step, rounded up to an even count.
inline int moment_slots(int nm, bool dbl) { return dbl ? 2 * ((nm + 1) / 2) : nm; }

// Launch plan of one moment set: partial slots [c0, c1) form one ring
// segment (the first holds ring + 2 slots, C_0 and C_1 included, the others
// ring), and inside a segment the recursion takes k-step launches while all k
// steps fit, then one launch of the 2 .. k - 1 steps that still fit, and single
// steps otherwise.  visit(kind, m, c0) is called for every recursion launch
// (kind = steps of the launch, first moment slot m) and segment(c0, c1, m0)
// once a segment's launches are done.
template <typename F, typename G>
void moment_plan(int slots, int ring, bool dbl, int k, F visit, G segment) {
    const int per_step = dbl ? 2 : 1;
    for (int c0 = 0; c0 < slots;) {
        const int c1 = std::min(slots, c0 == 0 ? ring + 2 : c0 + ring);
        const int m0 = std::max(c0, 2);
        for (int m = m0; m < c1;) {
            const int fit = (c1 - m) / per_step;          // whole steps left in the segment
            const int kind = k > 1 ? std::max(1, std::min(k, fit)) : 1;
            visit(kind, m, c0);
            m += kind * per_step;
        }
        segment(c0, c1, m0);
        c0 = c1;
    }
}

// The sweep that reduces the partials of launches of sw: partials of
// vector-major launches are [slot][nwg][planes], which is the layout of
// 2^vshift vectors side by side with vshift = log2(planes).
kpm::Sweep reduce_sweep(const kpm::Sweep &sw) {
    kpm::Sweep r = sw;
    if (sw.nplanes > 1) {
        int v = 0;
        while ((1 << v) < sw.nplanes) ++v;
        r.vshift = v;
        r.nplanes = 1;
        r.pstride = 0;
    }
    return r;
}

// Launches of one moment set (Alg. 5) on stream s: the first step, the
// recursion steps and the ring reductions into sys->dmom.  `events` brackets
// each uninterrupted run of recursion steps for kpm_set_timing.  In the
// doubling form phil is phir, recursion step n fills slots 2n and 2n + 1, and
// a final kernel turns the doubling sums into moments.  States rotate through
// a_buf, b_buf (and x0_buf, x1_buf for multi-step launches); group partials
// go to `partial`, the reduced moments to `dmom`; phir is only read.
template <typename V>
kpm_status enqueue_moments(kpm_system *sys, const kpm_launch &l, const kpm::Sweep &sw, int ring,
                           hipStream_t s, bool events, bool dbl, bool re, const V *phil,
                           const V *phir, int nm, V *a_buf, V *b_buf, V *x0_buf, V *x1_buf,
                           double2 *partial, double2 *dmom, int64_t stride_r, int64_t offset) {
    const kpm::Ell h = sys->ell_for(l);
    const int k = sys->multi_steps(sw.vshift, l);
    const kpm::Lat2 lat = sys->lat2(l, k, sw.nwg);
    V *pool[4] = {a_buf, b_buf, x0_buf, x1_buf};
    const int npool = k > 1 ? 4 : 2;
    // a pool state that is none of x, y, z
    auto free_state = [&](const V *x, const V *y, const V *z) -> V * {
        for (int q = 0; q < npool; ++q)
            if (pool[q] != x && pool[q] != y && pool[q] != z) return pool[q];
        return nullptr;
    };
    // C_0 and C_1 (phi_0 = phi_R, phi_1 = H~ phi_0)
    kpm::launch_moment_step<V>(h, sw, true, phir, nullptr, a_buf, phil, partial, 0, s);
    // phi_m = 2 H~ phi_{m-1} - phi_{m-2}; a single step writes over phi_{m-2}
    // (when it is scratch), a two-step launch into two other states
    const V *p0 = phir;
    V *p1 = a_buf;
    const int slots = moment_slots(nm, dbl);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool open = false;
    int64_t in_run = 0;                       // launches in the open timed run
    kpm_status st = KPM_OK;
    moment_plan(
        slots, ring, dbl, k,
        [&](int kind, int m, int c0) {
            if (st != KPM_OK) return;
            if (events && !open) {
                if ((st = sys->event_pair(&e0, &e1, kpm_system::sweep_elems(sw))) != KPM_OK)
                    return;
                if (hipEventRecord(e0, s) != hipSuccess) {
                    st = fail(KPM_ERR_DEVICE, "event record");
                    return;
                }
                open = true;
                in_run = 0;
            }
            ++in_run;
            if (kind > 1) {
                V *o1 = free_state(p0, p1, nullptr);
                V *o2 = free_state(p0, p1, o1);
                if (!kpm::launch_moment_multi<V>(
                        h, sw, kind == k ? lat : sys->lat2(l, kind, sw.nwg), p1, p0, o1, o2,
                        phil, partial, m - c0, dbl, re, s)) {
                    st = fail(KPM_ERR_UNSUPPORTED, "no multi-step kernel for %d steps", kind);
                    return;
                }
                p0 = o1;
                p1 = o2;
                return;
            }
            bool scratch = false;
            for (int q = 0; q < npool; ++q) scratch = scratch || pool[q] == p0;
            V *out = scratch ? const_cast<V *>(p0) : free_state(p0, p1, nullptr);
            if (dbl)
                kpm::launch_moment_step_doubled<V>(h, sw, p1, p0, out, partial, m - c0, s);
            else
                kpm::launch_moment_step<V>(h, sw, false, p1, p0, out, phil, partial, m - c0, s);
            p0 = p1;
            p1 = out;
        },
        [&](int c0, int c1, int) {
            if (st != KPM_OK) return;
            if (open) {
                if (hipEventRecord(e1, s) != hipSuccess) st = fail(KPM_ERR_DEVICE, "event record");
                sys->close_run(in_run);
                open = false;
            }
            kpm::launch_reduce(partial, reduce_sweep(sw), std::min(c1, nm) - c0, dmom, stride_r,
                               offset + c0, s);
        });
    KPM_TRY(st);
    const kpm::Sweep rs = reduce_sweep(sw);
    if (dbl) kpm::launch_undouble(dmom, rs.nseg << rs.vshift, stride_r, offset, nm, s);
    return KPM_OK;
}

// Chebyshev moments of Alg. 5 for n_vec vector pairs (every sample), reduced
// into sys->dmom[(s * R + r) * stride_r + offset + m] (complex).  With graphs
// enabled the launch sequence is captured once per set of buffers and
// replayed.  dbl selects the doubling form (phil must equal phir).  re: the
// caller uses only the real parts of the moments (their imaginary parts may
// then be left at 0).
template <typename V>
kpm_status run_moments(kpm_system *sys, int vshift, const V *phil, const V *phir, int nm,
                       V *a_buf, V *b_buf, int64_t stride_r, int64_t offset, bool dbl = false,
                       bool re = false, const kpm_launch *planes = nullptr) {
    // planes: run the 2^vshift vectors as vector-major planes under this shape
    const kpm_launch *lp = planes ? planes : &sys->shape(vshift, dbl);
    // real parts of FP64 states in vector-major planes: the eight-step strips
    // take ten steps per pass (in groups of at least kBlock threads, whose LDS
    // holds the ten-step pass's per-thread sums with two groups per CU)
    kpm_launch lre;
    if (re && !dbl && std::is_same<V, double2>::value && vshift > 0 &&
        lp->vectors_per_wave == 1 && lp->tiled >= 3 && lp->steps == kpm::kMaxMarchSteps &&
        (lp->group_size == 0 || lp->group_size >= kpm::kBlock)) {
        lre = *lp;
        lre.steps = kpm::kReMarchSteps;
        lp = &lre;
    }
    const kpm_launch &l = *lp;
    kpm::Sweep sw;
    KPM_TRY(planes ? sys->sweep_planes(vshift, l, &sw) : sys->sweep_for(vshift, l, &sw));
    const int k = sys->multi_steps(sw.vshift, l);
    if (k > 1) KPM_TRY(sys->ensure_xbuf(vshift));
    // Group partials live in a ring of moment slots that is reduced into
    // sys->dmom whenever it fills, bounding its size at any N_m; the ring is
    // a multiple of the slots of one k-step launch.
    const int slots = moment_slots(nm, dbl);
    const int per_launch = k * (dbl ? 2 : 1);
    const int ring = std::min(std::max(slots, 2), kPartialRing - kPartialRing % per_launch);
    KPM_TRY(sys->ensure_partial(ring + 2, sw.nwg, 1 << vshift));
    int64_t n1 = 0, n2 = 0;
    moment_plan(slots, ring, dbl, k, [&](int kind, int, int) { (kind > 1 ? n2 : n1) += 1; },
                [](int, int, int) {});
    const int64_t b1 = sys->sweep_step_bytes(sw, l, dbl), b2 = sys->step2_bytes(dbl) * sw.nplanes;
    const int steps = dbl ? slots / 2 - 1 : std::max(nm - 2, 0);   // recursion steps
    sys->stats.step_rows = kpm_system::sweep_elems(sw);
    sys->stats.step_bytes = n2 > 0 ? b2 : b1;
    sys->stats.site_updates += (int64_t)(steps + 1) * kpm_system::sweep_elems(sw);
    if (sys->timing) {
        sys->stats.step_launches += n1 + n2;
        sys->stats.step_bytes_total += n1 * b1 + n2 * b2;
    }
    if (!sys->graphs)
        return enqueue_moments<V>(sys, l, sw, ring, sys->stream, sys->timing, dbl, re, phil, phir,
                                  nm, a_buf, b_buf, (V *)sys->xbuf[0], (V *)sys->xbuf[1],
                                  sys->partial, sys->dmom, stride_r, offset);
    kpm_system::GraphKey key{phil, phir, a_buf, b_buf, sys->partial, sys->dmom, nm, vshift,
                             l.groups_per_cu, l.ilp, l.streaming, l.compact, l.tiled, l.steps,
                             dbl ? 1 : 0, re ? 1 : 0, sw.nplanes, sw.nwg, l.group_size,
                             stride_r, offset};
    hipGraphExec_t exec = sys->find_graph(key);
    if (!exec) {
        KPM_TRY(sys->ensure_capture_stream());
        KPM_HIP(hipStreamBeginCapture(sys->cap, hipStreamCaptureModeThreadLocal));
        kpm_status st = enqueue_moments<V>(sys, l, sw, ring, sys->cap, false, dbl, re, phil, phir,
                                           nm, a_buf, b_buf, (V *)sys->xbuf[0],
                                           (V *)sys->xbuf[1], sys->partial, sys->dmom, stride_r,
                                           offset);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(sys->cap, &graph);
        if (st != KPM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (ec != hipSuccess) return fail(KPM_ERR_DEVICE, "graph capture: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(KPM_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
        sys->graph_cache.push_back({key, exec});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (sys->timing) {
        KPM_TRY(sys->event_pair(&e0, &e1, kpm_system::sweep_elems(sw), n1 + n2));
        KPM_HIP(hipEventRecord(e0, sys->stream));
    }
    KPM_HIP(hipGraphLaunch(exec, sys->stream));
    if (sys->timing) KPM_HIP(hipEventRecord(e1, sys->stream));
    return KPM_OK;
}

// acc = [add +] U(sign dt) in  (Alg. 6).  Scratch a_buf, b_buf.
template <typename V>
kpm_status run_evolve(kpm_system *sys, int vshift, const V *in, V *acc, const V *add,
                      double dt, int sign, int np, V *a_buf, V *b_buf) {
    const kpm::Ell h = sys->ell_for(sys->launch[vshift]);
    kpm::Sweep sw;
    KPM_TRY(sys->sweep(vshift, &sw));
    std::vector<double2> c;
    const double2 *tab = nullptr;
    KPM_TRY(sys->bessel(dt, sign, np, c, &tab));
    hipStream_t s = sys->stream;
    kpm::launch_evolve_step<V>(h, sw, true, in, nullptr, a_buf, acc, add,
                               step_coef(c, tab, np, 0), step_coef(c, tab, np, 1), s);
    const V *p0 = in;
    V *p1 = a_buf;
    int m = 2;
    // Several steps per pass in the moment sets' marching strips (one sample,
    // one vector per row): the new states go to two of the four scratch
    // states that the pass does not read (never to `in`), and a last pass
    // takes the remaining steps when there are at least two
    const kpm_launch &l = sys->launch[vshift];
    const int k = sys->multi_steps(sw.vshift, l);
    if (k > 1 && l.tiled >= 3 && sys->d_flags && !tab && np - m >= 2) {
        KPM_TRY(sys->ensure_xbuf(vshift));
        V *pool[4] = {a_buf, b_buf, (V *)sys->xbuf[0], (V *)sys->xbuf[1]};
        while (np - m >= 2) {
            const int kk = std::min({k, np - m, kpm::kMaxMarchSteps});
            V *o[2];
            int no = 0;
            for (V *q : pool)
                if (q != p1 && q != p0 && no < 2) o[no++] = q;
            kpm::CoefK ck{};
            for (int j = 0; j < kk; ++j) ck.c[j] = c[m + j];
            if (!kpm::launch_evolve_multi<V>(h, sw, sys->lat2(l, kk, sw.nwg), p1, p0, o[0], o[1],
                                             acc, ck, s))
                return fail(KPM_ERR_UNSUPPORTED, "no propagator kernel for %d steps", kk);
            p0 = o[0];
            p1 = o[1];
            m += kk;
        }
    }
    for (; m < np; ++m) {
        V *out = (m == 2) ? b_buf : const_cast<V *>(p0);
        kpm::launch_evolve_step<V>(h, sw, false, p1, p0, out, acc, nullptr,
                                   step_coef(c, tab, np, 0), step_coef(c, tab, np, m), s);
        p0 = p1;
        p1 = out;
    }
    sys->stats.site_updates += (int64_t)(np - 1) * kpm_system::sweep_elems(sw);
    return KPM_OK;
}

// accx = [X, U(dt)] in, accu = U(dt) in  (Alg. 7 with Eq. 36 alongside).
template <typename V>
kpm_status run_evolve_x(kpm_system *sys, int vshift, const V *in, V *accx, V *accu,
                        double dt, int np, V *pa, V *pb, V *qa, V *qb) {
    const kpm::Ell h = sys->ell_for(sys->launch[vshift]);
    kpm::Sweep sw;
    KPM_TRY(sys->sweep(vshift, &sw));
    std::vector<double2> c;
    const double2 *tab = nullptr;
    KPM_TRY(sys->bessel(dt, +1, np, c, &tab));
    hipStream_t s = sys->stream;
    kpm::launch_evolve_x_step<V>(h, sw, true, in, nullptr, pa, nullptr, nullptr, qa, accx,
                                 accu, step_coef(c, tab, np, 0), step_coef(c, tab, np, 1), s);
    const V *p0 = in, *q0 = nullptr;
    V *p1 = pa, *q1 = qa;
    int m = 2;
    // Up to three coupled steps per pass in marching strips where the moment
    // sets use strips and the commutator weights follow the neighbour patterns;
    // each recursion's new states go to two of its four scratch states that the
    // pass does not read
    // the coupled strips run in groups of kBlock threads whatever the shape's
    // group size
    kpm_launch l = sys->launch[vshift];
    l.group_size = 0;
    const int k = std::min(sys->multi_steps(sw.vshift, l), 3);
    if (k > 1 && l.tiled >= 3 && sys->d_flags && sys->d_pxw && !tab && np - m >= 2) {
        KPM_TRY(sys->ensure_xbuf(vshift, 4));
        V *pool_p[4] = {pa, pb, (V *)sys->xbuf[0], (V *)sys->xbuf[1]};
        V *pool_q[4] = {qa, qb, (V *)sys->xbuf[2], (V *)sys->xbuf[3]};
        auto pick = [](V *const *pool, const V *a, const V *b, V **o) {
            int no = 0;
            for (int i = 0; i < 4; ++i)
                if (pool[i] != a && pool[i] != b && no < 2) o[no++] = pool[i];
        };
        while (np - m >= 2) {
            const int kk = std::min(k, np - m);
            V *po[2], *qo[2];
            pick(pool_p, p1, p0, po);
            pick(pool_q, q1, q0, qo);
            kpm::CoefK ck{};
            for (int j = 0; j < kk; ++j) ck.c[j] = c[m + j];
            if (!kpm::launch_evolve_x_multi<V>(h, sw, sys->lat2(l, kk, sw.nwg), sys->d_pxw, p1,
                                               p0, po[0], po[1], q1, q0, qo[0], qo[1], accx,
                                               accu, ck, s))
                return fail(KPM_ERR_UNSUPPORTED, "no coupled propagator kernel for %d steps", kk);
            p0 = po[0];
            p1 = po[1];
            q0 = qo[0];
            q1 = qo[1];
            m += kk;
        }
    }
    for (; m < np; ++m) {
        V *pout = (m == 2) ? pb : const_cast<V *>(p0);
        V *qout = (m == 2) ? qb : const_cast<V *>(q0);
        kpm::launch_evolve_x_step<V>(h, sw, false, p1, p0, pout, q1, q0, qout, accx, accu,
                                     step_coef(c, tab, np, 0), step_coef(c, tab, np, m), s);
        p0 = p1;
        p1 = pout;
        q0 = q1;
        q1 = qout;
    }
    sys->stats.site_updates += 2 * (int64_t)(np - 1) * kpm_system::sweep_elems(sw);
    return KPM_OK;
}

kpm_status check_common(kpm_system *sys, int n_vec, int *vshift) {
    if (!sys) return fail(KPM_ERR_INVALID, "null system");
    *vshift = vshift_of(n_vec);
    if (*vshift < 0) return fail(KPM_ERR_INVALID, "n_vec must be 1, 2, 4, ..., 64 (got %d)", n_vec);
    return KPM_OK;
}

kpm_status finish_moments(kpm_system *sys, size_t elems, double2 *host,
                          const double2 *src = nullptr) {
    KPM_HIP(hipMemcpyAsync(host, src ? src : sys->dmom, elems * sizeof(double2),
                           hipMemcpyDeviceToHost, sys->stream));
    KPM_HIP(hipStreamSynchronize(sys->stream));
    KPM_HIP(hipGetLastError());
    if (sys->timing) KPM_TRY(sys->harvest_events());
    for (size_t k = 0; k < elems; ++k)
        if (!std::isfinite(host[k].x) || !std::isfinite(host[k].y))
            return fail(KPM_ERR_NUMERIC, "non-finite moment at index %zu", k);
    return KPM_OK;
}

// The caller's state src ([n_sites][n_vec]) into the device buffer dst in
// the layout of the call (vector-major when planar), and back.
template <typename V>
kpm_status stage_in(kpm_system *sys, int vshift, const void *src, V *dst) {
    if (sys->planar(vshift))
        kpm::launch_planar<V>((const V *)src, dst, sys->n, vshift, true, sys->stream);
    else
        KPM_HIP(hipMemcpyAsync(dst, src, sys->state_bytes(vshift), hipMemcpyDeviceToDevice,
                               sys->stream));
    return KPM_OK;
}
template <typename V>
kpm_status stage_out(kpm_system *sys, int vshift, const V *src, void *dst) {
    if (sys->planar(vshift))
        kpm::launch_planar<V>(src, (V *)dst, sys->n, vshift, false, sys->stream);
    else
        KPM_HIP(hipMemcpyAsync(dst, src, sys->state_bytes(vshift), hipMemcpyDeviceToDevice,
                               sys->stream));
    return KPM_OK;
}

template <typename V>
kpm_status moments_impl(kpm_system *sys, int vshift, const void *phil, const void *phir,
                        int nm, double *mu, bool dbl) {
    const bool pl = sys->planar(vshift);
    KPM_TRY(sys->ensure_vecs(pl ? 4 : 2, vshift));
    const size_t elems = (size_t)sys->nseg * ((size_t)1 << vshift) * nm;
    KPM_TRY(sys->ensure_dmom(elems));
    V *a = (V *)sys->vecs[0], *b = (V *)sys->vecs[1];
    const V *l = (const V *)phil, *r = (const V *)phir;
    if (pl) {           // vector-major copies of the operands
        V *sl = (V *)sys->vecs[2], *sr = (V *)sys->vecs[3];
        KPM_TRY(stage_in<V>(sys, vshift, phil, sl));
        if (phir != phil) KPM_TRY(stage_in<V>(sys, vshift, phir, sr));
        l = sl;
        r = phir != phil ? sr : sl;
    }
    KPM_TRY(run_moments<V>(sys, vshift, l, r, nm, a, b, nm, 0, dbl));
    return finish_moments(sys, elems, (double2 *)mu);
}

// moments_impl (direct form) without allocating: the recursion states (two,
// or four under a multi-step launch shape), the group partials and the
// reduced moments are carved from the device's fixed scratch, which each call
// overwrites; no graph capture and no timing events.
template <typename V>
kpm_status moments_noalloc_impl(kpm_system *sys, int vshift, const void *phil, const void *phir,
                                int nm, double *mu) {
    if (!sys->static_scratch)
        return fail(KPM_ERR_DEVICE, "no fixed scratch on device %d", sys->device);
    const kpm_launch &l = sys->shape(vshift, false);
    kpm::Sweep sw;
    KPM_TRY(sys->sweep_with(vshift, l, &sw, false));
    const int k = sys->multi_steps(vshift, l);
    const int slots = moment_slots(nm, false);
    const int ring = std::min(std::max(slots, 2), kPartialRing - kPartialRing % k);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t nvec = (size_t)1 << vshift;
    const size_t sb = up(sys->state_bytes(vshift));
    const size_t nstates = k > 1 ? 4 : 2;
    const size_t pb = up((size_t)(ring + 2) * sw.nwg * nvec * sizeof(double2));
    const size_t elems = (size_t)sys->nseg * nvec * nm;
    const size_t db = up(elems * sizeof(double2));
    const size_t need = nstates * sb + pb + db;
    if (need > kpm::kStaticScratchBytes)
        return fail(KPM_ERR_OOM,
                    "kpm_moments_noalloc needs %zu bytes of scratch (%zu states of %zu bytes, "
                    "partials, moments), more than its fixed %zu bytes",
                    need, nstates, sb, (size_t)kpm::kStaticScratchBytes);
    char *base = (char *)sys->static_scratch;
    V *st[4] = {nullptr, nullptr, nullptr, nullptr};
    for (size_t q = 0; q < nstates; ++q) st[q] = (V *)(base + q * sb);
    double2 *partial = (double2 *)(base + nstates * sb);
    double2 *dmom = (double2 *)(base + nstates * sb + pb);
    sys->stats.step_rows = sw.total;
    sys->stats.step_bytes = k > 1 ? sys->step2_bytes(false) : sys->step_bytes(vshift, false);
    sys->stats.site_updates += (int64_t)std::max(nm - 1, 1) * sw.total;
    KPM_TRY(enqueue_moments<V>(sys, l, sw, ring, sys->stream, false, false, false, (const V *)phil,
                               (const V *)phir, nm, st[0], st[1], st[2], st[3], partial, dmom,
                               nm, 0));
    return finish_moments(sys, elems, (double2 *)mu, dmom);
}

template <typename V>
kpm_status evolve_impl(kpm_system *sys, int vshift, void *phi, double dt, int sign, int np) {
    const bool pl = sys->planar(vshift);
    KPM_TRY(sys->ensure_vecs(pl ? 4 : 3, vshift));
    V *a = (V *)sys->vecs[0], *b = (V *)sys->vecs[1], *acc = (V *)sys->vecs[2];
    const V *in = (const V *)phi;
    if (pl) {
        KPM_TRY(stage_in<V>(sys, vshift, phi, (V *)sys->vecs[3]));
        in = (const V *)sys->vecs[3];
    }
    KPM_TRY(run_evolve<V>(sys, vshift, in, acc, nullptr, dt, sign, np, a, b));
    KPM_TRY(stage_out<V>(sys, vshift, acc, phi));
    KPM_HIP(hipGetLastError());
    return KPM_OK;
}

template <typename V>
kpm_status evolve_x_impl(kpm_system *sys, int vshift, const void *phi, void *outx, void *outu,
                         double dt, int np) {
    const bool pl = sys->planar(vshift);
    KPM_TRY(sys->ensure_vecs(pl ? 7 : 5, vshift));
    V *pa = (V *)sys->vecs[0], *pb = (V *)sys->vecs[1], *qa = (V *)sys->vecs[2],
      *qb = (V *)sys->vecs[3], *u = (V *)sys->vecs[4];
    if (!pl) {
        KPM_TRY(run_evolve_x<V>(sys, vshift, (const V *)phi, (V *)outx, outu ? (V *)outu : u,
                                dt, np, pa, pb, qa, qb));
    } else {
        V *in = (V *)sys->vecs[5], *ox = (V *)sys->vecs[6];
        KPM_TRY(stage_in<V>(sys, vshift, phi, in));
        KPM_TRY(run_evolve_x<V>(sys, vshift, in, ox, u, dt, np, pa, pb, qa, qb));
        KPM_TRY(stage_out<V>(sys, vshift, ox, outx));
        if (outu) KPM_TRY(stage_out<V>(sys, vshift, u, outu));
    }
    KPM_HIP(hipGetLastError());
    return KPM_OK;
}

// VAC loop of Alg. 2 (Eq. 42-43) from the state psi = U^dag(t_k) phi,
// rr = U^dag(t_k) V phi: n steps of U(-dt) on both, then the moments
// <V psi| T_m |rr>.  start: psi holds phi, rr is set to V phi here, and the
// moments at t_k come first.  psi_io and rr_io are updated in place (the
// final state is copied back when it ends in a scratch buffer).  out: host
// [n_sys][n_vec][n_steps + start][nm] real parts.
template <typename V>
kpm_status vac_run(kpm_system *sys, int vshift, V *psi_io, V *rr_io, bool start, int nsteps,
                   double dt, int np, int nm, double *out) {
    KPM_TRY(sys->ensure_vecs(7, vshift));
    const int rows = nsteps + (start ? 1 : 0);
    const int64_t per_r = (int64_t)rows * nm;
    const size_t elems = (size_t)sys->nseg * ((size_t)1 << vshift) * per_r;
    KPM_TRY(sys->ensure_dmom(elems));
    V *a = (V *)sys->vecs[0], *b = (V *)sys->vecs[1];
    V *psi2 = (V *)sys->vecs[3], *rr2 = (V *)sys->vecs[5], *ll = (V *)sys->vecs[6];
    const kpm::Ell h = sys->ell_for(sys->launch[vshift]);
    kpm::Sweep sw;
    KPM_TRY(sys->sweep(vshift, &sw));
    const kpm::Coef alpha = sys->alpha();
    V *psi = psi_io, *rr = rr_io;
    int row = 0;
    if (start) {
        // R_0 = V phi; L_0 = V psi_0 = R_0
        kpm::launch_apply_d<V>(h, sw, psi, rr, alpha, sys->stream);
        KPM_TRY(run_moments<V>(sys, vshift, rr, rr, nm, a, b, per_r, 0, false, true));
        row = 1;
    }
    for (int k = 1; k <= nsteps; ++k, ++row) {
        KPM_TRY(run_evolve<V>(sys, vshift, psi, psi2, nullptr, dt, -1, np, a, b));
        std::swap(psi, psi2);
        KPM_TRY(run_evolve<V>(sys, vshift, rr, rr2, nullptr, dt, -1, np, a, b));
        std::swap(rr, rr2);
        kpm::launch_apply_d<V>(h, sw, psi, ll, alpha, sys->stream);
        KPM_TRY(run_moments<V>(sys, vshift, ll, rr, nm, a, b, per_r, (int64_t)row * nm, false,
                               true));
    }
    const size_t bytes = sys->state_bytes(vshift);
    if (psi != psi_io) KPM_HIP(hipMemcpyAsync(psi_io, psi, bytes, hipMemcpyDeviceToDevice, sys->stream));
    if (rr != rr_io) KPM_HIP(hipMemcpyAsync(rr_io, rr, bytes, hipMemcpyDeviceToDevice, sys->stream));
    std::vector<double2> host(elems);
    KPM_TRY(finish_moments(sys, host.size(), host.data()));
    for (size_t q = 0; q < host.size(); ++q) out[q] = host[q].x;
    return KPM_OK;
}

template <typename V>
kpm_status vac_impl(kpm_system *sys, int vshift, const void *phi, int nsteps, double dt, int np,
                    int nm, double *out) {
    KPM_TRY(sys->ensure_vecs(9, vshift));
    V *psi = (V *)sys->vecs[7], *rr = (V *)sys->vecs[8];
    KPM_TRY(stage_in<V>(sys, vshift, phi, psi));
    return vac_run<V>(sys, vshift, psi, rr, true, nsteps, dt, np, nm, out);
}

// MSD loop of Alg. 3 (Eq. 44) from the state psi' = U(t_k) phi, y = Y_k =
// [X, U(t_k)] phi: n steps of Y <- U(dt) Y + [X, U(dt)] psi', psi' <- U(dt)
// psi', then the moments of Y (in the doubling form when dbl).  start: psi'
// holds phi and Y_0 = 0 (y's contents are ignored); the zero moments at t_k
// come first.  In/out buffers and out as for vac_run.
template <typename V>
kpm_status msd_run(kpm_system *sys, int vshift, V *psi_io, V *y_io, bool start, int nsteps,
                   double dt, int np, int nm, bool dbl, double *out) {
    KPM_TRY(sys->ensure_vecs(7, vshift));
    const int rows = nsteps + (start ? 1 : 0);
    const int64_t per_r = (int64_t)rows * nm;
    const size_t elems = (size_t)sys->nseg * ((size_t)1 << vshift) * per_r;
    KPM_TRY(sys->ensure_dmom(elems));
    V *pa = (V *)sys->vecs[0], *pb = (V *)sys->vecs[1], *qa = (V *)sys->vecs[2],
      *qb = (V *)sys->vecs[3];
    V *y2 = (V *)sys->vecs[4], *xu = (V *)sys->vecs[5], *psi2 = (V *)sys->vecs[6];
    // Y_0 = [X, U(0)] phi = 0: its moments are exactly zero.
    if (start) KPM_HIP(hipMemsetAsync(sys->dmom, 0, elems * sizeof(double2), sys->stream));
    V *psi = psi_io, *y = y_io;
    bool y_zero = start;
    int row = start ? 1 : 0;
    for (int k = 1; k <= nsteps; ++k, ++row) {
        // [X, U(dt)] psi'_{k-1} and psi'_k = U(dt) psi'_{k-1}
        KPM_TRY(run_evolve_x<V>(sys, vshift, psi, xu, psi2, dt, np, pa, pb, qa, qb));
        std::swap(psi, psi2);
        if (y_zero) {
            std::swap(y, xu);                     // Y_1 = U(dt) 0 + [X, U(dt)] phi
            y_zero = false;
        } else {
            KPM_TRY(run_evolve<V>(sys, vshift, y, y2, xu, dt, +1, np, pa, pb));
            std::swap(y, y2);                     // Y_k = U(dt) Y_{k-1} + [X, U(dt)] psi'
        }
        KPM_TRY(run_moments<V>(sys, vshift, y, y, nm, pa, pb, per_r, (int64_t)row * nm, dbl,
                               true));
    }
    const size_t bytes = sys->state_bytes(vshift);
    if (psi != psi_io) KPM_HIP(hipMemcpyAsync(psi_io, psi, bytes, hipMemcpyDeviceToDevice, sys->stream));
    if (y != y_io) KPM_HIP(hipMemcpyAsync(y_io, y, bytes, hipMemcpyDeviceToDevice, sys->stream));
    std::vector<double2> host(elems);
    KPM_TRY(finish_moments(sys, host.size(), host.data()));
    for (size_t q = 0; q < host.size(); ++q) out[q] = host[q].x;
    return KPM_OK;
}

template <typename V>
kpm_status msd_impl(kpm_system *sys, int vshift, const void *phi, int nsteps, double dt, int np,
                    int nm, double *out, bool dbl) {
    KPM_TRY(sys->ensure_vecs(9, vshift));
    V *psi = (V *)sys->vecs[7], *y = (V *)sys->vecs[8];
    KPM_TRY(stage_in<V>(sys, vshift, phi, psi));
    return msd_run<V>(sys, vshift, psi, y, true, nsteps, dt, np, nm, dbl, out);
}

// VAC (Alg. 2) and MSD (Alg. 3) of the same phi in one pass over the time
// steps: both loops advance together and, at every t_k > 0, the VAC moment set
// <L_k|T_m|R_k> and the MSD set <Y_k|T_m|Y_k> run as the two vector planes of
// one launch sequence, with half the one-vector grid per plane (so each strip
// is about twice as long and half as many launches run).  The recursion states
// are those of vac_run and msd_run, the moments theirs up to the order of the
// inner-product sums.  One vector on a one-sample lattice whose moment sets take
// the marching strips; otherwise the two loops run one after the other.  With
// dos_out the DOS moments <phi|T_m|phi> (real: H~ is Hermitian) come along: in
// the joint form they are the second plane of the t_0 set, beside the VAC set
// of t_0 (whose MSD set is zero), so every moment set of the call runs on two
// planes; otherwise they are the real parts of kpm_moments.
template <typename V>
kpm_status vac_msd_impl(kpm_system *sys, int vshift, const void *phi, int nsteps, double dt,
                        int np, int nm, double *vac_out, double *msd_out,
                        double *dos_out = nullptr) {
    const kpm_launch &l0 = sys->launch[0];
    const bool joint = vshift == 0 && sys->nseg == 1 && sys->d_flags && l0.tiled >= 3 &&
                       sys->multi_steps(0, l0) > 1;
    if (!joint) {
        if (dos_out) {
            const size_t nmu = (size_t)sys->nseg * ((size_t)1 << vshift) * nm;
            std::vector<double> mu(2 * nmu);
            KPM_TRY(moments_impl<V>(sys, vshift, phi, phi, nm, mu.data(), false));
            for (size_t q = 0; q < nmu; ++q) dos_out[q] = mu[2 * q];
        }
        KPM_TRY(vac_impl<V>(sys, vshift, phi, nsteps, dt, np, nm, vac_out));
        return msd_impl<V>(sys, vshift, phi, nsteps, dt, np, nm, msd_out, false);
    }
    kpm::Sweep sw0;
    KPM_TRY(sys->sweep_with(0, l0, &sw0));
    // the one-vector shape on two planes: its wavefronts shared between the
    // planes, in groups of kBlock threads whatever the one-vector group size
    // (two-plane passes in groups of 64 threads measured 2.5 % slower on the
    // paper-scale sheet than in groups of 256)
    kpm_launch l2 = l0;
    l2.vectors_per_wave = 1;
    l2.group_size = 0;
    // both sets keep only real parts: with FP64 states the eight-step strips
    // take ten steps per pass (measured on the paper-scale sheet: 17.6 us per
    // step over both planes, against 17.8 with nine and 19.8 with eight)
    if (std::is_same<V, double2>::value && l0.steps == kpm::kMaxMarchSteps && l0.tiled >= 3)
        l2.steps = kpm::kReMarchSteps;
    const int waves = sw0.nwg * strip_waves(l0);
    l2.plane_groups = std::max(kpm::kXcds, waves / (kpm::kBlock / kpm::kWave) / 2 / kpm::kXcds *
                                               kpm::kXcds);
    KPM_TRY(sys->ensure_vecs(19, 1));                 // every scratch state holds two planes
    auto vec = [&](int i) { return (V *)sys->vecs[i]; };
    const size_t sb = sys->state_bytes(0);           // one plane
    V *ma = vec(0), *mb = vec(1), *pl = vec(2), *pr = vec(3);
    V *a = vec(4), *b = vec(5), *pa = vec(6), *pb = vec(7), *qa = vec(8), *qb = vec(9);
    V *psi = vec(10), *psi2 = vec(11), *rr = vec(12), *rr2 = vec(13);
    V *ps = vec(14), *ps2 = vec(15), *y = vec(16), *y2 = vec(17), *xu = vec(18);
    V *pl1 = (V *)((char *)pl + sb), *pr1 = (V *)((char *)pr + sb);
    const int64_t per = (int64_t)(nsteps + 1) * nm;
    const size_t elems = 2 * (size_t)per;            // [VAC, MSD][t_k][m]
    KPM_TRY(sys->ensure_dmom(elems));
    hipStream_t s = sys->stream;
    KPM_HIP(hipMemsetAsync(sys->dmom, 0, elems * sizeof(double2), s));    // MSD(0) = 0
    const kpm::Ell h = sys->ell_for(l0);
    const kpm::Coef alpha = sys->alpha();
    KPM_HIP(hipMemcpyAsync(psi, phi, sb, hipMemcpyDeviceToDevice, s));
    KPM_HIP(hipMemcpyAsync(ps, phi, sb, hipMemcpyDeviceToDevice, s));
    // t_0: R_0 = L_0 = V phi, the VAC set alone (Y_0 = 0), or beside the DOS set
    // of phi, whose moments fill the MSD set's slots of t_0 until read out
    kpm::launch_apply_d<V>(h, sw0, psi, rr, alpha, s);
    if (dos_out) {
        KPM_HIP(hipMemcpyAsync(pl, rr, sb, hipMemcpyDeviceToDevice, s));
        KPM_HIP(hipMemcpyAsync(pr, rr, sb, hipMemcpyDeviceToDevice, s));
        KPM_HIP(hipMemcpyAsync(pl1, phi, sb, hipMemcpyDeviceToDevice, s));
        KPM_HIP(hipMemcpyAsync(pr1, phi, sb, hipMemcpyDeviceToDevice, s));
        KPM_TRY(run_moments<V>(sys, 1, pl, pr, nm, ma, mb, per, 0, false, true, &l2));
    } else {
        KPM_TRY(run_moments<V>(sys, 0, rr, rr, nm, ma, mb, per, 0, false, true));
    }
    for (int k = 1; k <= nsteps; ++k) {
        // VAC: psi_k = U(-dt) psi_{k-1}, R_k = U(-dt) R_{k-1}, L_k = V psi_k
        KPM_TRY(run_evolve<V>(sys, 0, psi, psi2, nullptr, dt, -1, np, a, b));
        std::swap(psi, psi2);
        KPM_TRY(run_evolve<V>(sys, 0, rr, rr2, nullptr, dt, -1, np, a, b));
        std::swap(rr, rr2);
        kpm::launch_apply_d<V>(h, sw0, psi, pl, alpha, s);
        KPM_HIP(hipMemcpyAsync(pr, rr, sb, hipMemcpyDeviceToDevice, s));
        // MSD: [X, U(dt)] psi'_{k-1}, psi'_k = U(dt) psi'_{k-1}, Y_k = U(dt) Y_{k-1} + [X, U(dt)] psi'_{k-1}
        KPM_TRY(run_evolve_x<V>(sys, 0, ps, xu, ps2, dt, np, pa, pb, qa, qb));
        std::swap(ps, ps2);
        if (k == 1) {
            std::swap(y, xu);
        } else {
            KPM_TRY(run_evolve<V>(sys, 0, y, y2, xu, dt, +1, np, pa, pb));
            std::swap(y, y2);
        }
        KPM_HIP(hipMemcpyAsync(pl1, y, sb, hipMemcpyDeviceToDevice, s));
        KPM_HIP(hipMemcpyAsync(pr1, y, sb, hipMemcpyDeviceToDevice, s));
        KPM_TRY(run_moments<V>(sys, 1, pl, pr, nm, ma, mb, per, (int64_t)k * nm, false, true, &l2));
    }
    std::vector<double2> host(elems);
    KPM_TRY(finish_moments(sys, host.size(), host.data()));
    for (int64_t q = 0; q < per; ++q) {
        vac_out[q] = host[q].x;
        msd_out[q] = host[per + q].x;
    }
    if (dos_out)
        for (int m = 0; m < nm; ++m) {
            dos_out[m] = msd_out[m];
            msd_out[m] = 0.0;                          // [X, U(0)] = 0
        }
    return KPM_OK;
}

// The resumable loops on the caller's two state buffers: run in place, or
// for vector-major states on staged copies converted back at the end (Y_0
// and R_0 are not read when the loop starts).
template <typename V>
kpm_status continue_impl(kpm_system *sys, int vshift, void *a_io, void *b_io, bool start,
                         int nsteps, double dt, int np, int nm, int kind, double *out) {
    // kind: 0 VAC, 1 MSD, 2 MSD in the doubling form
    auto run = [&](V *a, V *b) {
        return kind == 0 ? vac_run<V>(sys, vshift, a, b, start, nsteps, dt, np, nm, out)
                         : msd_run<V>(sys, vshift, a, b, start, nsteps, dt, np, nm, kind == 2,
                                      out);
    };
    if (!sys->planar(vshift)) return run((V *)a_io, (V *)b_io);
    KPM_TRY(sys->ensure_vecs(11, vshift));
    V *a = (V *)sys->vecs[9], *b = (V *)sys->vecs[10];
    KPM_TRY(stage_in<V>(sys, vshift, a_io, a));
    if (!start) KPM_TRY(stage_in<V>(sys, vshift, b_io, b));
    KPM_TRY(run(a, b));
    KPM_TRY(stage_out<V>(sys, vshift, a, a_io));
    KPM_TRY(stage_out<V>(sys, vshift, b, b_io));
    KPM_HIP(hipStreamSynchronize(sys->stream));
    return KPM_OK;
}

// Y_n = [X, U(n dt)] phi by the recursion of Eq. 44, copied to out.
template <typename V>
kpm_status xu_state_impl(kpm_system *sys, int vshift, const void *phi_v, int nsteps, double dt,
                         int np, void *out) {
    KPM_TRY(sys->ensure_vecs(9, vshift));
    V *pa = (V *)sys->vecs[0], *pb = (V *)sys->vecs[1], *qa = (V *)sys->vecs[2],
      *qb = (V *)sys->vecs[3];
    V *y = (V *)sys->vecs[4], *y2 = (V *)sys->vecs[5], *xu = (V *)sys->vecs[6];
    V *psi = (V *)sys->vecs[7], *psi2 = (V *)sys->vecs[8];
    const V *cur = (const V *)phi_v;
    if (sys->planar(vshift)) {
        KPM_TRY(sys->ensure_vecs(10, vshift));
        KPM_TRY(stage_in<V>(sys, vshift, phi_v, (V *)sys->vecs[9]));
        cur = (const V *)sys->vecs[9];
    }
    for (int k = 1; k <= nsteps; ++k) {
        KPM_TRY(run_evolve_x<V>(sys, vshift, cur, xu, psi2, dt, np, pa, pb, qa, qb));
        std::swap(psi, psi2);
        cur = psi;
        if (k == 1) {
            std::swap(y, xu);
        } else {
            KPM_TRY(run_evolve<V>(sys, vshift, y, y2, xu, dt, +1, np, pa, pb));
            std::swap(y, y2);
        }
    }
    KPM_TRY(stage_out<V>(sys, vshift, y, out));
    KPM_HIP(hipGetLastError());
    return KPM_OK;
}

// Fourier moments of Alg. 4: F_n = <phi_L| U(n dtau) |phi_R>, n = -nm .. nm,
// reduced into sys->dmom[(s * R + r) * (2 nm + 1) + nm + n].
template <typename V>
kpm_status fourier_impl(kpm_system *sys, int vshift, const void *phil_v, const void *phir_v,
                        int nm, double dtau, int np, double *f) {
    KPM_TRY(sys->ensure_vecs(4, vshift));
    const int64_t per_r = 2 * (int64_t)nm + 1;
    const size_t elems = (size_t)sys->nseg * ((size_t)1 << vshift) * per_r;
    KPM_TRY(sys->ensure_dmom(elems));
    kpm::Sweep sw;
    KPM_TRY(sys->sweep(vshift, &sw));
    KPM_TRY(sys->ensure_partial(1, sw.nwg, 1 << vshift));
    V *a = (V *)sys->vecs[0], *b = (V *)sys->vecs[1], *psi = (V *)sys->vecs[2],
      *psi2 = (V *)sys->vecs[3];
    const V *phil = (const V *)phil_v, *phir = (const V *)phir_v;
    if (sys->planar(vshift)) {
        KPM_TRY(sys->ensure_vecs(6, vshift));
        a = (V *)sys->vecs[0];
        b = (V *)sys->vecs[1];
        psi = (V *)sys->vecs[2];
        psi2 = (V *)sys->vecs[3];
        KPM_TRY(stage_in<V>(sys, vshift, phil_v, (V *)sys->vecs[4]));
        KPM_TRY(stage_in<V>(sys, vshift, phir_v, (V *)sys->vecs[5]));
        phil = (const V *)sys->vecs[4];
        phir = (const V *)sys->vecs[5];
    }
    hipStream_t s = sys->stream;
    auto dot_into = [&](const V *x, int64_t idx) {
        kpm::launch_dot<V>(sw, phil, x, sys->partial, 0, s);
        kpm::launch_reduce(sys->partial, reduce_sweep(sw), 1, sys->dmom, per_r, idx, s);
    };
    dot_into(phir, nm);
    for (int dir = +1; dir >= -1; dir -= 2) {
        const V *cur = phir;
        for (int k = 1; k <= nm; ++k) {
            KPM_TRY(run_evolve<V>(sys, vshift, cur, psi2, nullptr, dtau, dir, np, a, b));
            std::swap(psi, psi2);
            cur = psi;
            dot_into(cur, nm + dir * k);
        }
    }
    return finish_moments(sys, elems, (double2 *)f);
}

// The launch shapes kpm_autotune times for 2^vs vectors on this system.
// Candidates: single steps (grid x ILP x streaming x neighbour form x
// traversal; all vectors of a row in adjacent lanes); then on chain lattices
// several recursion steps per pass: for one vector two steps in LDS tiles, 2,
// 3 or 4 steps in register tiles of 8 or 4 chains and 3 .. 8 steps in
// marching strips where the slots follow the graphene order, for several
// vectors one vector per wavefront in 4, 6 or 8-step strips (grid per plane
// from groups_per_cu or 16 .. 128 groups per plane); strips also in
// work-groups of 64, 128 and 512 threads.  Batches of chain lattices: strips
// per sample (one vector per wavefront for several vectors).
std::vector<kpm_launch> autotune_candidates(const kpm_system *sys, int vs) {
    static const int groups[] = {4, 8, 16};
    static const int ilps[] = {1, 2, 4};
    const int forms = sys->d_pid ? 2 : 1;
    bool can_tile = false;
    for (int32_t c : sys->chain) can_tile = can_tile || c >= 2 * tile_rows(vs);
    // row order and the base tile (wider tiles measured slower on every shape tried)
    const int tilings = can_tile ? 2 : 1;
    std::vector<kpm_launch> cand;
    for (int g : groups)
        for (int q = 0; q < 6 * forms * tilings; ++q) {
            kpm_launch l{};
            l.groups_per_cu = g;
            l.ilp = ilps[q % 3];
            l.streaming = (q / 3) % 2;
            l.compact = forms == 2 ? (q / 6) % 2 : 0;
            l.tiled = tilings == 2 ? q / (6 * forms) : 0;
            l.steps = 1;
            cand.push_back(l);
        }
    // several vectors on a one-sample chain lattice: one vector per wavefront
    // (vector-major states) in marching strips, the grid per plane from
    // groups_per_cu or a few groups per plane (longer strips)
    if (sys->d_flags && vs > 0 && sys->nseg == 1) {
        for (int ksteps : {4, 6, 8})
            for (int pg : {0, 16, 32, 64, 128})
                cand.push_back(kpm_launch{2, 1, 0, 1, 5, ksteps, 1, pg, 0});
        // work-groups of 64, 128 and 512 threads (the wavefronts per plane of 16
        // groups of 256)
        for (int gs : {64, 128, 512})
            cand.push_back(kpm_launch{2 * 256 / gs, 1, 0, 1, 5, 8, 1, 16 * 256 / gs, gs});
    }
    // a batch of chain lattices: 4, 6 or 8-step strips in groups of one, two or
    // four wavefronts, one vector per wavefront for several vectors (about
    // 2048 wavefronts over all planes, or two or four times that, shared out
    // among the samples in proportion to their rows; at least 8 groups per
    // sample)
    if (sys->bstrips) {
        const int64_t minpg = 8 * (int64_t)sys->nseg;
        for (int ksteps : {4, 6, 8})
            for (int gs : {64, 128, 256}) {
                const int wpg = gs / kpm::kWave;
                if (vs == 0) {
                    cand.push_back(kpm_launch{8 / wpg, 1, 0, 1, 5, ksteps, 0, 0, gs});
                    continue;
                }
                for (int mult : {1, 2, 4}) {
                    const int64_t per = ((int64_t)sys->cus * 8 * mult / wpg) >> vs;
                    const int64_t pg = std::max(minpg, std::min<int64_t>(65536, per / 8 * 8));
                    cand.push_back(kpm_launch{2, 1, 0, 1, 5, ksteps, 1, (int)pg, gs});
                }
            }
    }
    if (sys->d_code && vs == 0) {
        for (int g : {2, 3, 4, 6})
            for (int nt : {0, 1}) cand.push_back(kpm_launch{g, 1, nt, 1, 0, 2});
        if (sys->d_flags) {
            for (int ksteps : {2, 3, 4})
                for (int tiled : {1, 2})
                    for (int g : {1, 2, 3, 4, 6, 8})
                        cand.push_back(kpm_launch{g, 1, 0, 1, tiled, ksteps});
            // eight-step strips in work-groups of 64, 128 and 512 threads (two
            // wavefronts per SIMD)
            for (int gs : {64, 128, 512})
                cand.push_back(kpm_launch{2 * 256 / gs, 1, 0, 1, 5, 8, 0, 0, gs});
            for (int ksteps : {3, 4, 5, 6, 7, 8}) {
                for (int g : {2, 3, 4}) cand.push_back(kpm_launch{g, 1, 0, 1, 5, ksteps});
                if (ksteps <= 6)
                    for (int tiled : {3, 4}) cand.push_back(kpm_launch{2, 1, 0, 1, tiled, ksteps});
            }
        }
    }
    // each shape once (the grid formulas above can meet)
    std::vector<kpm_launch> uniq;
    for (const kpm_launch &l : cand) {
        bool seen = false;
        for (const kpm_launch &u : uniq)
            seen = seen || std::memcmp(&u, &l, sizeof(kpm_launch)) == 0;
        if (!seen) uniq.push_back(l);
    }
    return uniq;
}

template <typename V>
kpm_status autotune_impl(kpm_system *sys, int vs, const V *phi, int reps, kpm_launch *best) {
    KPM_TRY(sys->ensure_vecs(2, vs));
    V *a = (V *)sys->vecs[0], *b = (V *)sys->vecs[1];
    hipStream_t s = sys->stream;
    const size_t bytes = sys->state_bytes(vs);
    hipEvent_t e0, e1;
    KPM_HIP(hipEventCreate(&e0));
    KPM_HIP(hipEventCreate(&e1));
    kpm_status st = KPM_OK;
    // Each candidate runs the real two-buffer recursion (the output of one
    // step is the gathered input of the next) on copies of phi, three times;
    // the fastest round counts.
    auto time_shape = [&](const kpm_launch &l, bool dbl, float *out_ms) -> kpm_status {
        const kpm::Ell h = sys->ell_for(l);
        kpm::Sweep sw;
        KPM_TRY(l.vectors_per_wave == 1 && vs > 0 && (sys->nseg == 1 || sys->bstrips)
                    ? sys->sweep_planes(vs, l, &sw)
                    : sys->sweep_with(vs, l, &sw));
        const int ks = sys->multi_steps(sw.vshift, l);
        if (ks > 1) KPM_TRY(sys->ensure_xbuf(vs));
        KPM_TRY(sys->ensure_partial(2 * ks, sw.nwg, 1 << vs));
        const kpm::Lat2 lat = sys->lat2(l, ks, sw.nwg);
        // whole passes only (a long moment set has no tail to speak of), at
        // least one
        const int steps = ks > 1 ? std::max(1, reps / ks) * ks : reps;
        float best = 1e30f;
        for (int round = 0; round < 3; ++round) {
            KPM_HIP(hipMemcpyAsync(a, phi, bytes, hipMemcpyDeviceToDevice, s));
            KPM_HIP(hipMemcpyAsync(b, phi, bytes, hipMemcpyDeviceToDevice, s));
            V *p0 = b, *p1 = a, *o1 = (V *)sys->xbuf[0], *o2 = (V *)sys->xbuf[1];
            KPM_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < steps; ++k) {
                if (ks > 1 && k + ks <= steps) {
                    if (!kpm::launch_moment_multi<V>(h, sw, lat, p1, p0, o1, o2, phi,
                                                     sys->partial, 0, dbl, false, s))
                        return fail(KPM_ERR_UNSUPPORTED, "no multi-step kernel for %d steps", ks);
                    std::swap(p0, o1);
                    std::swap(p1, o2);
                    k += ks - 1;
                    continue;
                }
                if (dbl)
                    kpm::launch_moment_step_doubled<V>(h, sw, p1, p0, p0, sys->partial, 0, s);
                else
                    kpm::launch_moment_step<V>(h, sw, false, p1, p0, p0, phi, sys->partial, 0, s);
                std::swap(p0, p1);
            }
            KPM_HIP(hipEventRecord(e1, s));
            KPM_HIP(hipEventSynchronize(e1));
            float ms = 0;
            KPM_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        *out_ms = best * (float)reps / (float)steps;     // per reps recursion steps
        return KPM_OK;
    };
    const std::vector<kpm_launch> cand = autotune_candidates(sys, vs);
    // Each form (direct, doubling) keeps its current shape as the incumbent; a
    // candidate replaces it only when more than 2 % faster, so near-ties keep
    // a stable choice.
    // The direct form's pick fixes the layout of the states (vectors per
    // wavefront), so the doubling form then only considers shapes of that layout.
    kpm_launch pick = sys->launch[vs], pick_dbl = sys->launch_dbl[vs];
    for (int form = 0; form < 2 && st == KPM_OK; ++form) {
        const bool dbl = form == 1;
        kpm_launch &p = dbl ? pick_dbl : pick;
        if (dbl && p.vectors_per_wave != pick.vectors_per_wave) p = pick;
        float best_ms = 1e30f;
        st = time_shape(p, dbl, &best_ms);
        for (const kpm_launch &l : cand) {
            if (st != KPM_OK) break;
            if (dbl && l.vectors_per_wave != pick.vectors_per_wave) continue;
            float ms = 0;
            if ((st = time_shape(l, dbl, &ms)) != KPM_OK) break;
            if (ms < 0.98f * best_ms) {
                best_ms = ms;
                p = l;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != KPM_OK) return st;
    KPM_HIP(hipGetLastError());
    sys->launch[vs] = pick;
    sys->launch_dbl[vs] = pick_dbl;
    if (best) *best = pick;
    return KPM_OK;
}

// Builds the device system from validated samples laid side by side.
kpm_status build_system(std::vector<Packed> &parts, kpm_precision prec, int device,
                        void *hip_stream, kpm_system **out) {
    const int nseg = (int)parts.size();
    int64_t n = 0;
    int w = 0;
    bool any_hop = false, all_dx = true;
    for (const Packed &p : parts) {
        n += p.n;
        w = std::max(w, p.w);
        any_hop = any_hop || !p.hop.empty();
        all_dx = all_dx && !p.dx.empty();
    }
    if (n >= ((int64_t)1 << 31)) return fail(KPM_ERR_INVALID, "total rows %lld exceed 2^31", (long long)n);

    kpm_system *sys = new (std::nothrow) kpm_system();
    if (!sys) return fail(KPM_ERR_OOM, "host allocation");
    auto bail = [&](kpm_status st) {
        delete sys;
        return st;
    };
    sys->device = device;
    sys->stream = (hipStream_t)hip_stream;
    sys->prec = prec;
    sys->n = n;
    sys->w = w;
    sys->nseg = nseg;
    sys->has_dx = all_dx;
    sys->off.assign(nseg + 1, 0);
    sys->es.resize(nseg);
    for (int s = 0; s < nseg; ++s) {
        sys->off[s + 1] = sys->off[s] + parts[s].n;
        sys->es[s] = parts[s].e_scale;
    }
    for (int v = 0; v < 7; ++v) {
        const kpm_status st = env_launch(v, prec, &sys->launch[v]);
        if (st != KPM_OK) return bail(st);
        sys->launch_dbl[v] = sys->launch[v];
    }
    if (const char *env = std::getenv("KPM_SCRATCH_LIMIT_MB"))
        sys->scratch_limit = (size_t)(std::max(0.0, atof(env)) * 1048576.0);
    sys->chain.resize(nseg);
    for (int s = 0; s < nseg; ++s) sys->chain[s] = chain_length(parts[s].nbr, parts[s].w, parts[s].n);

    // Concatenate and shift indices by the sample offset; per-slot weights
    // carry 1/E_s of their sample.
    std::vector<int32_t> nbr((size_t)w * n, -1);
    std::vector<double> ons(n), hop(any_hop ? (size_t)w * n : 0), xw(all_dx ? (size_t)w * n : 0);
    sys->seg_t.resize(nseg);
    bool ons_float = std::getenv("KPM_COMPACT") == nullptr || atoi(std::getenv("KPM_COMPACT")) != 0;
    const bool try_compact = ons_float && w <= kpm::kMaxWidth;
    for (int s = 0; s < nseg; ++s) {
        const Packed &p = parts[s];
        const int64_t o = sys->off[s];
        const double inv = 1.0 / p.e_scale;
        sys->seg_t[s] = p.t * inv;
        for (int64_t r = 0; r < p.n; ++r) {
            ons[o + r] = p.ons[r];
            ons_float = ons_float && (double)(float)p.ons[r] == p.ons[r];
            for (int k = 0; k < p.w; ++k) {
                const size_t q = (size_t)k * p.n + r, qq = (size_t)k * n + o + r;
                const int32_t m = p.nbr[q];
                nbr[qq] = m >= 0 ? (int32_t)(m + o) : -1;
                const double hv = p.hop.empty() ? p.t : p.hop[q];
                if (any_hop) hop[qq] = m >= 0 ? hv * inv : 0.0;
                if (all_dx) xw[qq] = m >= 0 ? p.dx[q] * hv * inv : 0.0;
            }
        }
    }
    sys->uniform_hop = !any_hop;
    // Compact neighbour form: one byte per row selects one of at most
    // kMaxPatterns offset patterns (a lattice has only a few).
    std::vector<uint8_t> pid;
    std::vector<int32_t> pat;
    if (try_compact) {
        std::vector<std::array<int32_t, kpm::kMaxWidth>> pats;
        pid.resize(n);
        std::array<int32_t, kpm::kMaxWidth> cur{};
        int last = -1;
        for (int64_t r = 0; r < n && !pid.empty(); ++r) {
            for (int k = 0; k < kpm::kMaxWidth; ++k) {
                const int32_t m = k < w ? nbr[(size_t)k * n + r] : -1;
                cur[k] = m < 0 ? kpm::kEmptySlot : (int32_t)(m - r);
            }
            int id = (last >= 0 && pats[last] == cur) ? last : -1;
            for (int q = 0; id < 0 && q < (int)pats.size(); ++q)
                if (pats[q] == cur) id = q;
            if (id < 0) {
                if ((int)pats.size() == kpm::kMaxPatterns) {
                    pid.clear();
                    break;
                }
                pats.push_back(cur);
                id = (int)pats.size() - 1;
            }
            pid[r] = (uint8_t)id;
            last = id;
        }
        if (!pid.empty()) {
            for (const auto &a : pats) pat.insert(pat.end(), a.begin(), a.end());
            sys->npat = (int)pats.size();
        }
    }
    // Chain-lattice codes of the two-step sweep (one sample, compact width-3
    // form with uniform hopping).
    std::vector<uint32_t> code;
    std::vector<uint8_t> seen;
    const bool lat2 = nseg == 1 && !pid.empty() && w == 3 && !any_hop && sys->chain[0] > 0 &&
                      lattice_codes(nbr, w, n, 0, n, sys->chain[0], pid, sys->npat, code, seen);
    // a batch whose every sample is such a lattice of at least kMinChains
    // chains (and no wider than the strips' 32-bit row offsets allow): its
    // moment sets can take the marching strips, one vector per row, with
    // per-row ids of the distinct step codes of all samples (whatever the
    // compact form, whose patterns hold sample-specific row offsets)
    bool bstrips = nseg > 1 && w == 3 && !any_hop;
    std::vector<uint32_t> rcode, bcode, bflags;
    std::vector<uint8_t> sid;
    for (int s = 0; s < nseg && bstrips; ++s) {
        const int64_t nx = sys->chain[s], rows = sys->off[s + 1] - sys->off[s];
        bstrips = nx > 0 && rows / nx >= kpm::kMinChains &&
                  nx * (int64_t)sizeof(double2) < ((int64_t)1 << 31) &&
                  row_codes(nbr, w, n, sys->off[s], sys->off[s + 1], nx, rcode);
    }
    if (bstrips) {
        sid.resize(n);
        for (int64_t r = 0; r < n && bstrips; ++r) {
            size_t id = 0;
            while (id < bcode.size() && bcode[id] != rcode[r]) ++id;
            if (id == bcode.size()) {
                if (bcode.size() >= (size_t)kpm::kMaxPatterns) bstrips = false;
                bcode.push_back(rcode[r]);
            }
            sid[r] = (uint8_t)id;
        }
        rcode.clear();
        bstrips = bstrips && graphene_flags(bcode, bflags);
    }
    if (!ons_float) {
        for (int s = 0; s < nseg; ++s)
            for (int64_t r = sys->off[s]; r < sys->off[s + 1]; ++r) ons[r] /= parts[s].e_scale;
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return bail(fail(KPM_ERR_DEVICE, "no HIP device %d", device));
    DeviceGuard guard(device);
    if (hipDeviceGetAttribute(&sys->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        sys->cus = 256;
    auto upload = [&](void **dst, const void *src, size_t bytes) -> kpm_status {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return fail(KPM_ERR_OOM, "hipMalloc %zu bytes: %s", bytes, hipGetErrorString(e));
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(KPM_ERR_DEVICE, "upload: %s", hipGetErrorString(e));
        return KPM_OK;
    };
    kpm_status st = upload((void **)&sys->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t));
    if (st == KPM_OK && !pid.empty()) {
        st = upload((void **)&sys->d_pid, pid.data(), pid.size());
        if (st == KPM_OK) st = upload((void **)&sys->d_pat, pat.data(), pat.size() * sizeof(int32_t));
    }
    if (st == KPM_OK && lat2) {
        st = upload((void **)&sys->d_code, code.data(), code.size() * sizeof(uint32_t));
        sys->l2nx = sys->chain[0];
        sys->l2ny = (int32_t)(n / sys->chain[0]);
        std::vector<uint32_t> flags;
        if (st == KPM_OK && sys->l2ny >= 16 && graphene_flags(code, flags)) {
            st = upload((void **)&sys->d_flags, flags.data(), flags.size() * sizeof(uint32_t));
            // per-pattern commutator weights of the coupled strips, where every
            // row of a pattern carries the same ones (as on a builder lattice)
            if (st == KPM_OK && all_dx) {
                std::vector<double> pxw((size_t)sys->npat * 4, 0.0);
                std::vector<uint8_t> seen(sys->npat, 0);
                bool same = true;
                for (int64_t r = 0; r < n && same; ++r) {
                    const int q = pid[r];
                    for (int k = 0; k < 3; ++k) {
                        const double v = xw[(size_t)k * n + r];
                        if (!seen[q]) pxw[(size_t)q * 4 + k] = v;
                        else same = same && pxw[(size_t)q * 4 + k] == v;
                    }
                    seen[q] = 1;
                }
                if (same)
                    st = upload((void **)&sys->d_pxw, pxw.data(), pxw.size() * sizeof(double));
            }
        }
    }
    if (st == KPM_OK && bstrips) {
        st = upload((void **)&sys->d_flags, bflags.data(), bflags.size() * sizeof(uint32_t));
        if (st == KPM_OK) st = upload((void **)&sys->d_sid, sid.data(), sid.size());
        sys->nsp = (int)bcode.size();
        sys->bstrips = st == KPM_OK;
    }
    if (st == KPM_OK && ons_float) {
        std::vector<float> of(ons.begin(), ons.end());
        st = upload((void **)&sys->d_onsf, of.data(), of.size() * sizeof(float));
    } else if (st == KPM_OK) {
        st = upload((void **)&sys->d_ons, ons.data(), ons.size() * sizeof(double));
    }
    if (st == KPM_OK && any_hop) st = upload((void **)&sys->d_hop, hop.data(), hop.size() * sizeof(double));
    if (st == KPM_OK && all_dx) st = upload((void **)&sys->d_xw, xw.data(), xw.size() * sizeof(double));
    if (st == KPM_OK && nseg > 1) {
        std::vector<double2> al(nseg);
        for (int s = 0; s < nseg; ++s) al[s] = make_double2(0.0, -sys->es[s] / kHbar);
        st = upload((void **)&sys->d_alpha, al.data(), al.size() * sizeof(double2));
    }
    // several vectors on a one-sample graphene lattice that takes the strips:
    // one vector per wavefront in eight-step strips by default (measured fastest on the
    // paper-scale sheet with 64 vectors, in FP64 and with FP32 states), with
    // about 1024 work-groups over all planes; not when a KPM_* launch
    // override is set
    if (st == KPM_OK && nseg == 1 && sys->d_flags && sys->multi_steps(0, sys->launch[0]) > 1 &&
        !launch_env_set()) {
        for (int v = 1; v < 7; ++v) {
            const kpm_launch l{2, 1, 0, 1, 5, 8, 1, std::max(16, 1024 >> v)};
            sys->launch[v] = sys->launch_dbl[v] = l;
        }
    }
    // a batch whose moment sets can take the strips: eight-step strips, one
    // vector per wavefront for several vectors with about 1024 groups over all
    // planes and at least 8 per sample (the autotuner's pick for the 32-sample
    // batch of 8 vectors)
    if (st == KPM_OK && sys->bstrips && !launch_env_set()) {
        sys->launch[0] = sys->launch_dbl[0] = kpm_launch{2, 1, 0, 1, 5, 8, 0, 0, 0};
        for (int v = 1; v < 7; ++v) {
            const int pg = std::max(8 * nseg, 1024 >> v);
            if (pg > 65536) break;
            const kpm_launch l{2, 1, 0, 1, 5, 8, 1, pg, 0};
            sys->launch[v] = sys->launch_dbl[v] = l;
        }
    }
    if (st == KPM_OK) {
        const hipError_t e = kpm::static_scratch(device, &sys->static_scratch);
        if (e != hipSuccess)
            st = fail(KPM_ERR_DEVICE, "fixed scratch address: %s", hipGetErrorString(e));
    }
    // segment tables of the starting launch shapes (the allocation-free entry
    // point only looks them up)
    for (int v = 0; v < 7 && st == KPM_OK && nseg > 1; ++v) {
        kpm::Sweep sw;
        st = sys->sweep_with(v, sys->launch[v], &sw);
    }
    if (st != KPM_OK) return bail(st);
    *out = sys;
    return KPM_OK;
}

kpm_status check_loop(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                      int n_bessel, int n_moments, double *out, int *vs) {
    KPM_TRY(check_common(sys, n_vec, vs));
    if (!phi || !out) return fail(KPM_ERR_INVALID, "null buffer");
    if (!sys->has_dx) return fail(KPM_ERR_INVALID, "system has no dx (velocity operator)");
    if (n_steps < 0) return fail(KPM_ERR_INVALID, "n_steps must be >= 0");
    if (n_bessel < 2) return fail(KPM_ERR_INVALID, "n_bessel must be >= 2");
    if (n_moments < 1) return fail(KPM_ERR_INVALID, "n_moments must be >= 1");
    if (!std::isfinite(dt_fs) || dt_fs < 0) return fail(KPM_ERR_INVALID, "dt_fs");
    return KPM_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

kpm_status kpm_system_create(const kpm_system_desc *d, kpm_precision prec, int device,
                             void *hip_stream, kpm_system **out) {
    return kpm_batch_create(1, d, prec, device, hip_stream, out);
}

kpm_status kpm_batch_create(int n_sys, const kpm_system_desc *descs, kpm_precision prec,
                            int device, void *hip_stream, kpm_system **out) {
    if (!descs || !out) return fail(KPM_ERR_INVALID, "null descriptor or output");
    *out = nullptr;
    if (n_sys < 1 || n_sys > 4096) return fail(KPM_ERR_INVALID, "n_sys must be 1..4096");
    if (prec != KPM_FP64 && prec != KPM_FP32_STATES && prec != KPM_FP32)
        return fail(KPM_ERR_INVALID, "precision");
    std::vector<Packed> parts(n_sys);
    for (int s = 0; s < n_sys; ++s) KPM_TRY(pack_desc(&descs[s], s, parts[s]));
    return build_system(parts, prec, device, hip_stream, out);
}

kpm_status kpm_system_destroy(kpm_system *sys) {
    if (!sys) return KPM_OK;
    {
        DeviceGuard g(sys->device);
        (void)hipStreamSynchronize(sys->stream);
    }
    delete sys;
    return KPM_OK;
}

kpm_status kpm_system_set_stream(kpm_system *sys, void *hip_stream) {
    if (!sys) return fail(KPM_ERR_INVALID, "null system");
    sys->stream = (hipStream_t)hip_stream;
    return KPM_OK;
}

int64_t kpm_system_n_sites(const kpm_system *sys) { return sys ? sys->n : -1; }

int32_t kpm_system_n_samples(const kpm_system *sys) { return sys ? sys->nseg : -1; }

kpm_status kpm_system_offsets(const kpm_system *sys, int64_t *offsets) {
    if (!sys || !offsets) return fail(KPM_ERR_INVALID, "null argument");
    for (int s = 0; s <= sys->nseg; ++s) offsets[s] = sys->off[s];
    return KPM_OK;
}

kpm_status kpm_moments(kpm_system *sys, int n_vec, const void *phil, const void *phir,
                       int n_moments, double *mu) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phil || !phir || !mu) return fail(KPM_ERR_INVALID, "null buffer");
    if (n_moments < 1) return fail(KPM_ERR_INVALID, "n_moments must be >= 1");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64 ? moments_impl<double2>(sys, vs, phil, phir, n_moments, mu, false)
                                 : moments_impl<float2>(sys, vs, phil, phir, n_moments, mu, false);
}

kpm_status kpm_moments_noalloc(kpm_system *sys, int n_vec, const void *phil, const void *phir,
                               int n_moments, double *mu) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phil || !phir || !mu) return fail(KPM_ERR_INVALID, "null buffer");
    if (n_moments < 1) return fail(KPM_ERR_INVALID, "n_moments must be >= 1");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? moments_noalloc_impl<double2>(sys, vs, phil, phir, n_moments, mu)
               : moments_noalloc_impl<float2>(sys, vs, phil, phir, n_moments, mu);
}

kpm_status kpm_moments_doubled(kpm_system *sys, int n_vec, const void *phi, int n_moments,
                               double *mu) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi || !mu) return fail(KPM_ERR_INVALID, "null buffer");
    if (n_moments < 1) return fail(KPM_ERR_INVALID, "n_moments must be >= 1");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64 ? moments_impl<double2>(sys, vs, phi, phi, n_moments, mu, true)
                                 : moments_impl<float2>(sys, vs, phi, phi, n_moments, mu, true);
}

kpm_status kpm_evolve(kpm_system *sys, int n_vec, void *phi, double dt_fs, int sign,
                      int n_bessel) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi) return fail(KPM_ERR_INVALID, "null buffer");
    if (sign != 1 && sign != -1) return fail(KPM_ERR_INVALID, "sign must be +1 or -1");
    if (n_bessel < 2) return fail(KPM_ERR_INVALID, "n_bessel must be >= 2");
    if (!std::isfinite(dt_fs) || dt_fs < 0) return fail(KPM_ERR_INVALID, "dt_fs");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64 ? evolve_impl<double2>(sys, vs, phi, dt_fs, sign, n_bessel)
                                 : evolve_impl<float2>(sys, vs, phi, dt_fs, sign, n_bessel);
}

kpm_status kpm_evolve_x(kpm_system *sys, int n_vec, const void *phi, void *out_x, void *out_u,
                        double dt_fs, int n_bessel) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi || !out_x) return fail(KPM_ERR_INVALID, "null buffer");
    if (out_x == phi || out_u == phi || (out_u && out_u == out_x))
        return fail(KPM_ERR_INVALID, "outputs must not alias the input or each other");
    if (!sys->has_dx) return fail(KPM_ERR_INVALID, "system has no dx (position operator)");
    if (n_bessel < 2) return fail(KPM_ERR_INVALID, "n_bessel must be >= 2");
    if (!std::isfinite(dt_fs) || dt_fs < 0) return fail(KPM_ERR_INVALID, "dt_fs");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? evolve_x_impl<double2>(sys, vs, phi, out_x, out_u, dt_fs, n_bessel)
               : evolve_x_impl<float2>(sys, vs, phi, out_x, out_u, dt_fs, n_bessel);
}

kpm_status kpm_vac(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                   int n_bessel, int n_moments, double *out) {
    int vs;
    KPM_TRY(check_loop(sys, n_vec, phi, n_steps, dt_fs, n_bessel, n_moments, out, &vs));
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? vac_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out)
               : vac_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out);
}

kpm_status kpm_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                   int n_bessel, int n_moments, double *out) {
    int vs;
    KPM_TRY(check_loop(sys, n_vec, phi, n_steps, dt_fs, n_bessel, n_moments, out, &vs));
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? msd_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out, false)
               : msd_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out, false);
}

kpm_status kpm_vac_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                       int n_bessel, int n_moments, double *vac_out, double *msd_out) {
    int vs;
    KPM_TRY(check_loop(sys, n_vec, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out, &vs));
    if (!msd_out) return fail(KPM_ERR_INVALID, "null buffer");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? vac_msd_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out,
                                       msd_out)
               : vac_msd_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out,
                                      msd_out);
}

kpm_status kpm_dos_vac_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                           double dt_fs, int n_bessel, int n_moments, double *dos_out,
                           double *vac_out, double *msd_out) {
    int vs;
    KPM_TRY(check_loop(sys, n_vec, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out, &vs));
    if (!msd_out || !dos_out) return fail(KPM_ERR_INVALID, "null buffer");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? vac_msd_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out,
                                       msd_out, dos_out)
               : vac_msd_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, vac_out,
                                      msd_out, dos_out);
}

kpm_status kpm_msd_doubled(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                           double dt_fs, int n_bessel, int n_moments, double *out) {
    int vs;
    KPM_TRY(check_loop(sys, n_vec, phi, n_steps, dt_fs, n_bessel, n_moments, out, &vs));
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? msd_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out, true)
               : msd_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, n_moments, out, true);
}

static kpm_status check_continue(kpm_system *sys, int n_vec, void *a, void *b, int start,
                                 int n_steps, double dt_fs, int n_bessel, int n_moments,
                                 double *out, int *vs) {
    KPM_TRY(check_loop(sys, n_vec, a, n_steps, dt_fs, n_bessel, n_moments, out, vs));
    if (!b || a == b) return fail(KPM_ERR_INVALID, "null or aliased state buffers");
    if (start != 0 && start != 1) return fail(KPM_ERR_INVALID, "start must be 0 or 1");
    if (!start && n_steps < 1) return fail(KPM_ERR_INVALID, "n_steps must be >= 1 when continuing");
    return KPM_OK;
}

kpm_status kpm_vac_continue(kpm_system *sys, int n_vec, void *psi, void *r, int start,
                            int n_steps, double dt_fs, int n_bessel, int n_moments, double *out) {
    int vs;
    KPM_TRY(check_continue(sys, n_vec, psi, r, start, n_steps, dt_fs, n_bessel, n_moments, out, &vs));
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? continue_impl<double2>(sys, vs, psi, r, start != 0, n_steps, dt_fs, n_bessel,
                                        n_moments, 0, out)
               : continue_impl<float2>(sys, vs, psi, r, start != 0, n_steps, dt_fs, n_bessel,
                                       n_moments, 0, out);
}

kpm_status kpm_msd_continue(kpm_system *sys, int n_vec, void *psi, void *y, int start,
                            int n_steps, double dt_fs, int n_bessel, int n_moments, int doubled,
                            double *out) {
    int vs;
    KPM_TRY(check_continue(sys, n_vec, psi, y, start, n_steps, dt_fs, n_bessel, n_moments, out, &vs));
    if (doubled != 0 && doubled != 1) return fail(KPM_ERR_INVALID, "doubled must be 0 or 1");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? continue_impl<double2>(sys, vs, psi, y, start != 0, n_steps, dt_fs, n_bessel,
                                        n_moments, doubled ? 2 : 1, out)
               : continue_impl<float2>(sys, vs, psi, y, start != 0, n_steps, dt_fs, n_bessel,
                                       n_moments, doubled ? 2 : 1, out);
}

kpm_status kpm_xu_state(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                        int n_bessel, void *out) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi || !out || phi == out) return fail(KPM_ERR_INVALID, "null or aliased buffer");
    if (!sys->has_dx) return fail(KPM_ERR_INVALID, "system has no dx (velocity operator)");
    if (n_steps < 1) return fail(KPM_ERR_INVALID, "n_steps must be >= 1");
    if (n_bessel < 2) return fail(KPM_ERR_INVALID, "n_bessel must be >= 2");
    if (!std::isfinite(dt_fs) || dt_fs < 0) return fail(KPM_ERR_INVALID, "dt_fs");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? xu_state_impl<double2>(sys, vs, phi, n_steps, dt_fs, n_bessel, out)
               : xu_state_impl<float2>(sys, vs, phi, n_steps, dt_fs, n_bessel, out);
}

kpm_status kpm_fourier_moments(kpm_system *sys, int n_vec, const void *phi_l, const void *phi_r,
                               int n_moments, double dtau_fs, int n_bessel, double *f) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi_l || !phi_r || !f) return fail(KPM_ERR_INVALID, "null buffer");
    if (n_moments < 0) return fail(KPM_ERR_INVALID, "n_moments must be >= 0");
    if (n_bessel < 2) return fail(KPM_ERR_INVALID, "n_bessel must be >= 2");
    if (!std::isfinite(dtau_fs) || dtau_fs < 0) return fail(KPM_ERR_INVALID, "dtau_fs");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64
               ? fourier_impl<double2>(sys, vs, phi_l, phi_r, n_moments, dtau_fs, n_bessel, f)
               : fourier_impl<float2>(sys, vs, phi_l, phi_r, n_moments, dtau_fs, n_bessel, f);
}

kpm_status kpm_ftm_sum(int n_rows, int n_moments, const double *f, int n_energies,
                       const double *energies, double dtau_fs, double area_nm2, int hanning,
                       void *hip_stream, double *out) {
    if (n_rows < 1 || n_moments < 0 || n_energies < 1) return fail(KPM_ERR_INVALID, "sizes");
    if (!f || !energies || !out) return fail(KPM_ERR_INVALID, "null buffer");
    if (!(dtau_fs > 0) || !(area_nm2 > 0)) return fail(KPM_ERR_INVALID, "dtau / area");
    const int nf = 2 * n_moments + 1;
    std::vector<double> w(nf), theta(n_energies);
    for (int j = 0; j < nf; ++j)     // Hanning window, Eq. 28
        w[j] = hanning ? 0.5 * (1.0 + std::cos(kPi * (j - n_moments) / (n_moments + 1.0))) : 1.0;
    for (int k = 0; k < n_energies; ++k) {
        if (!std::isfinite(energies[k])) return fail(KPM_ERR_INVALID, "energy %d", k);
        theta[k] = energies[k] * dtau_fs / kHbar;
    }
    const double pref = dtau_fs / (kPi * kHbar * area_nm2);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nin = (size_t)n_rows * nf, nout = (size_t)n_rows * n_energies;
    double *buf = nullptr;
    const size_t total = 2 * nin + nf + (size_t)n_energies + nout;
    KPM_HIP(hipMalloc(&buf, total * sizeof(double)));
    double *dfv = buf, *dw = dfv + 2 * nin, *dth = dw + nf, *dout = dth + n_energies;
    kpm_status st = KPM_OK;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && st == KPM_OK) st = fail(KPM_ERR_DEVICE, "ftm_sum: %s", hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(dfv, f, 2 * nin * sizeof(double), hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dth, theta.data(), theta.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (st == KPM_OK) {
        kpm::launch_ftm_sum((const double2 *)dfv, n_rows, n_moments, dw, dth, n_energies, pref,
                            dout, s);
        chk(hipGetLastError());
    }
    chk(hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, s));
    chk(hipStreamSynchronize(s));
    (void)hipFree(buf);
    return st;
}

kpm_status kpm_kpm_sum(int n_rows, int n_moments, const double *moments, int n_energies,
                       const double *energies, double e_scale, double area_nm2, int jackson,
                       void *hip_stream, double *out) {
    if (n_rows < 1 || n_moments < 1 || n_energies < 1) return fail(KPM_ERR_INVALID, "sizes");
    if (!moments || !energies || !out) return fail(KPM_ERR_INVALID, "null buffer");
    if (!(e_scale > 0) || !(area_nm2 > 0)) return fail(KPM_ERR_INVALID, "e_scale / area");
    std::vector<double> w(n_moments), eps(n_energies), pref(n_energies);
    const double a = 1.0 / (n_moments + 1);
    for (int m = 0; m < n_moments; ++m) {
        // Jackson damping, Eq. 35
        const double g = jackson ? (1 - m * a) * std::cos(kPi * m * a) +
                                       a * std::sin(kPi * m * a) / std::tan(kPi * a)
                                 : 1.0;
        w[m] = g * (m == 0 ? 1.0 : 2.0);
    }
    for (int k = 0; k < n_energies; ++k) {
        eps[k] = energies[k] / e_scale;
        if (!(std::fabs(eps[k]) < 1.0)) return fail(KPM_ERR_INVALID, "energy %d outside (-E_s, E_s)", k);
        pref[k] = 2.0 / (kPi * area_nm2 * e_scale * std::sqrt(1.0 - eps[k] * eps[k]));
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nmom = (size_t)n_rows * n_moments, nout = (size_t)n_rows * n_energies;
    double *buf = nullptr;
    const size_t total = nmom + n_moments + 2 * (size_t)n_energies + nout;
    KPM_HIP(hipMalloc(&buf, total * sizeof(double)));
    double *dm = buf, *dw = dm + nmom, *de = dw + n_moments, *dp = de + n_energies,
           *dout = dp + n_energies;
    kpm_status st = KPM_OK;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && st == KPM_OK) st = fail(KPM_ERR_DEVICE, "kpm_sum: %s", hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(dm, moments, nmom * sizeof(double), hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(de, eps.data(), eps.size() * sizeof(double), hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dp, pref.data(), pref.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (st == KPM_OK) {
        kpm::launch_kpm_sum(dm, n_rows, n_moments, dw, de, dp, n_energies, dout, s);
        chk(hipGetLastError());
    }
    chk(hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, s));
    chk(hipStreamSynchronize(s));
    (void)hipFree(buf);
    return st;
}

kpm_status kpm_default_launch(int n_vec, kpm_precision precision, kpm_launch *out) {
    const int vs = vshift_of(n_vec);
    if (vs < 0) return fail(KPM_ERR_INVALID, "n_vec must be 1, 2, 4, ..., 64 (got %d)", n_vec);
    if (precision != KPM_FP64 && precision != KPM_FP32_STATES && precision != KPM_FP32)
        return fail(KPM_ERR_INVALID, "precision");
    if (!out) return fail(KPM_ERR_INVALID, "null output");
    return env_launch(vs, precision, out);
}

kpm_status kpm_set_launch(kpm_system *sys, int n_vec, const kpm_launch *l) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!l || !valid_launch(*l)) return fail(KPM_ERR_INVALID, "launch shape out of range");
    sys->launch[vs] = *l;
    sys->launch_dbl[vs] = *l;
    if (sys->nseg > 1) {      // its segment table, for the allocation-free entry point
        DeviceGuard g(sys->device);
        kpm::Sweep sw;
        KPM_TRY(sys->sweep_with(vs, *l, &sw));
    }
    return KPM_OK;
}

kpm_status kpm_get_launch(kpm_system *sys, int n_vec, kpm_launch *out) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!out) return fail(KPM_ERR_INVALID, "null output");
    *out = sys->launch[vs];
    return KPM_OK;
}

kpm_status kpm_set_launch_doubled(kpm_system *sys, int n_vec, const kpm_launch *l) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!l || !valid_launch(*l)) return fail(KPM_ERR_INVALID, "launch shape out of range");
    sys->launch_dbl[vs] = *l;
    return KPM_OK;
}

kpm_status kpm_get_launch_doubled(kpm_system *sys, int n_vec, kpm_launch *out) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!out) return fail(KPM_ERR_INVALID, "null output");
    *out = sys->launch_dbl[vs];
    return KPM_OK;
}

kpm_status kpm_autotune_candidates(kpm_system *sys, int n_vec, kpm_launch *out, int32_t capacity,
                                   int32_t *count) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!count || (capacity > 0 && !out) || capacity < 0)
        return fail(KPM_ERR_INVALID, "null output or negative capacity");
    const std::vector<kpm_launch> cand = autotune_candidates(sys, vs);
    *count = (int32_t)cand.size();
    for (int32_t q = 0; q < std::min<int32_t>(capacity, *count); ++q) out[q] = cand[q];
    return KPM_OK;
}

kpm_status kpm_autotune(kpm_system *sys, int n_vec, const void *phi, int reps, kpm_launch *best) {
    int vs;
    KPM_TRY(check_common(sys, n_vec, &vs));
    if (!phi) return fail(KPM_ERR_INVALID, "null buffer");
    if (reps < 1 || reps > 1000) return fail(KPM_ERR_INVALID, "reps must be 1..1000");
    DeviceGuard g(sys->device);
    return sys->prec == KPM_FP64 ? autotune_impl<double2>(sys, vs, (const double2 *)phi, reps, best)
                                 : autotune_impl<float2>(sys, vs, (const float2 *)phi, reps, best);
}

kpm_status kpm_set_graphs(kpm_system *sys, int enable) {
    if (!sys) return fail(KPM_ERR_INVALID, "null system");
    DeviceGuard g(sys->device);
    if (!enable) sys->drop_graphs();
    sys->graphs = enable != 0;
    return KPM_OK;
}

kpm_status kpm_set_timing(kpm_system *sys, int enable) {
    if (!sys) return fail(KPM_ERR_INVALID, "null system");
    sys->timing = enable != 0;
    return KPM_OK;
}

kpm_status kpm_get_stats(kpm_system *sys, kpm_stats *out) {
    if (!sys || !out) return fail(KPM_ERR_INVALID, "null argument");
    *out = sys->stats;
    return KPM_OK;
}

kpm_status kpm_reset_stats(kpm_system *sys) {
    if (!sys) return fail(KPM_ERR_INVALID, "null system");
    sys->stats = kpm_stats{};
    return KPM_OK;
}

}  // extern "C"
