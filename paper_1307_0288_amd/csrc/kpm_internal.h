// Internal interface between the host driver (kpm_host.cpp) and the gfx950
// kernels (kpm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpm {

constexpr int kBlock = 256;       // work-group size of the sweep kernels
constexpr int kMaxStripBlock = 512;   // largest work-group of the marching strips
constexpr int kWave = 64;         // CDNA wavefront
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies
constexpr int kMaxWidth = 4;      // neighbour-list slots per row
constexpr int kMaxPatterns = 256; // distinct neighbour-offset patterns of the compact form
constexpr int32_t kEmptySlot = INT32_MIN;   // pattern entry of an empty slot

// Scaled sparse Hamiltonian on the device (neighbour-list layout of Alg. 8).
// Neighbours come either from the explicit list `nbr` or, in the compact
// form, from a one-byte pattern id per row: slot k of row i holds row
// i + pat[pid[i]][k] (kEmptySlot = no bond).  Lattices repeat a handful of
// offset patterns, so this replaces 4 bytes per slot with 1 byte per row.
// On-site terms come from `ons` (H_nn / E_s) or, when every H_nn is exactly
// a float, from `onsf` (H_nn in eV) times the sample's 1/E_s.
struct Ell {
    const int32_t *nbr;   // [w][n] neighbour row, -1 = empty slot (or nullptr)
    const uint8_t *pid;   // [n] pattern id (compact form) or nullptr
    const int32_t *pat;   // [npat][kMaxWidth] row offsets (compact form)
    int npat;
    const double *hop;    // [w][n] H_nm / E_s, or nullptr (uniform hopping)
    const double *xw;     // [w][n] (X_n - X_m) H_nm / E_s, or nullptr
    const double *ons;    // [n] H_nn / E_s, or nullptr
    const float *onsf;    // [n] H_nn in eV, or nullptr
    int64_t n;            // rows
    int w;                // slots per row
};

// A segment is one independent sample of a batch: a contiguous element range
// [e0, e1), the contiguous work-groups [g0, g0 + nwg) that sweep it (g0 and
// nwg multiples of 8), its uniform hopping t / E_s and its 1 / E_s.  A plain
// system is a single segment.
//
// Tiled traversal (tnx > 0): the segment's rows form chains of tnx rows (a
// lattice whose vertical bonds join row i to row i +- tnx).  Blocks are then
// visited strip by strip: strip s holds columns [s tw, (s + 1) tw) of every
// chain, chain after chain, so the vertical neighbour of a row is gathered
// shortly after (or before) it is read in the neighbouring chain's tile, from
// L2, however many vectors a row carries.  tw is a power of two with tw << R
// a multiple of the block; the last strip is padded (masked elements).
struct Seg {
    int64_t e0, e1;
    int32_t g0, nwg;
    double t, inv_es;
    int32_t tnx, tw;       // chain length and tile width in rows; tnx = 0: row order
    // t / nch as (t * div_m) >> (32 + div_l), div_l = ceil(log2 nch), div_m =
    // ceil(2^(32 + div_l) / nch) < 2^33 (Granlund and Montgomery, PLDI 1994): exact
    // for t < 2^32, and t * div_m fits 64 bits for the tile indices t < 2^31 used
    uint64_t div_m;
    int32_t div_l;
    // marching strips of a batch (one vector per row): the sample's chain
    // length and the chains per strip
    int32_t snx, sj;
};

// Persistent, XCD-aware sweep.  Work-groups are dispatched round-robin over
// the XCDs, so group g runs on XCD g % 8.  Inside its segment, the element
// blocks are cut into 8 contiguous ranges, one per XCD, and the segment's
// groups on an XCD stride through that range together: rows that share
// neighbours are then served by the same L2.
struct Sweep {
    int64_t total;        // elements of the whole system (rows << vshift)
    int nwg;              // work-groups in the grid (multiple of 8)
    int vshift;           // log2(vectors per row)
    int ilp;              // elements per thread per pass in the moment step (1, 2, 4)
    int nt;               // streaming (non-temporal) access to phi_0, phi_L and the output
    int nseg;             // segments
    const Seg *seg;       // [nseg] device table, or nullptr for one segment
    const int32_t *wg_seg;// [nwg] device table: segment of each group (with seg)
    Seg one;              // the segment when seg is nullptr
    // Vector-major states: nplanes planes of pstride elements, one vector
    // each (then vshift = 0 and total = rows); the grid's second dimension
    // is the plane, and group partials are [slot][nwg][nplanes].  nplanes = 1
    // and pstride = 0 for states with every vector of a row side by side.
    int64_t pstride;
    int nplanes;
    int wpg;              // wavefronts per work-group of the marching strips (1 .. 8)
};

// Chain-lattice geometry of a one-sample system for the multi-step moment
// sweeps: row j * nx + i is column i of chain j, and slot k of every row with
// pattern p holds the row dj chains and di columns away (each -1, 0 or 1,
// periodic wrap), code[p] byte k = (dj + 1) * 3 + (di + 1), or 0xFF for an
// empty slot.  k recursion steps per pass (2 .. 6).  reg = 0: the LDS form
// (k = 2; tiles of tj = 16 chains x kTileCols columns, nti x ntj of them).
// reg = 1: the register-tiled form (tiles of tj = 4 or 8 chains x (64 - 2k)
// columns per wavefront) and reg = 2 its marching form (strips of tj chains
// walked row by row, kMarchRows rows per loop pass, so a strip of tj chains
// costs tj + 2k rounded up to a multiple of kMarchRows), for samples whose
// slots follow the graphene builder's order: flags[p] bit k = slot k filled,
// bit 3 = slot 2 joins the next chain.  All multi-step forms need at least
// kMinChains chains (their windows wrap around the sample at most once).
constexpr int kTileCols = 64;
constexpr int kMarchRows = 12;
constexpr int kMinChains = 24;
struct Lat2 {
    int32_t nx, ny;
    int32_t k, reg, tj;
    int32_t nti, ntj;
    const uint32_t *code;    // [npat]
    const uint32_t *flags;   // [npat], or nullptr
    int32_t arith32;         // FP32 states: strip levels in FP32 arithmetic (KPM_FP32)
    // per-row pattern ids of the strips and their number (flags per id):
    // the compact form's on one sample, on a batch the distinct (chain,
    // column) step codes of all its samples
    const uint8_t *sid;
    int32_t nsp;
};

// Coefficient of a step: the value for segment s is tab[s * stride + idx]
// when tab is set, else val.
struct Coef {
    const double2 *tab;
    int stride;
    int idx;
    double2 val;
};

inline Coef coef_val(double2 v) { return Coef{nullptr, 0, 0, v}; }
inline Coef coef_tab(const double2 *t, int stride, int idx, double2 v) {
    return Coef{t, stride, idx, v};
}

// --- launchers (all asynchronous on `s`) ----------------------------------
// Chebyshev moment step (Alg. 5 fused with Alg. 8 and the inner product):
//   first: out = H~ in; partial[slot] = <L|in>, partial[slot+1] = <L|out>.
//   else : out = 2 H~ p1 - p0 (out may alias p0); partial[slot] = <L|out>.
// partial: [slots][nwg][vectors] complex.
template <typename V>
void launch_moment_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                        const V *p0, V *out, const V *phil, double2 *partial,
                        int slot, hipStream_t s);

// Doubling step for phi_L = phi_R: out = 2 H~ p1 - p0 (out may alias p0);
// partial[slot] = <p1|p1>, partial[slot+1] = <p1|out>.
template <typename V>
void launch_moment_step_doubled(const Ell &h, const Sweep &sw, const V *p1, const V *p0,
                                V *out, double2 *partial, int slot, hipStream_t s);

// lat.k recursion steps per pass on a chain lattice (one vector per row,
// width-3 compact form, one sample): from p1 = phi_n and p0 = phi_{n-1},
// out1 = phi_{n+k-1} and out2 = phi_{n+k}; out1 and out2 must not alias p1,
// p0 or each other.  Non-doubling: partial[slot + s - 1] = <L|phi_{n+s}>,
// s = 1 .. k; doubling (phil unused): partial[slot + 2 (s - 1)] =
// <phi_{n+s-1}|phi_{n+s-1}> and partial[slot + 2 (s - 1) + 1] =
// <phi_{n+s-1}|phi_{n+s}>.  re: only the real parts are needed (the marching
// strips then skip the imaginary parts, which read 0; other forms ignore it).
// The multi-step launchers return false, launching nothing, for a step count
// or form that has no kernel (lat.k outside 2 .. 8 for strips, 2 .. 4 for
// register tiles, 2 for LDS tiles; the propagators need strips, and the
// coupled one 2 or 3 steps).
template <typename V>
bool launch_moment_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const V *p1,
                         const V *p0, V *out1, V *out2, const V *phil, double2 *partial,
                         int slot, bool dbl, bool re, hipStream_t s);

// Coefficients of the K steps of one multi-step propagator pass.
constexpr int kMaxMarchSteps = 8;
// Most steps per pass of the real-part strips with FP64 states (the VAC and
// MSD moment sets): two more than the other strips take
constexpr int kReMarchSteps = 10;
// Launch of those real-part strips of 9 or 10 steps (kpm_march_long.hip);
// false for any other step count or a lattice that does not take the strips.
bool launch_moment_march_re_long(const Ell &h, const Sweep &sw, const Lat2 &lat,
                                 const double2 *p1, const double2 *p0, double2 *out1,
                                 double2 *out2, const double2 *phil, double2 *partial, int slot,
                                 hipStream_t s);
struct CoefK {
    double2 c[kMaxMarchSteps];
};

// K = lat.k steps of the Chebyshev-Bessel propagator (Alg. 6) in marching
// strips (lat.reg == 2): from p1 = phi_n and p0 = phi_{n-1}, out1 = phi_{n+K-1},
// out2 = phi_{n+K} (neither aliasing p1, p0 or each other) and acc += c_m
// phi_m for m = n+1 .. n+K, c_m = ck.c[m - n - 1], in step order.
template <typename V>
bool launch_evolve_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const V *p1,
                         const V *p0, V *out1, V *out2, V *acc, const CoefK &ck,
                         hipStream_t s);

// K = lat.k = 2 or 3 coupled steps of Alg. 7 (Eq. 37-41) in marching strips:
// from p1, p0 (T_n psi, T_{n-1} psi) and q1, q0 ([X, T_n] psi, [X, T_{n-1}] psi;
// q0 may be nullptr for 0) the last two states of each recursion, and accu +=
// c_m p_m, accx += c_m q_m for m = n+1 .. n+K (c_m = ck.c[m - n - 1]).  pxw:
// [npat][4] commutator weight of each slot per pattern.  Outputs alias no input.
template <typename V>
bool launch_evolve_x_multi(const Ell &h, const Sweep &sw, const Lat2 &lat, const double *pxw,
                           const V *p1, const V *p0, V *pout1, V *pout2, const V *q1,
                           const V *q0, V *qout1, V *qout2, V *accx, V *accu, const CoefK &ck,
                           hipStream_t s);

// The strip launchers above for FP32 states with the recursion levels in FP32
// registers (lat.arith32; kpm_march32.hip); the same contracts.
bool launch_moment_multi_f32(const Ell &h, const Sweep &sw, const Lat2 &lat, const float2 *p1,
                             const float2 *p0, float2 *out1, float2 *out2, const float2 *phil,
                             double2 *partial, int slot, bool dbl, bool re, hipStream_t s);
bool launch_evolve_multi_f32(const Ell &h, const Sweep &sw, const Lat2 &lat, const float2 *p1,
                             const float2 *p0, float2 *out1, float2 *out2, float2 *acc,
                             const CoefK &ck, hipStream_t s);

// mom[t * stride + offset + j] = 2 mom[...j] - mom[...j % 2] for 2 <= j < nm,
// t < rows: moments from the doubling sums.
void launch_undouble(double2 *mom, int rows, int64_t stride, int64_t offset, int nm,
                     hipStream_t s);

// Chebyshev-Bessel propagator step (Alg. 6):
//   first: out = H~ in; acc = add + c0 in + c out   (add may be nullptr)
//   else : out = 2 H~ p1 - p0 (out may alias p0); acc += c out
template <typename V>
void launch_evolve_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                        const V *p0, V *out, V *acc, const V *add, Coef c0, Coef c,
                        hipStream_t s);

// Coupled T_m / [X, T_m] step (Alg. 7, Eq. 38-41), accumulating both sums:
//   first: pout = H~ in, qout = D in; accx = c qout; accu = c0 in + c pout
//   else : pout = 2 H~ p1 - p0; qout = 2 D p1 + 2 H~ q1 - q0 (q0 may be
//          nullptr = 0); accx += c qout; accu += c pout
template <typename V>
void launch_evolve_x_step(const Ell &h, const Sweep &sw, bool first, const V *p1,
                          const V *p0, V *pout, const V *q1, const V *q0, V *qout,
                          V *accx, V *accu, Coef c0, Coef c, hipStream_t s);

// y = alpha D x, D = [X, H~].
template <typename V>
void launch_apply_d(const Ell &h, const Sweep &sw, const V *x, V *y, Coef alpha,
                    hipStream_t s);

// State of R = 2^vshift >= 2 vectors from rows-major [n][R] (vectors of a
// row side by side, the caller's layout) to vector-major [R][n] (to_planar)
// or back; src and dst must not overlap.
template <typename V>
void launch_planar(const V *src, V *dst, int64_t n, int vshift, bool to_planar, hipStream_t s);

// partial[slot] = <a|b> per work-group and vector.
template <typename V>
void launch_dot(const Sweep &sw, const V *a, const V *b, double2 *partial, int slot,
                hipStream_t s);

// out[t][k] = pref sum_n w_n Re[exp(i theta_k n) f[t][n]], n = -nm .. nm
// (Fourier sum, Eq. 22-24).
void launch_ftm_sum(const double2 *f, int rows, int nm, const double *w, const double *theta,
                    int ne, double pref, double *out, hipStream_t s);

// dst[(seg * R + r) * stride_r + offset + j] = sum over the segment's groups g
// of partial[j][g][r], j < slots, in a fixed order (deterministic).
void launch_reduce(const double2 *partial, const Sweep &sw, int slots, double2 *dst,
                   int64_t stride_r, int64_t offset, hipStream_t s);

// out[t][k] = pref_k sum_m w_m T_m(e_k) mom[t][m]  (KPM sum, Eq. 29-31).
void launch_kpm_sum(const double *mom, int rows, int nm, const double *w,
                    const double *eps, const double *pref, int ne, double *out,
                    hipStream_t s);

// Fixed device scratch of the entry point that allocates nothing
// (kpm_moments_noalloc): a file-scope device array of kStaticScratchBytes per
// GPU.  static_scratch returns its address on `device`, which must be the
// current device; the address is looked up once per device and kept.
constexpr size_t kStaticScratchBytes = (size_t)320 << 20;
hipError_t static_scratch(int device, void **ptr);

}  // namespace kpm
