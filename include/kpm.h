/*
 * kpm.h -- C ABI of the MI355X library for linear-scaling Kubo-Greenwood
 * transport (Fan, Uppstu, Siro, Harju, "Efficient linear-scaling quantum
 * transport calculations on graphics processing units and applications on
 * electron transport in graphene").
 *
 * The library runs the Chebyshev recursion of a sparse tight-binding
 * Hamiltonian on complex state vectors in three forms -- Chebyshev moments
 * (Eq. 46), Chebyshev-Bessel time evolution (Eq. 36) and the commutator
 * propagator (Eq. 37, recursion Eq. 38-41) -- and the two time loops built
 * from them: the velocity auto-correlation (Alg. 2, Eq. 42-43) and the mean
 * square displacement (Alg. 3, Eq. 44).  It also performs the host-side
 * reconstruction (Jackson damping Eq. 35, KPM sums Eq. 29-31, running
 * conductivities Eq. 6, 9, 11).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: energies eV, times fs, lengths nm, hbar = 0.6582119569 eV fs.
 * Scaling: H~ = H / e_scale; e_scale must bound the spectrum (the library
 *   checks e_scale >= the Gershgorin bound).  No shift is applied.
 * States: device memory, complex numbers stored as (re, im) pairs,
 *   layout [n_sites][n_vec] with the vector index fastest; element type
 *   double for KPM_FP64 systems and float for KPM_FP32_STATES and KPM_FP32 systems.
 *   n_vec must be 1, 2, 4, 8, 16, 32 or 64.  States must be zero on removed
 *   (inactive) sites; the library keeps them zero there.
 * Streams: every call enqueues its work on the system's HIP stream.  Calls
 *   that return host results synchronise that stream before returning.
 * Errors: every call returns a kpm_status; kpm_last_error() gives a message
 *   for the last failing call on the calling thread.  No exception crosses
 *   the ABI.  On error the output buffers are unspecified.
 * Threads: one system may be used by one host thread at a time.
 */
#ifndef KPM_H
#define KPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KPM_OK = 0,
    KPM_ERR_INVALID = 1,     /* bad argument, descriptor or size            */
    KPM_ERR_OOM = 2,         /* device or host allocation failed            */
    KPM_ERR_DEVICE = 3,      /* HIP runtime error                           */
    KPM_ERR_UNSUPPORTED = 4, /* valid request this build does not support   */
    KPM_ERR_NUMERIC = 5      /* non-finite moments                          */
} kpm_status;

typedef enum {
    KPM_FP64 = 0,            /* states and arithmetic in double            */
    KPM_FP32_STATES = 1,     /* states stored as float; recursion arithmetic,
                                inner products and moments in double       */
    KPM_FP32 = 2             /* states stored as float, the recursion levels
                                of the multi-step strips computed in float
                                (other steps as KPM_FP32_STATES); inner
                                products and moments in double             */
} kpm_precision;

enum { KPM_MAX_WIDTH = 4 };

/* Lattice geometries of the paper's samples (Sec. 2). */
typedef enum {
    KPM_SHEET = 0,  /* periodic in x and y, transport along x (zigzag)      */
    KPM_ZGNR = 1,   /* periodic in x, open in y, transport along x          */
    KPM_AGNR = 2    /* open in x, periodic in y, transport along y          */
} kpm_geometry;

typedef struct kpm_system kpm_system;

/*
 * Sparse Hamiltonian in neighbour-list (ELL) form, the data structure of
 * Alg. 8: slot k of row n holds the k-th neighbour of site n; arrays are
 * slot-major ([width][n_sites], index k * n_sites + n) so that consecutive
 * rows read consecutive memory.  All arrays are host memory owned by the
 * caller and copied by kpm_system_create.
 *   n_sites    number of rows N (removed sites included), 1 <= N < 2^31.
 *   width      slots per row, 1..KPM_MAX_WIDTH (3 for graphene).
 *   nbr        [width][N] neighbour index m, or -1 for an empty slot.
 *   hop        [width][N] H_nm in eV, or NULL: every filled slot is t_uniform.
 *   t_uniform  hopping in eV used when hop is NULL (-2.7 in the paper, Eq. 13).
 *   onsite     [N] diagonal H_nn in eV, or NULL for zero.
 *   dx         [width][N] X_n - X_m in nm along the transport axis for the
 *              bond in that slot (minimum image under periodic boundaries),
 *              or NULL; the velocity operator V = (i/hbar)[H, X] (Eq. 15)
 *              needs it, so kpm_vac, kpm_msd and kpm_evolve_x reject a
 *              system built without it.
 *   active     [N] 0 marks a removed site (vacancy, Sec. 2), or NULL.
 *              Removed sites get no bonds and zero on-site energy.
 *   e_scale    E_s in eV (see Conventions).
 * There is no spectral shift field: the graphene spectra this library targets
 * are symmetric about zero, so H~ = H / e_scale (shift b = 0); a caller with
 * a shifted spectrum subtracts b from the on-site energies.  There is no area
 * field either: the area Omega enters only the sums (kpm_kpm_sum,
 * kpm_ftm_sum, the learned targets), which take it as an argument.
 * Validation: indices in range, H real symmetric (each bond listed from both
 * ends with equal hopping), dx antisymmetric, e_scale >= Gershgorin bound.
 * Device form (chosen at creation, results agree to rounding): when the rows
 * repeat at most 256 distinct neighbour-offset patterns (any lattice does),
 * neighbours are also stored as one pattern byte per row (kpm_launch.compact
 * selects the form a launch reads), and when every on-site energy is exactly
 * a float it is stored as a float.  The environment variable KPM_COMPACT=0
 * keeps only the explicit forms.
 * Scratch: each system allocates its working memory (recursion states, group
 * partials, moment staging) on first use and keeps it until destroy.  With
 * KPM_SCRATCH_LIMIT_MB=M set at creation, a call whose working memory would
 * exceed M MiB returns KPM_ERR_OOM before allocating anything; the system
 * stays usable for smaller calls.
 */
typedef struct {
    int64_t n_sites;
    int32_t width;
    const int32_t *nbr;
    const double *hop;
    double t_uniform;
    const double *onsite;
    const double *dx;
    const uint8_t *active;
    double e_scale;
} kpm_system_desc;

/*
 * Nearest-neighbour graphene lattice (Sec. 2, Eq. 13-15) in the descriptor's
 * layout, built on the host.  Site (i, j), i < nx along the zigzag chains,
 * j < ny across them, has index j*nx + i and sits at x = i sqrt(3) a / 2,
 * y = 3 j a / 2 + (a/2 if i + j is odd), a = 0.142 nm.  Slots: 0 = (i-1, j),
 * 1 = (i+1, j), 2 = (i, j+1) if i + j is odd else (i, j-1).  Periodic
 * directions need an even size (nx >= 4, ny >= 2).
 *   nbr  [3][nx*ny] output (caller-allocated host memory), -1 = no bond.
 *   dx   [3][nx*ny] output, X_n - X_m (nm) along the transport axis, or NULL.
 *   active  [nx*ny] or NULL; bonds to removed sites are left empty.
 */
kpm_status kpm_build_graphene(int64_t nx, int64_t ny, kpm_geometry geometry,
                              const uint8_t *active, int32_t *nbr, double *dx);

/*
 * Host-only check of one descriptor against every rule kpm_system_create
 * applies (listed under kpm_system_desc), without touching a device.  When
 * the structure is valid, *gershgorin (may be NULL) receives the Gershgorin
 * bound max_n (|H_nn| + sum_m |H_nm|) in eV: the smallest e_scale for which
 * the scaled spectrum lies in [-1, 1] as the Chebyshev expansion (Eq. 46)
 * requires.  It is written also when e_scale itself is rejected, so a
 * caller may validate with e_scale = 0 to learn the bound.
 * Returns KPM_OK, or KPM_ERR_INVALID with the first violated rule.
 */
kpm_status kpm_validate(const kpm_system_desc *desc, double *gershgorin);

/*
 * Create a system on `device` whose work runs on `hip_stream` (a
 * hipStream_t, or NULL for the default stream).  Copies the descriptor
 * arrays to device memory; the system owns them and all recursion scratch.
 */
kpm_status kpm_system_create(const kpm_system_desc *desc, kpm_precision precision,
                             int device, void *hip_stream, kpm_system **out);
kpm_status kpm_system_destroy(kpm_system *sys);
kpm_status kpm_system_set_stream(kpm_system *sys, void *hip_stream);
/* n_sites of the system (rows of every state buffer). */
int64_t kpm_system_n_sites(const kpm_system *sys);

/*
 * Ragged batch: n_sys independent samples (each its own descriptor, size,
 * width, disorder and e_scale) laid side by side in one system, so that every
 * recursion step of all samples is one kernel launch.  Sample s occupies rows
 * offsets[s] .. offsets[s+1]-1 of every state buffer (offsets from
 * kpm_system_offsets; n_sites is their total).  Each sample is scaled by its
 * own e_scale (time steps use each sample's Bessel argument) and gets its own
 * inner products: host outputs of kpm_moments, kpm_vac and kpm_msd gain a
 * leading sample dimension ([n_sys][n_vec][...]).  Every entry point that
 * takes a system accepts a batch.  kpm_system_create is the batch of one.
 * n_sys <= 4096; the total rows must stay below 2^31.
 */
kpm_status kpm_batch_create(int n_sys, const kpm_system_desc *descs, kpm_precision precision,
                            int device, void *hip_stream, kpm_system **out);
/* Number of samples (1 for kpm_system_create). */
int32_t kpm_system_n_samples(const kpm_system *sys);
/* Row offsets of the samples, offsets[0 .. n_samples] (host output). */
kpm_status kpm_system_offsets(const kpm_system *sys, int64_t *offsets);

/*
 * Chebyshev moments C_m = <phi_L| T_m(H~) |phi_R>, m = 0 .. n_moments-1, for
 * each of the n_vec vector pairs (Eq. 46, Alg. 5).  phi_l, phi_r: device
 * states (may be the same buffer).  mu: host output [n_vec][n_moments][2]
 * (re, im).  n_moments >= 1.  Synchronises the stream.
 */
kpm_status kpm_moments(kpm_system *sys, int n_vec, const void *phi_l,
                       const void *phi_r, int n_moments, double *mu);

/*
 * kpm_moments for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same moments from the same kernels and launch shape, with every scratch
 * buffer (the recursion states, the per-group partial sums and the reduced
 * moments) taken from a fixed device array of 320 MiB per GPU that the
 * library holds until the process ends.  It calls no hipMalloc or hipFree
 * and records no graph or timing event.  Sizes whose scratch exceeds the
 * array (two states, or four under a multi-step launch shape, of n_sites x
 * n_vec complex values, plus partials and moments) return KPM_ERR_OOM with
 * the bytes needed in kpm_last_error; the paper-scale sheet (3,998,792
 * sites, one FP64 vector) fits.  Every call on a GPU shares that GPU's array
 * and overwrites it: calls that overlap on one GPU (other streams, threads or
 * systems) race and must be serialised by the caller.  Arguments, output and
 * errors otherwise as kpm_moments; synchronises the stream.
 */
kpm_status kpm_moments_noalloc(kpm_system *sys, int n_vec, const void *phi_l,
                               const void *phi_r, int n_moments, double *mu);

/*
 * The moments of kpm_moments for phi_l = phi_r = phi (the DOS of Eq. 29), from
 * half the recursion steps: with phi_n = T_n(H~) phi, the product identities
 * T_{2n} = 2 T_n^2 - T_0 and T_{2n+1} = 2 T_{n+1} T_n - T_1 of the Chebyshev
 * polynomials (the KPM review the paper cites for Eq. 29-35) give
 * C_{2n} = 2 <phi_n|phi_n> - C_0 and C_{2n+1} = 2 <phi_n|phi_{n+1}> - C_1.
 * This is not the order of Alg. 5 (same values up to rounding, about
 * ceil(n_moments / 2) recursion steps instead of n_moments - 1, and phi is
 * read once per step instead of twice).  phi: device states; mu: host output
 * [n_vec][n_moments][2] as for kpm_moments.  Synchronises the stream.
 */
kpm_status kpm_moments_doubled(kpm_system *sys, int n_vec, const void *phi, int n_moments,
                               double *mu);

/*
 * phi <- U(sign * dt) phi, U(t) = exp(-i H t / hbar), by the Chebyshev-Bessel
 * expansion with n_bessel terms (Eq. 36, Alg. 6); sign = +1 or -1 (U(-dt) =
 * U(dt)^dagger).  phi: device state, in place.  n_bessel >= 2.  Asynchronous.
 * Where the moment sets of this system and n_vec run several steps per pass in
 * marching strips (kpm_launch steps > 1, tiled >= 3), so does the recursion
 * here after its first step, with the same result as single steps.
 */
kpm_status kpm_evolve(kpm_system *sys, int n_vec, void *phi, double dt_fs,
                      int sign, int n_bessel);

/*
 * out_x <- [X, U(dt)] phi (Eq. 37 with the recursion Eq. 38-41, Alg. 7) and,
 * if out_u is not NULL, out_u <- U(dt) phi from the same recursion.  Device
 * states; out_x and out_u must not alias phi or each other.  Asynchronous.
 * As for kpm_evolve, the coupled recursion takes up to three steps per pass in
 * marching strips where the moment sets use strips and the commutator weights
 * are the same for every row of a neighbour pattern; same result as single
 * steps.
 */
kpm_status kpm_evolve_x(kpm_system *sys, int n_vec, const void *phi, void *out_x,
                        void *out_u, double dt_fs, int n_bessel);

/*
 * Velocity auto-correlation moments (Alg. 2, Eq. 32 and 42-43):
 * out[r][k][m] = Re <V U^dagger(t_k) phi_r| T_m(H~) |U^dagger(t_k) V phi_r>
 * for t_k = k dt, k = 0 .. n_steps, with V = (i/hbar)[H, X].  Units nm^2/fs^2.
 * phi: device states (unchanged).  out: host [n_vec][n_steps+1][n_moments].
 * Synchronises the stream.
 */
kpm_status kpm_vac(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                   double dt_fs, int n_bessel, int n_moments, double *out);

/*
 * Mean-square-displacement moments (Alg. 3, Eq. 33 and 44):
 * out[r][k][m] = Re <[X, U(t_k)] phi_r| T_m(H~) |[X, U(t_k)] phi_r>, t_k = k dt,
 * k = 0 .. n_steps ([X, U(0)] = 0 gives zeros at k = 0).  Units nm^2.
 * phi: device states (unchanged).  out: host [n_vec][n_steps+1][n_moments].
 * Synchronises the stream.
 */
kpm_status kpm_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                   double dt_fs, int n_bessel, int n_moments, double *out);

/*
 * kpm_vac and kpm_msd of the same phi in one call (Alg. 2 and 3): vac_out and
 * msd_out as the two calls give them, up to the order of the inner-product
 * sums.  With one vector on a one-sample lattice whose moment sets take the
 * marching strips, both loops advance together and at every t_k > 0 the two
 * moment sets run as two vector planes of one launch sequence (half the
 * one-vector grid per plane: longer strips, half the launches); otherwise the
 * loops run one after the other.  Host outputs [n_vec][n_steps+1][n_moments]
 * each.  Synchronises the stream.
 */
kpm_status kpm_vac_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                       int n_bessel, int n_moments, double *vac_out, double *msd_out);

/*
 * The whole Kubo-Greenwood hot path of one set of random vectors in one call
 * (Alg. 1 with Alg. 2, 3 and 5): dos_out[r][m] = <phi_r|T_m(H~)|phi_r> (real,
 * H~ Hermitian; the real parts of kpm_moments(phi, phi)), and vac_out and
 * msd_out as kpm_vac_msd gives them.  Where kpm_vac_msd runs its loops jointly,
 * the DOS set runs as the second vector plane of the VAC set of t_0 (whose
 * MSD set is zero), so every moment set of the call is a two-plane launch
 * sequence; otherwise the DOS set runs first, on its own.  phi: device states
 * (unchanged).  Host outputs [n_vec][n_moments] and [n_vec][n_steps+1]
 * [n_moments] (a leading sample axis for a batch).  KPM_ERR_INVALID for a
 * null output.  Synchronises the stream.
 */
kpm_status kpm_dos_vac_msd(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                           double dt_fs, int n_bessel, int n_moments, double *dos_out,
                           double *vac_out, double *msd_out);

/*
 * kpm_msd with the moments of each [X, U(t_k)] phi taken in the doubling form
 * of kpm_moments_doubled (the bra and ket of Eq. 44 are the same state).  Same
 * arguments and output.
 */
kpm_status kpm_msd_doubled(kpm_system *sys, int n_vec, const void *phi, int n_steps,
                           double dt_fs, int n_bessel, int n_moments, double *out);

/*
 * Resumable forms of kpm_vac and kpm_msd for long correlation times: the loop
 * state lives in two caller-owned device buffers (same layout as phi) that are
 * updated in place, so a run can be split into pieces, checkpointed (copy the
 * two buffers and the moments out) and resumed, with results bit-identical to
 * one uninterrupted call on the same system.
 *  kpm_vac_continue: state psi = U^dagger(t_k) phi, r = U^dagger(t_k) V phi.
 *  kpm_msd_continue: state psi = U(t_k) phi, y = [X, U(t_k)] phi (Eq. 44);
 *                    doubled = 1 takes the moments in the doubling form.
 * start = 1 begins at t = 0: psi holds phi on entry, r (y) is set here, and
 * the moments at t = 0 come first.  start = 0 continues from t_k.  The call
 * advances n_steps steps of dt; out: host [n_sys][n_vec][n_steps + start]
 * [n_moments].  kpm_vac(phi, n) equals kpm_vac_continue(start = 1, n) on a
 * copy of phi, and also start = 1 for n1 steps followed by start = 0 for
 * n - n1 steps (likewise for the MSD).  Synchronises the stream.
 */
kpm_status kpm_vac_continue(kpm_system *sys, int n_vec, void *psi, void *r, int start,
                            int n_steps, double dt_fs, int n_bessel, int n_moments, double *out);
kpm_status kpm_msd_continue(kpm_system *sys, int n_vec, void *psi, void *y, int start,
                            int n_steps, double dt_fs, int n_bessel, int n_moments, int doubled,
                            double *out);

/*
 * Fourier moments of the FTM (Alg. 4, Eq. 25-27):
 * F_n = <phi_L| U(n dtau) |phi_R> for n = -n_moments .. n_moments, each step
 * of dtau by the Chebyshev-Bessel expansion with n_bessel terms (forward for
 * n > 0, backward for n < 0).  The aliasing-free step for a spectrum scaled to
 * [-E_s, E_s] is dtau = pi hbar / E_s (Sec. 4.2; Bessel argument pi).
 * phi_l, phi_r: device states.  f: host output [n_sys][n_vec][2 n_moments + 1][2]
 * (re, im), index n + n_moments.  Synchronises the stream.
 */
kpm_status kpm_fourier_moments(kpm_system *sys, int n_vec, const void *phi_l,
                               const void *phi_r, int n_moments, double dtau_fs,
                               int n_bessel, double *f);

/*
 * FTM sum (Eq. 22-24) on the device:
 * out[t][k] = dtau / (pi hbar Omega) sum_n w_n Re[exp(i E_k n dtau / hbar) F_n]
 * with w_n the Hanning window (Eq. 28) when hanning != 0, else 1.
 * f: host [n_rows][2 n_moments + 1][2]; energies: host [n_energies] eV;
 * out: host [n_rows][n_energies].  Runs on `hip_stream` and synchronises it.
 */
kpm_status kpm_ftm_sum(int n_rows, int n_moments, const double *f, int n_energies,
                       const double *energies, double dtau_fs, double area_nm2, int hanning,
                       void *hip_stream, double *out);

/*
 * KPM sum (Eq. 29-31) on the device:
 * out[t][k] = 2 / (pi Omega E_s sqrt(1 - e_k^2)) sum_m g_m (2 - delta_m0)
 *             T_m(e_k) moments[t][m],  e_k = energies[k] / E_s,
 * with g_m the Jackson factors (Eq. 35) when jackson != 0, else 1.
 * moments: host [n_rows][n_moments] (real parts); energies: host
 * [n_energies] eV, |E| < E_s; out: host [n_rows][n_energies].
 * Runs on `hip_stream` and synchronises it.
 */
kpm_status kpm_kpm_sum(int n_rows, int n_moments, const double *moments,
                       int n_energies, const double *energies, double e_scale,
                       double area_nm2, int jackson, void *hip_stream, double *out);

/*
 * Running electrical conductivities in units of e^2/h on the host, from
 * rows sampled at t_k = k dt (k = 0 .. n_times-1), each of n_energies:
 *  kpm_sigma_gk: from rho*C_vv (Eq. 6): 2 pi hbar * cumulative trapezoid.
 *  kpm_sigma_e1: from rho*MSD (Eq. 9): pi hbar * d/dt, centred differences
 *                (one-sided at both ends).
 *  kpm_sigma_e2: from rho*MSD (Eq. 11): pi hbar * value / t, 0 at t = 0.
 * in/out: host [n_times][n_energies]; out may not alias in.
 */
kpm_status kpm_sigma_gk(int n_times, int n_energies, const double *rho_vac,
                        double dt_fs, double *out);
kpm_status kpm_sigma_e1(int n_times, int n_energies, const double *rho_msd,
                        double dt_fs, double *out);
kpm_status kpm_sigma_e2(int n_times, int n_energies, const double *rho_msd,
                        double dt_fs, double *out);

/*
 * Transport quantities on the host (Sec. 5), all arrays [n_times][n_energies]
 * at t_k = k dt unless stated; lengths and widths in nm, conductivities and
 * conductances in e^2/h.  Invalid sizes or null pointers give
 * KPM_ERR_INVALID; undefined entries are NaN as stated.
 *
 * kpm_length: L(E, t) = 2 sqrt(Delta X^2(E, t)) (Eq. 50) with the per-state
 *   MSD Delta X^2 = rho_msd / rho (rho_msd: KPM sum of MSD moments, rho:
 *   [n_energies] DOS).  NaN where rho = 0 or Delta X^2 < 0.
 * kpm_conductance: G(E, L) = (W / L(E, t)) sigma(E, t) (Eq. 51, Eq. 59).
 *   NaN where L <= 0 or is NaN (t = 0).
 * kpm_ballistic_conductance: G(E) = (W/2) e^2 rho sqrt(v^2) (Eq. 52) with
 *   v^2 = Delta X^2(E, t_k) / t_k^2 at each t_k > 0, i.e. pi hbar W rho
 *   sqrt(v^2) in e^2/h.  Row 0 is NaN.
 * kpm_sigma_sc_max: sigma_sc(E) = max over t_k > 0 of sigma(E, t_k) (Eq. 53).
 *   n_times >= 2; out [n_energies].
 * kpm_sigma_sc_average: sigma_sc(E) = (1/(t2 - t1)) int_{t1}^{t2} sigma dt
 *   (Eq. 55) by the trapezoid rule, t1 = k1 dt, t2 = k2 dt,
 *   0 <= k1 < k2 < n_times; out [n_energies].
 * kpm_pade_fit: [m/n] Pade approximant of Eq. 58,
 *   y(t) ~ sum_{j=0}^{m} a_j t^j / (1 + sum_{k=1}^{n} b_k t^k) (the k = 0
 *   term of the printed denominator is taken as absent: it duplicates the 1),
 *   fitted over n_pts points by least squares on the linearised residual
 *   y q - p, re-weighted by 1 / |q| of the previous solution `sweeps` times
 *   (Sanathanan-Koerner iteration, which approaches the least-squares fit of
 *   y - p/q); each solve is a Householder QR in t / max|t|.  a: [m+1], b: [n]
 *   host outputs.  n_pts >= m + n + 1, m + n < 32, 0 <= sweeps <= 64;
 *   KPM_ERR_NUMERIC if a system is rank deficient.
 * kpm_pade_eval: value (and, if deriv is not NULL, d/dt) of that approximant
 *   at n_pts times; sigma_E1 of a fitted MSD is pi hbar rho times deriv.
 * kpm_typical_conductance: G_typ(E) = exp(<ln G(E)>) over n_real
 *   realisations (Eq. 60); g: [n_real][n_energies], all > 0; out [n_energies].
 */
kpm_status kpm_length(int n_times, int n_energies, const double *rho_msd, const double *rho,
                      double *out);
kpm_status kpm_conductance(int n_times, int n_energies, const double *sigma,
                           const double *length_nm, double width_nm, double *out);
kpm_status kpm_ballistic_conductance(int n_times, int n_energies, const double *rho_msd,
                                     const double *rho, double dt_fs, double width_nm,
                                     double *out);
kpm_status kpm_sigma_sc_max(int n_times, int n_energies, const double *sigma, double *out);
kpm_status kpm_sigma_sc_average(int n_times, int n_energies, const double *sigma, int k1,
                                int k2, double *out);
kpm_status kpm_pade_fit(int n_pts, const double *t, const double *y, int m, int n, int sweeps,
                        double *a, double *b);
kpm_status kpm_pade_eval(int m, int n, const double *a, const double *b, int n_pts,
                         const double *t, double *value, double *deriv);
kpm_status kpm_typical_conductance(int n_real, int n_energies, const double *g, double *out);

/*
 * Learned moment-to-spectrum reconstruction (not part of the paper's method;
 * plain Jackson-damped KPM of the full moment set stays the reference and the
 * fallback).  A fully connected network of n_layers weight layers with widths
 * widths[0 .. n_layers]: hidden a_{l+1} = tanh(a_l W_l^T + b_l), linear output,
 * trained on the mean squared error with Adam (Kingma and Ba), FP32 throughout.
 * Parameters are packed [W_0 (widths[1] x widths[0], row-major), b_0, W_1,
 * b_1, ...].  x, y: device [batch][widths[0]] and [batch][widths[n_layers]]
 * float arrays, batch <= max_batch.  All work on hip_stream; calls that return
 * host values synchronise it.  Parameters start at zero; kpm_mlp_set_params
 * also resets the Adam state.
 */
typedef struct kpm_mlp kpm_mlp;
typedef struct {
    float lr, beta1, beta2, eps;
} kpm_adam;
kpm_status kpm_mlp_create(int n_layers, const int32_t *widths, int max_batch, int device,
                          void *hip_stream, kpm_mlp **out);
kpm_status kpm_mlp_destroy(kpm_mlp *net);
int64_t kpm_mlp_n_params(const kpm_mlp *net);
kpm_status kpm_mlp_set_params(kpm_mlp *net, const float *params);   /* host [n_params] */
kpm_status kpm_mlp_get_params(kpm_mlp *net, float *params);         /* host [n_params] */
/* y <- network(x). */
kpm_status kpm_mlp_forward(kpm_mlp *net, int batch, const float *x, float *y);
/* loss = mean (network(x) - y)^2 (host); grads (host [n_params], may be NULL). */
kpm_status kpm_mlp_gradients(kpm_mlp *net, int batch, const float *x, const float *y,
                             double *loss, float *grads);
/* One Adam step on the batch; loss (host, may be NULL) is that of the parameters
 * before it.  With loss NULL the call does not synchronise the stream. */
kpm_status kpm_mlp_train_step(kpm_mlp *net, int batch, const float *x, const float *y,
                              const kpm_adam *opt, double *loss);

/*
 * Features and targets of the learned reconstruction, from moments of
 * n_samples samples with n_vec random vectors each (real parts, host
 * [n_samples][n_vec][n_moments]; averaged over the vectors first): with mu the
 * DOS moments (Eq. 46) and c the MSD moments at one time t* (Eq. 44),
 *   x = [mu_n / mu_0, n < n_in] + [c_n / c_0, n < n_in] + [ln(c_0 / mu_0)]
 *       (host float [n_samples][2 n_in + 1]),
 *   y = [10 eV rho(E_k) Omega / (2 mu_0)] + [0.25 sigma_E2(E_k, t*) / (e^2/h)]
 *       (host float [n_samples][2 n_energies]),
 * rho and rho Delta X^2 being the Jackson-damped KPM sums (Eq. 29-31) of all
 * n_moments moments on the device (hip_stream) and sigma_E2 = pi hbar rho
 * Delta X^2 / t* (Eq. 11).
 */
kpm_status kpm_learned_features(int n_samples, int n_vec, int n_moments, const double *mu_dos,
                                const double *mu_msd, int n_in, float *x);
kpm_status kpm_learned_targets(int n_samples, int n_vec, int n_moments, const double *mu_dos,
                               const double *mu_msd, int n_energies, const double *energies,
                               double e_scale, double area_nm2, double t_star_fs,
                               void *hip_stream, float *y);

/*
 * [X, U(n_steps dt)] phi by the recursion of Eq. 44 (the state whose moments
 * kpm_msd takes at t = n_steps dt), written to the device buffer out (same
 * layout as phi, must not alias it).  n_steps >= 1.  Asynchronous.
 */
kpm_status kpm_xu_state(kpm_system *sys, int n_vec, const void *phi, int n_steps, double dt_fs,
                        int n_bessel, void *out);

/*
 * Launch shape of the Chebyshev moment step for a given n_vec: work-groups
 * per compute unit of the persistent grid (1..32; the grid is rounded to a
 * multiple of the 8 XCDs), elements per thread per pass (ilp: 1, 2 or 4),
 * streaming (non-temporal) access to the operands read or written once per
 * step (0 or 1), and whether neighbours are read in the compact pattern form
 * (1) or from the explicit list (0; the explicit list is used regardless when
 * the system has no compact form).  tiled = 1, 2 or 3 visits the rows of a
 * lattice sample strip by strip (tiles of 64, 128 or 256 consecutive columns
 * of successive chains, at least 256 / n_vec columns times 1, 2 or 4; the
 * chain length found from the most common neighbour offset beyond 1) so that a
 * row's vertical neighbour is reused from cache even when a row carries many
 * vectors; tiled = 0, and samples without such a chain structure or with
 * chains shorter than two tiles, keep row order.  steps = 2 .. 8 advances
 * the recursion that many steps per pass: from phi_n and phi_{n-1} a pass
 * writes only the last two states, so each row's states cross HBM once per
 * pass instead of once per step.  It applies to one vector per row on a
 * single-sample lattice in the compact width-3 form whose every bond joins
 * rows at most one column and one chain apart (chains of at least 68 rows, at
 * least 24 chains); other calls take single steps.  A batch whose every
 * sample is such a lattice (with uniform hopping and the builder's slot
 * order) runs its moment sets in the strips below (tiled >= 3; each
 * work-group walks strips of its own sample, with that sample's chain length,
 * strip height and scale); its propagators take single steps.  Two steps run in tiles of
 * 16 chains x 64 columns staged in LDS (tiled = 0) or, where the slots follow
 * the order of kpm_build_graphene, in register tiles of one wavefront each, 8
 * chains (tiled = 1) or 4 (tiled = 2) by 64 - 2 steps columns, or in strips
 * of 64 - 2 steps columns that one wavefront walks chain by chain, 16 or 32
 * chains long (tiled = 3, 4) or of the length (8 .. 64 chains) that lets the
 * grid's wavefronts finish all strips in the fewest passes of 12 rows
 * (tiled = 5).
 * 3 and 4 steps need the register forms (else 2 steps apply), 5 .. 8 steps
 * the strips.  Under steps > 1 any single steps keep row order.  Default for
 * one vector: groups_per_cu 2, steps 8, tiled 5; for more vectors single
 * steps, except on one-sample graphene lattices and batches that take the
 * strips: eight-step strips with one vector per wavefront (below), about
 * 1024 work-groups over all planes (at least 8 per sample of a batch).  At a fixed grid size, traversal and step count the moments are
 * bit-identical for every ilp, streaming and compact choice; the recursion
 * states are bit-identical for every shape (up to the sign of zero), and the
 * shape changes only the order of the inner-product partial sums (in the
 * doubling form the strips accumulate only the real parts, the moments of
 * phi_L = phi_R being real).
 *
 * vectors_per_wave selects, for n_vec > 1 on a one-sample system (or a
 * batch whose moment sets take the strips), how a
 * wavefront's 64 lanes cover the states: 0 (default) puts the n_vec vectors
 * of a row in adjacent lanes (64 / n_vec rows per wavefront, one structure
 * read per row for all vectors); 1 gives every wavefront one vector: the
 * library then keeps its recursion states vector-major (one plane of
 * n_sites values per vector, converted from and to the caller's
 * [n_sites][n_vec] layout at the start and end of each call), every launch
 * sweeps all planes (the plane is the grid's second dimension), and the
 * multi-step shapes above apply to each plane as to one vector.
 * plane_groups (vectors_per_wave = 1 only) is the number of work-groups per
 * plane, a multiple of 8 up to 65536, or 0 for the grid groups_per_cu gives
 * one vector; fewer groups per plane make the strips of tiled = 5 longer (up
 * to the whole sample), so fewer boundary chains are recomputed.  A batch
 * shares a plane's groups out among its samples in proportion to their rows
 * (at least 8 each).  Other batches and n_vec = 1 ignore both fields, and the
 * layout of a call follows the direct form's shape (kpm_set_launch) also for
 * doubling-form moment sets.
 *
 * group_size: threads per work-group of the marching strips (64, 128, 256 or
 * 512; 0 = 256).  Each wavefront walks its own strips, so the group size
 * changes how the grid's wavefronts are grouped (groups_per_cu then counts
 * groups of that size; 8 x 64, 4 x 128, 2 x 256 and 1 x 512 threads per CU
 * all give two wavefronts per SIMD); the coupled strips of Alg. 7 and all
 * other kernels keep 256.
 */
typedef struct {
    int32_t groups_per_cu;
    int32_t ilp;
    int32_t streaming;
    int32_t compact;
    int32_t tiled;
    int32_t steps;
    int32_t vectors_per_wave;
    int32_t plane_groups;
    int32_t group_size;
} kpm_launch;

/* The shape a new system starts with for n_vec vectors per row (both forms):
 * the default above with the environment overrides KPM_GROUPS_PER_CU,
 * KPM_ILP, KPM_STREAMING, KPM_COMPACT_LAUNCH, KPM_TILED and KPM_STEPS applied,
 * each clamped to its range and combined into a valid shape (more than 4
 * steps select the strips, a traversal below 3 caps the steps at 4, single
 * steps take a traversal of at most 3).  Host only; kpm_system_create reads
 * the same environment.  KPM_ERR_INVALID for a bad n_vec or precision. */
kpm_status kpm_default_launch(int n_vec, kpm_precision precision, kpm_launch *out);

/* kpm_set_launch sets the shape of both forms (direct and doubling);
 * kpm_get_launch returns the direct form's. */
kpm_status kpm_set_launch(kpm_system *sys, int n_vec, const kpm_launch *launch);
kpm_status kpm_get_launch(kpm_system *sys, int n_vec, kpm_launch *out);
/* The shape of moment sets in the doubling form (kpm_moments_doubled,
 * kpm_msd_doubled), which kpm_autotune chooses separately. */
kpm_status kpm_set_launch_doubled(kpm_system *sys, int n_vec, const kpm_launch *launch);
kpm_status kpm_get_launch_doubled(kpm_system *sys, int n_vec, kpm_launch *out);

/*
 * Autotuner: times `reps` moment steps of every candidate shape
 * (groups_per_cu in {4, 8, 16} x ilp in {1, 2, 4} x streaming in {0, 1} x
 * compact in {0, 1} when the system has the compact form x tiled in {0, 1}
 * for lattices with long chains; plus, where the multi-step sweeps apply,
 * steps = 2 in LDS tiles with groups_per_cu in {2, 3, 4, 6} x streaming in
 * {0, 1}, steps in {2, 3, 4} in register tiles (tiled in {1, 2}) with
 * groups_per_cu in {1, 2, 3, 4, 6, 8}, and steps in {3, .., 8} in marching
 * strips (tiled 5 with groups_per_cu in {2, 3, 4}; up to 6 steps also tiled
 * in {3, 4} with groups_per_cu 2)) on the device state
 * `phi` ([n_sites][n_vec], read only; only system scratch is written), for
 * the direct and, separately, the doubling form, keeps the fastest of each
 * for this n_vec and returns the direct form's in *best (may be NULL).
 * Synchronises the stream.
 */
/* The candidate shapes kpm_autotune times for n_vec vectors on this system
 * (the incumbent shape is timed first as well): *count receives their number
 * and out[0 .. min(capacity, count) - 1] the shapes (out may be NULL when
 * capacity is 0).  Host only. */
kpm_status kpm_autotune_candidates(kpm_system *sys, int n_vec, kpm_launch *out, int32_t capacity,
                                   int32_t *count);
kpm_status kpm_autotune(kpm_system *sys, int n_vec, const void *phi, int reps,
                        kpm_launch *best);

/*
 * hipGraph replay of the moment sets.  When enabled, the launch sequence of a
 * moment set (first step, recursion steps, partial-sum reductions) is
 * captured once per combination of buffers, sizes and launch shape and
 * replayed on the system's stream; results are bit-identical to direct
 * launches.  Graphs are dropped when scratch is reallocated or graphs are
 * disabled.  Capture runs on an internal stream, so it also works when the
 * system's stream is the null stream.
 */
kpm_status kpm_set_graphs(kpm_system *sys, int enable);

/*
 * Timing of the hot recursion kernel.  When enabled, the library brackets
 * every uninterrupted run of Chebyshev moment steps with HIP events on the
 * system's stream and accumulates their elapsed time and launch count (with
 * graphs, the events bracket each replayed moment set, whose first step and
 * reductions then count towards the time).
 */
typedef struct {
    double step_ms;           /* summed event time of moment-step runs      */
    int64_t step_launches;    /* moment-step kernel launches in those runs  */
    int64_t step_rows;        /* rows x vectors per launch (last run)       */
    int64_t site_updates;     /* all recursion site-updates issued          */
    int64_t step_bytes;       /* algorithmic bytes per moment-step launch:
                                 4 state accesses per row and vector plus
                                 the row structure once per row (last run;
                                 5 accesses per row for a multi-step launch,
                                 4 in the doubling form)                     */
    int64_t step_bytes_total; /* algorithmic bytes of all launches in the
                                 timed moment-step runs                     */
    double wide_ms;           /* event time of the timed runs whose launches
                                 cover the most rows x vectors (wide_rows)  */
    int64_t wide_launches;    /* moment-step launches in those runs         */
    int64_t wide_rows;        /* rows x vectors per launch of those runs    */
} kpm_stats;

kpm_status kpm_set_timing(kpm_system *sys, int enable);
kpm_status kpm_get_stats(kpm_system *sys, kpm_stats *out);
kpm_status kpm_reset_stats(kpm_system *sys);

/* Message of the last failing call on this thread ("" if none). */
const char *kpm_last_error(void);
/* Library version string. */
const char *kpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KPM_H */
