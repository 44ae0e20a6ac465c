/*
 * Plain CPU oracle for linear-scaling Kubo-Greenwood transport (Fan, Uppstu,
 * Siro, Harju, "Efficient linear-scaling quantum transport calculations on
 * graphics processing units and applications on electron transport in
 * graphene").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code with the GPU library: its own lattice builder (CSR), its own
 * Bessel routine, its own recursions and dot products.
 *
 * Everything is complex128 (C99 double complex), written in the order the
 * paper states the steps.  Dot products use Neumaier-compensated summation so
 * that the oracle is the more accurate side of every comparison, and run
 * serially.  When built with OpenMP, the row loops of the sparse products and
 * the element-wise vector updates are split over threads (static partition of
 * the rows); each value is still computed by the same operations in the same
 * order, so results are bit-identical for every thread count.
 *
 * Units: energies in eV, times in fs, lengths in nm, hbar = 0.6582119569 eV fs.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Row loops shorter than this run on one thread: on small lattices the
 * thread start-up would cost more than the loop. */
#define ORC_PAR_MIN 32768

/* With ORC_PROGRESS set in the environment, the time loops report each
 * finished time step on stderr (long runs at paper scale). */
static void progress(const char *loop, int k, int n)
{
    if (getenv("ORC_PROGRESS")) {
        fprintf(stderr, "[oracle] %s time step %d/%d done\n", loop, k, n);
        fflush(stderr);
    }
}

/* Threads of the parallel row loops (1 when built without OpenMP). */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

#define ORC_BOND_NM 0.142 /* carbon-carbon distance a (Sec. 2, lattice paragraph) */

enum { ORC_SHEET = 0, ORC_ZGNR = 1, ORC_AGNR = 2 };

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. 2): an nx x ny graphene sample, nx dimer lines along the     */
/* zigzag direction and ny zigzag chains.  Site (i, j) has index j*nx + i and */
/* sits at x = i*sqrt(3)a/2, y = 3ja/2 + (a/2 if i+j is odd).  Each site is   */
/* bonded to (i-1, j), (i+1, j) inside its chain, and to (i, j+1) when i+j is */
/* odd or (i, j-1) when i+j is even.  Sheet: periodic in x and y, transport  */
/* along x.  ZGNR: periodic in x, open in y, transport along x.  AGNR: open  */
/* in x, periodic in y, transport along y.  Vacancies (Sec. 2, last          */
/* paragraph) are removed from the Hilbert space: no bonds touch them.       */
/*                                                                          */
/* Output CSR over all nx*ny rows; a removed site has an empty row.  For   */
/* each stored entry: hop = H_nm (eV) and dx = X_n - X_m, the bond vector   */
/* component along the transport axis (nm).  With periodic boundaries this  */
/* is the minimum-image displacement of the bond.                           */
/* Returns nnz, or -1 on invalid sizes.  col/hop/dx must hold 3*nx*ny.      */
/* ------------------------------------------------------------------------ */
int64_t orc_graphene(int64_t nx, int64_t ny, int geometry, double t_ev,
                     const unsigned char *active, int64_t *row_ptr,
                     int64_t *col, double *hop, double *dx)
{
    int pbc_x = (geometry == ORC_SHEET || geometry == ORC_ZGNR);
    int pbc_y = (geometry == ORC_SHEET || geometry == ORC_AGNR);
    int along_y = (geometry == ORC_AGNR);
    if (nx < 2 || ny < 1) return -1;
    if (pbc_x && (nx % 2 != 0 || nx < 4)) return -1;
    if (pbc_y && (ny % 2 != 0 || ny < 2)) return -1;
    if (geometry < 0 || geometry > 2) return -1;

    const double a = ORC_BOND_NM;
    const double hx = sqrt(3.0) * a / 2.0;
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t j = 0; j < ny; ++j) {
        for (int64_t i = 0; i < nx; ++i) {
            int64_t n = j * nx + i;
            int odd = (int)((i + j) & 1);
            if (active == NULL || active[n]) {
                /* three candidate bonds: (di, dj, bond vector from m to n) */
                int64_t mi[3], mj[3];
                double bx[3], by[3];
                /* left neighbour (i-1, j): X_n - X_m = +hx; Y_n - Y_m = +a/2 if odd else -a/2 */
                mi[0] = i - 1; mj[0] = j; bx[0] = hx;  by[0] = odd ? a / 2 : -a / 2;
                /* right neighbour (i+1, j) */
                mi[1] = i + 1; mj[1] = j; bx[1] = -hx; by[1] = odd ? a / 2 : -a / 2;
                /* vertical neighbour */
                if (odd) { mi[2] = i; mj[2] = j + 1; bx[2] = 0.0; by[2] = -a; }
                else     { mi[2] = i; mj[2] = j - 1; bx[2] = 0.0; by[2] = a; }
                for (int k = 0; k < 3; ++k) {
                    int64_t ii = mi[k], jj = mj[k];
                    if (ii < 0 || ii >= nx) {
                        if (!pbc_x) continue;
                        ii = (ii + nx) % nx;
                    }
                    if (jj < 0 || jj >= ny) {
                        if (!pbc_y) continue;
                        jj = (jj + ny) % ny;
                    }
                    int64_t m = jj * nx + ii;
                    if (active != NULL && !active[m]) continue;
                    col[nnz] = m;
                    hop[nnz] = t_ev;
                    dx[nnz] = along_y ? by[k] : bx[k];
                    ++nnz;
                }
            }
            row_ptr[n + 1] = nnz;
        }
    }
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Sparse products.  H~ = H / E_s (spectrum scaled into [-1, 1], Sec. 3.1,  */
/* end of the delta-function subsection; no shift).  D = [X, H~] has        */
/* entries (X_n - X_m) H~_nm (Eq. 15 without the i/hbar).                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int64_t *col;
    const double *hop;
    const double *dx;
    const double *onsite;   /* may be NULL */
    double e_scale;
} orc_ham;

static void apply_h(const orc_ham *h, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static) if (h->n >= ORC_PAR_MIN)
    for (int64_t n = 0; n < h->n; ++n) {
        cplx s = 0.0;
        if (h->onsite) s = h->onsite[n] * x[n];
        for (int64_t e = h->row_ptr[n]; e < h->row_ptr[n + 1]; ++e)
            s += h->hop[e] * x[h->col[e]];
        y[n] = s / h->e_scale;
    }
}

static void apply_d(const orc_ham *h, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static) if (h->n >= ORC_PAR_MIN)
    for (int64_t n = 0; n < h->n; ++n) {
        cplx s = 0.0;
        for (int64_t e = h->row_ptr[n]; e < h->row_ptr[n + 1]; ++e)
            s += h->dx[e] * (h->hop[e] / h->e_scale) * x[h->col[e]];
        y[n] = s;
    }
}

/* <a|b> = sum conj(a_n) b_n, Neumaier-compensated per component. */
static cplx dot(int64_t n, const cplx *a, const cplx *b)
{
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (int64_t k = 0; k < n; ++k) {
        cplx p = conj(a[k]) * b[k];
        double v = creal(p), t = sr + v;
        cr += (fabs(sr) >= fabs(v)) ? (sr - t) + v : (v - t) + sr;
        sr = t;
        v = cimag(p); t = si + v;
        ci += (fabs(si) >= fabs(v)) ? (si - t) + v : (v - t) + si;
        si = t;
    }
    return (sr + cr) + I * (si + ci);
}

static cplx *cvec(int64_t n) { return (cplx *)calloc((size_t)n, sizeof(cplx)); }

/* ------------------------------------------------------------------------ */
/* Chebyshev moments C_m = <phi_L| T_m(H~) |phi_R>, m = 0 .. nm-1           */
/* (Eq. 46 and Alg. 5): phi_0 = phi_R, phi_1 = H~ phi_0,                    */
/* phi_m = 2 H~ phi_{m-1} - phi_{m-2}.                                       */
/* ------------------------------------------------------------------------ */
static int moments(const orc_ham *h, const cplx *phil, const cplx *phir,
                   int nm, cplx *mu)
{
    int64_t n = h->n;
    cplx *p0 = cvec(n), *p1 = cvec(n), *p2 = cvec(n);
    if (!p0 || !p1 || !p2) { free(p0); free(p1); free(p2); return -2; }
    memcpy(p0, phir, (size_t)n * sizeof(cplx));
    mu[0] = dot(n, phil, p0);
    if (nm > 1) {
        apply_h(h, p0, p1);
        mu[1] = dot(n, phil, p1);
    }
    for (int m = 2; m < nm; ++m) {
        apply_h(h, p1, p2);
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
        for (int64_t k = 0; k < n; ++k) p2[k] = 2.0 * p2[k] - p0[k];
        mu[m] = dot(n, phil, p2);
        cplx *tmp = p0; p0 = p1; p1 = p2; p2 = tmp;
    }
    free(p0); free(p1); free(p2);
    return 0;
}

int orc_moments(int64_t n, const int64_t *row_ptr, const int64_t *col,
                const double *hop, const double *dx, const double *onsite,
                double e_scale, const double *phil, const double *phir,
                int nm, double *mu)
{
    if (nm < 1 || e_scale <= 0) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    return moments(&h, (const cplx *)phil, (const cplx *)phir, nm, (cplx *)mu);
}

/* ------------------------------------------------------------------------ */
/* Bessel functions J_0(x) .. J_{count-1}(x) of the first kind by Miller's  */
/* backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1}, started far above    */
/* the wanted orders from (0, tiny) and normalised with the sum rule        */
/* J_0 + 2 sum_k J_{2k} = 1.  x >= 0.                                       */
/* ------------------------------------------------------------------------ */
int orc_bessel_j(int count, double x, double *out)
{
    if (count < 1 || x < 0 || !isfinite(x)) return -1;
    for (int k = 0; k < count; ++k) out[k] = 0.0;
    if (x == 0.0) { out[0] = 1.0; return 0; }
    double top = (count > x ? count : x);
    int start = (int)(top + 30.0 + 10.0 * sqrt(top));
    if (start % 2) ++start;
    double *j = (double *)calloc((size_t)start + 2, sizeof(double));
    if (!j) return -2;
    j[start + 1] = 0.0;
    j[start] = 1e-300;
    for (int k = start; k >= 1; --k) {
        j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1];
        if (fabs(j[k - 1]) > 1e250) {       /* rescale to stay finite */
            for (int q = k - 1; q <= start + 1; ++q) j[q] *= 1e-250;
        }
    }
    double norm = j[0];
    for (int k = 2; k <= start; k += 2) norm += 2.0 * j[k];
    for (int k = 0; k < count; ++k) out[k] = j[k] / norm;
    free(j);
    return 0;
}

/* Expansion coefficients of Eq. 36: c_m = (2 - delta_m0) (-i s)^m J_m(x), */
/* s = +1 for U(+dt) and -1 for U(-dt) = U(dt)^dagger; x = E_s dt / hbar.  */
static int bessel_coeffs(int np, double x, int sign, cplx *c)
{
    double *jm = (double *)malloc((size_t)np * sizeof(double));
    if (!jm) return -2;
    int rc = orc_bessel_j(np, x, jm);
    if (rc) { free(jm); return rc; }
    cplx unit = (sign > 0) ? -I : I, pw = 1.0;
    for (int m = 0; m < np; ++m) {
        c[m] = (m == 0 ? 1.0 : 2.0) * pw * jm[m];
        pw *= unit;
    }
    free(jm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* out = U(sign*dt) in (Eq. 36, Alg. 6): out = sum_m c_m T_m(H~) in.        */
/* ------------------------------------------------------------------------ */
static int evolve(const orc_ham *h, double hbar, double dt, int sign, int np,
                  const cplx *in, cplx *out)
{
    int64_t n = h->n;
    cplx *c = cvec(np);
    cplx *p0 = cvec(n), *p1 = cvec(n), *p2 = cvec(n);
    int rc = (c && p0 && p1 && p2) ? 0 : -2;
    if (!rc) rc = bessel_coeffs(np, h->e_scale * dt / hbar, sign, c);
    if (!rc) {
        memcpy(p0, in, (size_t)n * sizeof(cplx));
        apply_h(h, p0, p1);
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
        for (int64_t k = 0; k < n; ++k) out[k] = c[0] * p0[k] + c[1] * p1[k];
        for (int m = 2; m < np; ++m) {
            apply_h(h, p1, p2);
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t k = 0; k < n; ++k) {
                p2[k] = 2.0 * p2[k] - p0[k];
                out[k] += c[m] * p2[k];
            }
            cplx *tmp = p0; p0 = p1; p1 = p2; p2 = tmp;
        }
    }
    free(c); free(p0); free(p1); free(p2);
    return rc;
}

int orc_evolve(int64_t n, const int64_t *row_ptr, const int64_t *col,
               const double *hop, const double *dx, const double *onsite,
               double e_scale, double hbar, double dt, int sign, int np,
               const double *in, double *out)
{
    if (np < 2 || e_scale <= 0 || (sign != 1 && sign != -1)) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    return evolve(&h, hbar, dt, sign, np, (const cplx *)in, (cplx *)out);
}

/* ------------------------------------------------------------------------ */
/* outx = [X, U(dt)] in  (Eq. 37, Alg. 7), with the recursion of Eq. 39-41: */
/*   [X,T_0] = 0, [X,T_1] = D, [X,T_m] = 2 D T_{m-1} + 2 H~ [X,T_{m-1}]     */
/*   - [X,T_{m-2}], applied to `in`.  D = [X, H~].                          */
/* If outu is not NULL it also receives U(dt) in (Eq. 36 with the same     */
/* T_m(H~) in), which the mean-square-displacement loop needs next.        */
/* ------------------------------------------------------------------------ */
static int evolve_x(const orc_ham *h, double hbar, double dt, int np,
                    const cplx *in, cplx *outx, cplx *outu)
{
    int64_t n = h->n;
    cplx *c = cvec(np);
    cplx *p0 = cvec(n), *p1 = cvec(n), *p2 = cvec(n);
    cplx *q0 = cvec(n), *q1 = cvec(n), *q2 = cvec(n), *tmpv = cvec(n);
    int rc = (c && p0 && p1 && p2 && q0 && q1 && q2 && tmpv) ? 0 : -2;
    if (!rc) rc = bessel_coeffs(np, h->e_scale * dt / hbar, +1, c);
    if (!rc) {
        memcpy(p0, in, (size_t)n * sizeof(cplx));          /* T_0 in      */
        /* q0 = [X,T_0] in = 0 (cvec is zeroed)                              */
        apply_h(h, p0, p1);                                /* T_1 in      */
        apply_d(h, in, q1);                                /* [X,T_1] in  */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
        for (int64_t k = 0; k < n; ++k) {
            outx[k] = c[1] * q1[k];
            if (outu) outu[k] = c[0] * p0[k] + c[1] * p1[k];
        }
        for (int m = 2; m < np; ++m) {
            apply_h(h, p1, p2);                            /* H~ T_{m-1}  */
            apply_d(h, p1, tmpv);                          /* D T_{m-1}   */
            apply_h(h, q1, q2);                            /* H~ [X,T_{m-1}] */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t k = 0; k < n; ++k) {
                q2[k] = 2.0 * tmpv[k] + 2.0 * q2[k] - q0[k];
                p2[k] = 2.0 * p2[k] - p0[k];
                outx[k] += c[m] * q2[k];
                if (outu) outu[k] += c[m] * p2[k];
            }
            cplx *t;
            t = p0; p0 = p1; p1 = p2; p2 = t;
            t = q0; q0 = q1; q1 = q2; q2 = t;
        }
    }
    free(c); free(p0); free(p1); free(p2); free(q0); free(q1); free(q2); free(tmpv);
    return rc;
}

int orc_evolve_x(int64_t n, const int64_t *row_ptr, const int64_t *col,
                 const double *hop, const double *dx, const double *onsite,
                 double e_scale, double hbar, double dt, int np,
                 const double *in, double *outx, double *outu)
{
    if (np < 2 || e_scale <= 0) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    return evolve_x(&h, hbar, dt, np, (const cplx *)in, (cplx *)outx, (cplx *)outu);
}

/* V = (i/hbar)[H, X] = -i (E_s/hbar) D (Eq. 15). */
static void apply_v(const orc_ham *h, double hbar, const cplx *x, cplx *y)
{
    apply_d(h, x, y);
    cplx f = -I * (h->e_scale / hbar);
#pragma omp parallel for schedule(static) if (h->n >= ORC_PAR_MIN)
    for (int64_t k = 0; k < h->n; ++k) y[k] *= f;
}

/* ------------------------------------------------------------------------ */
/* Velocity auto-correlation moments (Alg. 2, Eq. 42-43, Eq. 32):           */
/*   t_k = k dt, k = 0 .. nsteps;  R_k = U(-dt)^k V phi,  psi_k =            */
/*   U(-dt)^k phi,  L_k = V psi_k;  out[k][m] = Re <L_k| T_m(H~) |R_k>.      */
/* Units nm^2/fs^2.  k = 0 is included (the VAC at zero time).              */
/* ------------------------------------------------------------------------ */
int orc_vac(int64_t n, const int64_t *row_ptr, const int64_t *col,
            const double *hop, const double *dx, const double *onsite,
            double e_scale, double hbar, const double *phi, int nsteps,
            double dt, int np, int nm, double *out)
{
    if (np < 2 || nm < 1 || nsteps < 0 || e_scale <= 0) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    cplx *psi = cvec(n), *r = cvec(n), *l = cvec(n), *tmp = cvec(n);
    cplx *mu = cvec(nm);
    int rc = (psi && r && l && tmp && mu) ? 0 : -2;
    if (!rc) {
        memcpy(psi, phi, (size_t)n * sizeof(cplx));
        apply_v(&h, hbar, psi, r);
    }
    for (int k = 0; !rc && k <= nsteps; ++k) {
        if (k > 0) {
            rc = evolve(&h, hbar, dt, -1, np, psi, tmp);
            if (rc) break;
            memcpy(psi, tmp, (size_t)n * sizeof(cplx));
            rc = evolve(&h, hbar, dt, -1, np, r, tmp);
            if (rc) break;
            memcpy(r, tmp, (size_t)n * sizeof(cplx));
        }
        apply_v(&h, hbar, psi, l);
        rc = moments(&h, l, r, nm, mu);
        for (int m = 0; !rc && m < nm; ++m) out[(int64_t)k * nm + m] = creal(mu[m]);
        progress("vac", k, nsteps);
    }
    free(psi); free(r); free(l); free(tmp); free(mu);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Mean-square-displacement moments (Alg. 3, Eq. 44, Eq. 33):               */
/*   Y_0 = [X, U(0)] phi = 0, psi'_0 = phi;                                  */
/*   Y_k = U(dt) Y_{k-1} + [X, U(dt)] psi'_{k-1},  psi'_k = U(dt) psi'_{k-1}; */
/*   out[k][m] = Re <Y_k| T_m(H~) |Y_k>.  Units nm^2.                        */
/* ------------------------------------------------------------------------ */
int orc_msd(int64_t n, const int64_t *row_ptr, const int64_t *col,
            const double *hop, const double *dx, const double *onsite,
            double e_scale, double hbar, const double *phi, int nsteps,
            double dt, int np, int nm, double *out)
{
    if (np < 2 || nm < 1 || nsteps < 0 || e_scale <= 0) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    cplx *y = cvec(n), *ya = cvec(n), *psi = cvec(n), *xu = cvec(n), *u = cvec(n);
    cplx *mu = cvec(nm);
    int rc = (y && ya && psi && xu && u && mu) ? 0 : -2;
    if (!rc) memcpy(psi, phi, (size_t)n * sizeof(cplx));
    for (int k = 0; !rc && k <= nsteps; ++k) {
        if (k > 0) {
            rc = evolve(&h, hbar, dt, +1, np, y, ya);           /* U(dt) Y_{k-1}     */
            if (!rc) rc = evolve_x(&h, hbar, dt, np, psi, xu, u); /* [X,U] psi', U psi' */
            if (rc) break;
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
            for (int64_t q = 0; q < n; ++q) y[q] = ya[q] + xu[q];
            memcpy(psi, u, (size_t)n * sizeof(cplx));
        }
        rc = moments(&h, y, y, nm, mu);
        for (int m = 0; !rc && m < nm; ++m) out[(int64_t)k * nm + m] = creal(mu[m]);
        progress("msd", k, nsteps);
    }
    free(y); free(ya); free(psi); free(xu); free(u); free(mu);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Fourier moments F_n = <phi_L| U(n dtau) |phi_R>, n = -nm .. nm (Alg. 4,   */
/* Eq. 25-28): phi'_R is propagated forward by U(dtau) for n > 0 and        */
/* backward by U(-dtau) = U(dtau)^dagger for n < 0, each step by the        */
/* Chebyshev-Bessel expansion with np terms.  f[n + nm] receives F_n.       */
/* ------------------------------------------------------------------------ */
int orc_fourier(int64_t n, const int64_t *row_ptr, const int64_t *col,
                const double *hop, const double *dx, const double *onsite,
                double e_scale, double hbar, const double *phil, const double *phir,
                int nm, double dtau, int np, double *f)
{
    if (nm < 0 || np < 2 || e_scale <= 0) return -1;
    orc_ham h = {n, row_ptr, col, hop, dx, onsite, e_scale};
    const cplx *l = (const cplx *)phil, *r = (const cplx *)phir;
    cplx *out = (cplx *)f;
    cplx *psi = cvec(n), *nxt = cvec(n);
    int rc = (psi && nxt) ? 0 : -2;
    if (!rc) out[nm] = dot(n, l, r);
    for (int dir = +1; !rc && dir >= -1; dir -= 2) {
        memcpy(psi, r, (size_t)n * sizeof(cplx));
        for (int k = 1; !rc && k <= nm; ++k) {
            rc = evolve(&h, hbar, dtau, dir, np, psi, nxt);
            if (rc) break;
            cplx *t = psi; psi = nxt; nxt = t;
            out[nm + dir * k] = dot(n, l, psi);
        }
    }
    free(psi); free(nxt);
    return rc;
}
