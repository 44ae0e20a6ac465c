// Running conductivities (Eq. 6, 9, 11) and the transport quantities derived
// from them (host side of the C ABI): length and conductance (Sec. 5.1, Eq. 50-52), semi-classical
// conductivity by maximum or time-block average (Sec. 5.2, Eq. 53 and 55),
// the Pade fit of a saturating MSD (Sec. 5.3, Eq. 58) and the typical
// conductance (Eq. 60).  Arrays are [n_times][n_energies], time t_k = k dt.
#include "kpm.h"
#include "kpm_error.h"

#include <cmath>
#include <limits>
#include <vector>

namespace {

constexpr double kHbar = 0.6582119569;   // eV fs
constexpr double kPi = 3.14159265358979323846;
constexpr double kNaN = std::numeric_limits<double>::quiet_NaN();

kpm_status bad(const char *what) { return kpm_detail::set_error(KPM_ERR_INVALID, what); }

// Delta X^2 = [rho Delta X^2] / rho, NaN where rho = 0.
inline double per_state(double rho_msd, double rho) { return rho != 0.0 ? rho_msd / rho : kNaN; }

// Least-squares solution of A x = y (A: rows x cols, column-major, rows >=
// cols) by Householder QR.  Returns false when A is rank deficient.
bool least_squares(int rows, int cols, std::vector<double> &a, std::vector<double> &y,
                   std::vector<double> &x) {
    auto at = [&](int i, int j) -> double & { return a[(size_t)j * rows + i]; };
    double amax = 0.0;
    for (double v : a) amax = std::fmax(amax, std::fabs(v));
    for (int j = 0; j < cols; ++j) {
        double norm = 0.0;
        for (int i = j; i < rows; ++i) norm = std::hypot(norm, at(i, j));
        if (!(norm > 1e-13 * amax * std::sqrt((double)rows))) return false;
        const double alpha = at(j, j) > 0 ? -norm : norm;
        // v = a_j - alpha e_j (stored in place), beta = 2 / (v.v)
        at(j, j) -= alpha;
        double vv = 0.0;
        for (int i = j; i < rows; ++i) vv += at(i, j) * at(i, j);
        for (int c = j + 1; c < cols; ++c) {
            double d = 0.0;
            for (int i = j; i < rows; ++i) d += at(i, j) * at(i, c);
            const double f = 2.0 * d / vv;
            for (int i = j; i < rows; ++i) at(i, c) -= f * at(i, j);
        }
        double d = 0.0;
        for (int i = j; i < rows; ++i) d += at(i, j) * y[i];
        const double f = 2.0 * d / vv;
        for (int i = j; i < rows; ++i) y[i] -= f * at(i, j);
        at(j, j) = alpha;                    // R_jj; the rest of column j is no longer needed
    }
    x.assign(cols, 0.0);
    for (int j = cols - 1; j >= 0; --j) {
        double s = y[j];
        for (int c = j + 1; c < cols; ++c) s -= at(j, c) * x[c];
        x[j] = s / at(j, j);
    }
    return true;
}

}  // namespace

extern "C" {

// Running conductivities in e^2/h from the per-time inputs: Green-Kubo
// (Eq. 6, trapezoid integral of the VAC), Einstein E1 (Eq. 9, derivative of
// the MSD, central differences inside, one-sided at the ends) and E2 (Eq. 11,
// MSD over time).
kpm_status kpm_sigma_gk(int nt, int ne, const double *in, double dt, double *out) {
    if (nt < 1 || ne < 1 || !in || !out || in == out || !(dt > 0))
        return bad("sigma_gk arguments");
    const double f = 2.0 * kPi * kHbar;
    for (int k = 0; k < ne; ++k) {
        double acc = 0.0;
        out[k] = 0.0;
        for (int t = 1; t < nt; ++t) {
            acc += 0.5 * (in[(size_t)t * ne + k] + in[(size_t)(t - 1) * ne + k]) * dt;
            out[(size_t)t * ne + k] = f * acc;
        }
    }
    return KPM_OK;
}

kpm_status kpm_sigma_e1(int nt, int ne, const double *in, double dt, double *out) {
    if (nt < 1 || ne < 1 || !in || !out || in == out || !(dt > 0))
        return bad("sigma_e1 arguments");
    const double f = kPi * kHbar;
    for (int k = 0; k < ne; ++k) {
        for (int t = 0; t < nt; ++t) {
            double d;
            if (nt == 1) d = 0.0;
            else if (t == 0) d = (in[(size_t)ne + k] - in[k]) / dt;
            else if (t == nt - 1) d = (in[(size_t)t * ne + k] - in[(size_t)(t - 1) * ne + k]) / dt;
            else d = (in[(size_t)(t + 1) * ne + k] - in[(size_t)(t - 1) * ne + k]) / (2.0 * dt);
            out[(size_t)t * ne + k] = f * d;
        }
    }
    return KPM_OK;
}

kpm_status kpm_sigma_e2(int nt, int ne, const double *in, double dt, double *out) {
    if (nt < 1 || ne < 1 || !in || !out || in == out || !(dt > 0))
        return bad("sigma_e2 arguments");
    const double f = kPi * kHbar;
    for (int k = 0; k < ne; ++k) out[k] = 0.0;
    for (int t = 1; t < nt; ++t)
        for (int k = 0; k < ne; ++k)
            out[(size_t)t * ne + k] = f * in[(size_t)t * ne + k] / (t * dt);
    return KPM_OK;
}

kpm_status kpm_length(int nt, int ne, const double *rho_msd, const double *rho, double *out) {
    if (nt < 1 || ne < 1 || !rho_msd || !rho || !out) return bad("length arguments");
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < ne; ++k) {
            const double x2 = per_state(rho_msd[(size_t)t * ne + k], rho[k]);
            out[(size_t)t * ne + k] = x2 >= 0.0 ? 2.0 * std::sqrt(x2) : kNaN;
        }
    return KPM_OK;
}

kpm_status kpm_conductance(int nt, int ne, const double *sigma, const double *length_nm,
                           double width_nm, double *out) {
    if (nt < 1 || ne < 1 || !sigma || !length_nm || !out || !(width_nm > 0))
        return bad("conductance arguments");
    for (size_t q = 0; q < (size_t)nt * ne; ++q)
        out[q] = length_nm[q] > 0.0 ? width_nm * sigma[q] / length_nm[q] : kNaN;
    return KPM_OK;
}

kpm_status kpm_ballistic_conductance(int nt, int ne, const double *rho_msd, const double *rho,
                                     double dt_fs, double width_nm, double *out) {
    if (nt < 1 || ne < 1 || !rho_msd || !rho || !out || !(dt_fs > 0) || !(width_nm > 0))
        return bad("ballistic_conductance arguments");
    for (int k = 0; k < ne; ++k) out[k] = kNaN;
    for (int t = 1; t < nt; ++t)
        for (int k = 0; k < ne; ++k) {
            // Delta X^2 = v^2 t^2  ->  G / (e^2/h) = pi hbar W rho sqrt(v^2)
            const double x2 = per_state(rho_msd[(size_t)t * ne + k], rho[k]);
            const double v = x2 >= 0.0 ? std::sqrt(x2) / (t * dt_fs) : kNaN;
            out[(size_t)t * ne + k] = kPi * kHbar * width_nm * rho[k] * v;
        }
    return KPM_OK;
}

kpm_status kpm_sigma_sc_max(int nt, int ne, const double *sigma, double *out) {
    if (nt < 2 || ne < 1 || !sigma || !out) return bad("sigma_sc_max arguments (n_times >= 2)");
    for (int k = 0; k < ne; ++k) {
        double m = sigma[(size_t)ne + k];
        for (int t = 2; t < nt; ++t) m = std::fmax(m, sigma[(size_t)t * ne + k]);
        out[k] = m;
    }
    return KPM_OK;
}

kpm_status kpm_sigma_sc_average(int nt, int ne, const double *sigma, int k1, int k2,
                                double *out) {
    if (nt < 2 || ne < 1 || !sigma || !out || k1 < 0 || k2 <= k1 || k2 >= nt)
        return bad("sigma_sc_average arguments (0 <= k1 < k2 < n_times)");
    for (int k = 0; k < ne; ++k) {
        double s = 0.5 * (sigma[(size_t)k1 * ne + k] + sigma[(size_t)k2 * ne + k]);
        for (int t = k1 + 1; t < k2; ++t) s += sigma[(size_t)t * ne + k];
        out[k] = s / (k2 - k1);
    }
    return KPM_OK;
}

kpm_status kpm_pade_fit(int n_pts, const double *t, const double *y, int m, int n, int sweeps,
                        double *a, double *b) {
    if (m < 0 || n < 0 || m + n + 1 > 32 || n_pts < m + n + 1 || sweeps < 0 || sweeps > 64 ||
        !t || !y || !a || (n > 0 && !b))
        return bad("pade_fit arguments (n_pts >= m + n + 1, m + n < 32, 0 <= sweeps <= 64)");
    double ts = 0.0;
    for (int i = 0; i < n_pts; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(y[i])) return bad("pade_fit: non-finite data");
        ts = std::fmax(ts, std::fabs(t[i]));
    }
    if (!(ts > 0)) return bad("pade_fit: all times are zero");
    // Linearised residual w (y q - p) in tau = t / ts, linear in (a, b); the
    // weight w = 1 / |q| of the previous solve (1 at first) is refreshed
    // `sweeps` times (Sanathanan-Koerner iteration).
    const int cols = m + n + 1;
    std::vector<double> tau(n_pts), w(n_pts, 1.0), mat, rhs, x;
    for (int i = 0; i < n_pts; ++i) tau[i] = t[i] / ts;
    for (int it = 0; it <= sweeps; ++it) {
        mat.assign((size_t)n_pts * cols, 0.0);
        rhs.resize(n_pts);
        for (int i = 0; i < n_pts; ++i) {
            double p = w[i];
            for (int j = 0; j <= m; ++j, p *= tau[i]) mat[(size_t)j * n_pts + i] = p;
            p = w[i] * tau[i];
            for (int k = 1; k <= n; ++k, p *= tau[i]) mat[(size_t)(m + k) * n_pts + i] = -y[i] * p;
            rhs[i] = w[i] * y[i];
        }
        if (!least_squares(n_pts, cols, mat, rhs, x))
            return kpm_detail::set_error(KPM_ERR_NUMERIC, "pade_fit: rank-deficient system");
        for (int i = 0; i < n_pts; ++i) {
            double q = 0.0;
            for (int k = n; k >= 1; --k) q = q * tau[i] + x[m + k];
            q = 1.0 + tau[i] * q;
            if (!(std::fabs(q) > 0.0))
                return kpm_detail::set_error(KPM_ERR_NUMERIC, "pade_fit: pole at a data point");
            w[i] = 1.0 / std::fabs(q);
        }
    }
    double f = 1.0;
    for (int j = 0; j <= m; ++j, f *= ts) a[j] = x[j] / f;
    f = ts;
    for (int k = 1; k <= n; ++k, f *= ts) b[k - 1] = x[m + k] / f;
    return KPM_OK;
}

kpm_status kpm_pade_eval(int m, int n, const double *a, const double *b, int n_pts,
                         const double *t, double *value, double *deriv) {
    if (m < 0 || n < 0 || n_pts < 0 || !a || (n > 0 && !b) || (n_pts > 0 && (!t || !value)))
        return bad("pade_eval arguments");
    for (int i = 0; i < n_pts; ++i) {
        // Horner for p, p', q, q'
        double p = 0.0, dp = 0.0;
        for (int j = m; j >= 0; --j) {
            dp = dp * t[i] + p;
            p = p * t[i] + a[j];
        }
        double q = 0.0, dq = 0.0;
        for (int k = n; k >= 1; --k) {
            dq = dq * t[i] + q;
            q = q * t[i] + b[k - 1];
        }
        // q(t) = 1 + t * (b_1 + b_2 t + ...): the loop above built the bracket
        dq = q + t[i] * dq;
        q = 1.0 + t[i] * q;
        value[i] = p / q;
        if (deriv) deriv[i] = (dp * q - p * dq) / (q * q);
    }
    return KPM_OK;
}

kpm_status kpm_typical_conductance(int n_real, int ne, const double *g, double *out) {
    if (n_real < 1 || ne < 1 || !g || !out) return bad("typical_conductance arguments");
    for (int k = 0; k < ne; ++k) {
        double s = 0.0;
        for (int r = 0; r < n_real; ++r) {
            const double v = g[(size_t)r * ne + k];
            if (!(v > 0)) return bad("typical_conductance: conductances must be positive");
            s += std::log(v);
        }
        out[k] = std::exp(s / n_real);
    }
    return KPM_OK;
}

}  // extern "C"
