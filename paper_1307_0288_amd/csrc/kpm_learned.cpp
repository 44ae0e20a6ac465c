// Features and targets of the learned moment-to-spectrum reconstruction
// (host side of the C ABI; the KPM sums of the targets run on the device
// through kpm_kpm_sum).
#include "kpm.h"
#include "kpm_error.h"

#include <cmath>
#include <vector>

namespace {

constexpr double kHbar = 0.6582119569;   // eV fs
constexpr double kPi = 3.14159265358979323846;
constexpr double kDosScale = 10.0;       // eV
constexpr double kSigmaScale = 0.25;     // 1 / (e^2/h)

kpm_status bad(const char *what) { return kpm_detail::set_error(KPM_ERR_INVALID, what); }

// Mean over the vectors of each sample: [S][R][nm] -> [S][nm].
std::vector<double> vector_mean(int ns, int nv, int nm, const double *mu) {
    std::vector<double> out((size_t)ns * nm, 0.0);
    for (int s = 0; s < ns; ++s)
        for (int r = 0; r < nv; ++r)
            for (int m = 0; m < nm; ++m)
                out[(size_t)s * nm + m] += mu[((size_t)s * nv + r) * nm + m];
    for (double &v : out) v /= nv;
    return out;
}

}  // namespace

extern "C" {

kpm_status kpm_learned_features(int ns, int nv, int nm, const double *mu_dos,
                                const double *mu_msd, int n_in, float *x) {
    if (ns < 1 || nv < 1 || nm < 1 || n_in < 1 || n_in > nm || !mu_dos || !mu_msd || !x)
        return bad("learned_features arguments (1 <= n_in <= n_moments)");
    const std::vector<double> mu = vector_mean(ns, nv, nm, mu_dos);
    const std::vector<double> c = vector_mean(ns, nv, nm, mu_msd);
    const int nx = 2 * n_in + 1;
    for (int s = 0; s < ns; ++s) {
        const double *ms = &mu[(size_t)s * nm], *cs = &c[(size_t)s * nm];
        if (!(ms[0] > 0) || !(cs[0] > 0)) return bad("learned_features: C_0 must be positive");
        float *xs = x + (size_t)s * nx;
        for (int n = 0; n < n_in; ++n) {
            xs[n] = (float)(ms[n] / ms[0]);
            xs[n_in + n] = (float)(cs[n] / cs[0]);
        }
        xs[2 * n_in] = (float)std::log(cs[0] / ms[0]);
    }
    return KPM_OK;
}

kpm_status kpm_learned_targets(int ns, int nv, int nm, const double *mu_dos, const double *mu_msd,
                               int ne, const double *energies, double e_scale, double area_nm2,
                               double t_star_fs, void *hip_stream, float *y) {
    if (ns < 1 || nv < 1 || nm < 1 || ne < 1 || !mu_dos || !mu_msd || !energies || !y)
        return bad("learned_targets arguments");
    if (!(t_star_fs > 0)) return bad("learned_targets: t* must be positive");
    const std::vector<double> mu = vector_mean(ns, nv, nm, mu_dos);
    const std::vector<double> c = vector_mean(ns, nv, nm, mu_msd);
    std::vector<double> rho((size_t)ns * ne), rx2((size_t)ns * ne);
    kpm_status st = kpm_kpm_sum(ns, nm, mu.data(), ne, energies, e_scale, area_nm2, 1, hip_stream,
                                rho.data());
    if (st != KPM_OK) return st;
    st = kpm_kpm_sum(ns, nm, c.data(), ne, energies, e_scale, area_nm2, 1, hip_stream, rx2.data());
    if (st != KPM_OK) return st;
    for (int s = 0; s < ns; ++s) {
        if (!(mu[(size_t)s * nm] > 0)) return bad("learned_targets: C_0 must be positive");
        const double fd = kDosScale * area_nm2 / (2.0 * mu[(size_t)s * nm]);
        const double fs = kSigmaScale * kPi * kHbar / t_star_fs;
        float *ys = y + (size_t)s * 2 * ne;
        for (int k = 0; k < ne; ++k) {
            ys[k] = (float)(fd * rho[(size_t)s * ne + k]);
            ys[ne + k] = (float)(fs * rx2[(size_t)s * ne + k]);
        }
    }
    return KPM_OK;
}

}  // extern "C"
