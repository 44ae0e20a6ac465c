// Host-only part of the C ABI: graphene lattice (Sec. 2, Eq. 13-15) and
// descriptor validation (the neighbour-list structure of Alg. 8).
#include "kpm_lattice.h"
#include "kpm_error.h"

#include <algorithm>
#include <cmath>

using kpm_detail::fail;
using kpm_detail::Packed;

namespace {
constexpr double kBond = 0.142;          // nm, carbon-carbon distance (Sec. 2)
}

kpm_status kpm_detail::pack_desc(const kpm_system_desc *d, int index, Packed &p, double *bound) {
    const int64_t n = d->n_sites;
    const int w = d->width;
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(KPM_ERR_INVALID, "sample %d: n_sites out of range", index);
    if (w < 1 || w > KPM_MAX_WIDTH) return fail(KPM_ERR_INVALID, "sample %d: width must be 1..%d", index, KPM_MAX_WIDTH);
    if (!d->nbr) return fail(KPM_ERR_INVALID, "sample %d: nbr is null", index);
    if (!std::isfinite(d->t_uniform)) return fail(KPM_ERR_INVALID, "sample %d: t_uniform", index);
    p.n = n;
    p.w = w;
    p.t = d->t_uniform;
    p.e_scale = d->e_scale;
    p.nbr.assign((size_t)w * n, -1);
    p.ons.assign(n, 0.0);
    if (d->hop) p.hop.assign((size_t)w * n, 0.0);
    if (d->dx) p.dx.assign((size_t)w * n, 0.0);
    auto alive = [&](int64_t s) { return !d->active || d->active[s] != 0; };
    for (int64_t s = 0; s < n; ++s) {
        p.ons[s] = (alive(s) && d->onsite) ? d->onsite[s] : 0.0;
        if (!std::isfinite(p.ons[s])) return fail(KPM_ERR_INVALID, "sample %d: non-finite onsite at %lld", index, (long long)s);
        for (int k = 0; k < w; ++k) {
            const size_t q = (size_t)k * n + s;
            int32_t m = d->nbr[q];
            if (m < -1 || m >= n)
                return fail(KPM_ERR_INVALID, "sample %d: neighbour index %d out of range at row %lld slot %d", index, m, (long long)s, k);
            if (m >= 0 && (!alive(s) || !alive(m))) m = -1;
            p.nbr[q] = m;
            if (d->hop) {
                p.hop[q] = m >= 0 ? d->hop[q] : 0.0;
                if (!std::isfinite(p.hop[q])) return fail(KPM_ERR_INVALID, "sample %d: non-finite hop", index);
            }
            if (d->dx) {
                p.dx[q] = m >= 0 ? d->dx[q] : 0.0;
                if (!std::isfinite(p.dx[q])) return fail(KPM_ERR_INVALID, "sample %d: non-finite dx", index);
            }
        }
    }
    // Symmetry: every bond listed from both ends with equal H and opposite dx.
    double gersh = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        double row = std::fabs(p.ons[s]);
        for (int k = 0; k < w; ++k) {
            const size_t q = (size_t)k * n + s;
            const int32_t m = p.nbr[q];
            if (m < 0) continue;
            const double hv = d->hop ? p.hop[q] : p.t;
            row += std::fabs(hv);
            bool found = false;
            for (int k2 = 0; k2 < w && !found; ++k2) {
                const size_t q2 = (size_t)k2 * n + m;
                if (p.nbr[q2] != s) continue;
                const double hb = d->hop ? p.hop[q2] : p.t;
                if (hb != hv) continue;
                if (d->dx && p.dx[q2] != -p.dx[q]) continue;
                found = true;
            }
            if (!found)
                return fail(KPM_ERR_INVALID, "sample %d: H not symmetric (or dx not antisymmetric) at row %lld slot %d", index, (long long)s, k);
        }
        gersh = std::max(gersh, row);
    }
    if (bound) *bound = gersh;
    if (!(d->e_scale > 0) || !std::isfinite(d->e_scale)) return fail(KPM_ERR_INVALID, "sample %d: e_scale", index);
    if (d->e_scale < gersh)
        return fail(KPM_ERR_INVALID, "sample %d: e_scale %.6g below the Gershgorin bound %.6g", index, d->e_scale, gersh);
    return KPM_OK;
}

extern "C" {

kpm_status kpm_build_graphene(int64_t nx, int64_t ny, kpm_geometry geometry,
                              const uint8_t *active, int32_t *nbr, double *dx) {
    const bool pbc_x = geometry == KPM_SHEET || geometry == KPM_ZGNR;
    const bool pbc_y = geometry == KPM_SHEET || geometry == KPM_AGNR;
    if (geometry < KPM_SHEET || geometry > KPM_AGNR) return fail(KPM_ERR_INVALID, "geometry");
    if (nx < 2 || ny < 1 || nx * ny >= (int64_t)1 << 31)
        return fail(KPM_ERR_INVALID, "lattice size %lld x %lld", (long long)nx, (long long)ny);
    if (pbc_x && (nx % 2 || nx < 4)) return fail(KPM_ERR_INVALID, "periodic x needs even nx >= 4");
    if (pbc_y && (ny % 2 || ny < 2)) return fail(KPM_ERR_INVALID, "periodic y needs even ny >= 2");
    if (!nbr) return fail(KPM_ERR_INVALID, "nbr is null");
    const int64_t n = nx * ny;
    const double half_zig = std::sqrt(3.0) * kBond / 2.0;
    for (int64_t j = 0; j < ny; ++j) {
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t s = j * nx + i;
            const bool up = ((i + j) & 1) != 0;             // odd sites bond upwards
            int64_t li = i - 1, ri = i + 1, vj = up ? j + 1 : j - 1;
            bool lok = true, rok = true, vok = true;
            if (li < 0) { lok = pbc_x; li += nx; }
            if (ri >= nx) { rok = pbc_x; ri -= nx; }
            if (vj < 0) { vok = pbc_y; vj += ny; }
            if (vj >= ny) { vok = pbc_y; vj -= ny; }
            const int64_t m[3] = {j * nx + li, j * nx + ri, vj * nx + i};
            const bool ok[3] = {lok, rok, vok};
            // displacement X_s - X_m of each slot along the transport axis
            double d[3];
            if (geometry == KPM_AGNR) {
                const double dy = up ? kBond / 2 : -kBond / 2;   // chain neighbours
                d[0] = dy;
                d[1] = dy;
                d[2] = up ? -kBond : kBond;
            } else {
                d[0] = half_zig;
                d[1] = -half_zig;
                d[2] = 0.0;
            }
            const bool alive = !active || active[s];
            for (int k = 0; k < 3; ++k) {
                const bool use = alive && ok[k] && (!active || active[m[k]]);
                nbr[k * n + s] = use ? (int32_t)m[k] : -1;
                if (dx) dx[k * n + s] = use ? d[k] : 0.0;
            }
        }
    }
    return KPM_OK;
}

kpm_status kpm_validate(const kpm_system_desc *desc, double *gershgorin) {
    if (!desc) return fail(KPM_ERR_INVALID, "null descriptor");
    Packed p;
    return kpm_detail::pack_desc(desc, 0, p, gershgorin);
}

}  // extern "C"
