// Host-only part of the C ABI: the graphene lattice builder and the validation
// and packing of sample descriptors (no HIP; also built on its own, with the
// host sanitizers, by the CPU tests).
#pragma once

#include "kpm.h"

#include <cstdint>
#include <vector>

namespace kpm_detail {

// One validated sample in neighbour-list form, energies in eV.  Removed
// sites lose every bond and their on-site energy.
struct Packed {
    int64_t n = 0;
    int w = 0;
    std::vector<int32_t> nbr;   // [w][n], -1 = empty
    std::vector<double> hop;    // [w][n] or empty (uniform t)
    std::vector<double> ons;    // [n]
    std::vector<double> dx;     // [w][n] or empty
    double t = 0;
    double e_scale = 1;
};

// Checks every rule of the descriptor (indices in range, H real symmetric, dx
// antisymmetric, finite values, e_scale at least the Gershgorin bound) and
// copies it into p with removed sites disconnected.  When the structure is
// valid, *bound (if not null) receives the Gershgorin bound in eV, also when
// e_scale itself is rejected.
kpm_status pack_desc(const kpm_system_desc *d, int index, Packed &p, double *bound = nullptr);

}  // namespace kpm_detail
