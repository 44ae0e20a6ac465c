// The real-part strips of nine and ten recursion steps per pass (FP64
// states): the VAC and MSD moment sets of the joint call, two vector planes
// per launch (Alg. 2, 3 and 5).  They sit in a file of their own because it is
// compiled with the instruction scheduler's max-ILP strategy, which
// interleaves the independent parts of consecutive levels and keeps the
// ten-step kernel within its 256 VGPRs; on the other kernels that strategy
// costs occupancy or spills, so they keep the default schedule.
#include "kpm_march.h"

namespace kpm {

bool launch_moment_march_re_long(const Ell &h, const Sweep &sw, const Lat2 &lat,
                                 const double2 *p1, const double2 *p0, double2 *out1,
                                 double2 *out2, const double2 *phil, double2 *partial, int slot,
                                 hipStream_t s) {
    if (lat.reg != 2 || lat.k <= kMaxMarchSteps || lat.k > kReMarchSteps) return false;
    const dim3 grid(sw.nwg, sw.nplanes), block(sw.wpg * kWave);
#define KPM_LONG(ONSF_, K_)                                                                   \
    hipLaunchKernelGGL((k_moment_march_re<double2, ONSF_, K_>), grid, block, 0, s, h, sw, lat, \
                       p1, p0, out1, out2, phil, partial, slot)
    const bool onsf = h.onsf != nullptr;
    if (lat.k == 10) {
        if (onsf) KPM_LONG(true, 10);
        else KPM_LONG(false, 10);
    } else {
        if (onsf) KPM_LONG(true, 9);
        else KPM_LONG(false, 9);
    }
#undef KPM_LONG
    return true;
}

}  // namespace kpm
