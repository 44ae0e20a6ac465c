"""Register budget of the marching strips: every strip kernel (moment sets,
propagator, FP32 arithmetic) keeps its level rings in registers, so a change
that pushes one of them into scratch memory slows it many times over without
changing its results.  The library build keeps the compiler's per-kernel
resource report; each strip kernel may spill at most a few registers."""
import pytest

from paper_1307_0288_amd import build as bld

MAX_SPILL = 8          # VGPRs spilled by any strip kernel


@pytest.mark.parametrize("src", ["kpm_kernels.hip", "kpm_march32.hip", "kpm_march_long.hip"])
def test_strip_kernels_keep_their_registers(src):
    res = bld.resources(src)
    if not res:
        pytest.skip(f"{src} not built here (run the library build first)")
    strips = {k: v for k, v in res.items() if "march" in k}
    assert strips, "no strip kernels in the report"
    worst = max(strips.items(), key=lambda kv: kv[1].get("VGPRs Spill", 0))
    assert worst[1].get("VGPRs Spill", 0) <= MAX_SPILL, worst
    # two wavefronts per SIMD at least (the strips' latency hiding)
    assert min(v.get("Occupancy", 0) for v in strips.values()) >= 2
