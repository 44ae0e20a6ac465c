"""kpm_moments_noalloc: the entry point whose scratch is the library's fixed
per-GPU device array (for callers that cannot allocate).  Its moments must
equal kpm_moments' on the same system, inputs and launch shape, on two calls
in a row, the second with a smaller input (the array keeps the first call's
contents), and sizes beyond the array are refused with an error."""
import numpy as np
import pytest

import oracle
from cases import gpu_system, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(c, nm, n_vec=1, precision="fp64", shape=None):
    sysg = gpu_system(c, precision)
    if shape is not None:
        kp.kpm_set_launch(sysg, n_vec, **shape)
    phi_h = phases(c, n_vec)
    d = sysg.upload(phi_h)
    print(f"noalloc case {c['geometry']} {c['nx']}x{c['ny']} n_vec={n_vec} {precision} "
          f"nm={nm} shape={kp.kpm_get_launch(sysg, n_vec)}", flush=True)
    got = kp.kpm_moments_noalloc(sysg, d, d, nm)
    ref = kp.kpm_moments(sysg, d, d, nm)
    return sysg, phi_h, got, ref


def test_two_calls_second_smaller_match_kpm_moments_and_oracle():
    _need_gpu()
    big = recipe("sheet", 256, 128, w=1.0, vac=0.01, seed=5)
    small = recipe("sheet", 64, 32, w=1.0, seed=6)
    for c, nm in ((big, 300), (small, 100)):
        sysg, phi_h, got, ref = _run(c, nm)
        assert got.shape == ref.shape == (1, nm)
        norm = float(np.vdot(phi_h, phi_h).real)
        # the same kernels, launch shape and partial layout: identical sums
        assert rel_err(got, ref, norm) <= 1e-15
        want = oracle.moments(oracle_lattice(c), c["e_scale"], phi_h[:, 0], phi_h[:, 0], nm)
        assert rel_err(got[0], want, norm) < 1e-10
        sysg.close()


def test_single_step_shape_several_vectors_and_fp32():
    _need_gpu()
    c = recipe("sheet", 64, 32, w=1.0, vac=0.02, seed=7)
    one = {"groups_per_cu": 4, "ilp": 2, "streaming": 0, "compact": 1, "tiled": 0, "steps": 1}
    for n_vec, prec, shape in ((4, "fp64", None), (1, "fp64", one), (2, "fp32", None)):
        sysg, phi_h, got, ref = _run(c, 120, n_vec, prec, shape)
        norm = float(np.max(np.sum(np.abs(phi_h) ** 2, axis=0)))
        assert rel_err(got, ref, norm) <= 1e-15
        sysg.close()


def test_ragged_batch():
    _need_gpu()
    import kpm_inputs as ki
    cases = [recipe("sheet", 24, 12, w=1.0, vac=0.02, seed=20),
             recipe("zgnr", 30, 7, w=0.5, seed=21)]
    sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                   onsite=c["onsite"], active=c["active"],
                                   e_scale=c["e_scale"]) for c in cases], "fp64")
    phi_h = np.concatenate([ki.random_phase(c["nx"] * c["ny"], 2, 3000 + 100 * s, c["active"])
                            for s, c in enumerate(cases)])
    d = sysg.upload(phi_h)
    got = kp.kpm_moments_noalloc(sysg, d, d, 80)
    ref = kp.kpm_moments(sysg, d, d, 80)
    assert got.shape == ref.shape == (2, 2, 80)
    assert np.array_equal(got, ref)
    sysg.close()


def test_batch_in_the_strips():
    """A batch whose samples are chain lattices: one vector takes the batch's
    eight-step strips on the fixed scratch array too (bit-equal to
    kpm_moments); two vectors run rows-major single steps there while
    kpm_moments keeps them vector-major in the strips."""
    _need_gpu()
    import kpm_inputs as ki
    cases = [recipe("sheet", 130, 26, w=1.0, vac=0.01, seed=22),
             recipe("agnr", 90, 40, w=2.0, seed=23)]
    sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                   onsite=c["onsite"], active=c["active"],
                                   e_scale=c["e_scale"]) for c in cases], "fp64")
    for n_vec in (1, 2):
        phi_h = np.concatenate([ki.random_phase(c["nx"] * c["ny"], n_vec, 3000 + 100 * s,
                                                c["active"]) for s, c in enumerate(cases)])
        d = sysg.upload(phi_h)
        got = kp.kpm_moments_noalloc(sysg, d, d, 150)
        ref = kp.kpm_moments(sysg, d, d, 150)
        assert got.shape == ref.shape == (2, n_vec, 150)
        if n_vec == 1:
            assert kp.kpm_get_launch(sysg, 1)["steps"] == 8
            assert rel_err(got, ref, float(np.abs(ref[..., 0]).max())) <= 1e-15
        else:
            assert rel_err(got, ref, float(np.abs(ref[..., 0]).max())) < 1e-13
    sysg.close()


def test_too_large_is_refused():
    _need_gpu()
    # 64 FP64 vectors on a 65536-site sheet need 2 x 64 MiB of states plus
    # partials and moments; 64 vectors on 262144 sites need 512 MiB of states
    c = recipe("sheet", 512, 512, w=1.0, seed=8)
    sysg = gpu_system(c)
    d = torch.zeros((c["nx"] * c["ny"], 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(kp.KpmError) as ei:
        kp.kpm_moments_noalloc(sysg, d, d, 10)
    assert "scratch" in str(ei.value)
    sysg.close()
