"""kpm_vac_msd: the VAC and MSD loops of one state in one call, their moment
sets at every t_k > 0 run as two vector planes of one launch sequence.  The
recursion states are those of kpm_vac and kpm_msd, so the moments equal theirs
up to the order of the inner-product sums, and the oracle's to the parity bar;
where the joint form does not apply (several vectors, batches, single-step
shapes) the call runs the two loops one after the other, with identical
results."""
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


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_arith"])
@pytest.mark.parametrize("geometry,nx,ny", [("sheet", 200, 38), ("zgnr", 130, 38),
                                             ("sheet", 68, 24)])
def test_joint_loops_equal_separate_calls_and_oracle(precision, geometry, nx, ny):
    """(68 x 24: the smallest lattice the strips take, whose ten-step windows
    of up to 44 chains wrap around the 24 chains of the periodic sheet.)"""
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.0, vac=0.02, seed=nx + ny)
    sysg = gpu_system(c, precision)
    phi = phases(c, 1, 7500)
    d = sysg.upload(phi)
    print(f"[vac_msd] {geometry} {nx}x{ny} {precision} {kp.kpm_get_launch(sysg, 1)}", flush=True)
    args = (3, 0.5, 20, 97)
    v2, m2 = kp.kpm_vac_msd(sysg, d, *args)
    v1, m1 = kp.kpm_vac(sysg, d, *args), kp.kpm_msd(sysg, d, *args)
    assert v2.shape == m2.shape == (1, 4, 97)
    assert np.all(m2[0, 0] == 0)
    assert rel_err(v2, v1) < 1e-12 and rel_err(m2, m1) < 1e-12
    assert np.array_equal(d.cpu().numpy(), phi.astype(d.cpu().numpy().dtype))
    if precision == "fp64":
        lat = oracle_lattice(c)
        assert rel_err(v2[0], oracle.vac(lat, c["e_scale"], phi[:, 0], *args)) < 1e-10
        assert rel_err(m2[0], oracle.msd(lat, c["e_scale"], phi[:, 0], *args)) < 1e-10
    sysg.close()


@pytest.mark.parametrize("case", ["joint", "two_vectors", "batch"])
def test_dos_vac_msd(case):
    """kpm_dos_vac_msd: the DOS moments <phi|T_m|phi> (real parts of
    kpm_moments) with kpm_vac_msd's VAC and MSD, in the joint form (DOS beside
    the VAC set of t_0) and where the sets run one after the other."""
    _need_gpu()
    args = (2, 0.5, 20, 93)
    if case == "batch":
        import kpm_inputs as ki
        cases = [recipe("sheet", 96, 30, w=1.0, vac=0.02, seed=80),
                 recipe("zgnr", 100, 26, w=0.5, seed=81)]
        sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                       onsite=c["onsite"], active=c["active"],
                                       e_scale=c["e_scale"]) for c in cases], "fp64")
        phi = np.concatenate([ki.random_phase(c["nx"] * c["ny"], 1, 3100 + 100 * s, c["active"])
                              for s, c in enumerate(cases)])
    else:
        c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=82)
        sysg = gpu_system(c)
        phi = phases(c, 2 if case == "two_vectors" else 1, 8200)
    d = sysg.upload(phi)
    dos, vac, msd = kp.kpm_dos_vac_msd(sysg, d, *args)
    v2, m2 = kp.kpm_vac_msd(sysg, d, *args)
    mu = kp.kpm_moments(sysg, d, d, args[-1])
    assert dos.shape == mu.shape and vac.shape == v2.shape
    assert rel_err(vac, v2) < 1e-12 and rel_err(msd, m2) < 1e-12
    assert rel_err(dos, mu.real) < 1e-12
    assert np.array_equal(d.cpu().numpy(), phi.astype(d.cpu().numpy().dtype))
    if case == "joint":
        lat = oracle_lattice(c)
        ref = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], args[-1])
        assert rel_err(dos[0], ref.real, np.vdot(phi, phi).real) < 1e-10
        assert np.all(msd[0, 0] == 0)
    sysg.close()


def test_joint_loops_float_onsite_and_long_tail():
    """The ten-step two-plane passes with 4-byte on-site terms (the float-exact
    draw), on a sheet whose chains end in a partial strip and whose moment
    count leaves a tail of nine steps in the last ring segment."""
    _need_gpu()
    c = recipe("sheet", 150, 30, w=1.0, vac=0.02, seed=71, onsite="f32")
    sysg = gpu_system(c)
    phi = phases(c, 1, 7100)
    d = sysg.upload(phi)
    args = (2, 0.5, 20, 101)             # 99 recursion steps: 9 ten-step passes and one of 9
    v2, m2 = kp.kpm_vac_msd(sysg, d, *args)
    v1, m1 = kp.kpm_vac(sysg, d, *args), kp.kpm_msd(sysg, d, *args)
    assert rel_err(v2, v1) < 1e-12 and rel_err(m2, m1) < 1e-12
    lat = oracle_lattice(c)
    assert rel_err(v2[0], oracle.vac(lat, c["e_scale"], phi[:, 0], *args)) < 1e-10
    assert rel_err(m2[0], oracle.msd(lat, c["e_scale"], phi[:, 0], *args)) < 1e-10
    sysg.close()


@pytest.mark.parametrize("case", ["two_vectors", "single_steps", "batch"])
def test_other_shapes_run_the_loops_in_turn(case):
    _need_gpu()
    args = (2, 0.5, 20, 61)
    if case == "batch":
        import kpm_inputs as ki
        cases = [recipe("sheet", 96, 30, w=1.0, vac=0.02, seed=60),
                 recipe("zgnr", 100, 26, w=0.5, seed=61)]
        sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                       onsite=c["onsite"], active=c["active"],
                                       e_scale=c["e_scale"]) for c in cases], "fp64")
        phi = np.concatenate([ki.random_phase(c["nx"] * c["ny"], 1, 3000 + 100 * s, c["active"])
                              for s, c in enumerate(cases)])
    else:
        c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=63)
        sysg = gpu_system(c)
        n_vec = 2 if case == "two_vectors" else 1
        if case == "single_steps":
            kp.kpm_set_launch(sysg, 1, 4, 1, 0, 1, 0, 1)
        phi = phases(c, n_vec, 7600)
    d = sysg.upload(phi)
    v2, m2 = kp.kpm_vac_msd(sysg, d, *args)
    assert np.array_equal(v2, kp.kpm_vac(sysg, d, *args))
    assert np.array_equal(m2, kp.kpm_msd(sysg, d, *args))
    sysg.close()


def test_widest_launches_are_timed_on_their_own():
    """kpm_get_stats splits out the runs of the widest launches: in the joint
    loops these are the two-plane moment sets of t_1 .. t_n (2 N rows per
    launch), the t_0 VAC set being a one-plane set."""
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, seed=7)
    sysg = gpu_system(c)
    d = sysg.upload(phases(c, 1, 7600))
    n = c["nx"] * c["ny"]
    kp.kpm_reset_stats(sysg)
    kp.kpm_set_timing(sysg, True)
    kp.kpm_vac_msd(sysg, d, 3, 0.5, 20, 97)
    st = kp.kpm_get_stats(sysg)
    kp.kpm_set_timing(sysg, False)
    assert st["wide_rows"] == st["step_rows"] == 2 * n
    # 97 moments (95 recursion steps after C_0, C_1): the one-plane t_0 set in
    # 11 eight-step passes and one of 7 steps, the two-plane sets in 9 ten-step
    # passes and one of 5 steps
    assert st["wide_launches"] == 3 * 10
    assert st["step_launches"] == 12 + 3 * 10
    assert 0 < st["wide_ms"] < st["step_ms"]
    sysg.close()


def test_joint_loops_replayed_from_graphs():
    """With hipGraph capture on, the joint call's moment sets (the one-plane
    t_0 set and the two-plane sets, one graph each, reused at every time step)
    replay bit-identical to direct launches, call after call."""
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=9)
    sysg = gpu_system(c)
    d = sysg.upload(phases(c, 1, 7700))
    args = (3, 0.5, 20, 97)
    ref = kp.kpm_vac_msd(sysg, d, *args)
    kp.kpm_set_graphs(sysg, True)
    for rep in range(3):
        got = kp.kpm_vac_msd(sysg, d, *args)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), rep
        e = d.clone()
        kp.kpm_evolve(sysg, e, 0.2, 1, 12)                 # eager work in between
        torch.cuda.synchronize()
    kp.kpm_set_graphs(sysg, False)
    sysg.close()
