"""Several vectors with one vector per wavefront (kpm_launch.vectors_per_wave =
1): the library keeps its states vector-major and every launch sweeps all
vector planes, so the multi-step strips serve n_vec > 1.

Each vector's recursion states are those of the one-vector path exactly
(same operations in the same order), so propagated states equal the
rows-major single-step path bit for bit, moments agree with it to summation
order and with the oracle, per vector, to the parity bound.  Sizes leave
ragged strips (200 columns = 4 x 48 + 8) and strip lengths that do not divide
the chains (38 chains)."""
import numpy as np
import pytest

import oracle
from cases import gpu_system, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

ROWS = dict(groups_per_cu=4, ilp=1, streaming=0, compact=1, tiled=0, steps=1)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _log(msg):
    print(f"[planar] {msg}", flush=True)


def planar(steps=8, plane_groups=0, groups=2):
    return dict(groups_per_cu=groups, ilp=1, streaming=0, compact=1, tiled=5, steps=steps,
                vectors_per_wave=1, plane_groups=plane_groups)


def _pair(c, n_vec, shape, precision="fp64"):
    rows, plan = gpu_system(c, precision), gpu_system(c, precision)
    kp.kpm_set_launch(rows, n_vec, **ROWS)
    kp.kpm_set_launch(plan, n_vec, **shape)
    assert kp.kpm_get_launch(plan, n_vec)["vectors_per_wave"] == 1
    return rows, plan


CASES = [("sheet", 200, 38), ("zgnr", 200, 30), ("agnr", 132, 26)]


@pytest.mark.parametrize("geometry,nx,ny", CASES)
@pytest.mark.parametrize("n_vec", [2, 8, 64])
@pytest.mark.parametrize("steps,pg", [(8, 0), (8, 16), (5, 8), (2, 0)])
def test_moments_per_vector_match_oracle(geometry, nx, ny, n_vec, steps, pg):
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.2, vac=0.02, seed=nx + 3 * ny)
    _log(f"moments {geometry} {nx}x{ny} n_vec={n_vec} steps={steps} plane_groups={pg}")
    rows, plan = _pair(c, n_vec, planar(steps, pg))
    phi = phases(c, n_vec, 6100)
    d = plan.upload(phi)
    nm = 107
    got = kp.kpm_moments(plan, d, d, nm)
    one = kp.kpm_moments(rows, d, d, nm)
    lat = oracle_lattice(c)
    for r in sorted({0, n_vec // 2, n_vec - 1}):
        ref = oracle.moments(lat, c["e_scale"], phi[:, r], phi[:, r], nm)
        assert rel_err(got[r], ref, np.vdot(phi[:, r], phi[:, r]).real) < 1e-10, r
    scale = float(np.max(np.sum(np.abs(phi) ** 2, axis=0)))
    assert rel_err(got, one, scale) < 1e-13
    # the input is not modified and the doubling form agrees as well
    assert np.array_equal(d.cpu().numpy(), phi)
    dbl = kp.kpm_moments_doubled(plan, d, nm)
    assert rel_err(dbl, one, scale) < 1e-12


@pytest.mark.parametrize("n_vec", [2, 16])
def test_distinct_left_and_right_states(n_vec):
    _need_gpu()
    c = recipe("sheet", 200, 38, w=0.9, vac=0.01, seed=77)
    rows, plan = _pair(c, n_vec, planar(8, 0))
    pl, pr = phases(c, n_vec, 6200), phases(c, n_vec, 6300)
    got = kp.kpm_moments(plan, plan.upload(pl), plan.upload(pr), 90)
    one = kp.kpm_moments(rows, rows.upload(pl), rows.upload(pr), 90)
    scale = float(np.sqrt(np.max(np.sum(np.abs(pl) ** 2, axis=0)) *
                          np.max(np.sum(np.abs(pr) ** 2, axis=0))))
    assert rel_err(got, one, scale) < 1e-13
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], pl[:, 1], pr[:, 1], 90)
    assert rel_err(got[1], ref, scale) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("steps,pg", [(8, 0), (3, 24)])
def test_propagators_equal_rows_major_path(precision, steps, pg):
    """U(dt) (Alg. 6) and [X, U(dt)] with U(dt) (Alg. 7): vector-major strips
    against rows-major single steps, bit for bit, for term counts that leave
    full passes, a short last pass and no pass at all."""
    _need_gpu()
    c = recipe("zgnr", 200, 30, w=1.0, vac=0.02, seed=41)
    n_vec = 4
    _log(f"propagators {precision} steps={steps} plane_groups={pg}")
    rows, plan = _pair(c, n_vec, planar(steps, pg), precision)
    lat = oracle_lattice(c)
    for sign, nb, dt in ((1, 40, 1.0), (-1, 11, 0.3), (1, 2, 0.05)):
        phi = phases(c, n_vec, 6400 + nb)
        d1, d2 = rows.upload(phi), plan.upload(phi)
        kp.kpm_evolve(rows, d1, dt, sign, nb)
        kp.kpm_evolve(plan, d2, dt, sign, nb)
        assert np.array_equal(d2.cpu().numpy(), d1.cpu().numpy()), (sign, nb)
        if precision == "fp64":
            ref = oracle.evolve(lat, c["e_scale"], phi[:, 3], dt, sign, nb)
            assert rel_err(d2.cpu().numpy()[:, 3], ref) < 1e-12
        outs = []
        for sysg in (rows, plan):
            d = sysg.upload(phi)
            ox, ou = sysg.new_state(n_vec), sysg.new_state(n_vec)
            kp.kpm_evolve_x(sysg, d, ox, ou, dt, nb)
            outs.append((ox.cpu().numpy(), ou.cpu().numpy()))
        assert np.array_equal(outs[1][0], outs[0][0]) and np.array_equal(outs[1][1], outs[0][1])
        if precision == "fp64":
            rx, ru = oracle.evolve_x(lat, c["e_scale"], phi[:, 2], dt, nb)
            assert rel_err(outs[1][0][:, 2], rx) < 1e-12 and rel_err(outs[1][1][:, 2], ru) < 1e-12


@pytest.mark.parametrize("kind", ["vac", "msd", "msd_doubled"])
def test_time_loops_per_vector_match_oracle(kind):
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=43)
    n_vec = 4
    _log(f"{kind} n_vec={n_vec}")
    rows, plan = _pair(c, n_vec, planar(8, 0))
    phi = phases(c, n_vec, 6500)
    fn = {"vac": kp.kpm_vac, "msd": kp.kpm_msd, "msd_doubled": kp.kpm_msd_doubled}[kind]
    got = fn(plan, plan.upload(phi), 3, 0.5, 20, 61)
    one = fn(rows, rows.upload(phi), 3, 0.5, 20, 61)
    assert got.shape == one.shape == (n_vec, 4, 61)
    assert rel_err(got, one) < 1e-12
    ofn = oracle.vac if kind == "vac" else oracle.msd
    lat = oracle_lattice(c)
    for r in (0, 3):
        ref = ofn(lat, c["e_scale"], phi[:, r], 3, 0.5, 20, 61)
        assert rel_err(got[r], ref) < 1e-10, r


@pytest.mark.parametrize("kind", ["vac", "msd"])
def test_resumed_loops_equal_one_call(kind):
    """The resumable loops on the caller's (rows-major) buffers: a split run
    equals one call bit for bit, and the buffers hold the rows-major states."""
    _need_gpu()
    c = recipe("zgnr", 200, 30, w=1.0, vac=0.02, seed=47)
    n_vec = 2
    rows, plan = _pair(c, n_vec, planar(8, 0))
    phi = phases(c, n_vec, 6600)
    fn = kp.kpm_vac if kind == "vac" else kp.kpm_msd
    cont = kp.kpm_vac_continue if kind == "vac" else kp.kpm_msd_continue
    whole = np.asarray(fn(plan, plan.upload(phi), 4, 0.5, 20, 45))
    psi, r = plan.upload(phi), plan.new_state(n_vec)
    first = np.asarray(cont(plan, psi, r, True, 2, 0.5, 20, 45))
    rest = np.asarray(cont(plan, psi, r, False, 2, 0.5, 20, 45))
    assert np.array_equal(np.concatenate([first, rest], axis=1), whole)
    psi1, r1 = rows.upload(phi), rows.new_state(n_vec)
    cont(rows, psi1, r1, True, 4, 0.5, 20, 45)
    assert np.array_equal(psi.cpu().numpy(), psi1.cpu().numpy())
    assert np.array_equal(r.cpu().numpy(), r1.cpu().numpy())


def test_xu_state_and_fourier_moments():
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=53)
    n_vec = 2
    rows, plan = _pair(c, n_vec, planar(8, 0))
    phi = phases(c, n_vec, 6700)
    outs = [kp.kpm_xu_state(sysg, sysg.upload(phi), 3, 0.5, 20).cpu().numpy()
            for sysg in (rows, plan)]
    assert np.array_equal(outs[1], outs[0])
    f1 = kp.kpm_fourier_moments(rows, rows.upload(phi), rows.upload(phi), 6, 0.3, 15)
    f2 = kp.kpm_fourier_moments(plan, plan.upload(phi), plan.upload(phi), 6, 0.3, 15)
    assert rel_err(f2, f1) < 1e-13


def test_fp32_states_moments():
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=59)
    n_vec = 8
    rows, plan = _pair(c, n_vec, planar(8, 0), "fp32")
    phi = phases(c, n_vec, 6800)
    d = plan.upload(phi)
    got = kp.kpm_moments(plan, d, d, 120)
    one = kp.kpm_moments(rows, d, d, 120)
    scale = float(np.max(np.sum(np.abs(phi) ** 2, axis=0)))
    # the FP32 states are those of the rows-major path: only the FP64
    # summation order of the inner products differs
    assert rel_err(got, one, scale) < 1e-12
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 5], phi[:, 5], 120)
    assert rel_err(got[5], ref, scale) < 1e-4


def test_batches_take_vector_major_strips_only_when_every_sample_can():
    """A batch of chain lattices (every sample at least 68 x 24) keeps its
    states vector-major under such a shape and matches its single-step
    moments to summation order; with one sample too short for the strips the
    shape's vectors_per_wave is ignored and the moments are bit-identical."""
    _need_gpu()
    import kpm_inputs as ki

    def run(cases):
        sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                       onsite=c["onsite"], active=c["active"],
                                       e_scale=c["e_scale"]) for c in cases], "fp64")
        phi = np.concatenate([ki.random_phase(c["nx"] * c["ny"], 2, 3000 + 100 * s,
                                              c["active"]) for s, c in enumerate(cases)])
        d = sysg.upload(phi)
        ref = kp.kpm_moments(sysg, d, d, 60)
        kp.kpm_set_launch(sysg, 2, **planar(8, 16))
        got = kp.kpm_moments(sysg, d, d, 60)
        sysg.close()
        return got, ref

    strips = [recipe("sheet", 96, 30, w=1.0, vac=0.02, seed=60),
              recipe("zgnr", 100, 26, w=0.5, seed=61)]
    got, ref = run(strips)
    assert rel_err(got, ref, float(np.abs(ref[..., 0]).max())) < 1e-13
    got, ref = run(strips + [recipe("sheet", 80, 12, w=1.0, seed=62)])
    assert np.array_equal(got, ref)


def test_autotuner_considers_vector_major_strips():
    """The autotuner times vector-major strip shapes for several vectors on a
    chain lattice and keeps a shape whose moments still match the oracle."""
    _need_gpu()
    c = recipe("sheet", 400, 96, w=1.0, vac=0.02, seed=67)
    sysg = gpu_system(c)
    n_vec = 8
    phi = phases(c, n_vec, 6900)
    d = sysg.upload(phi)
    best = kp.kpm_autotune(sysg, d, 16)
    _log(f"autotuned shape for 8 vectors: {best}")
    assert best == kp.kpm_get_launch(sysg, n_vec)
    got = kp.kpm_moments(sysg, d, d, 80)
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 7], phi[:, 7], 80)
    assert rel_err(got[7], ref, np.vdot(phi[:, 7], phi[:, 7]).real) < 1e-10


def test_noalloc_keeps_rows_major_path():
    """kpm_moments_noalloc under a vector-major shape takes rows-major single
    steps in its fixed scratch: the same moments to summation order."""
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=71)
    rows, plan = _pair(c, 4, planar(8, 0))
    phi = phases(c, 4, 7000)
    d = plan.upload(phi)
    got = kp.kpm_moments_noalloc(plan, d, d, 70)
    one = kp.kpm_moments(plan, d, d, 70)
    scale = float(np.max(np.sum(np.abs(phi) ** 2, axis=0)))
    assert rel_err(got, one, scale) < 1e-13


def test_default_shape_for_several_vectors():
    """A one-sample graphene system starts several vectors in vector-major
    eight-step strips with about 1024 work-groups over all planes."""
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, seed=73)
    sysg = gpu_system(c)
    assert kp.kpm_get_launch(sysg, 1)["steps"] == 8
    assert "vectors_per_wave" not in kp.kpm_get_launch(sysg, 1)
    for n_vec in (2, 8, 64):
        assert kp.kpm_get_launch(sysg, n_vec) == planar(8, max(16, 1024 // n_vec))
    sysg.close()
    # a ribbon of 16 chains takes no strips: several vectors stay side by side
    r = recipe("zgnr", 200, 16, w=1.0, seed=74)
    rib = gpu_system(r)
    assert kp.kpm_get_launch(rib, 8).get("vectors_per_wave", 0) == 0
    rib.close()


@pytest.mark.parametrize("n_vec", [1, 8])
def test_fp32_arithmetic_strips(n_vec):
    """Precision fp32_arith (KPM_FP32): FP32 states with the strips' recursion
    levels in FP32 registers.  Moments, the propagator and the VAC / MSD loops
    agree with the FP32-states path (FP64 arithmetic) and with the oracle to
    single-precision rounding."""
    _need_gpu()
    c = recipe("sheet", 200, 38, w=1.0, vac=0.02, seed=79)
    s64 = gpu_system(c, "fp32")
    s32 = gpu_system(c, "fp32_arith")
    if n_vec > 1:
        for s in (s64, s32):
            kp.kpm_set_launch(s, n_vec, **planar(8, 0))
    phi = phases(c, n_vec, 7100)
    lat = oracle_lattice(c)
    scale = float(np.max(np.sum(np.abs(phi) ** 2, axis=0)))
    d = s32.upload(phi)
    got = kp.kpm_moments(s32, d, d, 150)
    assert rel_err(got, kp.kpm_moments(s64, d, d, 150), scale) < 1e-5
    ref = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], 150)
    assert rel_err(got[0], ref, scale) < 1e-4
    dbl = kp.kpm_moments_doubled(s32, d, 150)
    assert rel_err(dbl[0], ref, scale) < 1e-4
    e = s32.upload(phi)
    kp.kpm_evolve(s32, e, 1.0, 1, 40)
    ru = oracle.evolve(lat, c["e_scale"], phi[:, 0], 1.0, 1, 40)
    assert rel_err(e.cpu().numpy()[:, 0], ru) < 1e-5
    for fn, ofn in ((kp.kpm_vac, oracle.vac), (kp.kpm_msd, oracle.msd)):
        g = fn(s32, d, 2, 0.5, 20, 61)
        r = ofn(lat, c["e_scale"], phi[:, 0], 2, 0.5, 20, 61)
        assert rel_err(g[0], r) < 1e-4
    s32.close()
    s64.close()


@pytest.mark.parametrize("n_vec,precision", [(1, "fp64"), (8, "fp64"), (8, "fp32_arith")])
@pytest.mark.parametrize("group_size", [64, 128, 512])
def test_strip_group_sizes(n_vec, precision, group_size):
    """Strips in work-groups of 64, 128 and 512 threads: each wavefront walks
    its own strips, so propagated states equal the 256-thread groups' bit for
    bit and moments differ only in the order of the group partial sums."""
    _need_gpu()
    c = recipe("zgnr", 200, 30, w=1.0, vac=0.02, seed=83)
    base, other = gpu_system(c, precision), gpu_system(c, precision)
    g = 2 * 256 // group_size
    if n_vec == 1:
        kp.kpm_set_launch(base, 1, 2, 1, 0, 1, 5, 8)
        kp.kpm_set_launch(other, 1, g, 1, 0, 1, 5, 8, 0, 0, group_size)
    else:
        kp.kpm_set_launch(base, n_vec, **planar(8, 16))
        kp.kpm_set_launch(other, n_vec, **dict(planar(8, 16 * 256 // group_size), groups_per_cu=g,
                                               group_size=group_size))
    _log(f"group size {group_size}, n_vec={n_vec}, {precision}: {kp.kpm_get_launch(other, n_vec)}")
    phi = phases(c, n_vec, 7200)
    d = base.upload(phi)
    scale = float(np.max(np.sum(np.abs(phi) ** 2, axis=0)))
    m1, m2 = kp.kpm_moments(base, d, d, 130), kp.kpm_moments(other, d, d, 130)
    assert rel_err(m2, m1, scale) < 1e-13
    if precision == "fp64":
        ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], 130)
        assert rel_err(m2[0], ref, scale) < 1e-10
    e1, e2 = base.upload(phi), other.upload(phi)
    kp.kpm_evolve(base, e1, 1.0, -1, 40)
    kp.kpm_evolve(other, e2, 1.0, -1, 40)
    assert np.array_equal(e2.cpu().numpy(), e1.cpu().numpy())
    v1 = kp.kpm_vac(base, d, 2, 0.5, 20, 41)
    v2 = kp.kpm_vac(other, d, 2, 0.5, 20, 41)
    assert rel_err(v2, v1) < 1e-12
    base.close()
    other.close()


@pytest.mark.parametrize("n_vec", [1, 8])
def test_autotuner_axes(n_vec):
    """The autotuner's candidates cover work-group sizes 64 .. 512 and, for
    several vectors, both lane layouts (every vector of a row in adjacent lanes,
    one vector per wavefront); the shape it keeps gives the oracle's moments."""
    _need_gpu()
    c = recipe("sheet", 400, 96, w=1.0, vac=0.02, seed=89)
    sysg = gpu_system(c)
    cand = kp.kpm_autotune_candidates(sysg, n_vec)
    sizes = {cd.get("group_size", 0) or 256 for cd in cand}
    assert {64, 128, 256, 512} <= sizes
    layouts = {cd.get("vectors_per_wave", 0) for cd in cand}
    assert layouts == ({0, 1} if n_vec > 1 else {0})
    phi = phases(c, n_vec, 7300)
    d = sysg.upload(phi)
    best = kp.kpm_autotune(sysg, d, 16)
    _log(f"autotuned {n_vec} vector(s): {best}")
    assert best in cand or best == kp.kpm_get_launch(sysg, n_vec)
    got = kp.kpm_moments(sysg, d, d, 90)
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, -1], phi[:, -1], 90)
    assert rel_err(got[-1], ref, np.vdot(phi[:, -1], phi[:, -1]).real) < 1e-10
    sysg.close()
