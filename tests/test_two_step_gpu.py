"""Several recursion steps per pass (kpm_launch.steps = 2 .. 8) on chain lattices.

The sizes leave ragged tiles in both directions (130 columns = 64 + 64 + 2,
26 or 38 chains = 16 + 10 or 16 + 16 + 6), odd moment counts leave a final
single step, and every geometry's boundary (periodic sheet, open-y ZGNR,
open-x AGNR) goes through the periodic-wrap indexing of the tiles.  The
recursion states are the single-step states exactly, so the moments agree
with the single-step path to summation-order rounding and with the oracle
to the parity bound."""
import numpy as np
import pytest

import oracle
from cases import gpu_system, onsite_bytes, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

SHAPES = [("sheet", 130, 26), ("zgnr", 130, 38), ("agnr", 132, 26), ("sheet", 200, 40)]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _log(msg):
    print(f"[two-step] {msg}", flush=True)


def _pair(c, precision="fp64", tiled=0, steps=2):
    """Systems on the same sample: single steps, and `steps` steps per pass in
    LDS tiles of 16 chains (tiled = 0, two steps), register tiles of 8
    (tiled = 1) or 4 (tiled = 2) chains, or marching strips of 16, 32 or 64
    chains (tiled = 3, 4, 5)."""
    one, two = gpu_system(c, precision), gpu_system(c, precision)
    kp.kpm_set_launch(one, 1, 4, 1, 0, 1, 0, 1)
    kp.kpm_set_launch(two, 1, 3, 1, 0, 1, tiled, steps)
    return one, two


MULTI = [(2, 0), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 2), (2, 3), (3, 4), (4, 3), (4, 4),
         (4, 5), (5, 3), (6, 4), (5, 5), (6, 5), (7, 5), (8, 5), (7, 3), (8, 4)]


# on-site terms stored as doubles (the generator's draw) or, for the
# float-exact variant of a case, as floats
ONSITE = ["f64", "f32"]


@pytest.mark.parametrize("onsite", ONSITE)
@pytest.mark.parametrize("geometry,nx,ny", SHAPES)
@pytest.mark.parametrize("nm", [101, 64])
@pytest.mark.parametrize("steps,tiled", MULTI)
def test_moments_match_oracle_and_single_step(geometry, nx, ny, nm, steps, tiled, onsite):
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.5, vac=0.02, seed=nx + ny, onsite=onsite)
    ob = onsite_bytes(c)
    _log(f"moments {geometry} {nx}x{ny} nm={nm} steps={steps} tiled={tiled} onsite={onsite}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    phi = phases(c, 1, 4400)
    d = one.upload(phi)
    kp.kpm_set_timing(two, True)
    kp.kpm_reset_stats(two)
    m2 = kp.kpm_moments(two, d, d, nm)[0]
    st = kp.kpm_get_stats(two)
    m1 = kp.kpm_moments(one, d, d, nm)[0]
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], nm)
    scale = np.vdot(phi, phi).real
    assert rel_err(m2, ref, scale) < 1e-10
    assert rel_err(m2, m1, scale) < 1e-13
    n = nx * ny
    # 5 state accesses of 16 B, pattern byte and on-site term per row
    assert st["step_bytes"] == n * (5 * 16 + 1 + ob)
    # full passes, then one pass of the 2 .. steps - 1 steps left, or one single step
    n2, r = divmod(nm - 2, steps)
    n2, n1 = (n2 + 1, 0) if r >= 2 else (n2, r)
    assert st["step_launches"] == n2 + n1
    assert st["step_bytes_total"] == n2 * st["step_bytes"] + n1 * n * (4 * 16 + 1 + ob)


@pytest.mark.parametrize("onsite", ONSITE)
@pytest.mark.parametrize("geometry,nx,ny", SHAPES[:3])
@pytest.mark.parametrize("steps,tiled", MULTI)
def test_distinct_left_vector_and_doubling(geometry, nx, ny, steps, tiled, onsite):
    _need_gpu()
    c = recipe(geometry, nx, ny, w=0.8, vac=0.01, seed=7 * nx + ny, onsite=onsite)
    _log(f"phi_L != phi_R and doubling {geometry} {nx}x{ny} steps={steps} tiled={tiled}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    pl, pr = phases(c, 1, 4500), phases(c, 1, 4501)
    lat = oracle_lattice(c)
    got = kp.kpm_moments(two, two.upload(pl), two.upload(pr), 77)[0]
    ref = oracle.moments(lat, c["e_scale"], pl[:, 0], pr[:, 0], 77)
    assert rel_err(got, ref, np.sqrt(np.vdot(pl, pl).real * np.vdot(pr, pr).real)) < 1e-10
    for nm in (100, 99, 103, 97):        # 2 steps x 2 slots per launch; 2-slot tails
        dbl = kp.kpm_moments_doubled(two, two.upload(pr), nm)[0]
        ref = oracle.moments(lat, c["e_scale"], pr[:, 0], pr[:, 0], nm)
        assert rel_err(dbl, ref, np.vdot(pr, pr).real) < 1e-10, nm


@pytest.mark.parametrize("steps,tiled", [(2, 0), (3, 1), (3, 3), (8, 5)])
def test_double_onsite_form(steps, tiled):
    """On-site energies that differ from floats only below float precision
    still take the width-3 compact form with double on-site terms."""
    _need_gpu()
    c = recipe("sheet", 130, 26, w=1.0, vac=0.02, seed=3, onsite="f32")
    c["onsite"] = c["onsite"] + 1e-9 * np.sin(np.arange(c["onsite"].size))
    _log(f"double on-site sheet 130x26 steps={steps} tiled={tiled}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    phi = phases(c, 1, 4650)
    d = one.upload(phi)
    kp.kpm_reset_stats(two)
    kp.kpm_set_timing(two, True)
    m2 = kp.kpm_moments(two, d, d, 70)[0]
    assert kp.kpm_get_stats(two)["step_bytes"] == 130 * 26 * (5 * 16 + 1 + 8)
    m1 = kp.kpm_moments(one, d, d, 70)[0]
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], 70)
    scale = np.vdot(phi, phi).real
    assert rel_err(m2, ref, scale) < 1e-10 and rel_err(m2, m1, scale) < 1e-13


@pytest.mark.parametrize("steps,tiled", [(2, 0), (4, 2), (4, 4)])
def test_fp32_states_equal_single_step(steps, tiled):
    _need_gpu()
    c = recipe("sheet", 130, 26, w=1.0, vac=0.02, seed=5)
    _log(f"fp32 states sheet 130x26 steps={steps}")
    one, two = _pair(c, "fp32", tiled, steps)
    phi = phases(c, 1, 4600)
    d = one.upload(phi)
    m1 = kp.kpm_moments(one, d, d, 90)[0]
    m2 = kp.kpm_moments(two, d, d, 90)[0]
    scale = np.vdot(phi, phi).real
    assert rel_err(m2, m1, scale) < 1e-12
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], 90)
    assert rel_err(m2, ref, scale) < 1e-4


@pytest.mark.parametrize("onsite", ONSITE)
@pytest.mark.parametrize("kind", ["vac", "msd", "msd_doubled"])
@pytest.mark.parametrize("steps,tiled", [(2, 0), (3, 2), (4, 3), (8, 5)])
def test_time_loops_with_two_step_moments(kind, steps, tiled, onsite):
    _need_gpu()
    c = recipe("sheet", 130, 26, w=1.0, vac=0.02, seed=9, onsite=onsite)
    _log(f"{kind} sheet 130x26 steps={steps}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    phi = phases(c, 1, 4700)
    fn = {"vac": kp.kpm_vac, "msd": kp.kpm_msd, "msd_doubled": kp.kpm_msd_doubled}[kind]
    got = fn(two, two.upload(phi), 3, 0.5, 20, 61)
    lat = oracle_lattice(c)
    ofn = oracle.vac if kind == "vac" else oracle.msd
    ref = ofn(lat, c["e_scale"], phi[:, 0], 3, 0.5, 20, 61)
    assert got.shape == (1, 4, 61)
    assert rel_err(got[0], ref) < 1e-10


@pytest.mark.parametrize("kind", ["vac", "msd"])
def test_resumed_loops_in_strips_equal_one_call(kind):
    """A VAC / MSD run split into two resumable calls gives, bit for bit, the
    moments of one uninterrupted call, with moments and both propagators in
    eight-step strips."""
    _need_gpu()
    c = recipe("zgnr", 130, 38, w=1.0, vac=0.02, seed=31)
    _log(f"resumed {kind} zgnr 130x38 steps=8")
    _, two = _pair(c, tiled=5, steps=8)
    phi = phases(c, 1, 5300)
    fn = kp.kpm_vac if kind == "vac" else kp.kpm_msd
    cont = kp.kpm_vac_continue if kind == "vac" else kp.kpm_msd_continue
    whole = np.asarray(fn(two, two.upload(phi), 4, 0.5, 20, 45)).reshape(5, 45)
    psi, r = two.upload(phi), two.new_state(1)
    first = np.asarray(cont(two, psi, r, True, 2, 0.5, 20, 45)).reshape(3, 45)
    rest = np.asarray(cont(two, psi, r, False, 2, 0.5, 20, 45)).reshape(2, 45)
    assert np.array_equal(np.concatenate([first, rest]), whole)


EVOLVE = [(2, 5), (3, 5), (5, 5), (6, 5), (8, 5), (7, 3), (8, 4)]


@pytest.mark.parametrize("onsite", ONSITE)
@pytest.mark.parametrize("geometry,nx,ny", SHAPES[:3])
@pytest.mark.parametrize("steps,tiled", EVOLVE)
def test_propagator_in_strips_equals_single_steps(geometry, nx, ny, steps, tiled, onsite):
    """U(+-dt) with the recursion in marching strips (Alg. 6 several steps per
    pass): the same states and accumulator as single steps, and the oracle's
    result; Bessel term counts leave full passes, a short last pass, a
    single last step, or no multi-step pass at all."""
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.2, vac=0.02, seed=3 * nx + ny, onsite=onsite)
    _log(f"propagator {geometry} {nx}x{ny} steps={steps} tiled={tiled}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    lat = oracle_lattice(c)
    for sign, nb, dt in ((1, 40, 1.0), (-1, 13, 0.3), (1, 11, 0.2), (1, 3, 0.2), (-1, 2, 0.05)):
        phi = phases(c, 1, 4950 + nb)
        ref = oracle.evolve(lat, c["e_scale"], phi[:, 0], dt, sign, nb)
        d1, d2 = one.upload(phi), two.upload(phi)
        kp.kpm_evolve(one, d1, dt, sign, nb)
        kp.kpm_evolve(two, d2, dt, sign, nb)
        g1, g2 = d1.cpu().numpy()[:, 0], d2.cpu().numpy()[:, 0]
        assert np.array_equal(g2, g1), (sign, nb)
        assert rel_err(g2, ref) < 1e-12, (sign, nb)


@pytest.mark.parametrize("onsite", ONSITE)
@pytest.mark.parametrize("geometry,nx,ny", SHAPES[:3])
@pytest.mark.parametrize("steps,tiled", [(2, 5), (3, 5), (8, 5), (5, 3), (4, 4)])
def test_commutator_propagator_in_strips_equals_single_steps(geometry, nx, ny, steps, tiled,
                                                            onsite):
    """[X, U(dt)] psi and U(dt) psi (Alg. 7) with up to three coupled steps per
    pass in marching strips: the same results as single steps, and the
    oracle's; term counts leave full passes, a short last pass, a single last
    step, or no multi-step pass."""
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.1, vac=0.02, seed=5 * nx + ny, onsite=onsite)
    _log(f"commutator propagator {geometry} {nx}x{ny} steps={steps} tiled={tiled}")
    one, two = _pair(c, tiled=tiled, steps=steps)
    lat = oracle_lattice(c)
    for nb, dt in ((40, 1.0), (12, 0.3), (9, 0.2), (4, 0.2), (3, 0.1), (2, 0.05)):
        phi = phases(c, 1, 5050 + nb)
        rx, ru = oracle.evolve_x(lat, c["e_scale"], phi[:, 0], dt, nb)
        outs = []
        for sysg in (one, two):
            d = sysg.upload(phi)
            ox, ou = sysg.new_state(1), sysg.new_state(1)
            kp.kpm_evolve_x(sysg, d, ox, ou, dt, nb)
            outs.append((ox.cpu().numpy()[:, 0], ou.cpu().numpy()[:, 0]))
        assert np.array_equal(outs[1][0], outs[0][0]) and np.array_equal(outs[1][1], outs[0][1]), nb
        assert rel_err(outs[1][0], rx) < 1e-12 and rel_err(outs[1][1], ru) < 1e-12, nb


@pytest.mark.parametrize("steps,tiled", [(5, 5), (8, 5)])
def test_propagator_in_strips_fp32(steps, tiled):
    _need_gpu()
    c = recipe("zgnr", 130, 38, w=1.0, vac=0.02, seed=23)
    _log(f"propagator fp32 zgnr 130x38 steps={steps}")
    one, two = _pair(c, "fp32", tiled, steps)
    phi = phases(c, 1, 4990)
    d1, d2 = one.upload(phi), two.upload(phi)
    kp.kpm_evolve(one, d1, 0.8, 1, 30)
    kp.kpm_evolve(two, d2, 0.8, 1, 30)
    assert np.array_equal(d2.cpu().numpy(), d1.cpu().numpy())
    ref = oracle.evolve(oracle_lattice(c), c["e_scale"], phi[:, 0], 0.8, 1, 30)
    assert rel_err(d2.cpu().numpy()[:, 0], ref) < 1e-5
    outs = []
    for sysg, d in ((one, d1), (two, d2)):
        ox, ou = sysg.new_state(1), sysg.new_state(1)
        kp.kpm_evolve_x(sysg, d, ox, ou, 0.8, 30)
        outs.append((ox.cpu().numpy(), ou.cpu().numpy()))
    assert np.array_equal(outs[1][0], outs[0][0]) and np.array_equal(outs[1][1], outs[0][1])


@pytest.mark.parametrize("steps,tiled", [(8, 5), (5, 3), (4, 1)])
def test_real_part_moment_sets_equal_complex_ones(steps, tiled):
    """The VAC takes its moments as real parts only (the strips then skip the
    imaginary parts): at t = 0 (R_0 = L_0 = V phi) they equal, bit for bit, the
    real parts of kpm_moments on V phi under the same launch shape."""
    _need_gpu()
    c = recipe("sheet", 200, 40, w=1.0, vac=0.02, seed=29)
    _log(f"real-part moments sheet 200x40 steps={steps} tiled={tiled}")
    _, two = _pair(c, tiled=tiled, steps=steps)
    phi = phases(c, 1, 5200)
    psi, r = two.upload(phi), two.new_state(1)
    got = kp.kpm_vac_continue(two, psi, r, True, 0, 0.5, 20, 91)
    ref = kp.kpm_moments(two, r, r, 91)
    assert np.array_equal(np.asarray(got).reshape(-1), ref.real.reshape(-1))


@pytest.mark.parametrize("steps,tiled", [(2, 0), (4, 1), (4, 4), (8, 5)])
def test_graph_replays_match_eager(steps, tiled):
    _need_gpu()
    c = recipe("zgnr", 130, 38, w=1.0, vac=0.02, seed=11)
    _log(f"graphs zgnr 130x38 steps={steps}")
    _, two = _pair(c, tiled=tiled, steps=steps)
    phi = phases(c, 1, 4800)
    d = two.upload(phi)
    eager = kp.kpm_moments(two, d, d, 151)[0]
    kp.kpm_set_graphs(two, True)
    for _ in range(3):
        rep = kp.kpm_moments(two, d, d, 151)[0]
        torch.cuda.synchronize()
        assert np.array_equal(rep, eager)
    kp.kpm_set_graphs(two, False)


def test_not_applicable_falls_back_to_single_steps():
    """Chains shorter than 68 rows, fewer than 24 chains and several vectors
    per row take single steps under steps > 1, with the same results."""
    _need_gpu()
    c = recipe("sheet", 48, 20, w=1.0, vac=0.02, seed=13)
    one, two = _pair(c)
    kp.kpm_set_launch(two, 1, 4, 1, 0, 1, 0, 2)
    phi = phases(c, 1, 4900)
    d = one.upload(phi)
    assert np.array_equal(kp.kpm_moments(one, d, d, 40), kp.kpm_moments(two, d, d, 40))
    for ny in (4, 10, 22):
        c = recipe("sheet", 130, ny, w=1.0, vac=0.02, seed=14)
        _log(f"fallback sheet 130x{ny}")
        one, two = _pair(c, tiled=5, steps=5)
        kp.kpm_reset_stats(two)
        kp.kpm_set_timing(two, True)
        phi = phases(c, 1, 4902)
        d = one.upload(phi)
        assert np.array_equal(kp.kpm_moments(one, d, d, 40), kp.kpm_moments(two, d, d, 40))
        assert kp.kpm_get_stats(two)["step_launches"] == 38
    c = recipe("sheet", 130, 26, w=1.0, vac=0.02, seed=13)
    one, two = _pair(c)
    kp.kpm_set_launch(one, 2, 4, 1, 0, 1, 0, 1)
    kp.kpm_set_launch(two, 2, 4, 1, 0, 1, 0, 2)
    phi = phases(c, 2, 4901)
    d = one.upload(phi)
    assert np.array_equal(kp.kpm_moments(one, d, d, 40), kp.kpm_moments(two, d, d, 40))


def test_autotune_considers_two_steps():
    _need_gpu()
    c = recipe("sheet", 512, 256, w=0.5, vac=0.005, seed=17)
    _log("autotune sheet 512x256")
    sysg = gpu_system(c)
    phi = phases(c, 1, 5000)
    d = sysg.upload(phi)
    best = kp.kpm_autotune(sysg, d, 20)
    assert best["steps"] in range(1, 7)
    got = kp.kpm_moments(sysg, d, d, 50)[0]
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], 50)
    assert rel_err(got, ref, np.vdot(phi, phi).real) < 1e-10


def test_doubling_form_has_its_own_shape():
    """kpm_set_launch sets both forms, kpm_set_launch_doubled only the doubling
    one; the autotuner picks each form's shape; moments stay correct."""
    _need_gpu()
    c = recipe("sheet", 200, 40, w=1.0, vac=0.02, seed=19)
    sysg = gpu_system(c)
    kp.kpm_set_launch(sysg, 1, 2, 1, 0, 1, 2, 4)
    kp.kpm_set_launch_doubled(sysg, 1, 3, 1, 0, 1, 3, 3)
    assert kp.kpm_get_launch(sysg, 1)["tiled"] == 2
    assert kp.kpm_get_launch_doubled(sysg, 1) == dict(groups_per_cu=3, ilp=1, streaming=0,
                                                      compact=1, tiled=3, steps=3)
    phi = phases(c, 1, 5100)
    d = sysg.upload(phi)
    ref = oracle.moments(oracle_lattice(c), c["e_scale"], phi[:, 0], phi[:, 0], 81)
    scale = np.vdot(phi, phi).real
    assert rel_err(kp.kpm_moments_doubled(sysg, d, 81)[0], ref, scale) < 1e-10
    assert rel_err(kp.kpm_moments(sysg, d, d, 81)[0], ref, scale) < 1e-10
    kp.kpm_autotune(sysg, d, 8)
    assert kp.kpm_get_launch_doubled(sysg, 1)["steps"] in range(1, 7)
    assert rel_err(kp.kpm_moments_doubled(sysg, d, 81)[0], ref, scale) < 1e-10
