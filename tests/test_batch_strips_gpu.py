"""Batches of chain lattices in the marching strips (Alg. 5 with several
recursion steps per pass): every sample of the batch is a periodic sheet or a
ribbon with at least 68-site chains and 24 chains, so the moment sets of the
whole batch advance K steps per launch, each work-group sweeping strips of its
own sample (its chain length, strip height, t / E_s and 1 / E_s from the
segment table).  Several vectors take one vector per wavefront (vector-major
states).  Each sample and vector is checked against the oracle run on that
sample alone; sizes leave ragged last strips in both directions."""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import oracle_lattice, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

# (geometry, nx, ny, W, vacancies): chains of 68 .. 200 sites, 24 .. 60 chains
SAMPLES = [
    ("sheet", 130, 26, 1.0, 0.01),
    ("zgnr", 100, 31, 0.5, 0.0),
    ("agnr", 90, 40, 2.0, 0.02),
    ("sheet", 200, 60, 0.0, 0.0),
    ("zgnr", 68, 24, 1.0, 0.0),
]


def _log(msg):
    print(msg, flush=True)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(n_vec, precision="fp64", onsite="f64", samples=SAMPLES):
    cases = [recipe(g, nx, ny, w=w, vac=vac, seed=40 + s, onsite=onsite)
             for s, (g, nx, ny, w, vac) in enumerate(samples)]
    sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                   onsite=c["onsite"], active=c["active"],
                                   e_scale=c["e_scale"]) for c in cases], precision)
    phis = [ki.random_phase(c["nx"] * c["ny"], n_vec, 3000 + 100 * s, c["active"])
            for s, c in enumerate(cases)]
    return cases, sysg, phis


def _strip_shape(n_vec, k, gs, pg):
    """kpm_set_launch arguments of a strip shape: one vector per row (n_vec = 1),
    or one vector per wavefront with pg groups per plane."""
    if n_vec == 1:
        return dict(groups_per_cu=8 * 64 // gs, ilp=1, streaming=0, compact=1, tiled=5,
                    steps=k, group_size=gs)
    return dict(groups_per_cu=2, ilp=1, streaming=0, compact=1, tiled=5, steps=k,
                vectors_per_wave=1, plane_groups=pg, group_size=gs)


def _check_moments(cases, phis, got, nm, n_vec, bar=1e-10):
    for s, c in enumerate(cases):
        lat = oracle_lattice(c)
        for r in range(n_vec):
            ph = phis[s][:, r]
            ref = oracle.moments(lat, c["e_scale"], ph, ph, nm)
            scale = max(np.vdot(ph, ph).real, 1.0)
            assert rel_err(got[s, r], ref, scale) < bar, (s, r)


@pytest.mark.parametrize("n_vec,k,gs,pg", [
    (1, 8, 64, 0), (1, 4, 256, 0),
    (2, 8, 64, 48), (2, 6, 256, 40), (8, 8, 64, 64), (8, 4, 256, 40),
])
def test_batch_strip_moments_vs_oracle(n_vec, k, gs, pg):
    _need_gpu()
    cases, sysg, phis = _batch(n_vec)
    kp.kpm_set_launch(sysg, n_vec, **_strip_shape(n_vec, k, gs, pg))
    _log(f"batch strips: {n_vec} vectors, {k} steps, groups of {gs}, {pg} groups per plane")
    d = sysg.upload(np.concatenate(phis))
    nm = 203                       # a tail pass after the full ones, and a partial ring
    got = kp.kpm_moments(sysg, d, d, nm)
    assert got.shape == (len(cases), n_vec, nm)
    _check_moments(cases, phis, got, nm, n_vec)


def test_batch_strips_float_onsite_and_doubling():
    """4-byte on-site terms (float-exact draw) and the doubling form in the
    strips, both against the oracle."""
    _need_gpu()
    cases, sysg, phis = _batch(8, onsite="f32")
    kp.kpm_set_launch(sysg, 8, **_strip_shape(8, 8, 64, 64))
    kp.kpm_set_launch_doubled(sysg, 8, **_strip_shape(8, 8, 64, 64))
    d = sysg.upload(np.concatenate(phis))
    nm = 160
    _check_moments(cases, phis, kp.kpm_moments(sysg, d, d, nm), nm, 8)
    _check_moments(cases, phis, kp.kpm_moments_doubled(sysg, d, nm), nm, 8)


def test_batch_strips_match_single_step_shape():
    """The strips' moments against the same batch's single-step launches."""
    _need_gpu()
    cases, sysg, phis = _batch(8)
    d = sysg.upload(np.concatenate(phis))
    kp.kpm_set_launch(sysg, 8, 8, 1, 1, 1, 0)
    ref = kp.kpm_moments(sysg, d, d, 300)
    kp.kpm_set_launch(sysg, 8, **_strip_shape(8, 8, 64, 64))
    got = kp.kpm_moments(sysg, d, d, 300)
    assert rel_err(got, ref, float(np.abs(ref[..., 0]).max())) < 1e-13


def test_batch_strips_vac_msd_vs_oracle():
    """VAC and MSD of a batch whose states are kept vector-major for the strips
    (the propagators run as single steps on the planes)."""
    _need_gpu()
    cases, sysg, phis = _batch(2)
    kp.kpm_set_launch(sysg, 2, **_strip_shape(2, 8, 64, 48))
    args = (2, 0.3, 25, 48)
    d = sysg.upload(np.concatenate(phis))
    gv = kp.kpm_vac(sysg, d, *args)
    gm = kp.kpm_msd(sysg, d, *args)
    for s, c in enumerate(cases):
        lat = oracle_lattice(c)
        for r in range(2):
            assert rel_err(gv[s, r], oracle.vac(lat, c["e_scale"], phis[s][:, r], *args)) < 1e-10
            assert rel_err(gm[s, r], oracle.msd(lat, c["e_scale"], phis[s][:, r], *args)) < 1e-10


def test_batch_strips_fp32_close_to_fp64():
    """FP32 states (FP64 arithmetic) and FP32 strip arithmetic within 1e-5 of
    FP64 on the same batch in the same shape."""
    _need_gpu()
    _, s64, phis = _batch(8, "fp64")
    ph = np.concatenate(phis)
    kp.kpm_set_launch(s64, 8, **_strip_shape(8, 8, 64, 64))
    a = kp.kpm_moments(s64, s64.upload(ph), s64.upload(ph), 200)
    for prec in ("fp32", "fp32_arith"):
        _, s32, _ = _batch(8, prec)
        kp.kpm_set_launch(s32, 8, **_strip_shape(8, 8, 64, 64))
        b = kp.kpm_moments(s32, s32.upload(ph), s32.upload(ph), 200)
        for s in range(a.shape[0]):
            scale = max(float(np.abs(a[s, :, 0]).max()), 1.0)
            assert rel_err(b[s], a[s], scale) < 1e-5, (prec, s)


def test_batch_autotune_visits_strips_and_graphs_replay():
    """The autotuner's candidates for a batch of chain lattices include the
    strips; its pick reproduces the oracle's moments, and hipGraph replays of
    the pick equal direct launches bit for bit."""
    _need_gpu()
    cases, sysg, phis = _batch(8)
    cand = kp.kpm_autotune_candidates(sysg, 8)
    strips = [c for c in cand if c.get("vectors_per_wave") == 1 and c["steps"] > 1]
    assert {c["steps"] for c in strips} >= {4, 8}
    assert {c.get("group_size", 0) for c in strips} >= {64, 256}
    d = sysg.upload(np.concatenate(phis))
    best = kp.kpm_autotune(sysg, d, 16)
    _log(f"autotuned batch shape: {best}")
    nm = 120
    ref = kp.kpm_moments(sysg, d, d, nm)
    _check_moments(cases, phis, ref, nm, 8)
    kp.kpm_set_graphs(sysg, True)
    for rep in range(3):
        assert np.array_equal(kp.kpm_moments(sysg, d, d, nm), ref), rep
        torch.cuda.synchronize()
    kp.kpm_set_graphs(sysg, False)


def test_batch_with_short_sample_keeps_single_steps():
    """A sample below the strips' 24 chains keeps the whole batch on single
    steps under a strip shape; the moments still match the oracle."""
    _need_gpu()
    samples = SAMPLES[:2] + [("sheet", 80, 12, 1.0, 0.0)]
    cases, sysg, phis = _batch(2, samples=samples)
    kp.kpm_set_launch(sysg, 2, **_strip_shape(2, 8, 64, 48))
    d = sysg.upload(np.concatenate(phis))
    nm = 90
    _check_moments(cases, phis, kp.kpm_moments(sysg, d, d, nm), nm, 2)


def test_many_samples_beyond_the_compact_form():
    """30 samples of 30 different chain lengths: their neighbour patterns hold
    sample-specific row offsets, too many for the compact form, while the
    strips' own pattern ids (the samples' shared (chain, column) steps) still
    cover them; every sample and vector against the oracle."""
    _need_gpu()
    geos = ("sheet", "zgnr", "agnr")
    samples = [(geos[s % 3], 68 + 4 * s, 24 + 2 * (s % 5), (0.5, 1.0, 2.0)[s % 3], 0.0)
               for s in range(30)]
    cases, sysg, phis = _batch(2, samples=samples)
    kp.kpm_set_launch(sysg, 2, **_strip_shape(2, 8, 64, 256))
    d = sysg.upload(np.concatenate(phis))
    nm = 100
    got = kp.kpm_moments(sysg, d, d, nm)
    _check_moments(cases, phis, got, nm, 2)
    kp.kpm_set_launch(sysg, 2, 8, 1, 1, 1, 0)          # single steps, rows side by side
    ref = kp.kpm_moments(sysg, d, d, nm)
    assert rel_err(got, ref, float(np.abs(ref[..., 0]).max())) < 1e-13
