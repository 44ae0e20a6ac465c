"""Ragged batches (kpm_batch_create): several independent samples of different
size, geometry, disorder and E_s side by side in one system, each checked
against the oracle run on that sample alone."""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import oracle_lattice, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

SAMPLES = [
    ("sheet", 24, 12, 1.0, 0.02),
    ("zgnr", 30, 7, 0.5, 0.0),
    ("agnr", 9, 40, 2.0, 0.01),
    ("sheet", 64, 32, 1.0, 0.0),
    ("sheet", 8, 4, 0.0, 0.0),
    ("zgnr", 200, 5, 2.0, 0.03),
]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(n_vec, precision="fp64", samples=SAMPLES):
    cases = [recipe(g, nx, ny, w=w, vac=vac, seed=20 + s)
             for s, (g, nx, ny, w, vac) in enumerate(samples)]
    sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                   onsite=c["onsite"], active=c["active"],
                                   e_scale=c["e_scale"]) for c in cases], precision)
    phis = [ki.random_phase(c["nx"] * c["ny"], n_vec, 3000 + 100 * s, c["active"])
            for s, c in enumerate(cases)]
    return cases, sysg, phis


@pytest.fixture(scope="module")
def batch2():
    _need_gpu()
    cases, sysg, phis = _batch(2)
    lats = [oracle_lattice(c) for c in cases]
    return cases, sysg, phis, lats


def test_offsets(batch2):
    cases, sysg, phis, lats = batch2
    sizes = [c["nx"] * c["ny"] for c in cases]
    assert sysg.n_samples == len(cases)
    assert list(np.diff(sysg.offsets)) == sizes
    assert sysg.n_sites == sum(sizes)


def test_batch_moments_per_sample(batch2):
    cases, sysg, phis, lats = batch2
    nm = 150
    d = sysg.upload(np.concatenate(phis))
    got = kp.kpm_moments(sysg, d, d, nm)
    assert got.shape == (len(cases), 2, nm)
    for s, (c, lat) in enumerate(zip(cases, lats)):
        for r in range(2):
            ph = phis[s][:, r]
            ref = oracle.moments(lat, c["e_scale"], ph, ph, nm)
            scale = max(np.vdot(ph, ph).real, 1.0)
            assert rel_err(got[s, r], ref, scale) < 1e-10, (s, r)


def test_batch_vac_msd_per_sample(batch2):
    cases, sysg, phis, lats = batch2
    args = (2, 0.3, 25, 48)
    d = sysg.upload(np.concatenate(phis))
    gv = kp.kpm_vac(sysg, d, *args)
    gm = kp.kpm_msd(sysg, d, *args)
    for s, (c, lat) in enumerate(zip(cases, lats)):
        for r in range(2):
            rv = oracle.vac(lat, c["e_scale"], phis[s][:, r], *args)
            rm = oracle.msd(lat, c["e_scale"], phis[s][:, r], *args)
            assert rel_err(gv[s, r], rv) < 1e-10, (s, r)
            assert rel_err(gm[s, r], rm) < 1e-10, (s, r)


def test_batch_evolve_per_sample(batch2):
    cases, sysg, phis, lats = batch2
    d = sysg.upload(np.concatenate(phis))
    kp.kpm_evolve(sysg, d, 0.4, -1, 30)
    got = d.cpu().numpy()
    off = sysg.offsets
    for s, (c, lat) in enumerate(zip(cases, lats)):
        for r in range(2):
            ref = oracle.evolve(lat, c["e_scale"], phis[s][:, r], 0.4, -1, 30)
            assert rel_err(got[off[s]:off[s + 1], r], ref) < 1e-12, (s, r)


def test_batch_matches_single_systems():
    _need_gpu()
    cases, sysg, phis = _batch(8)
    d = sysg.upload(np.concatenate(phis))
    got = kp.kpm_moments(sysg, d, d, 100)
    for s, c in enumerate(cases):
        single = kp.graphene_system(c["nx"], c["ny"], c["geometry"], -2.7, c["onsite"],
                                    c["active"], c["e_scale"])
        ds = single.upload(phis[s])
        ref = kp.kpm_moments(single, ds, ds, 100)
        scale = max(float(np.abs(ref[:, 0]).max()), 1.0)
        assert rel_err(got[s], ref, scale) < 1e-13, s


def test_batch_fp32_close_to_fp64():
    _need_gpu()
    _, s64, phis = _batch(4, "fp64")
    _, s32, _ = _batch(4, "fp32")
    ph = np.concatenate(phis)
    a = kp.kpm_moments(s64, s64.upload(ph), s64.upload(ph), 200)
    b = kp.kpm_moments(s32, s32.upload(ph), s32.upload(ph), 200)
    for s in range(a.shape[0]):
        scale = max(float(np.abs(a[s, :, 0]).max()), 1.0)
        assert rel_err(b[s], a[s], scale) < 1e-5, s


def test_batch_launch_shapes_and_autotune():
    _need_gpu()
    cases, sysg, phis = _batch(8)
    d = sysg.upload(np.concatenate(phis))
    first = None
    for tiled in (0, 1):          # the 200-row zigzag chains of one sample are tiled
        ref = None
        for ilp in (1, 2, 4):
            for nt in (0, 1):
                for cp in (0, 1):
                    kp.kpm_set_launch(sysg, 8, 8, ilp, nt, cp, tiled)
                    mu = kp.kpm_moments(sysg, d, d, 30)
                    ref = mu if ref is None else ref
                    assert np.array_equal(mu, ref), (tiled, ilp, nt, cp)
        first = ref if first is None else first
        assert rel_err(ref, first, float(np.abs(first[..., 0]).max())) < 1e-13
    best = kp.kpm_autotune(sysg, d, 3)
    mu = kp.kpm_moments(sysg, d, d, 30)
    assert rel_err(mu, ref, float(np.abs(ref[..., 0]).max())) < 1e-13
    assert best["groups_per_cu"] in (4, 8, 16)


def test_graph_replays_match_eager():
    """Moment sets replayed from captured hipGraphs equal direct launches bit
    for bit, on every replay, with eager work and synchronisations between
    the replays (single system and batch; moments and the VAC loop)."""
    _need_gpu()
    cases, sysg, phis = _batch(2)
    d = sysg.upload(np.concatenate(phis))
    ref = kp.kpm_moments(sysg, d, d, 300)
    ref_v = kp.kpm_vac(sysg, d, 2, 0.3, 20, 64)
    kp.kpm_set_graphs(sysg, True)
    for rep in range(3):
        got = kp.kpm_moments(sysg, d, d, 300)
        assert np.array_equal(got, ref), rep
        got_v = kp.kpm_vac(sysg, d, 2, 0.3, 20, 64)
        assert np.array_equal(got_v, ref_v), rep
        e = d.clone()
        kp.kpm_evolve(sysg, e, 0.2, 1, 12)                 # eager work in between
        torch.cuda.synchronize()
    kp.kpm_set_graphs(sysg, False)
    assert np.array_equal(kp.kpm_moments(sysg, d, d, 300), ref)

    c = cases[3]
    single = kp.graphene_system(c["nx"], c["ny"], c["geometry"], -2.7, c["onsite"],
                                c["active"], c["e_scale"])
    ds = single.upload(phis[3])
    ref1 = kp.kpm_moments(single, ds, ds, 500)
    kp.kpm_set_graphs(single, True)
    for rep in range(3):
        assert np.array_equal(kp.kpm_moments(single, ds, ds, 500), ref1), rep
        torch.cuda.synchronize()


def test_batch_fourier_moments_per_sample(batch2):
    cases, sysg, phis, lats = batch2
    d = sysg.upload(np.concatenate(phis))
    nm, dtau = 6, 0.2
    got = kp.kpm_fourier_moments(sysg, d, d, nm, dtau, 20)
    for s, (c, lat) in enumerate(zip(cases, lats)):
        for r in range(2):
            ref = oracle.fourier_moments(lat, c["e_scale"], phis[s][:, r], phis[s][:, r], nm,
                                         dtau, 20)
            scale = max(np.vdot(phis[s][:, r], phis[s][:, r]).real, 1.0)
            assert rel_err(got[s, r], ref, scale) < 1e-10, (s, r)
