"""Learned moment-to-spectrum reconstruction on the GPU against the oracle's
float64 network (oracle/learned.py): forward pass, loss and gradients, Adam
steps, features and targets, the [X, U(t)] state that feeds the MSD moments,
and a small end-to-end training run.

Bars (FP32 network vs float64 oracle on the same float32 parameters and
inputs): outputs max|d| / max|ref| <= 2e-5; gradients per layer <= 1e-4; five
Adam steps (eps = 1e-3, a smooth update) parameters within 1e-4 of the
largest step; targets (FP64 KPM sums, float32 storage) <= 1e-6.
"""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from oracle import learned as ln
from cases import gpu_system, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

# widths not multiples of the 64 x 64 tiles or the 32-deep K chunks
SIZES = [37, 70, 45, 130]
# deep enough for products split over several K ranges (partials summed in order)
SIZES_SPLIT = [300, 200, 150, 96]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _log(msg):
    print(msg, flush=True)


def _net_and_data(sizes=SIZES, batch=33, seed=5):
    params = ki.mlp_init(sizes, seed)
    rng = np.random.default_rng(seed)
    params = [(w, (0.1 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64))
              for w, b in params]
    x = rng.standard_normal((batch, sizes[0])).astype(np.float32)
    y = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    net = kp.MLP(sizes, max_batch=max(64, batch))
    net.set_params(ln.flatten(params).astype(np.float32))
    return params, x, y, net


@pytest.mark.parametrize("sizes", [SIZES, SIZES_SPLIT])
def test_forward_matches_oracle(sizes):
    _need_gpu()
    params, x, y, net = _net_and_data(sizes)
    got = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = ln.forward(params, x.astype(np.float64))[-1]
    assert rel_err(got, ref) < 2e-5
    assert np.array_equal(net.get_params(), ln.flatten(params).astype(np.float32))


@pytest.mark.parametrize("batch,sizes", [(1, SIZES), (33, SIZES), (64, SIZES), (33, SIZES_SPLIT),
                                         (64, SIZES_SPLIT)])
def test_gradients_match_oracle(batch, sizes):
    _need_gpu()
    params, x, y, net = _net_and_data(sizes, batch=batch)
    loss, g = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    rl, rg = ln.loss_and_grads(params, x.astype(np.float64), y.astype(np.float64))
    assert loss == pytest.approx(rl, rel=1e-5)
    got = ln.unflatten(g.astype(np.float64), sizes)
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(got, rg)):
        assert rel_err(gw, rw) < 1e-4, l
        assert rel_err(gb, rb) < 1e-4, l


def test_full_size_network_matches_oracle():
    """The network of the learned workload (513 -> 1024 -> 1024 -> 2048, batch
    100, split-K products) against the oracle: outputs, loss and gradients."""
    _need_gpu()
    sizes = [513, 1024, 1024, 2048]
    params, x, y, net = _net_and_data(sizes, batch=100)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    got = net.forward(xd).cpu().numpy()
    acts = ln.forward(params, x.astype(np.float64))
    assert rel_err(got, acts[-1]) < 2e-5
    loss, g = net.gradients(xd, yd)
    rl, rg = ln.loss_and_grads(params, x.astype(np.float64), y.astype(np.float64))
    assert loss == pytest.approx(rl, rel=1e-5)
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(ln.unflatten(g.astype(np.float64), sizes), rg)):
        assert rel_err(gw, rw) < 1e-4, l
        assert rel_err(gb, rb) < 1e-4, l


@pytest.mark.parametrize("want_loss", [True, False])
def test_adam_steps_match_oracle(want_loss):
    """Five Adam steps, with the loss read back after each (a host sync) or
    not at all (the steps queue on the stream)."""
    _need_gpu()
    params, x, y, net = _net_and_data()
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    lr, eps = 1e-3, 1e-3
    state = ln.adam_init(params)
    ref = params
    for _ in range(5):
        loss = net.train_step(xd, yd, lr, 0.9, 0.999, eps, want_loss=want_loss)
        rl, rg = ln.loss_and_grads(ref, x.astype(np.float64), y.astype(np.float64))
        if want_loss:
            assert loss == pytest.approx(rl, rel=1e-4)
        else:
            assert loss is None
        ref, state = ln.adam_step(ref, rg, state, lr, eps=eps)
    got = net.get_params().astype(np.float64)
    moved = np.max(np.abs(ln.flatten(ref) - ln.flatten(params)))
    assert np.max(np.abs(got - ln.flatten(ref))) < 1e-4 * max(moved, lr)


def test_features_and_targets_match_oracle():
    _need_gpu()
    c = recipe("sheet", 32, 16, w=1.0, vac=0.01, seed=3)
    lat = oracle_lattice(c)
    es = 1.01 * (3 * 2.7 + 1.0)
    phi = phases(c, 2, 3000)
    mu = np.stack([oracle.moments(lat, es, phi[:, r], phi[:, r], 300) for r in range(2)])[None]
    cm = np.stack([oracle.msd(lat, es, phi[:, r], 3, 1.0, 30, 300)[3] for r in range(2)])[None]
    en = np.linspace(-7.5, 7.5, 129)
    y = kp.kpm_learned_targets(mu, cm, en, es, lat.area_nm2, 3.0)
    ref = ln.targets(mu, cm, en, es, lat.area_nm2, 3.0)
    assert rel_err(y[:, :129], ref[:, :129]) < 1e-6
    assert rel_err(y[:, 129:], ref[:, 129:]) < 1e-6
    x = kp.kpm_learned_features(mu, cm, 64)
    assert rel_err(x, ln.features(mu, cm, 64)) < 1e-6


def test_xu_state_gives_msd_moments():
    """Moments of [X, U(n dt)] phi equal row n of the MSD moments (Eq. 44)."""
    _need_gpu()
    c = recipe("sheet", 48, 20, w=1.0, vac=0.01, seed=9)
    sysg = gpu_system(c)
    lat = oracle_lattice(c)
    phi = phases(c, 2, 3000)
    d = sysg.upload(phi)
    y = kp.kpm_xu_state(sysg, d, 3, 0.8, 25)
    m = kp.kpm_moments_doubled(sysg, y, 100).real
    ref = oracle.msd(lat, c["e_scale"], phi[:, 1], 3, 0.8, 25, 100)[3]
    assert rel_err(m[1], ref) < 1e-10
    full = kp.kpm_msd(sysg, d, 3, 0.8, 25, 100)
    assert rel_err(m, full[:, 3]) < 1e-12


def test_small_training_run_learns():
    """Forty 32 x 16 sheets (W, vacancies varied), 64-moment features, 512-moment
    targets: training lowers the loss tenfold, and on eight held-out sheets the
    error is below that of predicting the mean training target (these 512-site
    spectra carry a large stochastic part that no feature predicts)."""
    _need_gpu()
    specs = ki.learned_sample_specs(48, 500)
    es = 1.01 * (3 * 2.7 + 1.0)
    nx, ny, nm, n_in = 32, 16, 512, 64
    en = np.linspace(-7.5, 7.5, 64)
    mus, cs = [], []
    for sp in specs:
        act = ki.vacancy_mask(nx * ny, sp["vac"], sp["vac_seed"])
        ons = ki.anderson_onsite(nx * ny, sp["w"], sp["onsite_seed"])
        sysg = kp.graphene_system(nx, ny, "sheet", -2.7, ons, act, es)
        d = sysg.upload(ki.random_phase(nx * ny, 4, sp["vec_seed"], act))
        mus.append(kp.kpm_moments_doubled(sysg, d, nm).real)
        cs.append(kp.kpm_moments_doubled(sysg, kp.kpm_xu_state(sysg, d, 4, 1.0, 35), nm).real)
        area = sysg.area_nm2
    mu, cm = np.stack(mus), np.stack(cs)
    x = kp.kpm_learned_features(mu, cm, n_in)
    y = kp.kpm_learned_targets(mu, cm, en, es, area, 4.0)
    sizes = [x.shape[1], 128, 128, y.shape[1]]
    net = kp.MLP(sizes, max_batch=40)
    net.set_params(ln.flatten(ki.mlp_init(sizes, 1)).astype(np.float32))
    xt, yt = torch.from_numpy(x[:40]).cuda(), torch.from_numpy(y[:40]).cuda()
    first = None
    for it in range(600):
        loss = net.train_step(xt, yt, 2e-3)
        first = loss if first is None else first
    assert loss < 0.1 * first
    pred = net.forward(torch.from_numpy(x[40:]).cuda()).cpu().numpy()
    err = np.mean((pred - y[40:]) ** 2)
    base = np.mean((y[:40].mean(axis=0) - y[40:]) ** 2)
    _log(f"held-out mse {err:.3e} vs mean-predictor {base:.3e}")
    assert err < 0.9 * base
