"""Pins of the oracle's learned-reconstruction network (oracle/learned.py):
gradients against central finite differences, a linear model trained by
gradient descent against the least-squares solution (numpy.linalg.lstsq),
Adam's first step (-lr g / (|g| + eps) after bias correction, Kingma and Ba),
invariance under a permutation of hidden units, tanh saturation, and the
normalisation of the features and targets."""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from oracle import learned as ln


def _tiny(sizes=(5, 4, 3), seed=7):
    return ki.mlp_init(list(sizes), seed)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = _tiny((5, 6, 4, 3))
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((7, 5))
    y = rng.standard_normal((7, 3))
    _, grads = ln.loss_and_grads(params, x, y)
    flat = ln.flatten(params)
    gflat = ln.flatten(grads)
    sizes = [5, 6, 4, 3]
    h = 1e-6
    num = np.zeros_like(flat)
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = ln.loss_and_grads(ln.unflatten(flat + e, sizes), x, y)
        lm, _ = ln.loss_and_grads(ln.unflatten(flat - e, sizes), x, y)
        num[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(num - gflat)) < 1e-8 * max(1.0, np.max(np.abs(gflat)))


def test_linear_model_descends_to_least_squares():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((40, 3))
    y = x @ np.array([[1.0, -2.0], [0.5, 0.0], [3.0, 1.0]]) + np.array([0.2, -0.1]) \
        + 0.05 * rng.standard_normal((40, 2))
    params = [(np.zeros((2, 3)), np.zeros(2))]
    for _ in range(4000):
        _, g = ln.loss_and_grads(params, x, y)
        params = [(params[0][0] - 1.0 * g[0][0], params[0][1] - 1.0 * g[0][1])]
    design = np.concatenate([x, np.ones((40, 1))], axis=1)
    sol = np.linalg.lstsq(design, y, rcond=None)[0]
    assert np.allclose(params[0][0], sol[:3].T, atol=1e-9)
    assert np.allclose(params[0][1], sol[3], atol=1e-9)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    params = _tiny()
    x, y = rng.standard_normal((4, 5)), rng.standard_normal((4, 3))
    _, grads = ln.loss_and_grads(params, x, y)
    lr, eps = 1e-2, 1e-8
    new, state = ln.adam_step(params, grads, ln.adam_init(params), lr, eps=eps)
    for (w, b), (gw, gb), (nw, nb) in zip(params, grads, new):
        assert np.allclose(nw - w, -lr * gw / (np.abs(gw) + eps), rtol=1e-9, atol=1e-15)
        assert np.allclose(nb - b, -lr * gb / (np.abs(gb) + eps), rtol=1e-9, atol=1e-15)
    assert state[0] == 1


def test_hidden_permutation_invariance():
    """Relabelling hidden units (rows of W_0 and b_0, columns of W_1) changes
    neither the output nor the loss, and permutes the gradients alike."""
    rng = np.random.default_rng(3)
    params = _tiny((5, 6, 3))
    params = [(w, rng.standard_normal(b.shape)) for w, b in params]
    perm = rng.permutation(6)
    (w0, b0), (w1, b1) = params
    pp = [(w0[perm], b0[perm]), (w1[:, perm], b1)]
    x, y = rng.standard_normal((9, 5)), rng.standard_normal((9, 3))
    assert np.allclose(ln.forward(params, x)[-1], ln.forward(pp, x)[-1], rtol=1e-13, atol=1e-14)
    l1, g1 = ln.loss_and_grads(params, x, y)
    l2, g2 = ln.loss_and_grads(pp, x, y)
    assert l1 == pytest.approx(l2, rel=1e-13)
    assert np.allclose(g1[0][0][perm], g2[0][0]) and np.allclose(g1[1][0][:, perm], g2[1][0])


def test_saturated_hidden_layer():
    """Huge biases saturate tanh at +-1: the output is W_1 sign(b_0) + b_1."""
    w0 = np.zeros((4, 2))
    b0 = np.array([50.0, -50.0, 50.0, 50.0])
    w1 = np.arange(12.0).reshape(3, 4)
    b1 = np.array([1.0, 2.0, 3.0])
    out = ln.forward([(w0, b0), (w1, b1)], np.ones((2, 2)))[-1]
    assert np.allclose(out, w1 @ np.sign(b0) + b1)


def test_feature_and_target_normalisation():
    """Features are moment ratios; the DOS target integrates to DOS_SCALE over
    the band (Eq. 29 normalisation); the sigma target is SIGMA_SCALE times
    sigma_E2 (Eq. 11) of the same moments at t*."""
    lat = oracle.graphene(16, 8, "sheet", -2.7, ki.anderson_onsite(128, 1.0, 5))
    es = 1.01 * (3 * 2.7 + 1.0)
    phi = ki.random_phase(128, 2, 3000)
    mu = np.stack([oracle.moments(lat, es, phi[:, r], phi[:, r], 400) for r in range(2)])[None]
    m = np.stack([oracle.msd(lat, es, phi[:, r], 4, 1.0, 30, 400) for r in range(2)])[None]
    c = m[:, :, 4]                                   # moments at t* = 4 fs
    x = ln.features(mu, c, 32)
    assert x.shape == (1, 65)
    assert x[0, 0] == 1.0 and x[0, 32] == 1.0
    assert x[0, 64] == pytest.approx(np.log(c.mean(axis=1)[0, 0] / mu.real.mean(axis=1)[0, 0]))
    en = np.linspace(-0.999 * es, 0.999 * es, 40001)
    y = ln.targets(mu, c, en, es, lat.area_nm2, 4.0)
    integral = np.trapezoid(y[0, :en.size], en) / ln.DOS_SCALE
    assert integral == pytest.approx(1.0, abs=2e-3)
    rho_x2 = oracle.kpm_sum(m.mean(axis=1)[0], en[::100], es, lat.area_nm2)
    s_e2 = oracle.sigma_e2(rho_x2, 1.0)[4]
    y2 = ln.targets(mu, c, en[::100], es, lat.area_nm2, 4.0)
    assert np.allclose(y2[0, en[::100].size:], ln.SIGMA_SCALE * s_e2, rtol=1e-12)
