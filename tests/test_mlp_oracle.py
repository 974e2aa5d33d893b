"""Pins of the learned-flux gradient oracle (CPU, FP64): backpropagation
against central finite differences, and the input/target normalisation on
special cases whose values follow by hand."""
import math

import numpy as np
import pytest

import oracle

G = 5.0 / 3.0


def _raw_samples(n, seed):
    rng = np.random.default_rng(seed)
    raw = np.zeros((n, 15))
    for s in range(n):
        qL = [rng.uniform(0.3, 3), rng.normal(0, 1), rng.normal(0, .5), rng.normal(0, .5), rng.uniform(.2, 3)]
        qR = [rng.uniform(0.3, 3), rng.normal(0, 1), rng.normal(0, .5), rng.normal(0, .5), rng.uniform(.2, 3)]
        qg, st, _ = oracle.riemann(qL, qR)
        raw[s, :5], raw[s, 5:10] = qL, qR
        raw[s, 10:] = [st["p"], st["u"], st["rhoL"], st["rhoR"], qg[0]]
    return raw


def _init(seed):
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.mlp_nparam())
    off = 0
    for nin, nout in ((10, 64), (64, 64), (64, 64), (64, 5)):
        lim = math.sqrt(6.0 / (nin + nout))
        P[off:off + nin * nout] = rng.uniform(-lim, lim, nin * nout)
        off += nin * nout
        P[off:off + nout] = rng.uniform(-0.1, 0.1, nout)
        off += nout
    assert off == P.size == 9349
    return P


def test_backprop_matches_central_differences():
    raw = _raw_samples(6, 1)
    x, y = oracle.mlp_normalize(raw)
    P = _init(2)
    loss, g = oracle.mlp_loss_grad(P, x, y)
    pat = oracle.mlp_relu_pattern(P, x)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(9349, 300, replace=False),
                          np.arange(640, 704), np.arange(9344, 9349)])
    checked = 0
    for i in idx:
        h = 1e-6 * max(1.0, abs(P[i]))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        if oracle.mlp_relu_pattern(Pp, x) != pat or oracle.mlp_relu_pattern(Pm, x) != pat:
            continue  # the perturbation crosses a ReLU kink
        lp, _ = oracle.mlp_loss_grad(Pp, x, y)
        lm, _ = oracle.mlp_loss_grad(Pm, x, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-7 * abs(g[i]), (i, fd, g[i])
        checked += 1
    assert checked > 300
    # forward consistency: the loss is the mean squared error of the forward pass
    yh = oracle.mlp_forward(P, x)
    assert loss == pytest.approx(((yh - y) ** 2).sum() / x.shape[0], rel=1e-14)


def test_normalisation_special_cases():
    # equal states at rest: rho and p normalise to 1 and 1/gamma, velocities to 0;
    # the solver returns p* = p, u* = u, so the pressure target is ln(1/gamma)
    q = [1.7, 0.0, 0.0, 0.0, 0.9]
    qg, st, _ = oracle.riemann(q, q)
    raw = np.array([q + q + [st["p"], st["u"], st["rhoL"], st["rhoR"], qg[0]]])
    x, y = oracle.mlp_normalize(raw)
    assert x[0] == pytest.approx([1, 0, 0, 0, 1 / G, 1, 0, 0, 0, 1 / G], abs=1e-14)
    assert y[0] == pytest.approx([math.log(1 / G), 0, 0, 0, 0], abs=1e-14)
    # a Galilean boost of both states shifts u and u* together: inputs unchanged
    r1 = _raw_samples(1, 9)[0]
    r2 = r1.copy()
    r2[[1, 6, 11]] += 2.5
    x1, y1 = oracle.mlp_normalize(r1[None])
    x2, y2 = oracle.mlp_normalize(r2[None])
    assert np.allclose(x1, x2, atol=1e-13) and np.allclose(y1, y2, atol=1e-13)
    # a uniform density / pressure rescaling (same sound speed) leaves x, y unchanged
    r3 = r1.copy()
    r3[[0, 5, 12, 13, 14]] *= 3.0
    r3[[4, 9, 10]] *= 3.0
    x3, y3 = oracle.mlp_normalize(r3[None])
    assert np.allclose(x1, x3, atol=1e-13) and np.allclose(y1, y3, atol=1e-13)


def test_training_domain_excludes_outlier_samples():
    # a face whose pressures sit at the floor (sound speeds ~ 1e-10) while its
    # velocities differ normalises to inputs far outside the training domain
    # (|x| > 64): it contributes nothing, and the loss stays normalised by the
    # batch size
    rng = np.random.default_rng(3)
    n = 40
    raw = np.zeros((n, 15))
    raw[:, 0] = rng.uniform(0.5, 2.0, n)
    raw[:, 1] = rng.normal(0, 0.3, n)
    raw[:, 4] = rng.uniform(0.5, 2.0, n)
    raw[:, 5] = rng.uniform(0.5, 2.0, n)
    raw[:, 6] = rng.normal(0, 0.3, n)
    raw[:, 9] = rng.uniform(0.5, 2.0, n)
    raw[:, 10] = 0.5 * (raw[:, 4] + raw[:, 9])
    raw[:, 11] = 0.5 * (raw[:, 1] + raw[:, 6])
    raw[:, 12:15] = raw[:, [0, 5, 0]]
    out = raw[:1].copy()
    out[0, 4] = out[0, 9] = 1e-20
    out[0, 1], out[0, 6] = 1.0, -1.0   # (u_L - ubar) / cbar ~ 1e10, finite
    x, y = oracle.mlp_normalize(raw)
    xo, yo = oracle.mlp_normalize(out)
    assert np.isfinite(xo).all() and np.abs(xo).max() > 64
    P = rng.normal(0, 0.1, 9349)
    l_in, g_in = oracle.mlp_loss_grad(P, x, y)
    l_all, g_all = oracle.mlp_loss_grad(P, np.vstack([x, xo]), np.vstack([y, yo]))
    assert l_all * (n + 1) == pytest.approx(l_in * n, rel=1e-12)
    assert np.allclose(g_all * (n + 1), g_in * n, rtol=1e-12, atol=1e-15)
