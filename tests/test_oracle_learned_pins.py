"""Pins of the learned-estimator oracle (proposal MLP, histogram loss, Adam).

Checked against closed forms and hand-built networks whose output is known,
finite differences of the oracle's own forward, and the first-step closed
form of Adam -- never against a re-typed copy of the same formula.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

H = 16


def zero_params(H):
    return np.zeros(oracle.mlp_param_count(H), np.float32)


def views(p, H):
    o = 0
    W1 = p[o:o + 39 * H].reshape(H, 39); o += 39 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def test_zero_network_is_softplus_of_bias():
    p = zero_params(H)
    x = scenes.rng(1).uniform(-2, 2, (50, 3))
    assert np.allclose(oracle.mlp_fwd(x, p, H), math.log(2.0), rtol=0, atol=1e-15)
    views(p, H)[5][0] = 1.25
    assert np.allclose(oracle.mlp_fwd(x, p, H), math.log1p(math.exp(1.25)), rtol=1e-15)


@pytest.mark.parametrize("feature", [0, 2, 3, 4, 3 + 12 + 2 * 5, 3 + 24 + 2 * 3 + 1])
def test_hand_built_network_selects_one_feature(feature):
    # W1 picks one feature into unit 0, W2 passes unit 0, w3 reads unit 0:
    # sigma = softplus(relu(relu(gamma_f))) with gamma the documented encoding
    p = zero_params(H)
    W1, b1, W2, b2, w3, b3 = views(p, H)
    W1[0, feature] = 1.0
    W2[0, 0] = 1.0
    w3[0] = 1.0
    x = scenes.rng(2).uniform(-1.4, 1.4, (200, 3))
    s = oracle.mlp_fwd(x, p, H, scale=1.5)
    xh = x / 1.5
    if feature < 3:
        g = xh[:, feature]
    else:
        a, rem = divmod(feature - 3, 12)
        k, c = divmod(rem, 2)
        g = (np.cos if c else np.sin)(2.0 ** k * np.pi * xh[:, a])
    expect = np.log1p(np.exp(np.maximum(g, 0.0)))
    np.testing.assert_allclose(s, expect, rtol=1e-14, atol=1e-15)


def test_scene_contraction():
    # inside the unit ball the map is the identity (then halved); outside it
    # lands in the radius-2 ball and is continuous across the sphere
    p = zero_params(H)
    W1, _, W2, _, w3, _ = views(p, H)
    W1[0, 0] = 1.0  # reads x_hat_0
    W2[0, 0] = 1.0
    w3[0] = 1.0
    x = np.array([[0.6, 0, 0], [1.5, 0, 0], [3.0, 0, 0], [150.0, 0, 0], [1.5 * 1.0000001, 0, 0]])
    s = oracle.mlp_fwd(x, p, H, scale=1.5, contract=True)
    xh = np.log(np.expm1(s))  # invert softplus: recovers the positive feature
    np.testing.assert_allclose(xh[:3], [0.2, 0.5, 0.75], rtol=1e-12)
    assert 0.99 < xh[3] / 1.0 < 1.0
    assert abs(xh[4] - 0.5) < 1e-6


def test_bf16_rounding_points():
    # exact bfloat16 values pass; halfway cases round to even; one-bit cases round up
    p = zero_params(H)
    W1, _, W2, _, w3, _ = views(p, H)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    w3[0] = 1.0
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9])
    x = np.stack([vals * 1.5, np.zeros(4), np.zeros(4)], 1)
    s = oracle.mlp_fwd(x, p, H, scale=1.5, emulate_bf16=True)
    feat = np.log(np.expm1(s))
    np.testing.assert_allclose(feat, [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7], rtol=1e-12)


def test_mlp_gradient_matches_finite_differences():
    g = scenes.rng(3)
    p = (g.standard_normal(oracle.mlp_param_count(H)) * 0.3).astype(np.float32)
    x = g.uniform(-1.4, 1.4, (24, 3))
    ds = g.standard_normal(24)
    grad = oracle.mlp_bwd(x, p, H, ds, scale=1.5)
    idx = g.choice(p.size, 60, replace=False)
    for i in idx:
        # step exactly representable in float32 around p_i
        h = np.float32(2.0 ** -10)
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        f = lambda q: float(np.dot(ds, oracle.mlp_fwd(x, q, H, scale=1.5)))
        fd = (f(pp) - f(pm)) / (float(pp[i]) - float(pm[i]))
        assert grad[i] == pytest.approx(fd, rel=2e-4, abs=2e-6), i


def _bf16_rne(v):
    # independent bfloat16 round-to-nearest-even through the float32 bit pattern
    u = np.array([v], np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return float(u.astype(np.uint32).view(np.float32)[0])


def test_emulated_adjoint_rounds_hidden_adjoints():
    # one point, one active path: x_hat_0 = 1 -> a1 = 1 -> a2 = 1 -> z = w3 + b3.
    # d2 = dz w3 and d1 = W2 d2 are rounded to bfloat16 in the emulated adjoint;
    # the bias gradients expose them directly.
    p = zero_params(H)
    W1, b1, W2, b2, w3, b3 = views(p, H)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.5
    w3[0] = 0.75
    b2[0] = -0.5
    x = np.array([[1.5, 0.0, 0.0]])
    ds = np.array([0.3])
    z = 0.75 * (1.5 * 1.0 - 0.5)
    dz = 0.3 / (1.0 + math.exp(-z))
    g = oracle.mlp_bwd(x, p, H, ds, scale=1.5, emulate_bf16=True)
    gb1 = g[39 * H:40 * H]
    gb2 = g[40 * H + H * H:41 * H + H * H]
    d2 = _bf16_rne(dz * 0.75)
    assert d2 != dz * 0.75  # the case does exercise a rounding
    assert gb2[0] == d2
    assert gb1[0] == _bf16_rne(1.5 * d2)
    assert np.count_nonzero(gb2) == 1 and np.count_nonzero(gb1) == 1
    # unrounded in the binary64 adjoint
    g64 = oracle.mlp_bwd(x, p, H, ds, scale=1.5)
    assert g64[40 * H + H * H] == pytest.approx(dz * 0.75, rel=1e-15)


def test_adjoint_term_magnitudes():
    # the same point with opposite upstream gradients: the gradient cancels to
    # exactly zero while the magnitude doubles that of one point
    g = scenes.rng(8)
    p = (g.standard_normal(oracle.mlp_param_count(H)) * 0.3).astype(np.float32)
    x1 = g.uniform(-1.4, 1.4, (1, 3))
    one, one_abs = oracle.mlp_bwd(x1, p, H, [0.7], emulate_bf16=True, want_abs=True)
    np.testing.assert_array_equal(one_abs, np.abs(one))
    two, two_abs = oracle.mlp_bwd(np.concatenate([x1, x1]), p, H, [0.7, -0.7],
                                  emulate_bf16=True, want_abs=True)
    assert np.all(two == 0.0)
    np.testing.assert_array_equal(two_abs, 2 * np.abs(one))
    assert np.count_nonzero(one) > p.size // 4


def test_emulated_adjoint_near_binary64():
    # bfloat16 quantisation (weights, features, activations, adjoints, and the
    # ReLU masks of units that sit near zero) moves the gradient by a few percent
    g = scenes.rng(9)
    p = scenes.mlp_init(H, seed=4)
    x = g.uniform(-1.4, 1.4, (64, 3))
    ds = g.standard_normal(64)
    ge = oracle.mlp_bwd(x, p, H, ds, emulate_bf16=True)
    g64 = oracle.mlp_bwd(x, p, H, ds)
    assert np.linalg.norm(ge - g64) / np.linalg.norm(g64) < 0.1
    assert np.dot(ge, g64) / (np.linalg.norm(ge) * np.linalg.norm(g64)) > 0.995


def test_hist_loss_zero_when_proposal_bounds_target():
    # proposal = target on the same bins: every bound equals its weight
    n_bins = 8
    edges = np.linspace(0.0, 1.0, n_bins + 1).astype(np.float32)[None]
    w = np.array([0.1, 0.0, 0.3, 0.2, 0.05, 0.0, 0.15, 0.1], np.float32)
    info = np.array([[0, n_bins]], np.int32)
    loss, d = oracle.hist_loss(info, edges[0, :-1], edges[0, 1:], w, edges, w[None])
    assert loss[0] == 0.0 and np.all(d == 0.0)


def test_hist_loss_hand_cases():
    # one target interval (0.25, 0.5) with weight 0.5 over two proposal bins
    # [0, 0.5) and [0.5, 1): only bin 0 overlaps (touching ends do not)
    edges = np.array([[0.0, 0.5, 1.0]], np.float32)
    info = np.array([[0, 1]], np.int32)
    t0 = np.array([0.25], np.float32)
    t1 = np.array([0.5], np.float32)
    w = np.array([0.5], np.float32)
    wp = np.array([[0.2, 0.7]], np.float32)
    loss, d = oracle.hist_loss(info, t0, t1, w, edges, wp, eps=0.0)
    gap = 0.5 - np.float64(np.float32(0.2))
    assert loss[0] == pytest.approx(gap * gap / 0.5, rel=1e-12)
    assert d[0, 0] == pytest.approx(-2 * gap / 0.5, rel=1e-12) and d[0, 1] == 0.0
    # straddling interval (0.4, 0.6) is bounded by both bins: 0.9 > 0.5 -> no loss
    loss2, _ = oracle.hist_loss(info, np.float32([0.4]), np.float32([0.6]), w, edges, wp)
    assert loss2[0] == 0.0


def test_hist_loss_gradient_finite_differences():
    g = scenes.rng(4)
    n, nb = 6, 10
    counts = g.integers(1, 8, n).astype(np.int32)
    info, S = oracle.exclusive_scan(counts)
    t0 = np.concatenate([np.sort(g.uniform(0, 0.9, c)) for c in counts]).astype(np.float32)
    t1 = (t0 + g.uniform(0.01, 0.1, S)).astype(np.float32)
    w = g.uniform(0.0, 0.3, S).astype(np.float32)
    edges = np.sort(g.uniform(0, 1, (n, nb + 1)), 1).astype(np.float32)
    wp = g.uniform(0, 0.2, (n, nb)).astype(np.float64)
    loss, d = oracle.hist_loss(info, t0, t1, w, edges, wp)
    for r in range(n):
        for j in range(nb):
            h = 2.0 ** -12
            a, b = wp.copy(), wp.copy()
            a[r, j] += h
            b[r, j] -= h
            la = oracle.hist_loss(info, t0, t1, w, edges, a.astype(np.float32))[0].mean()
            lb = oracle.hist_loss(info, t0, t1, w, edges, b.astype(np.float32))[0].mean()
            fd = (la - lb) / (float(np.float32(a[r, j])) - float(np.float32(b[r, j])))
            assert d[r, j] == pytest.approx(fd, rel=1e-3, abs=1e-6)
    assert np.all(loss >= 0)


def test_adam_first_steps_closed_form():
    # with bias correction, m_hat = g and v_hat = g^2 at step 1, so the update is
    # lr * g / (|g| + eps); with a constant gradient the same holds at step 2
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = oracle.adam(p0, np.zeros(4), np.zeros(4), g, lr=0.1, eps=1e-15, step=1)
    np.testing.assert_allclose(p1, p0 - 0.1 * np.sign(g), rtol=1e-12)
    p2, _, _ = oracle.adam(p1, m, v, g, lr=0.1, eps=1e-15, step=2)
    np.testing.assert_allclose(p2, p0 - 0.2 * np.sign(g), rtol=1e-12)
