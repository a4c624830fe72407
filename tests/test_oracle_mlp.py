"""Pins of the oracle's learned-guess network (CPU only).

The network is a heuristic, so it has no exact answer to compare with; the
oracle's forward, backward and Adam arithmetic are pinned instead by
  * the definition of bfloat16 round-to-nearest-even (hand-worked values),
  * a constructed network whose output is a known closed form,
  * invariance under a relabelling of hidden units,
  * central finite differences of the FP64 loss (backprop),
  * Adam's closed form after one and two steps from a zero state,
  * the textbook prim -> cons relations for the features and the inverse of
    the target transform.
"""
import math

import numpy as np
import pytest

from oracle import orc
from paper_2510_13965_amd import inputs as I

OFF = orc.MLP_OFF


def rand_params(seed, scale=0.3):
    r = np.random.default_rng(seed)
    p = np.zeros(orc.MLP_NBLOCK)
    p[:orc.MLP_NPARAM] = r.normal(0.0, scale, orc.MLP_NPARAM)
    p[OFF["mean"]:OFF["mean"] + 8] = r.normal(0.0, 1.0, 8)
    p[OFF["istd"]:OFF["istd"] + 8] = r.uniform(0.5, 2.0, 8)
    return p


def test_bf16_round_to_nearest_even():
    # ulp of bf16 at 1 is 2^-7; halfway cases go to the even neighbour
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -8, 1.0),                          # tie, 1.0 is even
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),          # tie between 1+2^-7 (odd) and 1+2^-6 (even)
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # just above the tie
        (-(1.0 + 2.0 ** -8 + 2.0 ** -20), -(1.0 + 2.0 ** -7)),
        (3.0 * 2.0 ** -130, 3.0 * 2.0 ** -130),          # subnormal with few bits stays exact
        (65280.0, 65280.0),                              # 0xff00 * 1: exact
        (float("inf"), float("inf")),
    ]
    got = orc.bf16([c[0] for c in cases])
    for (x, want), g in zip(cases, got):
        assert g == np.float32(want), (x, g, want)
    assert np.isnan(orc.bf16([float("nan")])[0])


def test_constructed_network_closed_form():
    """W1 routes feature k to hidden unit 2k+1 with gain (k+1); W2 is a
    non-symmetric permutation; W3 random: y = W3 P relu(W1 z) exactly."""
    p = np.zeros(orc.MLP_NBLOCK)
    W1 = np.zeros((64, 8))
    for k in range(8):
        W1[2 * k + 1, k] = k + 1.0
    perm = (np.arange(64) * 5 + 3) % 64   # h2[n] = h1[perm[n]]
    W2 = np.zeros((64, 64))
    W2[np.arange(64), perm] = 1.0
    r = np.random.default_rng(5)
    W3 = np.round(r.normal(size=(2, 64)) * 8) / 8    # exactly representable
    b3 = np.array([0.5, -0.25])
    p[OFF["W1"]:OFF["W1"] + 512] = W1.ravel()
    p[OFF["W2"]:OFF["W2"] + 4096] = W2.ravel()
    p[OFF["W3"]:OFF["W3"] + 128] = W3.ravel()
    p[OFF["b3"]:OFF["b3"] + 2] = b3
    p[OFF["mean"]:OFF["mean"] + 8] = 1.0
    p[OFF["istd"]:OFF["istd"] + 8] = 0.5
    X = np.array([[3.0, 5.0, -1.0, 9.0, 1.0, 2.0, 7.0, 0.0]], dtype=np.float32)
    z = (X[0] - 1.0) * 0.5
    h1 = np.zeros(64)
    for k in range(8):
        h1[2 * k + 1] = max((k + 1.0) * z[k], 0.0)
    h2 = h1[perm]
    want = W3 @ h2 + b3
    for em in (0, 1):
        Y = orc.mlp_forward(p, X, emulate=em)
        assert np.array_equal(Y[0], want), (em, Y, want)


def test_hidden_unit_relabelling_invariance():
    p = rand_params(11)
    r = np.random.default_rng(12)
    X = r.normal(size=(32, 8)).astype(np.float32)
    q = p.copy()
    s1 = r.permutation(64)
    s2 = r.permutation(64)
    W1 = p[OFF["W1"]:OFF["W1"] + 512].reshape(64, 8)
    b1 = p[OFF["b1"]:OFF["b1"] + 64]
    W2 = p[OFF["W2"]:OFF["W2"] + 4096].reshape(64, 64)
    b2 = p[OFF["b2"]:OFF["b2"] + 64]
    W3 = p[OFF["W3"]:OFF["W3"] + 128].reshape(2, 64)
    q[OFF["W1"]:OFF["W1"] + 512] = W1[s1].ravel()
    q[OFF["b1"]:OFF["b1"] + 64] = b1[s1]
    q[OFF["W2"]:OFF["W2"] + 4096] = W2[s2][:, s1].ravel()
    q[OFF["b2"]:OFF["b2"] + 64] = b2[s2]
    q[OFF["W3"]:OFF["W3"] + 128] = W3[:, s2].ravel()
    for em in (0, 1):
        Ya = orc.mlp_forward(p, X, emulate=em)
        Yb = orc.mlp_forward(q, X, emulate=em)
        assert np.allclose(Ya, Yb, rtol=1e-13, atol=1e-13), em


def test_gradient_matches_finite_differences():
    p = rand_params(21)
    r = np.random.default_rng(22)
    n = 6
    X = r.normal(size=(n, 8)).astype(np.float32)
    T = r.normal(size=(n, 2)).astype(np.float32)
    loss, g = orc.mlp_grad(p, X, T, emulate=0)
    idx = np.concatenate([r.choice(np.arange(OFF["W1"], OFF["W1"] + 512), 25),
                          r.choice(np.arange(OFF["b1"], OFF["b1"] + 64), 10),
                          r.choice(np.arange(OFF["W2"], OFF["W2"] + 4096), 40),
                          r.choice(np.arange(OFF["b2"], OFF["b2"] + 64), 10),
                          np.arange(OFF["W3"], OFF["W3"] + 128, 9), [OFF["b3"], OFF["b3"] + 1]])
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pm = p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = orc.mlp_grad(pp, X, T, emulate=0)
        lm, _ = orc.mlp_grad(pm, X, T, emulate=0)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # loss is the stated mean squared error
    Y = orc.mlp_forward(p, X, emulate=0)
    assert loss == pytest.approx(0.5 * np.sum((Y - T) ** 2) / n, rel=1e-12)


def test_emulated_gradient_close_to_fp64():
    """bf16 rounding perturbs the gradient by about the bf16 unit roundoff,
    not more (a misplaced rounding or a dropped term would show here)."""
    p = rand_params(31)
    r = np.random.default_rng(32)
    X = r.normal(size=(64, 8)).astype(np.float32)
    T = r.normal(size=(64, 2)).astype(np.float32)
    _, g0 = orc.mlp_grad(p, X, T, emulate=0)
    _, g1 = orc.mlp_grad(p, X, T, emulate=1)
    for name, lo, hi in (("W1", 0, 512), ("W2", 576, 4672), ("W3", 4736, 4864)):
        rel = np.linalg.norm(g1[lo:hi] - g0[lo:hi]) / np.linalg.norm(g0[lo:hi])
        assert 0 < rel < 3e-2, (name, rel)


def test_adam_closed_form():
    r = np.random.default_rng(41)
    n = orc.MLP_NPARAM
    p0 = r.normal(size=orc.MLP_NBLOCK)
    g1 = r.normal(size=n)
    g2 = r.normal(size=n)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-3
    p = p0.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    orc.mlp_adam(p, g1, m, v, 1, lr, b1, b2, eps)
    want1 = p0[:n] - lr * g1 / (np.abs(g1) + eps)
    assert np.allclose(p[:n], want1, rtol=1e-14, atol=1e-15)
    assert np.array_equal(p[n:], p0[n:])   # normalisation constants untouched
    orc.mlp_adam(p, g2, m, v, 2, lr, b1, b2, eps)
    mh = ((1 - b1) * b1 * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = ((1 - b2) * b2 * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    want2 = want1 - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(p[:n], want2, rtol=1e-13, atol=1e-15)


def test_features_textbook_flat_hydro():
    """Flat metric, B = 0: D = rho W, tau = rho h W^2 - p - D, S_i = rho h W^2 v_i
    (h the specific enthalpy), so q = tau/D and r^2 = (h W)^2 v^2."""
    rho, eps, Gam = 1e-4, 0.3, 2.0
    p = (Gam - 1) * rho * eps
    v = np.array([0.3, -0.2, 0.1])
    W = 1 / math.sqrt(1 - v @ v)
    hs = 1 + eps + p / rho
    D = rho * W
    tau = rho * hs * W * W - p - D
    S = rho * hs * W * W * v
    cons = np.array([D, 0.1 * D, tau, *S])
    gdn = np.array([1.0, 0, 0, 1.0, 0, 1.0])
    x = orc.mlp_features(cons, np.zeros(3), gdn, gdn)
    q = tau / D
    r2 = (hs * W) ** 2 * (v @ v)
    assert x[0] == pytest.approx(math.log10(D), rel=1e-14)
    assert x[1] == pytest.approx(math.log10(q), rel=1e-13)
    assert x[2] == pytest.approx(math.log10(r2), rel=1e-13)
    assert x[3] == pytest.approx(-30.0, rel=1e-12)
    assert x[4] == 0.0
    assert x[5] == pytest.approx(math.log10(1 + q), rel=1e-13)
    assert x[6] == pytest.approx(math.log10(r2 / (1 + q) ** 2), rel=1e-13)


def test_features_frame_invariant():
    """The features are scalars: an invertible change of spatial frame
    (gamma -> A^T gamma A, S_i -> A^T S, B^i -> A^-1 B) leaves them unchanged."""
    r = np.random.default_rng(51)
    G = np.eye(3) + 0.1 * r.normal(size=(3, 3))
    G = G @ G.T
    A = np.eye(3) + 0.3 * r.normal(size=(3, 3))
    cons = np.array([2e-4, 2e-5, 5e-5, 1e-5, -3e-5, 2e-5])
    B = np.array([1e-3, -2e-3, 5e-4])

    def pack(M):
        return np.array([M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]])

    x0 = orc.mlp_features(cons, B, pack(G), pack(np.linalg.inv(G)))
    G2 = A.T @ G @ A
    cons2 = cons.copy()
    cons2[3:] = A.T @ cons[3:]
    B2 = np.linalg.solve(A, B)
    x1 = orc.mlp_features(cons2, B2, pack(G2), pack(np.linalg.inv(G2)))
    assert np.allclose(x0, x1, rtol=1e-11, atol=1e-11), (x0, x1)


def test_targets_invert_to_roots():
    b = np.array([-0.3, 0.05])
    for mu in ([0.7, 0.3], [0.999, 0.5], [1e-3, 1e-3 * 0.25], [1.0, 1.0]):
        t = orc.mlp_targets(1.0, b, np.array(mu))
        assert np.exp(t[0] + b[0]) == pytest.approx(mu[0], rel=1e-14)
        assert np.exp(t[1] + b[1]) * mu[0] == pytest.approx(mu[1], rel=1e-14)
    t = orc.mlp_targets(2.0, np.zeros(2), np.array([0.25, 0.2]))
    assert t[0] == pytest.approx(math.log(0.5)) and t[1] == pytest.approx(math.log(0.8))


def _textbook_state(rho, eps, Gam, v_up, gdn3):
    """Undensitized (D, Y_e D, tau, S_i) of an ideal-gas fluid without field:
    D = rho W, S_i = rho h W^2 v_i, tau = rho h W^2 - p - D."""
    p = (Gam - 1) * rho * eps
    vd = gdn3 @ v_up
    W = 1 / math.sqrt(1 - v_up @ vd)
    hs = 1 + eps + p / rho
    D = rho * W
    return np.array([D, 0.1 * D, rho * hs * W * W - p - D, *(rho * hs * W * W * vd)]), p, hs, W


def test_baseline_exact_without_field():
    """App. D: with calB = 0, rbar(mu) = r for every mu, so the auxiliary root is
    mu_+ = 1/sqrt(h0^2 + r^2) and the first target (log fraction less the
    baseline) vanishes to the root solver's accuracy.  For a fluid at rest
    (r = 0, mu_+ = 1/h0) mu = 1/h while 1 + q = 1 + eps, so the second target is
    log((1 + eps)/h) in closed form.  The roots come from the oracle's own
    bracketed solver, so this also pins its auxiliary root."""
    e = orc.make_eos(I.EOS_IDEAL2)
    r = np.random.default_rng(61)
    def pack(M):
        return np.array([M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]])
    for n in range(40):
        G = np.eye(3) + 0.1 * r.normal(size=(3, 3))
        G = G @ G.T
        Gi = np.linalg.inv(G)
        rho = 10 ** r.uniform(-8, -3)
        eps = 10 ** r.uniform(-4, 0)
        still = n % 4 == 0
        v = np.zeros(3) if still else r.normal(size=3)
        if not still:
            v *= r.uniform(0.05, 0.95) / math.sqrt(v @ G @ v)
        cons, p, hs, W = _textbook_state(rho, eps, 2.0, v, G)
        _, prim, mu, _ = orc.c2p_point(e, cons, np.zeros(3), pack(G), pack(Gi), 1.0)
        b = orc.mlp_baseline(1.0, cons, pack(Gi))
        t = orc.mlp_targets(1.0, b, mu)
        assert abs(t[0]) <= 2e-14, (n, t)
        if still:
            assert t[1] == pytest.approx(math.log((1 + eps) / hs), rel=1e-10, abs=1e-14), (n, t)


def test_baseline_mu_plus_for_moving_fluid_flat():
    """Flat metric, B = 0, moving fluid: b0 = -log(1 + r^2)/2 with r = h W |v|
    (h0 = 1), written out from the textbook state."""
    cons, p, hs, W = _textbook_state(1e-4, 0.3, 2.0, np.array([0.3, -0.2, 0.1]), np.eye(3))
    gup = np.array([1.0, 0, 0, 1.0, 0, 1.0])
    b = orc.mlp_baseline(1.0, cons, gup)
    r2 = (hs * W) ** 2 * 0.14
    assert b[0] == pytest.approx(-0.5 * math.log(1 + r2), rel=1e-13)
    q = cons[2] / cons[0]
    assert b[1] == pytest.approx(-math.log(1 + q) + 0.5 * math.log(1 + r2), rel=1e-13)
