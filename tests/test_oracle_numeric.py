"""Pins of the floating-point oracles (saxpy, sum-reduce, N-body, cost-model MLP)
against exact arithmetic, closed forms, conservation laws and finite differences."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth


# ---------------------------------------------------------------- saxpy
def _round_f32(q: Fraction) -> np.float32:
    """Round an exact rational to the nearest float32, ties to even (brute force
    over the neighbours of a first guess)."""
    c = np.float32(float(q))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = None
    for x in cands:
        d = abs(Fraction(float(x)) - q)
        if best is None or d < best[0] or (d == best[0] and (x.view(np.uint32) & 1) == 0):
            best = (d, x)
    return best[1]


def test_saxpy_single_rounding_exact(orc):
    rng = np.random.default_rng(0)
    n = 3000
    v = synth.vector(1, n)
    w = synth.vector(2, n)
    # include cancellation-prone and tiny values
    v[:10] = np.float32(1.0) + np.float32(2 ** -23) * np.arange(10, dtype=np.float32)
    w[:10] = -v[:10]
    for a in (synth.saxpy_coeff(rng), np.float32(1.0), np.float32(-3.25)):
        out = orc.saxpy(v, w, a)
        for i in range(n):
            q = Fraction(float(np.float32(a))) * Fraction(float(v[i])) + Fraction(float(w[i]))
            assert out[i] == _round_f32(q), i


def test_saxpy_zero_coefficient(orc):
    v, w = synth.vector(3, 100), synth.vector(4, 100)
    assert (orc.saxpy(v, w, 0.0) == w).all()


def test_reverse(orc):
    v = synth.vector(5, 101)
    assert (orc.reverse(v) == v[::-1]).all()
    assert (orc.reverse(orc.reverse(v)) == v).all()


def test_f32_chain_order(orc):
    v, w1, w2 = synth.vector(6, 50), synth.vector(7, 50), synth.vector(8, 50)
    st = [("saxpy", {"a": 1.5}), ("mirror", {}), ("saxpy", {"a": -2.0})]
    out, (s, a) = orc.run_f32_chain(v, st, [w1, w2], "sum")
    ref = orc.saxpy(orc.reverse(orc.saxpy(v, w1, 1.5)), w2, -2.0)
    assert (out == ref).all()
    assert abs(s - math.fsum(float(x) for x in ref)) <= 1e-12 * a


# ------------------------------------------------------------------ sum
def test_sum_against_exact_fsum(orc):
    v = synth.vector(9, 200001)
    s, a = orc.sum_f32(v)
    exact = math.fsum(float(x) for x in v)
    assert abs(s - exact) <= 1e-12 * a
    assert a == pytest.approx(math.fsum(abs(float(x)) for x in v), rel=1e-12)


def test_sum_all_ones(orc):
    s, a = orc.sum_f32(np.ones(1 << 20, np.float32))
    assert s == float(1 << 20) and a == float(1 << 20)


# ---------------------------------------------------------------- N-body
def test_single_body_never_moves(orc):
    pos = np.array([[0.3, -0.2, 0.7, 1.1]], np.float32)
    acc = orc.nbody_accel(pos)
    assert (acc == 0).all()
    p, v = orc.nbody_run(pos, np.zeros((1, 4), np.float32), 5)
    assert (p == pos.astype(np.float64)).all() and (v == 0).all()


def test_two_body_closed_form_first_step(orc):
    d, m, eps, G, dt = 0.25, 0.8, 1e-2, 1.0, 1e-3
    pos = np.array([[-d, 0, 0, m], [d, 0, 0, m]], np.float64)
    acc = orc.nbody_accel(pos, G=G, eps=eps)
    r = 2 * d
    amag = G * m * r / (r * r + eps * eps) ** 1.5          # softened inverse square
    assert acc[0] == pytest.approx([amag, 0, 0], rel=1e-14, abs=0)
    assert acc[1] == pytest.approx([-amag, 0, 0], rel=1e-14, abs=0)
    p, v = orc.nbody_run(pos, np.zeros((2, 3)), 1, G=G, eps=eps, dt=dt)
    # kick then drift from rest: v = dt*a, x = x0 + dt*v
    assert v[0, 0] == pytest.approx(dt * amag, rel=1e-14)
    assert p[0, 0] == pytest.approx(-d + dt * dt * amag, rel=1e-14)


def test_unsoftened_limit_is_inverse_square(orc):
    pos = np.array([[0, 0, 0, 2.0], [3.0, 4.0, 0, 1.0]], np.float64)
    acc = orc.nbody_accel(pos, G=1.0, eps=1e-9)
    # |a_0| = G m_1 / r^2 toward body 1 (r = 5), Newton's third law for body 1
    assert acc[0] == pytest.approx(np.array([3.0, 4.0, 0]) / 5.0 * (1.0 / 25.0), rel=1e-12)
    assert 2.0 * acc[0] == pytest.approx(-1.0 * acc[1], rel=1e-12)


def test_two_equal_masses_stay_antisymmetric(orc):
    pos = np.array([[-0.3, 0.1, -0.2, 1.0], [0.3, -0.1, 0.2, 1.0]], np.float64)
    vel = np.array([[0.0, 0.5, 0.0], [0.0, -0.5, 0.0]])
    p, v = orc.nbody_run(pos, vel, 50)
    assert (p[0, :3] == -p[1, :3]).all() and (v[0] == -v[1]).all()


def test_symmetric_cross_centre_feels_no_force(orc):
    pts = [[0, 0, 0, 1.0]]
    for ax in range(3):
        for sgn in (-1, 1):
            q = [0.0, 0.0, 0.0, 0.7]
            q[ax] = 0.5 * sgn
            pts.append(q)
    acc = orc.nbody_accel(np.array(pts, np.float64))
    assert np.abs(acc[0]).max() < 1e-15


def test_momentum_and_centre_of_mass_conserved(orc):
    pos, vel = synth.nbody(31, 64)
    p0 = pos.astype(np.float64)
    m = p0[:, 3]
    com0 = (m[:, None] * p0[:, :3]).sum(0) / m.sum()
    p, v = orc.nbody_run(pos, vel, 20)
    mom = (m[:, None] * v).sum(0)
    scale = (m[:, None] * np.abs(v)).sum()
    assert np.abs(mom).max() <= 1e-12 * scale
    com = (m[:, None] * p[:, :3]).sum(0) / m.sum()
    assert np.abs(com - com0).max() < 1e-12


def test_far_field_monopole(orc):
    # A compact cluster seen from far away pulls like a point of its total mass.
    pos, _ = synth.nbody(32, 32)
    cl = pos.astype(np.float64)
    cl[:, :3] *= 1e-3
    probe = np.array([[100.0, 0, 0, 1e-6]])
    acc = orc.nbody_accel(np.vstack([cl, probe]))
    M = cl[:, 3].sum()
    assert acc[-1, 0] == pytest.approx(-M / 100.0 ** 2, rel=1e-4)


# ------------------------------------------------------------------- MLP
def _mlp():
    from oracle import mlp
    return mlp


def test_mlp_param_count():
    mlp = _mlp()
    assert mlp.N_PARAMS == 5825 == synth.mlp_init(0).size


def test_mlp_gradient_central_differences():
    mlp = _mlp()
    rng = np.random.default_rng(1)
    theta = synth.mlp_init(2)
    theta[1536:1600] = rng.uniform(-0.1, 0.1, 64)     # nonzero biases
    X = rng.normal(size=(40, 24))
    t = rng.normal(size=40)
    L, g = mlp.loss_and_grad(theta, X, t)
    assert L == pytest.approx(mlp.loss(theta, X, t), rel=1e-15)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss(tp, X, t) - mlp.loss(tm, X, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, k


def test_mlp_linear_regime_collapses_to_affine_map():
    mlp = _mlp()
    rng = np.random.default_rng(3)
    W1 = np.abs(rng.normal(size=(64, 24)))
    W2 = np.abs(rng.normal(size=(64, 64)))
    W3 = rng.normal(size=(1, 64))
    b1, b2, b3 = np.ones(64), np.ones(64), np.array([0.5])
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = np.abs(rng.normal(size=(10, 24)))            # every pre-activation positive
    y, _ = mlp.forward(theta, X)
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    assert y == pytest.approx((X @ A.T + c)[:, 0], rel=1e-12)
    # all-negative first layer: output is the constant W3 relu(b2) + b3
    theta2 = theta.copy()
    theta2[:1536] = -np.abs(theta2[:1536])
    theta2[1536:1600] = -1.0
    y2, _ = mlp.forward(theta2, X)
    assert y2 == pytest.approx(np.full(10, float((W3 @ np.maximum(b2, 0))[0] + b3[0])), rel=1e-14)


def test_adam_first_step_closed_form():
    mlp = _mlp()
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2  =>  step = lr * g / (|g| + eps)
    assert new == pytest.approx(th - 1e-3 * g / (np.abs(g) + 1e-8), rel=1e-14)


def test_mlp_training_lowers_loss_on_analytic_target():
    mlp = _mlp()
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, size=(512, 24))
    # t = log(bytes / BW + launches * c): a smooth synthetic runtime law
    t = np.log(np.exp(3 * X[:, 0]) + 0.5 * (1 + 4 * X[:, 1]))
    theta0 = synth.mlp_init(6)
    perms = [rng.permutation(512) for _ in range(60)]
    theta, hist = mlp.train(theta0, X, t, 60, 64, perms, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
