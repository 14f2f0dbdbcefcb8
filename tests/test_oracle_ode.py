"""Pins of the oracle's integrators against closed forms and convergence orders."""

import math

import numpy as np
import pytest

from oracle import net, ode
from oracle.sample import simulate_event
from workload import configs, events, params


def _euler_product(alpha, beta, K, t0=0.0, t1=1.0):
    h = (t1 - t0) / K
    g = 1.0
    for k in range(K):
        g *= 1.0 + h * (alpha + beta * (t0 + k * h))
    return g


def _rk4_product(alpha, beta, K, t0=0.0, t1=1.0):
    """Growth factor of one classic RK4 run on x' = (alpha + beta t) x.

    With a = lam(t_k), m = lam(t_k + h/2), e = lam(t_k + h) the stage slopes are
    k1 = a, k2 = m (1 + h a/2), k3 = m (1 + h k2/2), k4 = e (1 + h k3) (times x), so one
    step multiplies x by 1 + h/6 (k1 + 2 k2 + 2 k3 + k4).
    """
    h = (t1 - t0) / K
    g = 1.0
    for k in range(K):
        t = t0 + k * h
        a, m, e = alpha + beta * t, alpha + beta * (t + h / 2), alpha + beta * (t + h)
        k1 = a
        k2 = m * (1 + h * k1 / 2)
        k3 = m * (1 + h * k2 / 2)
        k4 = e * (1 + h * k3)
        g *= 1 + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return g


def _midpoint_product(alpha, beta, K, t0=0.0, t1=1.0):
    """Growth factor of the explicit midpoint rule on x' = (alpha + beta t) x: one step
    multiplies x by 1 + h m (1 + h a / 2), a = lam(t_k), m = lam(t_k + h/2)."""
    h = (t1 - t0) / K
    g = 1.0
    for k in range(K):
        t = t0 + k * h
        a, m = alpha + beta * t, alpha + beta * (t + h / 2)
        g *= 1 + h * m * (1 + h * a / 2)
    return g


@pytest.mark.parametrize("scheme", [ode.EULER, ode.RK4, ode.MIDPOINT])
@pytest.mark.parametrize("K", [1, 3, 16, 50])
def test_linear_field_exact_product(scheme, K):
    alpha, beta = -0.7, 1.9
    x0 = np.array([[1.0, -2.0, 0.5]])
    x = ode.integrate(lambda x, t: (alpha + beta * t) * x, x0, scheme, K)
    g = {ode.EULER: _euler_product, ode.RK4: _rk4_product,
         ode.MIDPOINT: _midpoint_product}[scheme](alpha, beta, K)
    np.testing.assert_allclose(x, g * x0, rtol=1e-13)


def test_linear_field_converges_to_exponential_at_the_right_order():
    alpha, beta = 0.8, 1.1      # leading error terms of both schemes do not cancel here
    exact = math.exp(alpha + beta / 2)          # x(1) = x0 exp(int_0^1 alpha + beta t dt)
    x0 = np.ones((1, 1))
    errs = {}
    for scheme in (ode.EULER, ode.RK4, ode.MIDPOINT):
        errs[scheme] = [abs(ode.integrate(lambda x, t: (alpha + beta * t) * x, x0, scheme, K)[0, 0]
                            - exact) for K in (8, 16, 32, 64)]
    for a, b in zip(errs[ode.EULER], errs[ode.EULER][1:]):
        assert 0.85 < math.log2(a / b) < 1.15
    for a, b in zip(errs[ode.MIDPOINT], errs[ode.MIDPOINT][1:]):
        assert 1.85 < math.log2(a / b) < 2.15
    for a, b in zip(errs[ode.RK4], errs[ode.RK4][1:]):
        assert 3.7 < math.log2(a / b) < 4.3


def test_stage_times():
    assert ode.stage_times(ode.EULER, 4) == [0.0, 0.25, 0.5, 0.75]
    assert ode.stage_times(ode.RK4, 2) == [0.0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1.0]
    assert ode.stage_times(ode.MIDPOINT, 2) == [0.0, 0.25, 0.5, 0.75]
    with pytest.raises(ValueError):
        ode.integrate(lambda x, t: x, np.ones(1), ode.EULER, 0)


def test_time_dependence_enters_at_stage_times():
    """x' = t^3 integrates exactly by RK4 (Simpson) and to the left Riemann sum by Euler."""
    K = 5
    x = ode.integrate(lambda x, t: np.full_like(x, t ** 3), np.zeros(1), ode.RK4, K)
    assert math.isclose(x[0], 0.25, rel_tol=1e-14)
    xe = ode.integrate(lambda x, t: np.full_like(x, t ** 3), np.zeros(1), ode.EULER, K)
    assert math.isclose(xe[0], sum((k / K) ** 3 for k in range(K)) / K, rel_tol=1e-14)
    # midpoint: the midpoint quadrature sum of t^3
    xm = ode.integrate(lambda x, t: np.full_like(x, t ** 3), np.zeros(1), ode.MIDPOINT, K)
    assert math.isclose(xm[0], sum(((k + 0.5) / K) ** 3 for k in range(K)) / K, rel_tol=1e-14)


def _tiny_problem():
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, seed=0, perturbed=True)
    P = net.unpack(flat, cfg)
    off, feat = events.truth_events(1, ("fixed", 4), seed=5)
    x0 = np.random.default_rng(6).standard_normal((4, 9))
    return P, feat.astype(np.float64), x0


def test_convergence_orders_on_the_network():
    """Observed orders log2(e_K / e_2K) of Euler (1) and RK4 (4) on the real network."""
    P, u, x0 = _tiny_problem()
    v = lambda x, t: net.velocity(P, u, x, t)       # noqa: E731
    ref = ode.integrate(v, x0, ode.RK4, 512)
    e_euler = [np.abs(ode.integrate(v, x0, ode.EULER, K) - ref).max() for K in (64, 128, 256)]
    e_rk4 = [np.abs(ode.integrate(v, x0, ode.RK4, K) - ref).max() for K in (8, 16, 32)]
    p_euler = [math.log2(a / b) for a, b in zip(e_euler, e_euler[1:])]
    p_rk4 = [math.log2(a / b) for a, b in zip(e_rk4, e_rk4[1:])]
    assert all(0.8 < p < 1.2 for p in p_euler), p_euler
    assert all(3.4 < p < 4.6 for p in p_rk4), p_rk4


def test_zero_head_keeps_noise_and_bias_shifts_it():
    """W_out = 0: v is the constant b_out, so x_K = x0 + (t1 - t0) b_out for both schemes."""
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, seed=0)
    nm = params.named(cfg, flat)
    nm["W_out"][:] = 0.0
    nm["b_out"][:] = np.arange(9, dtype=np.float32) * 0.25 - 1.0
    P = net.unpack(flat, cfg)
    _, u, x0 = _tiny_problem()
    for scheme, K in ((ode.EULER, 7), (ode.RK4, 3)):
        x = simulate_event(P, u, x0, scheme, K)
        np.testing.assert_allclose(x, x0 + P["b_out"], rtol=1e-14, atol=1e-14)
