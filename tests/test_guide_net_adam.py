"""Pins of the FP64 reference Adam step (Kingma and Ba, "Adam: a method for
stochastic optimization", ICLR 2015, Algorithm 1) that trains the guide.

What fixes each expected value (none of it is the reference's own formula):
  * first step: both moment estimates are exactly unbiased after the bias
    correction, so every parameter moves by -lr g / (|g| + eps) (Sec. 2:
    m-hat = g, v-hat = g^2 at t = 1);
  * a constant gradient: m-hat = g and v-hat = g^2 at every step (the bias
    correction divides out 1 - beta^t exactly, Sec. 3), so after T steps every
    parameter has moved by -T lr g / (|g| + eps);
  * a hand-worked two-step case: g = 1 then g = -2, lr = 0.1, eps = 0, worked
    out in exact decimals (m_2 = -0.11, v_2 = 0.004999, m-hat = -11/19,
    v-hat = 4999/1999, so the second step is +0.0366103527035845565...);
  * scale invariance (Sec. 2.1): with eps = 0, multiplying every gradient by
    c > 0 leaves the trajectory unchanged;
  * eps enters outside the square root: a gradient of 1e-8 with eps = 1e-8
    moves a parameter by lr / 2 on the first step.

Each pin is a function of the implementation, so the planted-mistake test can
run the same pins against altered copies of the reference.
"""
import numpy as np
import pytest

from oracle import guide_net as ref


def run_steps(adam, grads, lr, b1=0.9, b2=0.999, eps=1e-8, theta0=None):
    g0 = np.asarray(grads[0], np.float64)
    theta = np.zeros_like(g0) if theta0 is None else np.array(theta0, np.float64)
    m = np.zeros_like(g0)
    v = np.zeros_like(g0)
    path = [theta.copy()]
    for t, g in enumerate(grads, start=1):
        theta, m, v = adam(theta, m, v, np.asarray(g, np.float64), t, lr, b1, b2, eps)
        path.append(theta.copy())
    return np.array(path)


def pin_first_step(adam):
    g = np.array([3.0, -0.5, 1e-3, -7e-6, 0.0])
    th0 = np.array([0.25, -1.0, 2.0, 0.0, 5.0])
    p = run_steps(adam, [g], 0.01, theta0=th0)
    want = th0 - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p[1], want, rtol=1e-13, atol=1e-15), (p[1], want)


def pin_constant_gradient(adam):
    g = np.array([0.3, -2.0, 1e-4])
    T, lr, eps = 25, 1e-3, 1e-8
    p = run_steps(adam, [g] * T, lr, eps=eps)
    want = -np.arange(T + 1)[:, None] * lr * g / (np.abs(g) + eps)
    assert np.allclose(p, want, rtol=1e-11, atol=1e-15), np.max(np.abs(p - want))


def pin_two_steps(adam):
    p = run_steps(adam, [[1.0], [-2.0]], 0.1, eps=0.0)
    assert p[1][0] == pytest.approx(-0.1, rel=1e-14)
    assert p[2][0] - p[1][0] == pytest.approx(0.0366103527035845565282265431, rel=1e-12)


def pin_scale_invariance(adam):
    rng = np.random.default_rng(4)
    grads = [rng.normal(size=6) for _ in range(12)]
    a = run_steps(adam, grads, 0.05, eps=0.0)
    b = run_steps(adam, [1000.0 * g for g in grads], 0.05, eps=0.0)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-15)


def pin_eps_outside_root(adam):
    p = run_steps(adam, [[1e-8]], 1.0, eps=1e-8)
    assert p[1][0] == pytest.approx(-0.5, rel=1e-12)


PINS = [pin_first_step, pin_constant_gradient, pin_two_steps, pin_scale_invariance,
        pin_eps_outside_root]


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_reference_adam(pin):
    pin(ref.adam)
