"""Pins for the proximal maps: closed forms, prox optimality, firm non-expansiveness, Moreau."""
import numpy as np
import pytest

from oracle import prox
from paper_1502_05037_amd import synth


def test_soft_closed_form_and_ties():
    v = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.5])
    np.testing.assert_array_equal(prox.soft(v, 1.0), [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.5])
    np.testing.assert_array_equal(prox.soft(v, 0.0), v)
    tau = np.array([0, 1, 2, 3, 0.1, 0.5, 3.0])
    np.testing.assert_allclose(prox.soft(v, tau), [-3.0, 0.0, 0.0, 0.0, 0.4, 0.5, 0.0])


def test_soft_is_prox_of_l1():
    # prox_{tau|.|}(v) minimises tau|p| + (p - v)^2 / 2: brute force on a fine grid
    g = synth.rng(97, 0, 0)
    grid = np.linspace(-5, 5, 200001)
    for v, tau in zip(g.normal(size=20) * 2, g.uniform(0, 2, size=20)):
        p = grid[np.argmin(tau * np.abs(grid) + 0.5 * (grid - v) ** 2)]
        assert prox.soft(np.array([v]), tau)[0] == pytest.approx(p, abs=1e-4)


def test_soft_moreau_identity():
    # v = prox_{tau f}(v) + tau prox_{f*/tau}(v / tau), f* = indicator of the l_inf unit ball
    g = synth.rng(97, 1, 0)
    v = g.normal(size=100) * 3
    tau = 0.7
    np.testing.assert_allclose(prox.soft(v, tau) + tau * np.clip(v / tau, -1, 1), v, atol=1e-15)


def test_ball_projection_cases():
    c = np.array([1.0 + 1j, -2.0 + 0.5j])
    inside = c + np.array([0.1, -0.1j])
    np.testing.assert_array_equal(prox.ball(inside, c, 1.0), inside)
    edge = c + np.array([0.6, 0.8j])          # exactly on the sphere of radius 1
    np.testing.assert_array_equal(prox.ball(edge, c, 1.0), edge)
    np.testing.assert_array_equal(prox.ball(c, c, 0.0), c)
    far = c + np.array([3.0, 4.0j])
    np.testing.assert_allclose(prox.ball(far, c, 1.0), c + np.array([0.6, 0.8j]))


def test_projection_optimality_and_firm_nonexpansive():
    g = synth.rng(97, 2, 0)
    m = 30
    c = g.normal(size=m) + 1j * g.normal(size=m)
    eps = 2.0
    for _ in range(50):
        t = c + 3 * (g.normal(size=m) + 1j * g.normal(size=m))
        p = prox.ball(t, c, eps)
        assert np.linalg.norm(p - c) <= eps * (1 + 1e-14)
        q = c + (g.normal(size=m) + 1j * g.normal(size=m))
        q = c + (q - c) * min(1.0, eps / np.linalg.norm(q - c)) * g.uniform()
        assert np.vdot(q - p, t - p).real <= 1e-12          # <t - p, q - p> <= 0
        t2 = c + 3 * (g.normal(size=m) + 1j * g.normal(size=m))
        p2 = prox.ball(t2, c, eps)
        assert np.linalg.norm(p - p2) ** 2 <= np.vdot(p - p2, t - t2).real + 1e-12
    v = g.normal(size=100)
    w = g.normal(size=100)
    assert np.linalg.norm(prox.positive(v) - prox.positive(w)) ** 2 <= np.dot(prox.positive(v) - prox.positive(w), v - w) + 1e-14
    np.testing.assert_array_equal(prox.positive(np.array([-1.0, 0.0, 2.0])), [0.0, 0.0, 2.0])
