"""Pins of the oracle's proximal operators (CPU only)."""
import numpy as np
import pytest

from oracle import prox


def test_soft_threshold_brute_force_real():
    lam = 0.7
    grid = np.linspace(-5, 5, 200001)                 # step 5e-5
    for x in [-3.0, -0.71, -0.7, -0.2, 0.0, 0.5, 0.7, 0.7000001, 2.5]:
        obj = lam * np.abs(grid) + 0.5 * (grid - x) ** 2
        best = grid[np.argmin(obj)]
        assert prox.soft_threshold(np.array([x]), lam)[0] == pytest.approx(best, abs=6e-5)


def test_soft_threshold_brute_force_complex():
    lam = 0.4
    g = np.linspace(-2, 2, 801)                       # step 5e-3
    V = g[None, :] + 1j * g[:, None]
    rng = np.random.default_rng(0)
    for _ in range(6):
        x = complex(rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5))
        obj = lam * np.abs(V) + 0.5 * np.abs(V - x) ** 2
        best = V.reshape(-1)[np.argmin(obj)]
        assert abs(prox.soft_threshold(np.array([x]), lam)[0] - best) < 8e-3


def test_soft_threshold_ties_and_moreau():
    lam = 0.5
    x = np.array([-0.5, 0.5, -2.0, 0.3, 1.7])
    s = prox.soft_threshold(x, lam)
    assert s[0] == 0 and s[1] == 0
    # Moreau: x = S_lam(x) + clip_lam(x), and clip_lam is the projection onto [-lam, lam]
    assert np.allclose(s + prox.clip_magnitude(x, lam), x, atol=0)
    assert np.allclose(prox.clip_magnitude(x, lam), np.clip(x, -lam, lam), atol=1e-16)


def test_l2ball_brute_force_2d():
    z = np.array([0.3, -0.2])
    eps = 0.8
    th = np.linspace(0, 2 * np.pi, 20001)
    r = np.linspace(0, eps, 401)
    pts = z[None, None, :] + r[:, None, None] * np.stack([np.cos(th), np.sin(th)], -1)[None]
    pts = pts.reshape(-1, 2)
    rng = np.random.default_rng(1)
    for _ in range(5):
        x = rng.uniform(-3, 3, 2)
        best = pts[np.argmin(np.sum((pts - x) ** 2, axis=1))]
        assert np.allclose(prox.proj_l2ball(x, z, eps), best, atol=3e-3)


def test_l2ball_inside_and_boundary_unchanged():
    z = np.array([1.0 + 1j, -2.0])
    x = z + np.array([0.3, 0.4j])          # distance exactly 0.5
    assert np.array_equal(prox.proj_l2ball(x, z, 0.5), x)
    assert np.array_equal(prox.proj_l2ball(x, z, 0.6), x)
    p = prox.proj_l2ball(x, z, 0.25)
    assert prox.l2_distance(p, z) == pytest.approx(0.25, rel=1e-15)
    # the projection moves along x - z
    assert np.allclose((p - z) / 0.25, (x - z) / 0.5)


def test_positivity_projection():
    x = np.array([-1.0, 0.0, 2.5, -0.0])
    assert np.array_equal(prox.proj_positive(x), [0.0, 0.0, 2.5, 0.0])
    assert np.array_equal(prox.proj_positive(np.array([1 - 2j, -3 + 1j])), [1.0, 0.0])
