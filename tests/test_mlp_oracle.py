"""Pins of the FP64 MLP reference: finite-difference gradients, Adam's
closed-form first step, BF16 rounding, and the invariance of the features
(and of the inversion they stand for) under rotations."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M


def _theta(rng, scale=0.5):
    return rng.normal(scale=scale, size=M.NPARAM)


def test_param_count():
    assert M.NPARAM == 4674


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    th = _theta(rng)
    X = rng.normal(size=(37, 5))
    T = rng.normal(size=(37, 2))
    Y, cache = M.forward(th, X)
    g = M.backward(th, cache, M.loss_grad(Y, T))
    idx = rng.choice(M.NPARAM, 300, replace=False)
    h = 1e-6
    worst = 0.0
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(M.forward(th + e, X)[0], T) - M.loss(M.forward(th - e, X)[0], T)) / (2 * h)
        # relative to the gradient's scale: central differences carry an
        # O(eps*|L|/h) ~ 1e-10 round-off floor
        worst = max(worst, abs(fd - g[i]) / (abs(g[i]) + 1e-4 * np.abs(g).max()))
    assert worst < 1e-6


def test_adam_first_step_closed_form():
    """With m0 = v0 = 0, the first bias-corrected Adam step is
    -lr * g / (|g| + eps): a move of lr against the gradient's sign."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    th, m, v = M.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-3, 65504.0])
    r = M.bf16_round(x)
    assert r[0] == 1.0
    # bf16 keeps 8 significant bits (7 stored): rounding error <= half an
    # ulp, i.e. 2^-8 relative
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    # exact on values with <= 8 significant bits; ties go to even
    assert M.bf16_round(np.array([1.5, 1.0 + 2 ** -7]))[1] == 1.0 + 2 ** -7
    assert M.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q if np.linalg.det(q) > 0 else -q


def test_features_rotation_invariant_and_sufficient():
    """Rotating S and B together leaves the features unchanged, and the
    oracle's inversion of the rotated state gives the same rho, p, Gamma --
    the features carry all the inversion depends on."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        rho, p = 10 ** rng.uniform(-1, 1), 10 ** rng.uniform(-2, 1)
        v = rng.normal(size=3)
        v *= rng.uniform(0, 0.95) / np.linalg.norm(v)
        B = rng.normal(size=3)
        pr = np.array([rho, *v, p, *B])
        u = O.prim2cons(pr)
        R = _rot(rng)
        ur = np.concatenate([[u[0]], R @ u[1:4], [u[4]], R @ u[5:8]])
        f = M.features(u[None, 0], u[None, 1:4], u[None, 4], u[None, 5:8])
        fr = M.features(ur[None, 0], ur[None, 1:4], ur[None, 4], ur[None, 5:8])
        np.testing.assert_allclose(f, fr, rtol=1e-12, atol=1e-14)
        rc1, p1, _, _, _ = O.con2prim(u, -1.0)
        rc2, p2, _, _, _ = O.con2prim(ur, -1.0)
        assert rc1 == rc2 == 0
        assert p1[0] == pytest.approx(p2[0], rel=1e-12)
        assert p1[4] == pytest.approx(p2[4], rel=1e-10)
        t1 = M.targets(p1[None, 0], p1[None, 1:4], p1[None, 4])
        np.testing.assert_allclose(t1, M.targets(np.array([rho]), v[None], np.array([p])), atol=1e-10)
