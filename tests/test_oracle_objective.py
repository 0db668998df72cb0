"""Pins of the FP64 objective oracle (oracle/objective.py) against facts other than itself:
Eq. 7's weight against its tanh closed form and its limits, the unweighted special case
(k = 0) against the C oracle's loss, finite differences with the weight held fixed; the TV
term of a linear ramp in closed form, its invariances and finite differences; the
coarse-to-fine step reproducing a quadratic exactly (Eq. 1 holds with no truncation error)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import objective as obj
from test_oracle_pins import _random_poly, _taylor_coeffs_of


def test_surface_weight_closed_form_and_limits():
    """2 sigmoid(z) - 1 = tanh(z / 2), so w'(d) = 1 - tanh(|k d| / 2) = 2 / (1 + exp(|k d|)):
    1 on the surface, 1/2 where |k d| = ln 3, and to 0 far from it, symmetric in d."""
    rng = np.random.default_rng(0)
    d = rng.normal(0, 1, size=1000)
    for k in (0.5, 7.0, 40.0):
        w = obj.surface_weight_1(d, k)
        # the definition loses relative accuracy where w is tiny (1 - a number near 1): compare absolutely
        np.testing.assert_allclose(w, 2.0 / (1.0 + np.exp(np.abs(k * d))), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(w, obj.surface_weight_1(-d, k), rtol=0, atol=1e-15)
        assert obj.surface_weight_1(0.0, k) == 1.0
        assert abs(obj.surface_weight_1(math.log(3.0) / k, k) - 0.5) < 1e-14
    assert obj.surface_weight_1(1e4, 10.0) == 0.0  # saturates without overflow trouble
    np.testing.assert_array_equal(obj.surface_weight_1(d, 0.0), 1.0)


def test_weight_takes_the_larger_of_predicted_and_true():
    """Eq. 7's max: a sample is weighted up when either distance is near the surface."""
    rng = np.random.default_rng(1)
    f, d = rng.normal(0, 0.5, size=200), rng.normal(0, 0.5, size=200)
    w = obj.surface_weight(f, d, 9.0)
    for i in range(200):
        wf = 2.0 / (1.0 + math.exp(abs(9.0 * f[i])))
        wd = 2.0 / (1.0 + math.exp(abs(9.0 * d[i])))
        assert abs(w[i] - max(wf, wd)) <= 1e-14
    # on either surface the weight is 1
    assert obj.surface_weight(0.0, 3.0, 9.0) == 1.0 and obj.surface_weight(3.0, 0.0, 9.0) == 1.0


def test_k0_is_the_unweighted_loss():
    rng = np.random.default_rng(2)
    n = 300
    f, d = rng.normal(0, 1, size=n), rng.normal(0, 1, size=n)
    grad = rng.normal(0, 1, size=(n, 3))
    loss, gf, gg = obj.weighted_sdf_loss(f, grad, d, 0.1, 0.0)
    ref, rgf, rgg = oracle.sdf_loss(f, grad, d, 0.1)
    np.testing.assert_allclose(loss, ref, rtol=1e-14)
    np.testing.assert_array_equal(gf, rgf)
    np.testing.assert_array_equal(gg, rgg)


def test_weighted_loss_gradient_matches_finite_differences():
    """With the weight held at its value, d L_recon / d f_i is a central difference of
    (1/n) sum_j w_j |f_j - d_j| (no sample sits on its kink)."""
    rng = np.random.default_rng(3)
    n = 50
    f = rng.normal(0, 0.3, size=n)
    d = f + rng.choice([-1, 1], size=n) * rng.uniform(0.01, 0.2, size=n)
    k = 12.0
    loss, gf, _ = obj.weighted_sdf_loss(f, None, d, 0.0, k)
    w = obj.surface_weight(f, d, k)
    recon = lambda ff: float(np.sum(w * np.abs(ff - d)) / n)
    assert abs(loss[1] - recon(f)) <= 1e-15 and loss[0] == loss[1]
    eps = 1e-6
    for i in range(n):
        fp, fm = f.copy(), f.copy()
        fp[i] += eps
        fm[i] -= eps
        fd = (recon(fp) - recon(fm)) / (2 * eps)
        assert abs(fd - gf[i]) <= 1e-9, (i, fd, gf[i])
    # the weight only scales: samples far from both surfaces count less
    assert np.all(np.abs(gf) <= 1.0 / n + 1e-18)


def _ramp(res, slopes):
    """A [res_z, res_y, res_x, 2] array: channel 0 a linear ramp in the vertex indices,
    channel 1 a constant."""
    dim = len(res)
    idx = np.meshgrid(*[np.arange(r) for r in res], indexing="ij")  # idx[a][i_x, i_y, i_z]
    ramp = sum(s * i for s, i in zip(slopes, idx))
    ramp = np.transpose(ramp, tuple(reversed(range(dim))))
    return np.stack([ramp, np.full(ramp.shape, 3.5)], axis=-1)


@pytest.mark.parametrize("res,slopes", [((4, 5, 6), (0.3, -1.2, 2.0)), ((7, 3), (1.5, 0.25))])
def test_tv_of_a_linear_ramp(res, slopes):
    """Every forward difference along axis a is slope_a except on the last layer of a, so a
    vertex contributes sqrt(sum of slope_a^2 over the axes where it is not on the last layer);
    counting vertices by that set of axes gives TV in closed form.  The constant channel adds 0."""
    dim = len(res)
    C = _ramp(res, slopes)
    total = 0.0
    for inner in itertools.product([True, False], repeat=dim):
        count = np.prod([res[a] - 1 if inner[a] else 1 for a in range(dim)])
        total += count * math.sqrt(sum(slopes[a] ** 2 for a in range(dim) if inner[a]))
    value, _ = obj.tv(C, dim)
    assert abs(value - total / np.prod(res)) <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_tv_invariances(dim):
    """TV ignores an added constant, scales with |lambda|, and its gradient sums to zero over
    the vertices of each channel (the value is invariant under a constant shift)."""
    rng = np.random.default_rng(4 + dim)
    shape = (5, 6, 4, 3) if dim == 3 else (6, 7, 3)
    C = rng.normal(0, 1, size=shape)
    v, g = obj.tv(C, dim)
    v2, g2 = obj.tv(C + 4.25, dim)
    assert abs(v - v2) <= 1e-12 * v
    np.testing.assert_allclose(g, g2, atol=1e-13)
    v3, _ = obj.tv(-2.5 * C, dim)
    assert abs(v3 - 2.5 * v) <= 1e-12 * v
    np.testing.assert_allclose(g.reshape(-1, shape[-1]).sum(axis=0), 0.0, atol=1e-13)
    # a constant field has zero TV and the zero subgradient
    v0, g0 = obj.tv(np.full(shape, 1.25), dim)
    assert v0 == 0.0 and not np.any(g0)


@pytest.mark.parametrize("dim", [2, 3])
def test_tv_gradient_matches_finite_differences(dim):
    rng = np.random.default_rng(6 + dim)
    shape = (3, 4, 3, 2) if dim == 3 else (4, 5, 3)
    C = rng.normal(0, 1, size=shape)
    _, g = obj.tv(C, dim)
    eps = 1e-6
    for idx in np.ndindex(*shape):
        cp, cm = C.copy(), C.copy()
        cp[idx] += eps
        cm[idx] -= eps
        fd = (obj.tv(cp, dim)[0] - obj.tv(cm, dim)[0]) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-8, (idx, fd, g[idx])


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("fine_order", [0, 1, 2])
def test_upsampling_reproduces_a_quadratic(dim, fine_order):
    """A coarse K=2 grid storing a quadratic's exact derivatives represents it exactly, so the
    fine grid's coefficients are the quadratic's derivatives at the fine vertices, whatever
    the fine resolution (fine vertices on and off the coarse faces)."""
    rng = np.random.default_rng(20 + dim)
    p = _random_poly(dim, 2, rng)
    if dim == 3:
        lo, hi = (-1.0, 0.25, -3.0), (2.0, 1.5, -0.5)
        coarse = oracle.Geometry(3, (4, 5, 3), 2, lo, hi)
        fine = oracle.Geometry(3, (7, 9, 6), fine_order, lo, hi)
    else:
        lo, hi = (-1.0, 0.25), (2.0, 1.5)
        coarse = oracle.Geometry(2, (5, 4), 2, lo, hi)
        fine = oracle.Geometry(2, (9, 10), fine_order, lo, hi)
    up = obj.upsample(coarse, _taylor_coeffs_of(p, coarse), fine)
    np.testing.assert_allclose(up, _taylor_coeffs_of(p, fine), rtol=0, atol=1e-10)
