"""Pins of the FP64 compositing oracle (oracle/radiance.py) against facts other than itself:
closed forms of the Max model (Sec. 3.3, Eq. 10) for one sample and for a homogeneous ray, the
product form of the transmittance, the telescoping sum of the weights, and central finite
differences of the photometric loss (Eq. 11)."""
import numpy as np

from oracle import radiance as rad


def test_single_sample_closed_form():
    rng = np.random.default_rng(0)
    f = rng.uniform(0.1, 3.0, size=(5, 1))
    delta = rng.uniform(0.01, 0.5, size=(5, 1))
    c = rng.uniform(0, 1, size=(5, 1, 3))
    rgb, T, _ = rad.composite(f, c, delta)
    np.testing.assert_allclose(T, 1.0)
    np.testing.assert_allclose(rgb, (1.0 - np.exp(-f * delta)) * c[:, 0, :], rtol=1e-14)


def test_homogeneous_ray_closed_form():
    """Constant density, colour and spacing: the weights telescope to 1 - exp(-sigma delta N)."""
    sigma, delta, n = 0.7, 0.05, 64
    c = np.array([0.2, 0.5, 0.9])
    rgb, T, _ = rad.composite(np.full((1, n), sigma), np.tile(c, (1, n, 1)), np.full((1, n), delta))
    np.testing.assert_allclose(rgb[0], (1.0 - np.exp(-sigma * delta * n)) * c, rtol=1e-13)
    np.testing.assert_allclose(T[0], np.exp(-sigma * delta * np.arange(n)), rtol=1e-13)


def test_transmittance_product_form_and_weight_sum():
    """T_i is the product of the earlier samples' (1 - alpha_j); sum_i T_i alpha_i = 1 - T_N."""
    rng = np.random.default_rng(1)
    f = rng.normal(0.5, 1.0, size=(7, 40))  # some negative: ReLU zeroes them
    delta = rng.uniform(0.0, 0.2, size=(7, 40))
    c = rng.uniform(0, 1, size=(7, 40, 3))
    _, T, alpha = rad.composite(f, c, delta)
    prod = np.cumprod(np.concatenate([np.ones((7, 1)), 1.0 - alpha[:, :-1]], axis=1), axis=1)
    np.testing.assert_allclose(T, prod, rtol=1e-12)
    end = T[:, -1] * (1.0 - alpha[:, -1])
    np.testing.assert_allclose((T * alpha).sum(axis=1), 1.0 - end, rtol=1e-12)
    # a sample of non-positive density is transparent
    assert np.all(alpha[f <= 0] == 0.0)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    R, N = 3, 6
    f = rng.uniform(0.2, 2.0, size=(R, N)) * rng.choice([1.0, -1.0], size=(R, N), p=[0.8, 0.2])
    delta = rng.uniform(0.05, 0.4, size=(R, N))
    c = rng.uniform(0, 1, size=(R, N, 3))
    target = rng.uniform(0, 1, size=(R, 3))
    loss, _, g_f, g_c = rad.composite_backward(f, c, delta, target)

    def L(ff, cc):
        return rad.photometric_loss(rad.composite(ff, cc, delta)[0], target)

    eps = 1e-6
    for r in range(R):
        for i in range(N):
            fp, fm = f.copy(), f.copy()
            fp[r, i] += eps
            fm[r, i] -= eps
            fd = (L(fp, c) - L(fm, c)) / (2 * eps)
            assert abs(fd - g_f[r, i]) <= 1e-8 + 1e-6 * abs(fd), (r, i, fd, g_f[r, i])
            for k in range(3):
                cp, cm = c.copy(), c.copy()
                cp[r, i, k] += eps
                cm[r, i, k] -= eps
                fd = (L(f, cp) - L(f, cm)) / (2 * eps)
                assert abs(fd - g_c[r, i, k]) <= 1e-8 + 1e-6 * abs(fd)
    assert np.isclose(loss, L(f, c))
    assert np.all(g_f[f < 0] == 0.0)
