"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself:
  * a library routine (scipy multilinear interpolation for order 0; torch.optim.Adam);
  * closed forms (exact reproduction of any polynomial of degree <= K whose derivatives are
    stored at the vertices; analytic loss values);
  * hand-worked examples (tests/golden/, Sec. 3.1 Eq. 1-4);
  * invariants (vertex property, C0 continuity, adjoint identity, clamping);
  * central finite differences (gradient, Hessian, dq, dC);
  * the independent NumPy brute force on tiny grids.
The last test plants mistakes in copies of the oracle source and shows that these pins fail.
"""
import itertools
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geom(dim, order, aniso=True):
    if dim == 2:
        return oracle.Geometry(2, (5, 7), order, (-1.0, 0.25), (2.0, 1.5)) if aniso else \
            oracle.Geometry(2, (6, 6), order, (0.0, 0.0), (1.0, 1.0))
    return oracle.Geometry(3, (5, 4, 6), order, (-1.0, 0.25, -3.0), (2.0, 1.5, -0.5)) if aniso else \
        oracle.Geometry(3, (5, 5, 5), order, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))


def _inside(geom, n, rng, margin=0.0):
    lo = np.array(geom.lo)
    hi = np.array(geom.hi)
    return rng.uniform(lo + margin, hi - margin, size=(n, geom.dim))


def _cell_coord(geom, q):
    lo = np.array(geom.lo)
    hi = np.array(geom.hi)
    h = (hi - lo) / (np.array(geom.res) - 1)
    return (np.clip(q, lo, hi) - lo) / h


def _away_from_faces(geom, q, gap):
    s = _cell_coord(geom, q)
    frac = s - np.floor(s)
    return np.all((frac > gap) & (frac < 1 - gap), axis=1)


# ----------------------------------------------------------------------------- golden
def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            vals[key] = np.array([float(x) for x in rest])
    return vals


@pytest.mark.parametrize("name", ["hand_2d_k2.txt", "hand_3d_k2.txt"])
def test_hand_worked_examples(name):
    v = _read_golden(name)
    dim = int(v["dim"][0])
    g = oracle.Geometry(dim, v["res"].astype(int), int(v["order"][0]), v["lo"], v["hi"])
    f, grad = oracle.forward(g, v["coeffs"], v["query"].reshape(1, dim))
    assert f[0] == v["f"][0]
    np.testing.assert_array_equal(grad[0], v["grad"])


# ----------------------------------------------------------------------------- library
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("aniso", [False, True])
def test_order0_is_multilinear_interpolation(dim, aniso):
    """K = 0 stores only values: the field is plain multilinear interpolation of the
    vertex values (the 'Linear' grid of the paper's comparisons)."""
    from scipy.interpolate import RegularGridInterpolator

    rng = np.random.default_rng(1)
    g = _geom(dim, 0, aniso)
    C = rng.normal(size=g.coeff_shape)
    q = _inside(g, 2000, rng)
    axes = [np.linspace(g.lo[a], g.hi[a], g.res[a]) for a in range(dim)]
    vals = np.transpose(C[..., 0])  # [x, y, (z)] for scipy
    ref = RegularGridInterpolator(axes, vals, method="linear")(q)
    f = oracle.forward(g, C, q, want_grad=False)
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-13)


def test_adam_matches_torch():
    import torch

    rng = np.random.default_rng(2)
    n = 1000
    theta0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * s for s in (1.0, 1e-3, 10.0, 1e-9)]
    for wd in (0.0, 0.01):
        p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
        opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
        th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
        for step, gr in enumerate(grads, start=1):
            p.grad = torch.tensor(gr, dtype=torch.float64)
            opt.step()
            th, m, v, ss = oracle.adam(th, m, v, gr, 1e-2, 0.9, 0.999, 1e-8, wd, step)
            np.testing.assert_allclose(th, p.detach().numpy(), rtol=0, atol=1e-14)
            np.testing.assert_allclose(ss, float(np.sum(gr * gr)), rtol=1e-14)
            # torch forms m with lerp; the two agree to rounding relative to the largest entry
            tm = opt.state[p]["exp_avg"].numpy()
            tv = opt.state[p]["exp_avg_sq"].numpy()
            np.testing.assert_allclose(m, tm, rtol=0, atol=1e-15 * np.abs(tm).max())
            np.testing.assert_allclose(v, tv, rtol=0, atol=1e-15 * np.abs(tv).max())


# ----------------------------------------------------------------------------- closed forms
def _random_poly(dim, degree, rng):
    """Random polynomial as {exponent tuple: coefficient}."""
    return {e: rng.normal() for e in itertools.product(range(degree + 1), repeat=dim) if sum(e) <= degree}


def _poly_derivative(poly, alpha):
    out = {}
    for e, c in poly.items():
        if all(ei >= ai for ei, ai in zip(e, alpha)):
            k = c
            for ei, ai in zip(e, alpha):
                for j in range(ai):
                    k *= ei - j
            ne = tuple(ei - ai for ei, ai in zip(e, alpha))
            out[ne] = out.get(ne, 0.0) + k
    return out


def _poly_eval(poly, x):
    x = np.atleast_2d(x)
    r = np.zeros(len(x))
    for e, c in poly.items():
        r += c * np.prod(x ** np.array(e), axis=1)
    return r


def _taylor_coeffs_of(poly, g):
    """Stored coefficients = exact derivatives d^alpha p at every vertex."""
    exps = oracle.exponents(g.dim, g.order)
    axes = [np.linspace(g.lo[a], g.hi[a], g.res[a]) for a in range(g.dim)]
    mesh = np.meshgrid(*axes, indexing="ij")  # [x, y, z]
    pts = np.stack([m.reshape(-1) for m in mesh], axis=1)
    C = np.stack([_poly_eval(_poly_derivative(poly, tuple(a)), pts) for a in exps], axis=1)
    C = C.reshape(tuple(g.res) + (len(exps),))
    return np.transpose(C, tuple(reversed(range(g.dim))) + (g.dim,))  # -> [z, y, x, C]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_polynomial_reproduction(dim, order):
    """Every corner's Taylor polynomial of a degree-<=K polynomial is the polynomial itself,
    and the interpolation weights sum to one, so the field reproduces it exactly (value and
    gradient), on an anisotropic box.  Fixes the 1/alpha! factors of Eq. 1, the world-unit
    offsets, the off-diagonal convention and the corner/vertex wiring."""
    rng = np.random.default_rng(10 + dim * 5 + order)
    g = _geom(dim, order, aniso=True)
    p = _random_poly(dim, order, rng)
    C = _taylor_coeffs_of(p, g)
    q = _inside(g, 500, rng)
    f, grad = oracle.forward(g, C, q)
    np.testing.assert_allclose(f, _poly_eval(p, q), rtol=0, atol=1e-11)
    for a in range(dim):
        e = tuple(1 if i == a else 0 for i in range(dim))
        np.testing.assert_allclose(grad[:, a], _poly_eval(_poly_derivative(p, e), q), rtol=0, atol=1e-10)


def test_higher_degree_is_not_reproduced():
    """Sanity: a degree-3 polynomial stored at order 2 is not reproduced (the test above
    has teeth)."""
    rng = np.random.default_rng(3)
    g = _geom(3, 2)
    p = {(3, 0, 0): 1.0}
    C = _taylor_coeffs_of(p, g)
    q = _inside(g, 100, rng)
    f = oracle.forward(g, C, q, want_grad=False)
    assert np.max(np.abs(f - _poly_eval(p, q))) > 1e-3


# ----------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("dim", [2, 3])
def test_vertex_property(dim):
    """At a vertex only that vertex has non-zero weight and the offset is zero: f = C[v][0]."""
    rng = np.random.default_rng(4)
    g = _geom(dim, 2, aniso=False)
    C = rng.normal(size=g.coeff_shape)
    idx = np.stack(np.meshgrid(*[np.arange(r) for r in g.res], indexing="ij"), -1).reshape(-1, dim)
    h = (np.array(g.hi) - np.array(g.lo)) / (np.array(g.res) - 1)
    q = np.array(g.lo) + idx * h
    f = oracle.forward(g, C, q, want_grad=False)
    flat = C.reshape(-1, g.num_coeffs)
    lin = np.zeros(len(idx), dtype=np.int64)
    for a in reversed(range(dim)):
        lin = lin * g.res[a] + idx[:, a]
    np.testing.assert_allclose(f, flat[lin, 0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_c0_continuity_across_faces(dim):
    rng = np.random.default_rng(5)
    g = _geom(dim, 2)
    C = rng.normal(size=g.coeff_shape)
    h = (np.array(g.hi) - np.array(g.lo)) / (np.array(g.res) - 1)
    for a in range(dim):
        q = _inside(g, 200, rng, margin=1e-3)
        k = rng.integers(1, g.res[a] - 1, size=len(q))
        q[:, a] = g.lo[a] + k * h[a]
        eps = 1e-9 * h[a]
        qm, qp = q.copy(), q.copy()
        qm[:, a] -= eps
        qp[:, a] += eps
        fm = oracle.forward(g, C, qm, want_grad=False)
        fp = oracle.forward(g, C, qp, want_grad=False)
        assert np.max(np.abs(fm - fp)) < 1e-7


@pytest.mark.parametrize("dim", [2, 3])
def test_clamping(dim):
    """Outside the box the field equals its value at the clamped point and the gradient is
    zero along clamped axes only."""
    rng = np.random.default_rng(6)
    g = _geom(dim, 2)
    C = rng.normal(size=g.coeff_shape)
    lo, hi = np.array(g.lo), np.array(g.hi)
    q = rng.uniform(lo - 1.0, hi + 1.0, size=(500, dim))
    f, grad = oracle.forward(g, C, q)
    fc, gc = oracle.forward(g, C, np.clip(q, lo, hi))
    np.testing.assert_allclose(f, fc, rtol=0, atol=1e-15)
    outside = (q < lo) | (q > hi)
    assert outside.any() and (~outside).any()
    assert np.all(grad[outside] == 0.0)
    np.testing.assert_allclose(grad[~outside], gc[~outside], rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- derivatives
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_gradient_and_hessian_match_finite_differences(dim, order):
    rng = np.random.default_rng(7 + dim + order)
    g = _geom(dim, order)
    C = rng.normal(size=g.coeff_shape)
    q = _inside(g, 400, rng, margin=1e-3)
    q = q[_away_from_faces(g, q, 1e-3)]
    f, grad, hess = oracle.forward(g, C, q, want_hess=True)
    h = (np.array(g.hi) - np.array(g.lo)) / (np.array(g.res) - 1)
    for a in range(dim):
        eps = 1e-6 * h[a]
        qp, qm = q.copy(), q.copy()
        qp[:, a] += eps
        qm[:, a] -= eps
        fp, gp = oracle.forward(g, C, qp)
        fm, gm = oracle.forward(g, C, qm)
        np.testing.assert_allclose(grad[:, a], (fp - fm) / (2 * eps), rtol=0, atol=1e-6 * max(1, np.abs(grad).max()))
        np.testing.assert_allclose(hess[:, :, a], (gp - gm) / (2 * eps), rtol=0, atol=1e-5 * max(1, np.abs(hess).max()))
    np.testing.assert_allclose(hess, np.swapaxes(hess, 1, 2), rtol=0, atol=1e-10 * np.abs(hess).max())


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_adjoint_identity(dim, order):
    """(f, grad f) is linear in C, so <dC(gf, gg), C'> = <gf, f(C')> + <gg, grad f(C')>
    for any C' -- including queries clamped outside the box."""
    rng = np.random.default_rng(8 + dim + order)
    g = _geom(dim, order)
    C = rng.normal(size=g.coeff_shape)
    lo, hi = np.array(g.lo), np.array(g.hi)
    q = rng.uniform(lo - 0.3, hi + 0.3, size=(300, dim))
    gf = rng.normal(size=len(q))
    gg = rng.normal(size=(len(q), dim))
    dC, _ = oracle.backward(g, C, q, gf, gg)
    for _ in range(3):
        Cp = rng.normal(size=g.coeff_shape)
        f, grad = oracle.forward(g, Cp, q)
        lhs = np.sum(dC * Cp)
        rhs = gf @ f + np.sum(gg * grad)
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs))


def test_dcoeff_matches_finite_differences():
    """Central differences in C are exact up to rounding for a linear map."""
    rng = np.random.default_rng(9)
    g = _geom(3, 2)
    C = rng.normal(size=g.coeff_shape)
    q = _inside(g, 200, rng)
    gf = rng.normal(size=len(q))
    gg = rng.normal(size=(len(q), 3))
    dC, _ = oracle.backward(g, C, q, gf, gg)
    flat = C.reshape(-1)
    for k in rng.choice(flat.size, size=40, replace=False):
        e = np.zeros_like(flat)
        e[k] = 0.5

        def obj(c):
            f, grad = oracle.forward(g, c.reshape(C.shape), q)
            return gf @ f + np.sum(gg * grad)

        fd = (obj(flat + e) - obj(flat - e)) / 1.0
        assert abs(fd - dC.reshape(-1)[k]) < 1e-10 * max(1.0, abs(fd))


@pytest.mark.parametrize("dim", [2, 3])
def test_dq_matches_finite_differences(dim):
    rng = np.random.default_rng(11 + dim)
    g = _geom(dim, 2)
    C = rng.normal(size=g.coeff_shape)
    q = _inside(g, 300, rng, margin=1e-3)
    q = q[_away_from_faces(g, q, 1e-3)]
    gf = rng.normal(size=len(q))
    gg = rng.normal(size=(len(q), dim))
    _, dq = oracle.backward(g, C, q, gf, gg, want_dq=True)
    h = (np.array(g.hi) - np.array(g.lo)) / (np.array(g.res) - 1)

    def obj_per_query(qq):
        f, grad = oracle.forward(g, C, qq)
        return gf * f + np.sum(gg * grad, axis=1)

    for a in range(dim):
        eps = 1e-6 * h[a]
        qp, qm = q.copy(), q.copy()
        qp[:, a] += eps
        qm[:, a] -= eps
        fd = (obj_per_query(qp) - obj_per_query(qm)) / (2 * eps)
        np.testing.assert_allclose(dq[:, a], fd, rtol=0, atol=1e-5 * max(1.0, np.abs(dq).max()))


def test_dq_zero_on_clamped_axes():
    rng = np.random.default_rng(12)
    g = _geom(3, 2)
    C = rng.normal(size=g.coeff_shape)
    lo, hi = np.array(g.lo), np.array(g.hi)
    q = rng.uniform(lo - 1.0, hi + 1.0, size=(300, 3))
    _, dq = oracle.backward(g, C, q, rng.normal(size=300), rng.normal(size=(300, 3)), want_dq=True)
    outside = (q < lo) | (q > hi)
    assert np.all(dq[outside] == 0.0)


# ----------------------------------------------------------------------------- brute force
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_oracle_matches_brute_force(dim, order):
    rng = np.random.default_rng(13 + dim + order)
    if dim == 2:
        g = oracle.Geometry(2, (4, 5), order, (-0.5, 0.0), (1.0, 2.0))
    else:
        g = oracle.Geometry(3, (3, 4, 3), order, (-0.5, 0.0, 1.0), (1.0, 2.0, 1.5))
    C = rng.normal(size=g.coeff_shape)
    lo, hi = np.array(g.lo), np.array(g.hi)
    q = rng.uniform(lo - 0.2, hi + 0.2, size=(40, dim))
    f, grad = oracle.forward(g, C, q)
    fb, gb = brute.forward(dim, g.res, order, g.lo, g.hi, C, q)
    np.testing.assert_allclose(f, fb, rtol=0, atol=1e-13)
    np.testing.assert_allclose(grad, gb, rtol=0, atol=1e-12)
    gf = rng.normal(size=len(q))
    gg = rng.normal(size=(len(q), dim))
    dC, _ = oracle.backward(g, C, q, gf, gg)
    dCb = brute.backward(dim, g.res, order, g.lo, g.hi, g.num_coeffs, q, gf, gg)
    np.testing.assert_allclose(dC.reshape(-1), dCb, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------- losses
def test_sdf_loss_closed_form():
    """A grid that reproduces p(x) = a.x + b has grad f = a everywhere, so the eikonal mean
    is (|a| - 1)^2; with targets d = p - delta the L1 mean is mean|delta|."""
    rng = np.random.default_rng(14)
    g = _geom(3, 2)
    a = np.array([0.6, -0.8, 0.5])
    b = 0.3
    poly = {(0, 0, 0): b, (1, 0, 0): a[0], (0, 1, 0): a[1], (0, 0, 1): a[2]}
    C = _taylor_coeffs_of(poly, g)
    q = _inside(g, 1000, rng)
    f, grad = oracle.forward(g, C, q)
    delta = rng.uniform(0.01, 0.1, size=len(q)) * rng.choice([-1.0, 1.0], size=len(q))
    d = _poly_eval(poly, q) - delta
    out, gf, gg = oracle.sdf_loss(f, grad, d, 0.1)
    np.testing.assert_allclose(out[1], np.mean(np.abs(delta)), rtol=1e-12)
    np.testing.assert_allclose(out[2], (np.linalg.norm(a) - 1) ** 2, rtol=1e-10)
    np.testing.assert_allclose(out[0], out[1] + 0.1 * out[2], rtol=1e-14)
    np.testing.assert_allclose(gf, np.sign(delta) / len(q), rtol=0, atol=1e-18)


def test_sdf_loss_gradients_match_finite_differences():
    rng = np.random.default_rng(15)
    n = 50
    f = rng.normal(size=n)
    d = f + rng.choice([-1, 1], size=n) * rng.uniform(0.1, 1.0, size=n)
    grad = rng.normal(size=(n, 3))
    out, gf, gg = oracle.sdf_loss(f, grad, d, 0.1)
    eps = 1e-6
    for i in range(0, n, 7):
        fp, fm = f.copy(), f.copy()
        fp[i] += eps
        fm[i] -= eps
        fd = (oracle.sdf_loss(fp, grad, d, 0.1)[0][0] - oracle.sdf_loss(fm, grad, d, 0.1)[0][0]) / (2 * eps)
        assert abs(fd - gf[i]) < 1e-8
        for a in range(3):
            gp, gm = grad.copy(), grad.copy()
            gp[i, a] += eps
            gm[i, a] -= eps
            fd = (oracle.sdf_loss(f, gp, d, 0.1)[0][0] - oracle.sdf_loss(f, gm, d, 0.1)[0][0]) / (2 * eps)
            assert abs(fd - gg[i, a]) < 1e-8


def test_sdf_loss_degenerate_cases():
    out, gf, gg = oracle.sdf_loss(np.zeros(4), np.zeros((4, 3)), np.zeros(4), 0.1)
    assert np.all(gf == 0) and np.all(gg == 0)  # sign(0) = 0; zero-norm gradient -> 0
    np.testing.assert_allclose(out, [0.1, 0.0, 1.0])
    out, gf, gg = oracle.sdf_loss(np.zeros(0), np.zeros((0, 3)), np.zeros(0), 0.1)
    assert np.all(out == 0)


# ----------------------------------------------------------------------------- planted mistakes
MUTATIONS = {
    "drop the 1/alpha! factor": ("        r /= factorial(alpha[a]);\n", ""),
    "offset sign flipped": ("K->d[a] = L->x[a] - v;", "K->d[a] = v - L->x[a];"),
    "weight factor swapped": ("factor[a] = ba ? L->t[a] : 1.0 - L->t[a];", "factor[a] = ba ? 1.0 - L->t[a] : L->t[a];"),
    "x and y strides transposed": ("stride *= g->res[a];", "stride *= g->res[g->dim - 1 - a];"),
    "weight-derivative term dropped in dC": ("contrib += s_g[a] * (K.dw[a] * m + K.w * monomial_d1(alpha, K.d, dim, a));",
                                            "contrib += s_g[a] * (K.w * monomial_d1(alpha, K.d, dim, a));"),
    "Hessian cross term dropped": ("K.dw[a] * dT[c] + K.dw[c] * dT[a]", "K.dw[a] * dT[c]"),
}


def _pins_pass(lib):
    """A compact run of the pins above against a given oracle build."""
    rng = np.random.default_rng(99)
    ok = True
    g = _geom(3, 2, aniso=True)
    p = _random_poly(3, 2, rng)
    C = _taylor_coeffs_of(p, g)
    q = _inside(g, 200, rng, margin=1e-3)
    q = q[_away_from_faces(g, q, 1e-3)]
    f, grad, hess = oracle.forward(g, C, q, want_hess=True, lib=lib)
    ok &= np.allclose(f, _poly_eval(p, q), atol=1e-10)
    gf = rng.normal(size=len(q))
    gg = rng.normal(size=(len(q), 3))
    Cr = rng.normal(size=g.coeff_shape)
    dC, dq = oracle.backward(g, Cr, q, gf, gg, want_dq=True, lib=lib)
    Cp = rng.normal(size=g.coeff_shape)
    fp, gp = oracle.forward(g, Cp, q, lib=lib)
    ok &= abs(np.sum(dC * Cp) - (gf @ fp + np.sum(gg * gp))) < 1e-9
    fr, gr, hr = oracle.forward(g, Cr, q, want_hess=True, lib=lib)
    h = (np.array(g.hi) - np.array(g.lo)) / (np.array(g.res) - 1)
    for a in range(3):
        e = 1e-6 * h[a]
        qp, qm = q.copy(), q.copy()
        qp[:, a] += e
        qm[:, a] -= e
        _, gpp = oracle.forward(g, Cr, qp, lib=lib)
        _, gmm = oracle.forward(g, Cr, qm, lib=lib)
        ok &= np.allclose(hr[:, :, a], (gpp - gmm) / (2 * e), atol=1e-4 * max(1, np.abs(hr).max()))
    return bool(ok)


def test_pins_pass_on_the_oracle():
    assert _pins_pass(None)


def _variant_main(name):
    """Child-process entry: build the mutated oracle and exit 0 iff the pins still pass.
    A mutation may also crash the child (an index out of bounds), which counts as caught."""
    old, new = MUTATIONS[name]
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.build_variant(oracle.source_text().replace(old, new), tmp)
        sys.exit(0 if _pins_pass(lib) else 1)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name):
    old, _ = MUTATIONS[name]
    assert oracle.source_text().count(old) >= 1, name
    here = os.path.dirname(os.path.abspath(__file__))
    code = (f"import sys; sys.path[:0] = [{os.path.dirname(here)!r}, {here!r}]; "
            f"import test_oracle_pins as t; t._variant_main({name!r})")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch: {name}"
