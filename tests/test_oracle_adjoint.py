"""Pins of the oracle's adjoint (gradients of L = 1/2 ||rf - obs||^2).

The adjoint is checked against central finite differences of the oracle's
own forward RF (a different computation: no derivative formula involved),
against the Euler identity of a function linear in the reflectivities, and
by the dot-product identity of a linear map and its transpose.
"""
import numpy as np
import pytest


def make(orc, convex=False, baffle=0, with_y=True, alpha=0.5):
    if convex:
        su = orc.Setup(n_elements=5, fc=3e6, pitch=0.5e-3, width=0.45e-3, height=13e-3,
                       elev_focus=60e-3, bandwidth=0.77, c=1540.0, alpha_db=alpha, fs=12e6,
                       radius=60e-3, nu=2, baffle=baffle)
        rng = np.random.default_rng(11)
        phi = rng.uniform(-0.3, 0.3, 4)
        rho = rng.uniform(70e-3, 90e-3, 4)
        x, z = rho * np.sin(phi), rho * np.cos(phi) - 60e-3
    else:
        su = orc.Setup(n_elements=4, fc=7.6e6, pitch=0.3e-3, width=0.27e-3, height=5e-3,
                       elev_focus=18e-3, bandwidth=0.77, c=1540.0, alpha_db=alpha, fs=30.4e6,
                       nu=2, baffle=baffle)
        rng = np.random.default_rng(7)
        x = rng.uniform(-2e-3, 2e-3, 4)
        z = rng.uniform(6e-3, 14e-3, 4)
    y = rng.uniform(-0.8e-3, 0.8e-3, x.size) if with_y else np.zeros(x.size)
    R = rng.standard_normal(x.size)
    N = su.n_elements
    delays = np.stack([np.zeros(N), np.linspace(0, 2e-7, N)])
    apod = np.stack([np.ones(N), np.linspace(0.5, 1.0, N)])
    g = orc.grid(su, delays, x, y, z)
    obs = orc.rf(su, g, delays, apod, x + 3e-5, y, z - 2e-5, R * 0.9)
    return su, g, delays, apod, x, y, z, R, obs


def loss(orc, su, g, delays, apod, x, y, z, R, obs):
    rf = orc.rf(su, g, delays, apod, x, y, z, R)
    return 0.5 * np.sum((rf - obs) ** 2), rf


@pytest.mark.parametrize("convex,baffle,with_y", [(False, 0, True), (False, 1, False),
                                                  (True, 0, False), (True, 2, True)])
def test_adjoint_matches_finite_differences(orc, convex, baffle, with_y):
    su, g, dl, ap, x, y, z, R, obs = make(orc, convex, baffle, with_y)
    L0, rf = loss(orc, su, g, dl, ap, x, y, z, R, obs)
    grad = orc.adjoint(su, g, dl, ap, x, y, z, R, rf - obs)
    h = 1e-8
    for s in range(x.size):
        for name, arr in (("x", x), ("y", y), ("z", z)):
            if name == "y" and not with_y:
                continue
            p, m = arr.copy(), arr.copy()
            p[s] += h
            m[s] -= h
            args = dict(x=x, y=y, z=z)
            Lp = loss(orc, su, g, dl, ap, **{**args, name: p}, R=R, obs=obs)[0]
            Lm = loss(orc, su, g, dl, ap, **{**args, name: m}, R=R, obs=obs)[0]
            fd = (Lp - Lm) / (2 * h)
            scale = max(abs(fd), 1e-3 * np.abs(grad[name]).max())
            assert abs(grad[name][s] - fd) < 2e-5 * scale, (name, s, grad[name][s], fd)
        # L is quadratic in R: the central difference is exact up to rounding
        p, m = R.copy(), R.copy()
        p[s] += 1e-3
        m[s] -= 1e-3
        fd = (loss(orc, su, g, dl, ap, x, y, z, p, obs)[0] - loss(orc, su, g, dl, ap, x, y, z, m, obs)[0]) / 2e-3
        assert abs(grad["R"][s] - fd) < 1e-8 * max(abs(fd), 1.0)


def test_adjoint_euler_identity(orc):
    """rf is linear in R, so sum_s R_s dL/dR_s = <rho, rf>."""
    su, g, dl, ap, x, y, z, R, obs = make(orc)
    _, rf = loss(orc, su, g, dl, ap, x, y, z, R, obs)
    rho = rf - obs
    grad = orc.adjoint(su, g, dl, ap, x, y, z, R, rho)
    lhs = np.sum(R * grad["R"])
    rhs = np.sum(rho * rf)
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)


def test_adjoint_reflectivity_dot_product(orc):
    """<J v, rho> = <v, J^T rho> for J = d rf / d R (a linear map)."""
    su, g, dl, ap, x, y, z, R, _ = make(orc, with_y=False)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(R.size)
    rho = rng.standard_normal((2, su.n_elements, g["n_t"]))
    Jv = orc.rf(su, g, dl, ap, x, y, z, v)
    JT = orc.adjoint(su, g, dl, ap, x, y, z, R, rho)["R"]
    assert abs(np.sum(Jv * rho) - np.sum(v * JT)) < 1e-10 * abs(np.sum(Jv * rho))


def test_adjoint_selection_matches_full(orc):
    su, g, dl, ap, x, y, z, R, obs = make(orc)
    _, rf = loss(orc, su, g, dl, ap, x, y, z, R, obs)
    full = orc.adjoint(su, g, dl, ap, x, y, z, R, rf - obs)
    part = orc.adjoint(su, g, dl, ap, x, y, z, R, rf - obs, sel=[2, 0])
    for k in "Rxyz":
        assert np.array_equal(part[k], full[k][[2, 0]])
