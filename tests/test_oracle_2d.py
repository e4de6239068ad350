"""Pins of the oracle's 2-D acoustics (Section V, Eqs. 35-38).

The 2-D Green's term is pinned against the 3-D one, which is pinned in
test_oracle_pins.py: Section V obtains 2-D as the limit h -> inf,
R_f -> inf of the 3-D model, where alpha_g -> -i k / (2 r) and
sqrt(pi / alpha_g) -> sqrt(2 i pi r / k).  With the four Gaussians of
Eq. (18) the 3-D term then tends to (sum_g A_g) sqrt(2 i pi / k) times the
2-D term.  The remaining pins are closed forms (on-axis echo, inverse
square-root spreading, directivity, RMS field) and invariants (y is not
used; finite-difference gradients).
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def sum_A():
    a = np.loadtxt(os.path.join(GOLD, "gauss4_eq18.txt"))
    return complex(np.sum(a[:, 0]), np.sum(a[:, 1]))


def setup(orc, **kw):
    base = dict(n_elements=1, fc=7.6e6, pitch=0.3e-3, width=0.27e-3, height=5e-3,
                elev_focus=18e-3, bandwidth=0.77, c=1540.0, alpha_db=0.0, fs=30.4e6, nu=1)
    base.update(kw)
    return orc.Setup(**base)


def test_2d_is_the_limit_of_3d(orc):
    """3-D with h = 10 km and R_f = inf against 2-D: ratio
    (sum A_g) sqrt(2 i pi / k) at every point, frequency and baffle."""
    sA = sum_A()
    assert abs(sA - 0.95) < 1e-12              # the conjugate pairs cancel
    for baffle in (0, 1, 2):
        s3 = setup(orc, height=1e4, elev_focus=math.inf, baffle=baffle, nu=2, n_elements=3)
        s2 = setup(orc, dim2=1, baffle=baffle, nu=2, n_elements=3)
        for f in (3e6, 7.6e6, 11e6):
            w = 2 * np.pi * f
            k = w / s3.c
            for n in range(6):
                for x, z in [(0.0, 10e-3), (2e-3, 25e-3), (-4e-3, 8e-3), (1e-3, 40e-3)]:
                    g3 = orc.green(s3, n, x, 0.0, z, w)
                    g2 = orc.green(s2, n, x, 0.0, z, w)
                    ratio = sA * np.sqrt(2j * np.pi / k)
                    assert abs(g3 - ratio * g2) < 1e-9 * abs(g3)


def test_2d_spreading_and_phase_on_axis(orc):
    """On axis (D = 1, no attenuation) the 2-D term is exp(i k z) / sqrt(z)."""
    su = setup(orc, dim2=1)
    w = 2 * np.pi * 5e6
    k = w / su.c
    for z in (5e-3, 12e-3, 37e-3):
        g = orc.green(su, 0, 0.0, 0.0, z, w)
        assert abs(g - np.exp(1j * k * z) / math.sqrt(z)) < 1e-12 * abs(g)
    g1, g2 = orc.green(su, 0, 0.0, 0.0, 10e-3, w), orc.green(su, 0, 0.0, 0.0, 20e-3, w)
    assert abs(abs(g2 / g1) - 1 / math.sqrt(2)) < 1e-12


def test_2d_ignores_y_and_keeps_the_directivity(orc):
    """The 2-D domain is the x-z plane: a point's y does not enter; the
    angular factor is the same sinc times cos(theta) as in 3-D."""
    su = setup(orc, dim2=1)
    w = 2 * np.pi * 7.6e6
    k = w / su.c
    b = su.width / 2
    r = 20e-3
    g0 = orc.green(su, 0, 0.0, 0.0, r, w)
    for th in np.radians([5, 20, 45]):
        x, z = r * math.sin(th), r * math.cos(th)
        g = orc.green(su, 0, x, 0.0, z, w)
        assert orc.green(su, 0, x, 3e-3, z, w) == g
        u = k * b * math.sin(th)
        assert abs(g / g0 - math.sin(u) / u * math.cos(th)) < 1e-12


def test_2d_on_axis_echo_closed_form(orc):
    """Eq. (38), one element, nu = 1, scatterer on axis at z0 with
    attenuation: X_j = 2b S_P S_T R exp(2 i (k + i k_a) z0) / z0."""
    su = setup(orc, dim2=1, alpha_db=0.5)
    z0 = 23e-3
    nfft = 2048
    bins = np.arange(100, 700, 41)
    X = orc.spectrum(su, nfft, np.zeros((1, 1)), np.ones((1, 1)), [0.0], [0.0], [z0], [1.3], bins)[0, 0]
    for j, xj in zip(bins, X):
        w = 2 * np.pi * j * su.fs / nfft
        k = w / su.c
        ka = su.alpha_db / 8.69 * (w / (2 * np.pi)) / 1e4
        P = orc.pulse_spectrum(su, w) * orc.transducer_spectrum(su, w)
        expected = su.width * P * 1.3 * np.exp(2j * (k + 1j * ka) * z0) / z0
        assert abs(xj - expected) < 1e-10 * abs(expected)


def test_2d_pfield_riemann_sum(orc):
    """Eqs. (37), (41), (42) in 2-D, one element on axis: |P|^2 = 2b |S_P|^2
    S_T / z0, so P_RMS^2 approaches 2b / z0 times the integral of |S_P|^2
    S_T over [0, 2 wc]."""
    from scipy.integrate import quad
    su = setup(orc, dim2=1)
    z0 = 15e-3
    wc = 2 * np.pi * su.fc
    integ, _ = quad(lambda w: abs(orc.pulse_spectrum(su, w)) ** 2 * orc.transducer_spectrum(su, w),
                    0, 2 * wc, limit=400)
    expected = math.sqrt(integ * su.width / z0)
    for nf in (64, 256):
        prms = orc.pfield(su, np.zeros(1), np.ones(1), nf, [0.0], [0.0], [z0])[0]
        assert abs(prms - expected) < 2e-3 * expected


@pytest.mark.parametrize("convex", [False, True])
def test_2d_adjoint_matches_finite_differences(orc, convex):
    """The oracle's analytic 2-D gradients against central differences of
    its own 2-D RF (positions: h = 1e-8 m; R enters linearly)."""
    rng = np.random.default_rng(5)
    if convex:
        su = setup(orc, dim2=1, n_elements=6, radius=20e-3, pitch=0.5e-3, width=0.45e-3, fc=3e6,
                   fs=12e6, nu=2, alpha_db=0.4)
    else:
        su = setup(orc, dim2=1, n_elements=6, nu=2, alpha_db=0.4)
    n = 5
    x = rng.uniform(-2e-3, 2e-3, n)
    z = rng.uniform(8e-3, 18e-3, n)
    y = np.zeros(n)
    R = rng.standard_normal(n)
    dl = np.linspace(0, 2e-7, 6)[None, :]
    ap = np.ones((1, 6))
    g = orc.grid(su, dl, x, y, z)
    rho = rng.standard_normal((1, 6, g["n_t"]))
    grads = orc.adjoint(su, g, dl, ap, x, y, z, R, rho)

    def L(xx, zz, RR):
        return float(np.sum(rho * orc.rf(su, g, dl, ap, xx, y, zz, RR)))

    h = 1e-8
    for s in range(n):
        for key, arr in (("x", x), ("z", z)):
            ap_, am_ = arr.copy(), arr.copy()
            ap_[s] += h
            am_[s] -= h
            if key == "x":
                fd = (L(ap_, z, R) - L(am_, z, R)) / (2 * h)
            else:
                fd = (L(x, ap_, R) - L(x, am_, R)) / (2 * h)
            assert abs(grads[key][s] - fd) < 1e-5 * (abs(fd) + 1e-3 * np.max(np.abs(grads[key]))), (key, s)
        assert abs(grads["y"][s]) == 0.0
