"""Seeded synthetic inputs: probes, transmit sequences and phantoms.

This module holds input recipes only -- no part of the RF synthesis itself.
Both the HIP path (tests, bench) and the FP64 oracle (tests) draw their
inputs from here, so that the two sides see bit-identical data.

Workloads follow the shapes of the paper's examples (SIMUS Part I, Figs. 8,
10-13): linear 7.6 MHz and convex 3 MHz probes, plane and diverging waves,
uniformly distributed point scatterers with N(0, 1) reflectivity.

Draw order inside one generator: scatterer counts (batched phantoms), then
x, z, reflectivity.  y = 0 (scatterers in the azimuth plane).
"""
from __future__ import annotations

import math

import numpy as np

MM = 1e-3


def linear_probe(n_elements: int = 128) -> dict:
    """Linear array: pitch 0.3 mm, width 0.27 mm, height 5 mm, elevation
    focus 18 mm, fc 7.6 MHz, 77 % pulse-echo bandwidth (cf. Figs. 8, 10)."""
    return dict(n_elements=n_elements, fc=7.6e6, pitch=0.3 * MM, width=0.27 * MM,
                height=5 * MM, elev_focus=18 * MM, bandwidth=0.77, radius=0.0,
                baffle=0, zeta=1.75)


def convex_probe(n_elements: int = 128) -> dict:
    """Convex array: radius 60 mm, pitch 0.5 mm, width 0.45 mm, height
    13 mm, elevation focus 60 mm, fc 3 MHz, 77 % bandwidth."""
    return dict(n_elements=n_elements, fc=3e6, pitch=0.5 * MM, width=0.45 * MM,
                height=13 * MM, elev_focus=60 * MM, bandwidth=0.77, radius=60 * MM,
                baffle=0, zeta=1.75)


def phased_probe(n_elements: int = 64) -> dict:
    """Phased array (cardiac, cf. Figs. 9 and 12): pitch 0.3 mm, width
    0.25 mm, height 14 mm, elevation focus 60 mm, fc 2.7 MHz, 74 %
    bandwidth."""
    return dict(n_elements=n_elements, fc=2.7e6, pitch=0.3 * MM, width=0.25 * MM,
                height=14 * MM, elev_focus=60 * MM, bandwidth=0.74, radius=0.0,
                baffle=0, zeta=1.75)


def element_centres(probe: dict) -> np.ndarray:
    """Element centres (x, z) [N, 2]; convex: apex at the origin, centre of
    curvature at (0, -R), chord pitch."""
    N = probe["n_elements"]
    e = np.arange(1, N + 1, dtype=np.float64)
    R = probe.get("radius", 0.0)
    if R <= 0:
        return np.stack([probe["pitch"] * (e - (N + 1) / 2), np.zeros(N)], -1)
    dphi = 2 * math.asin(probe["pitch"] / (2 * R))
    phi = (e - (N + 1) / 2) * dphi
    return np.stack([R * np.sin(phi), R * np.cos(phi) - R], -1)


def plane_wave_delays(probe: dict, angles_deg, c: float = 1540.0) -> np.ndarray:
    """Steered plane waves on a linear array: delays [T, N] in seconds,
    positive = fires later, min delay 0."""
    xe = element_centres(probe)[:, 0]
    out = []
    for a in np.atleast_1d(angles_deg):
        d = xe * math.sin(math.radians(a)) / c
        out.append(d - d.min())
    return np.asarray(out, dtype=np.float64)


def diverging_wave_delays(probe: dict, xv_list, zv: float, c: float = 1540.0) -> np.ndarray:
    """Diverging waves from virtual sources (xv, zv): delays [T, N]."""
    ec = element_centres(probe)
    out = []
    for xv in np.atleast_1d(xv_list):
        d = np.hypot(ec[:, 0] - xv, ec[:, 1] - zv) / c
        out.append(d - d.min())
    return np.asarray(out, dtype=np.float64)


def focused_delays(probe: dict, angles_deg, depth: float, c: float = 1540.0) -> np.ndarray:
    """Focused transmits steered to angles_deg at `depth` from the array
    centre: delays [T, N], min delay 0."""
    ec = element_centres(probe)
    out = []
    for a in np.atleast_1d(angles_deg):
        fx, fz = depth * math.sin(math.radians(a)), depth * math.cos(math.radians(a))
        d = np.hypot(ec[:, 0] - fx, ec[:, 1] - fz) / c
        out.append(d.max() - d)
    return np.asarray(out, dtype=np.float64)


def rect_phantom(rng, n: int, x_range, z_range, disks=()):
    """n scatterers uniform in a rectangle; N(0,1) reflectivity, zeroed
    inside the given anechoic disks (cx, cz, radius)."""
    x = rng.uniform(x_range[0], x_range[1], n)
    z = rng.uniform(z_range[0], z_range[1], n)
    R = rng.standard_normal(n)
    for cx, cz, rad in disks:
        R[(x - cx) ** 2 + (z - cz) ** 2 < rad ** 2] = 0.0
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(x=f(x), y=np.zeros(n, np.float32), z=f(z), R=f(R))


def sector_phantom(rng, n: int, radius: float, depth_max: float, half_angle_deg: float,
                   depth_min: float = 1 * MM):
    """n scatterers area-uniform in an annular sector about (0, -radius)."""
    phi = rng.uniform(-math.radians(half_angle_deg), math.radians(half_angle_deg), n)
    rho = np.sqrt(rng.uniform((radius + depth_min) ** 2, (radius + depth_max) ** 2, n))
    R = rng.standard_normal(n)
    x = rho * np.sin(phi)
    z = rho * np.cos(phi) - radius
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(x=f(x), y=np.zeros(n, np.float32), z=f(z), R=f(R))


def _common(probe, delays, phantoms, alpha_db, n_t, name, **extra):
    T, N = delays.shape
    return dict(name=name, probe=probe,
                medium=dict(c=1540.0, alpha_db=alpha_db),
                options=dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7,
                             nfft=0, n_t=n_t),
                delays=delays, apod=np.ones((T, N), np.float32), phantoms=phantoms, **extra)


def depth_samples(depth: float, fs: float, c: float = 1540.0) -> int:
    return int(math.ceil(fs * 2 * depth / c))


def workload(name: str, seed: int = 0, scale: float = 1.0) -> dict:
    """Named synthetic workloads.  `scale` shrinks scatterer counts (tests)."""
    rng = np.random.default_rng(seed)
    S = lambda n: max(1, int(round(n * scale)))
    if name == "pw32_s200":
        # 32-element linear array, one 0-degree plane wave, 200 scatterers
        # in x in [-5, 5] mm, z in [5, 30] mm, no attenuation.
        probe = linear_probe(32)
        ph = rect_phantom(rng, S(200), (-5 * MM, 5 * MM), (5 * MM, 30 * MM))
        return _common(probe, plane_wave_delays(probe, [0.0]), [ph], 0.0, 0, name)
    if name == "pw128_s50k":
        # 128 elements, 0-degree plane wave, 50,000 scatterers in 40 x 40 mm
        # from z = 5 mm, three 5 mm anechoic disks, 0.5 dB/cm/MHz, 50 mm depth.
        probe = linear_probe(128)
        disks = [(-10 * MM, 15 * MM, 2.5 * MM), (0.0, 25 * MM, 2.5 * MM), (10 * MM, 35 * MM, 2.5 * MM)]
        ph = rect_phantom(rng, S(50_000), (-20 * MM, 20 * MM), (5 * MM, 45 * MM), disks)
        n_t = depth_samples(50 * MM, 4 * probe["fc"])
        return _common(probe, plane_wave_delays(probe, [0.0]), [ph], 0.5, n_t, name)
    if name == "pw128x21_s200k":
        # 21 steered plane waves -10..10 degrees, 200,000 scatterers.
        probe = linear_probe(128)
        ph = rect_phantom(rng, S(200_000), (-20 * MM, 20 * MM), (5 * MM, 45 * MM))
        n_t = depth_samples(50 * MM, 4 * probe["fc"])
        return _common(probe, plane_wave_delays(probe, np.arange(-10, 11)), [ph], 0.5, n_t, name)
    if name == "cvx128x11_p16":
        # convex 128 elements, 11 diverging waves, 16 phantoms of 10k-500k
        # scatterers (log-uniform) in a 90-degree sector to 120 mm depth.
        probe = convex_probe(128)
        counts = np.round(np.exp(rng.uniform(math.log(1e4), math.log(5e5), 16))).astype(np.int64)
        phs = [sector_phantom(rng, S(int(n)), probe["radius"], 120 * MM, 45.0) for n in counts]
        dl = diverging_wave_delays(probe, np.linspace(-30 * MM, 30 * MM, 11), -60 * MM)
        n_t = depth_samples(120 * MM, 4 * probe["fc"])
        return _common(probe, dl, phs, 0.5, n_t, name)
    if name == "ph64x128_s40k":
        # 64-element 2.7 MHz phased array, 128 focused transmits steered over
        # -45..45 degrees (focus 60 mm), 40,000 scatterers in a 90-degree
        # sector to 120 mm (the shape of Fig. 12's sequence).
        probe = phased_probe(64)
        ph = sector_phantom(rng, S(40_000), 0.0, 120 * MM, 45.0, depth_min=5 * MM)
        dl = focused_delays(probe, np.linspace(-45, 45, 128), 60 * MM)
        n_t = depth_samples(120 * MM, 4 * probe["fc"])
        return _common(probe, dl, [ph], 0.5, n_t, name)
    if name == "pw128x5_s100k":
        # 5 plane waves (-8, -4, 0, 4, 8 degrees), 100,000 scatterers.
        probe = linear_probe(128)
        ph = rect_phantom(rng, S(100_000), (-20 * MM, 20 * MM), (5 * MM, 45 * MM))
        n_t = depth_samples(50 * MM, 4 * probe["fc"])
        return _common(probe, plane_wave_delays(probe, [-8, -4, 0, 4, 8]), [ph], 0.5, n_t, name)
    raise KeyError(name)


def concat_phantoms(phs):
    """Concatenated SoA scatterers of a list of phantoms and the offsets
    [P + 1] of each phantom's first scatterer."""
    x = np.concatenate([p["x"] for p in phs])
    y = np.concatenate([p["y"] for p in phs])
    z = np.concatenate([p["z"] for p in phs])
    R = np.concatenate([p["R"] for p in phs])
    off = np.cumsum([0] + [p["x"].size for p in phs]).astype(np.int64)
    return x, y, z, R, off


def perturbed(ph: dict, seed: int = 1, sigma_pos: float = 50e-6, sigma_R: float = 0.1) -> dict:
    """Observed phantom for the misfit: positions + N(0, 50 um), R + N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    n = ph["x"].size
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(x=f(ph["x"] + rng.normal(0, sigma_pos, n)), y=ph["y"].copy(),
                z=f(ph["z"] + rng.normal(0, sigma_pos, n)),
                R=f(ph["R"] + rng.normal(0, sigma_R, n)))


WORKLOADS = ["pw32_s200", "pw128_s50k", "pw128x21_s200k", "cvx128x11_p16", "pw128x5_s100k",
             "ph64x128_s40k"]
