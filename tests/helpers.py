"""Shared test helpers: build the oracle's setup and the library's arguments
from one workload recipe, and compare results."""
import math

import numpy as np

from paper_2102_02738_amd.inputs import concat_phantoms  # noqa: F401

ORACLE_KEYS = ["n_elements", "fc", "pitch", "width", "height", "elev_focus", "bandwidth", "radius",
               "baffle", "zeta"]


def oracle_setup(orc, w: dict, nu: int = 0):
    p = w["probe"]
    o = w["options"]
    return orc.Setup(**{k: p[k] for k in ORACLE_KEYS}, c=w["medium"]["c"],
                     alpha_db=w["medium"]["alpha_db"], fs=o["fs"], n_cycles=o["n_cycles"],
                     nu=nu or o.get("nu", 0), dim2=1 if o.get("flags", 0) & 8 else 0,
                     gauss=o.get("gauss"))


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(*arrs, device="cuda"):
    import torch
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
            for a in arrs]


def sample_bins(g: dict, k: int) -> np.ndarray:
    """k bins spread over the band, always including its first and last bin."""
    lo, n = g["j_lo"], g["n_bins"]
    return np.unique(np.round(np.linspace(0, n - 1, k)).astype(np.int64)) + lo


def assert_grid_matches(orc, w: dict, g: dict, x, y, z):
    """The library's grid (simus_rf_grid) equals the oracle's for the same
    call, integer for integer."""
    su = oracle_setup(orc, w)
    yy = np.zeros_like(x) if y is None else y
    og = orc.grid(su, w["delays"], x, yy, z, n_t=w["options"].get("n_t", 0),
                  eps=w["options"].get("spectral_eps", 1e-7))
    for k in ("nfft", "n_t", "j_lo", "n_bins"):
        assert g[k] == og[k], (k, g, og)


def oracle_spectrum_split(orc, su, nfft, delays, apod, x, y, z, R, bins, parts: int = 4):
    """The oracle's spectra at `bins`, computed as the sum of its spectra over
    `parts` disjoint slices of the scatterers, run concurrently (the spectra
    of Eqs. 31-34 are a sum over scatterers; the oracle parallelises over
    bins only, so few bins of many scatterers would use few cores)."""
    from concurrent.futures import ThreadPoolExecutor
    n = len(x)
    cuts = np.linspace(0, n, parts + 1).astype(np.int64)
    yy = np.zeros(n) if y is None else y

    def one(k):
        sl = slice(cuts[k], cuts[k + 1])
        return orc.spectrum(su, nfft, delays, apod, x[sl], yy[sl], z[sl], R[sl], bins)

    with ThreadPoolExecutor(max_workers=parts) as ex:
        return sum(ex.map(one, range(parts)))


def band_peak_bin(orc, su, g: dict) -> int:
    """Absolute index of the band's bin of largest |S_P S_T| (Eqs. 25, 27),
    from the oracle's spectra."""
    js = np.arange(g["j_lo"], g["j_lo"] + g["n_bins"])
    df = su.fs / g["nfft"]
    mag = [abs(orc.pulse_spectrum(su, 2 * np.pi * j * df)) * orc.transducer_spectrum(su, 2 * np.pi * j * df)
           for j in js]
    return int(js[int(np.argmax(mag))])
