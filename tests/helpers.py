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
                     nu=nu or o.get("nu", 0), dim2=1 if o.get("flags", 0) & 8 else 0)


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
