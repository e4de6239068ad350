"""CPU-side checks of libsimus: it loads, exports every declared symbol, its
host-only planning agrees with the oracle, and invalid arguments are
rejected on the host before any GPU call."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from tests.helpers import oracle_setup

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2102_02738_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    header = open(os.path.join(ROOT, "include", "simus.h")).read()
    declared = set(re.findall(r"\b(simus_[a-z_]+)\s*\(", header))
    assert declared, "no declarations parsed"
    lib = L.lib()
    missing = [s for s in sorted(declared) if not hasattr(lib, s)]
    assert not missing, missing
    assert set(L.EXPORTS) == declared
    assert lib.simus_version() == 201


@pytest.mark.parametrize("name,scale", [("pw32_s200", 1.0), ("pw128_s50k", 0.01),
                                        ("pw128x21_s200k", 0.002), ("cvx128x11_p16", 0.001),
                                        ("pw128x5_s100k", 0.003)])
def test_grid_agrees_with_oracle(L, orc, name, scale):
    from paper_2102_02738_amd import inputs
    w = inputs.workload(name, scale=scale)
    from tests.helpers import concat_phantoms
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = L.rf_grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    su = oracle_setup(orc, w)
    go = orc.grid(su, w["delays"], x, y, z, n_t=w["options"]["n_t"])
    for k in ("nfft", "n_t", "j_lo", "n_bins"):
        assert g[k] == go[k], (k, g, go)
    assert g["nu"] == su.resolved_nu()
    assert g["df"] == w["options"]["fs"] / g["nfft"]


def test_pfield_nf_agrees_with_oracle(L, orc):
    from paper_2102_02738_amd import inputs
    probe = inputs.linear_probe(64)
    dl = inputs.plane_wave_delays(probe, [10.0])[0]
    X, Z = np.meshgrid(np.linspace(-10e-3, 10e-3, 7), np.linspace(2e-3, 40e-3, 5))
    X, Z = X.ravel().astype(np.float32), Z.ravel().astype(np.float32)
    w = dict(probe=probe, medium=dict(c=1540.0, alpha_db=0.5),
             options=dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0))
    nf = L.pfield_nf(probe, w["medium"], w["options"], dl, X, None, Z)
    nfo = orc.pfield_nf(oracle_setup(orc, w), dl, X, np.zeros_like(X), Z)
    assert nf == nfo


def _base():
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.05)
    return w


def _grid_call(L, probe=None, medium=None, options=None, delays=None, x=None, z=None):
    w = _base()
    ph = w["phantoms"][0]
    return L.rf_grid(probe or w["probe"], medium or w["medium"], options or w["options"],
                     w["delays"] if delays is None else delays,
                     ph["x"] if x is None else x, None, ph["z"] if z is None else z)


@pytest.mark.parametrize("field,value,code", [
    ("n_elements", 0, -1), ("width", 0.5e-3, -1), ("bandwidth", 2.5, -1), ("height", -1.0, -1),
    ("baffle", 7, -1), ("elev_focus", 0.0, -1), ("fc", float("nan"), -1)])
def test_invalid_probe_rejected(L, field, value, code):
    w = _base()
    p = dict(w["probe"])
    p[field] = value
    with pytest.raises(L.SimusError) as ei:
        _grid_call(L, probe=p)
    assert ei.value.code == code


@pytest.mark.parametrize("field,value", [("fs", 1e6), ("spectral_eps", 1.5), ("nfft", 1001),
                                         ("nu", -2), ("n_cycles", 0.0), ("flags", 128),
                                         ("flags", -1)])
def test_invalid_options_rejected(L, field, value):
    w = _base()
    o = dict(w["options"])
    o[field] = value
    with pytest.raises(L.SimusError) as ei:
        _grid_call(L, options=o)
    assert ei.value.code == -1


def test_domain_errors(L):
    w = _base()
    ph = w["phantoms"][0]
    z = ph["z"].copy()
    z[3] = -1e-3
    with pytest.raises(L.SimusError) as ei:
        _grid_call(L, z=z)
    assert ei.value.code == -2
    x = ph["x"].copy()
    x[0] = np.nan
    with pytest.raises(L.SimusError) as ei:
        _grid_call(L, x=x)
    assert ei.value.code == -2
    # negative delays are invalid
    with pytest.raises(L.SimusError) as ei:
        _grid_call(L, delays=-np.ones_like(w["delays"]))
    assert ei.value.code == -1


def test_n_t_above_nfft_rejected(L):
    w = _base()
    o = dict(w["options"], nfft=512, n_t=600)
    with pytest.raises(L.SimusError):
        _grid_call(L, options=o)


def test_fixed_nfft_is_kept(L):
    w = _base()
    g = _grid_call(L, options=dict(w["options"], nfft=4000, n_t=1000))
    assert g["nfft"] == 4000 and g["n_t"] == 1000


def test_device_entry_points_validate_before_gpu(L):
    """Invalid calls fail on the host with EINVAL; the pointers passed are
    never dereferenced (there is no GPU here)."""
    w = _base()
    lib = L.lib()
    P, M = L.make_probe(w["probe"]), L.make_medium(w["medium"])
    d = np.ascontiguousarray(w["delays"], dtype=np.float64)
    a = np.ones_like(d, dtype=np.float32)
    off = np.array([0, 10], dtype=np.int64)
    fake = C.c_void_p(0x1000)
    pd = d.ctypes.data_as(C.POINTER(C.c_double))
    pa = a.ctypes.data_as(C.POINTER(C.c_float))
    po = off.ctypes.data_as(C.POINTER(C.c_int64))
    cases = [
        (L.make_options(w["options"], nfft=0), 1, po, 1),                 # nfft required
        (L.make_options(w["options"], nfft=1280), 0, po, 1),              # n_tx = 0
        (L.make_options(w["options"], nfft=1280), 1, po, 0),              # no phantom
        (L.make_options(w["options"], nfft=1280, n_t=2000), 1, po, 1),    # n_t > nfft
    ]
    for O, ntx, offs, nph in cases:
        rc = lib.simus_rf(C.byref(P), C.byref(M), C.byref(O), ntx, pd, pa, nph, offs,
                          fake, None, fake, fake, fake, None)
        assert rc == -1, lib.simus_last_error()
    bad = np.array([0, 10, 5], dtype=np.int64)
    rc = lib.simus_rf(C.byref(P), C.byref(M), C.byref(L.make_options(w["options"], nfft=1280)), 1,
                      pd, pa, 2, bad.ctypes.data_as(C.POINTER(C.c_int64)), fake, None, fake, fake,
                      fake, None)
    assert rc == -1 and b"non-decreasing" in lib.simus_last_error()
    # work items index scatterers with int32: 2^31 scatterers are rejected
    huge = np.array([0, 1 << 31], dtype=np.int64)
    rc = lib.simus_rf(C.byref(P), C.byref(M), C.byref(L.make_options(w["options"], nfft=1280)), 1,
                      pd, pa, 1, huge.ctypes.data_as(C.POINTER(C.c_int64)), fake, None, fake, fake,
                      fake, None)
    assert rc == -1 and b"too many scatterers" in lib.simus_last_error()
    rc = lib.simus_spectrum_to_rf(1001, 10, 1, 4, 1, fake, fake, None)
    assert rc == -1
    rc = lib.simus_spectrum_to_rf(1000, 10, 499, 4, 1, fake, fake, None)
    assert rc == -1


def test_plan_entry_points_validate_before_gpu(L):
    """Plan creation rejects invalid arguments on the host (EINVAL, no plan
    returned); execute and graph launch reject a NULL plan; destroy ignores
    NULL."""
    w = _base()
    lib = L.lib()
    P, M = L.make_probe(w["probe"]), L.make_medium(w["medium"])
    d = np.ascontiguousarray(w["delays"], dtype=np.float64)
    a = np.ones_like(d, dtype=np.float32)
    off = np.array([0, 10], dtype=np.int64)
    pd = d.ctypes.data_as(C.POINTER(C.c_double))
    pa = a.ctypes.data_as(C.POINTER(C.c_float))
    po = off.ctypes.data_as(C.POINTER(C.c_int64))
    h = C.c_void_p()
    for O, ntx, nph in [(L.make_options(w["options"], nfft=0), 1, 1),
                        (L.make_options(w["options"], nfft=1280), 0, 1),
                        (L.make_options(w["options"], nfft=1280), 1, 0),
                        (L.make_options(w["options"], nfft=1280, n_t=2000), 1, 1)]:
        rc = lib.simus_rf_plan_create(C.byref(P), C.byref(M), C.byref(O), ntx, pd, pa, nph, po, 0,
                                      None, C.byref(h))
        assert rc == -1, lib.simus_last_error()
        assert not h.value
    O = L.make_options(w["options"], nfft=1280)
    assert lib.simus_rf_plan_create(C.byref(P), C.byref(M), C.byref(O), 1, pd, pa, 1, po, 0, None,
                                    None) == -1
    fake = C.c_void_p(0x1000)
    assert lib.simus_rf_plan_execute(None, fake, None, fake, fake, fake, None) == -1
    assert lib.simus_rf_plan_graph_launch(None, fake, None, fake, fake, fake, None) == -1
    assert lib.simus_rf_plan_autotune(None, fake, None, fake, fake, fake, None, None, None) == -1
    lib.simus_rf_plan_destroy(None)


def test_package_raises_without_library(monkeypatch, tmp_path):
    """The product path fails loudly when the HIP library is missing."""
    from paper_2102_02738_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(_lib.SimusError):
        _lib.lib()


def test_binding_refuses_small_buffers(L):
    """The library takes raw device pointers; the binding refuses tensors
    smaller than what a call reads or writes, before any library call (CPU
    tensors of the right size are then refused as not on the device)."""
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.1)
    ph = w["phantoms"][0]
    n = ph["x"].size
    x, z, R = (torch.from_numpy(ph[k].astype(np.float32)) for k in ("x", "z", "R"))
    n_tx, N, n_t = w["delays"].shape[0], w["probe"]["n_elements"], 64
    o = dict(w["options"], nfft=128, n_t=n_t)
    args = (w["probe"], w["medium"], o, w["delays"], w["apod"])
    good = torch.empty(n_tx * N * n_t)
    with pytest.raises(L.SimusError, match="rf holds"):
        L.rf_into(good[:-1], *args, x, None, z, R)
    with pytest.raises(L.SimusError, match="refl holds"):
        L.rf_into(good, *args, x, None, z, R[:-1])
    with pytest.raises(L.SimusError, match="device tensor expected"):
        L.rf_into(good, *args, x, None, z, R)
    with pytest.raises(L.SimusError, match="drf holds"):
        L.rf_backward_into({}, *args, x, None, z, R, good[:-1])
    with pytest.raises(L.SimusError, match="gradient x holds"):
        L.rf_backward_into({"x": torch.empty(n - 1)}, *args, x, None, z, R, good)
    with pytest.raises(L.SimusError, match="p_rms holds"):
        L.pfield_into(torch.empty(n - 1), w["probe"], w["medium"], o, 10, w["delays"][0], None,
                      x, None, z)
    with pytest.raises(L.SimusError, match="spec holds"):
        L.spectrum_to_rf_into(torch.empty(4 * n_t), torch.empty(4 * 2 * 10 - 1), 128, n_t, 1, 10, 4)
    # offsets past the end of the scatterer arrays
    with pytest.raises(L.SimusError, match="scat_offsets end at"):
        L.rf_into(good, *args, x, None, z, R, offsets=[0, n + 1])
    with pytest.raises(L.SimusError, match="scat_offsets end at"):
        L.rf_backward_into({}, *args, x, None, z, R, good, offsets=[0, 2, n + 3])
    # n_t = 0 means nfft samples per channel
    o0 = dict(o, n_t=0)
    with pytest.raises(L.SimusError, match="rf holds"):
        L.rf_into(good, w["probe"], w["medium"], o0, w["delays"], w["apod"], x, None, z, R)
    with pytest.raises(L.SimusError, match="drf holds"):
        L.rf_backward_into({}, w["probe"], w["medium"], o0, w["delays"], w["apod"], x, None, z, R, good)
    # the spectra of rf_spectrum_into: [n_ph][n_tx][N][n_bins] complex
    n_bins = L.rf_grid(w["probe"], w["medium"], o, w["delays"], [], None, [])["n_bins"]
    with pytest.raises(L.SimusError, match="spec holds"):
        L.rf_spectrum_into(torch.empty(2 * n_tx * N * n_bins - 1), *args, x, None, z, R)
    with pytest.raises(L.SimusError, match="device tensor expected"):
        L.rf_spectrum_into(torch.empty(2 * n_tx * N * n_bins), *args, x, None, z, R)
    # float32 only
    with pytest.raises(L.SimusError, match="must be float32"):
        L.rf_into(good.double(), *args, x, None, z, R)
    with pytest.raises(L.SimusError, match="must be float32"):
        L.rf_into(good, *args, x.double(), None, z, R)
    # transmit arrays of the probe's shape
    with pytest.raises(L.SimusError, match="apod holds"):
        L.rf_into(good, w["probe"], w["medium"], o, w["delays"], w["apod"][:, :-1], x, None, z, R)
    with pytest.raises(L.SimusError, match="delays hold"):
        L.rf_into(good, w["probe"], w["medium"], o, w["delays"][:, :-1], None, x, None, z, R)
    with pytest.raises(L.SimusError, match="delays hold"):
        L.pfield_into(torch.empty(n), w["probe"], w["medium"], o, 10, w["delays"][0][:-1], None,
                      x, None, z)


def test_product_and_oracle_share_no_code():
    """The HIP path and the FP64 oracle are independent: no package source
    imports or includes anything under oracle/, and no oracle source imports
    the package (the seeded input generators are the only shared module, and
    the oracle receives their arrays from the tests)."""
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2102_02738_amd")
    bad = []
    for d, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(d, f), encoding="utf-8").read()
                if re.search(r"^\s*(from|import)\s+oracle\b|#include\s+[\"<][^\">]*oracle", src, re.M):
                    bad.append(os.path.join(d, f))
    for d, _, files in os.walk(os.path.join(root, "oracle")):
        for f in files:
            if f.endswith((".py", ".c", ".h")):
                src = open(os.path.join(d, f), encoding="utf-8").read()
                if re.search(r"^\s*(from|import)\s+paper_2102_02738_amd\b|#include\s+[\"<][^\">]*(simus\.h|csrc)", src, re.M):
                    bad.append(os.path.join(d, f))
    assert not bad, bad


def test_gaussian_set_validation(L):
    """options.gauss: at most 32 Gaussians, finite, Re B_g > 0; a valid set
    is accepted by the host planning."""
    from paper_2102_02738_amd import gaussians as GS
    w = _base()
    ok = dict(w["options"], gauss=GS.fit(6))
    _grid_call(L, options=ok)
    bad_b = GS.fit(4).copy()
    bad_b[1, 1] = -1.0 + 2.0j
    for gset in (bad_b, np.full((2, 2), np.nan + 0j), np.tile(GS.EQ18, (9, 1))):
        with pytest.raises(L.SimusError) as ei:
            _grid_call(L, options=dict(w["options"], gauss=gset))
        assert ei.value.code == -1


def test_tune_cache_arguments():
    """The autotuner's cache takes a path (copied), None or "" to switch it
    off, and refuses paths over 4095 bytes; its hit counter starts at zero
    in a process that never tuned."""
    import paper_2102_02738_amd as S
    from paper_2102_02738_amd._lib import SimusError
    assert S.tune_cache_hits() == 0
    S.tune_cache("/tmp/simus_tune_cache_test.txt")
    S.tune_cache("")
    S.tune_cache(None)
    with pytest.raises(SimusError, match="EINVAL"):
        S.tune_cache("a" * 4096)
