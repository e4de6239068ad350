"""simus_rf_noalloc, the entry point that allocates nothing (its workspace
is the library's static per-GPU scratch), against simus_rf through the C
ABI: two calls in a row, the second with a smaller input, each compared with
simus_rf on the same seeded inputs (relative L2 <= 1e-4, the RF bar, and bit
for bit where the default work-item partition fits the scratch).  A call
whose workspace cannot fit is refused on the host (SIMUS_ETOOBIG)."""
import ctypes as C

import numpy as np
import pytest

from tests.helpers import concat_phantoms, rel_l2, to_dev

TOL = 1e-4


def _case(S, name, scale):
    from paper_2102_02738_amd import inputs
    w = inputs.workload(name, scale=scale)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    return w, o, to_dev(x, z, R), x.size


@pytest.mark.gpu
def test_noalloc_matches_simus_rf_two_calls():
    import torch
    import paper_2102_02738_amd as S
    from paper_2102_02738_amd import _lib
    # calls in a row, each smaller than the one before: the 50,000-scatterer
    # single plane wave and 5 plane waves on 1,000 scatterers (matrix-core
    # path), whose default partitions need more than the scratch, so the
    # calls take longer work items; then 200 scatterers on 32 elements,
    # whose default partition fits (bit for bit the same as simus_rf)
    calls = [("pw128_s50k", 1.0, False), ("pw128x5_s100k", 0.01, False), ("pw32_s200", 1.0, True)]
    sizes = []
    for name, scale, bitwise in calls:
        w, o, (dx, dz, dR), n = _case(S, name, scale)
        sizes.append(n)
        T, N = w["delays"].shape
        ref = torch.empty((1, T, N, o["n_t"]), device="cuda")
        got = torch.full_like(ref, float("nan"))
        _lib.rf_into(ref, w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
        _lib.rf_noalloc_into(got, w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
        torch.cuda.synchronize()
        e = rel_l2(got.cpu().numpy(), ref.cpu().numpy())
        print(f"{name} x{scale}: {n} scatterers, noalloc vs simus_rf rel L2 {e:.3e}")
        assert torch.isfinite(got).all()
        assert e <= TOL
        if bitwise:
            assert torch.equal(got, ref)
    assert sizes[2] < sizes[1] < sizes[0]


def test_noalloc_refuses_calls_larger_than_its_scratch():
    """16 phantoms x 11 transmits x 128 elements x ~1,060 bins need about
    190 MB of spectra alone: refused with SIMUS_ETOOBIG on the host, before
    any GPU call (the device pointers are never dereferenced)."""
    from paper_2102_02738_amd import _lib, inputs
    w = inputs.workload("cvx128x11_p16", scale=0.0005)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = _lib.rf_grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = _lib.make_options(w["options"], nfft=3000, n_t=g["n_t"])
    P, M = _lib.make_probe(w["probe"]), _lib.make_medium(w["medium"])
    d = np.ascontiguousarray(w["delays"], dtype=np.float64)
    a = np.ascontiguousarray(w["apod"], dtype=np.float32)
    offs = np.ascontiguousarray(off, dtype=np.int64)
    fake = C.c_void_p(0x1000)
    lib = _lib.lib()
    rc = lib.simus_rf_noalloc(C.byref(P), C.byref(M), C.byref(o), d.shape[0],
                              d.ctypes.data_as(C.POINTER(C.c_double)),
                              a.ctypes.data_as(C.POINTER(C.c_float)), offs.size - 1,
                              offs.ctypes.data_as(C.POINTER(C.c_int64)), fake, None, fake, fake,
                              fake, None)
    assert rc == -5, lib.simus_last_error()
    assert b"scratch" in lib.simus_last_error()
