"""GPU checks of the forward plan (simus_rf_plan_*): its executions and its
captured HIP graph give simus_rf's results bit for bit, on the vector path
and on the matrix-core path, with static and persistent launches, across
several graph replays separated by other eager work, and after a pointer
change that forces a new capture; and the batched uneven-phantom launch
matches the FP64 oracle."""
import numpy as np
import pytest

from tests.helpers import concat_phantoms, oracle_setup, rel_l2, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2102_02738_amd as S
    S._lib.lib()
    return S


def _prep(S, w, flags=0, with_y=False):
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, y if with_y else None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"], flags=flags)
    dx, dy, dz, dR = to_dev(x, y if with_y else None, z, R)
    return g, o, (dx, dy, dz, dR), (x, y, z, R, off)


def _convex_uneven(n_tx):
    from paper_2102_02738_amd import inputs
    probe = inputs.convex_probe(48)
    rng = np.random.default_rng(11)
    phs = [inputs.sector_phantom(rng, n, probe["radius"], 60e-3, 30.0) for n in (300, 0, 1200, 37)]
    dl = inputs.diverging_wave_delays(probe, np.linspace(-12e-3, 12e-3, n_tx), -60e-3)
    apod = np.random.default_rng(n_tx).uniform(0.3, 1.0, dl.shape).astype(np.float32)
    return dict(probe=probe, medium=dict(c=1540.0, alpha_db=0.5),
                options=dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7, nfft=0, n_t=0),
                delays=dl, apod=apod, phantoms=phs)


@pytest.mark.parametrize("case", ["valu_static", "valu_persistent", "mfma_static", "mfma_persistent"])
def test_plan_and_graph_match_rf_bitwise(S, case):
    import torch
    from paper_2102_02738_amd import inputs
    persistent = case.endswith("persistent")
    if case.startswith("valu"):
        w = inputs.workload("pw128_s50k", scale=0.1)           # 1 transmit: vector path
    else:
        w = _convex_uneven(7)                                  # 7 transmits: matrix cores
    g, o, (dx, dy, dz, dR), (x, y, z, R, off) = _prep(S, w, 0 if persistent else S.FLAG_STATIC)
    offs = off
    ref = S.rf(w["probe"], w["medium"], dict(o, flags=0), w["delays"], w["apod"], dx, None, dz, dR,
               offsets=offs)
    plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=offs)
    got = plan.rf(dx, None, dz, dR, g["n_t"])
    torch.cuda.synchronize()
    print(case, "execute", torch.equal(got, ref))
    assert torch.equal(got, ref)
    out = torch.empty_like(ref)
    for rep in range(3):
        out.zero_()
        plan.graph_launch_into(out, dx, None, dz, dR)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"graph replay {rep}"
        # unrelated eager work on the same stream between replays
        tmp = S.rf(w["probe"], w["medium"], dict(o, flags=0), w["delays"], w["apod"], dx, None, dz,
                   dR * 0.5, offsets=offs)
        torch.cuda.synchronize()
        assert torch.allclose(tmp * 2, ref, rtol=1e-5, atol=1e-6 * float(ref.abs().max()))
    plan.close()


def test_graph_recaptures_on_new_pointers(S):
    import torch
    from paper_2102_02738_amd import inputs
    w = _convex_uneven(5)
    g, o, (dx, dy, dz, dR), (x, y, z, R, off) = _prep(S, w, S.FLAG_PERSISTENT)
    plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=off)
    a = plan.rf(dx, None, dz, dR, g["n_t"], graph=True)
    R2 = torch.from_numpy(np.random.default_rng(3).standard_normal(R.size).astype(np.float32)).cuda()
    b = plan.rf(dx, None, dz, R2, g["n_t"], graph=True)
    c = plan.rf(dx, None, dz, dR, g["n_t"], graph=True)
    ref_b = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, R2, offsets=off)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    assert torch.equal(b, ref_b)
    assert not torch.equal(a, b)
    plan.close()


@pytest.mark.parametrize("n_tx", [7, 20])
def test_batched_uneven_phantoms_graph_vs_oracle(S, orc, n_tx):
    """One persistent graph launch over 4 uneven phantoms (one empty) with 7
    diverging waves (the eight-bin kernel) or 20 (the four-bin kernel over a
    group of 32 columns) on the matrix-core path, against per-phantom oracle
    runs."""
    import torch
    w = _convex_uneven(n_tx)
    g, o, (dx, dy, dz, dR), (x, y, z, R, off) = _prep(S, w, S.FLAG_PERSISTENT)
    plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=off)
    rf = plan.rf(dx, None, dz, dR, g["n_t"], graph=True).cpu().numpy()
    su = oracle_setup(orc, w)
    for p in range(len(off) - 1):
        sl = slice(off[p], off[p + 1])
        ref = orc.rf(su, g, w["delays"], w["apod"], x[sl], np.zeros(off[p + 1] - off[p]), z[sl], R[sl])
        if off[p + 1] == off[p]:
            assert np.all(rf[p] == 0)
        else:
            e = rel_l2(rf[p], ref)
            print("phantom", p, "rel L2", e)
            assert e <= TOL
    plan.close()


def test_plan_with_y_and_argument_checks(S):
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.5)
    rng = np.random.default_rng(2)
    w["phantoms"][0]["y"] = rng.uniform(-1e-3, 1e-3, w["phantoms"][0]["x"].size).astype(np.float32)
    g, o, (dx, dy, dz, dR), _ = _prep(S, w, with_y=True)
    ref = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, dy, dz, dR)
    plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], n_scat=dx.numel(), has_y=True)
    got = plan.rf(dx, dy, dz, dR, g["n_t"], graph=True)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    with pytest.raises(S.SimusError):
        plan.rf(dx, None, dz, dR, g["n_t"])
    plan.close()
    with pytest.raises(S.SimusError):
        plan.rf(dx, dy, dz, dR, g["n_t"])


@pytest.mark.parametrize("path", ["valu", "mfma"])
def test_autotune_keeps_results(S, path):
    """The autotuned plan gives simus_rf's results for the options it chose,
    bit for bit (execution and graph), and matches the default options to
    rounding order."""
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128_s50k", scale=0.1) if path == "valu" else _convex_uneven(7)
    g, o, (dx, dy, dz, dR), (_, _, _, _, off) = _prep(S, w)
    plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=off)
    first = plan.rf(dx, None, dz, dR, g["n_t"], graph=True)
    ch = plan.autotune(dx, None, dz, dR, g["n_t"])
    print(path, "chosen", ch)
    assert ch["tile_scat"] > 0
    if path == "mfma":
        assert not ch["flags"] & S.FLAG_STATIC     # the matrix-core path is always persistent
    ref = S.rf(w["probe"], w["medium"], dict(o, **ch), w["delays"], w["apod"], dx, None, dz, dR,
               offsets=off)
    got = plan.rf(dx, None, dz, dR, g["n_t"])
    gr = plan.rf(dx, None, dz, dR, g["n_t"], graph=True)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(gr, ref)
    e = rel_l2(got.cpu().numpy(), first.cpu().numpy())
    print(path, "rel L2 vs default shape", e)
    assert e <= 3e-5     # shapes with FP32 or split-bf16 matrix-core products
    plan.close()


def test_autotune_cache(S, tmp_path):
    """With a cache file, the first autotune of a problem class appends one
    line; a second plan of the class takes the stored choice without timing
    (one more cache hit, no new line) and gives simus_rf's results for it,
    bit for bit."""
    import torch
    w = _convex_uneven(7)
    g, o, (dx, dy, dz, dR), (_, _, _, _, off) = _prep(S, w)
    path = tmp_path / "tune.txt"
    S.tune_cache(str(path))
    try:
        plan = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=off)
        ch = plan.autotune(dx, None, dz, dR, g["n_t"])
        plan.close()
        lines = path.read_text().splitlines()
        print("cache:", lines)
        assert len(lines) == 1 and lines[0].startswith("simus")
        hits = S.tune_cache_hits()
        plan2 = S.rf_plan(w["probe"], w["medium"], o, w["delays"], w["apod"], offsets=off)
        ch2 = plan2.autotune(dx, None, dz, dR, g["n_t"])
        assert S.tune_cache_hits() == hits + 1
        assert ch2 == ch
        assert len(path.read_text().splitlines()) == 1
        ref = S.rf(w["probe"], w["medium"], dict(o, **ch2), w["delays"], w["apod"], dx, None, dz, dR,
                   offsets=off)
        got = plan2.rf(dx, None, dz, dR, g["n_t"])
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        plan2.close()
    finally:
        S.tune_cache(None)
