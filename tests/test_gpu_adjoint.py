"""GPU parity of the adjoint (simus_rf_backward) against the FP64 oracle's
adjoint and against finite differences of the FP64 oracle forward.

Bar: relative L2 error <= 1e-3 per gradient group (reflectivity, x, z, y).
"""
import numpy as np
import pytest

from tests.helpers import concat_phantoms, oracle_setup, rel_l2, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2102_02738_amd as S
    S._lib.lib()
    return S


def small(n_el=8, n_tx=2, n_scat=40, seed=3, with_y=False, convex=False, baffle=0):
    from paper_2102_02738_amd import inputs
    rng = np.random.default_rng(seed)
    if convex:
        probe = inputs.convex_probe(n_el)
        probe["baffle"] = baffle
        ph = inputs.sector_phantom(rng, n_scat, probe["radius"], 40e-3, 20.0, depth_min=10e-3)
        dl = inputs.diverging_wave_delays(probe, np.linspace(-5e-3, 5e-3, n_tx), -60e-3)
    else:
        probe = inputs.linear_probe(n_el)
        probe["baffle"] = baffle
        ph = inputs.rect_phantom(rng, n_scat, (-2e-3, 2e-3), (6e-3, 16e-3))
        dl = inputs.plane_wave_delays(probe, np.linspace(-6, 6, n_tx))
    if with_y:
        ph["y"] = rng.uniform(-1e-3, 1e-3, n_scat).astype(np.float32)
    apod = rng.uniform(0.5, 1.0, dl.shape).astype(np.float32)
    w = dict(probe=probe, medium=dict(c=1540.0, alpha_db=0.5),
             options=dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7, nfft=0, n_t=0),
             delays=dl, apod=apod, phantoms=[ph])
    return w


def gpu_grads(S, w, rho, with_y=False, flags=0):
    import torch
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, y if with_y else None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"], flags=flags)
    dx, dy, dz, dR = to_dev(x, y if with_y else None, z, R)
    (drho,) = to_dev(rho)
    gr = S.rf_backward(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, dy, dz, dR, drho)
    torch.cuda.synchronize()
    return g, {k: v.cpu().numpy().astype(np.float64) for k, v in gr.items()}


def oracle_grads(orc, w, g, rho, with_y=False, sel=None):
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    yy = y if with_y else np.zeros_like(x)
    r = orc.adjoint(oracle_setup(orc, w), g, w["delays"], w["apod"], x, yy, z, R,
                    rho.astype(np.float64), sel=sel)
    r["refl"] = r.pop("R")
    return r


def _check(got, ref, keys):
    for k in keys:
        e = rel_l2(got[k], ref[k])
        print(f"  d{k}: rel L2 {e:.2e}")
        assert e <= TOL, (k, e)


# "alt" runs the other adjoint kernel (SIMUS_FLAG_ALT_SHAPE): these small
# probes take the vector kernel by default, the matrix-core one with it (up
# to 8 transmits with split-bf16 products; "alt_fp32" with FP32 products)
PATHS = ["default", "alt", "alt_fp32"]


def _path_flags(S, path):
    return {"default": 0, "alt": S.FLAG_ALT_SHAPE, "alt_fp32": S.FLAG_ALT_SHAPE | S.FLAG_FP32_PRODUCTS}[path]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("with_y,convex,baffle,flags", [
    (False, False, 0, 0), (False, False, 0, 4), (True, False, 0, 0), (False, True, 2, 0),
    (False, False, 1, 0)])
def test_adjoint_matches_oracle_adjoint(S, orc, with_y, convex, baffle, flags, path):
    w = small(with_y=with_y, convex=convex, baffle=baffle)
    flags |= _path_flags(S, path)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, y if with_y else None, z)
    rho = np.random.default_rng(7).standard_normal((1, len(w["delays"]), w["probe"]["n_elements"],
                                                    g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho, with_y, flags)
    ref = oracle_grads(orc, w, g, rho[0], with_y)
    _check(got, ref, ["refl", "x", "z"] + (["y"] if with_y else []))


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_scat", [7, 61, 137])
def test_adjoint_ragged_chunks(S, orc, n_scat, path):
    """Scatterer counts that leave a partial chunk (8 or, for nu = 2 and
    y = 0 on the matrix cores, 10 scatterers) and span one to three items
    of 60-64 scatterers."""
    w = small(n_tx=3, n_scat=n_scat, seed=n_scat)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    rho = np.random.default_rng(n_scat).standard_normal((1, 3, 8, g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho, flags=_path_flags(S, path))
    ref = oracle_grads(orc, w, g, rho[0])
    _check(got, ref, ["refl", "x", "z"])


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_tx", [1, 3, 5, 9])
def test_adjoint_transmit_groups(S, orc, n_tx, path):
    w = small(n_tx=n_tx, n_scat=30)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    rho = np.random.default_rng(n_tx).standard_normal((1, n_tx, 8, g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho, flags=_path_flags(S, path))
    ref = oracle_grads(orc, w, g, rho[0])
    _check(got, ref, ["refl", "x", "z"])


def test_gradient_matches_oracle_finite_differences(S, orc):
    """L = 1/2 ||rf - obs||^2 with obs the RF of a perturbed phantom (all
    FP64 oracle); GPU gradient at the base phantom vs central differences of
    the oracle's L."""
    from paper_2102_02738_amd import inputs
    w = small(n_el=6, n_tx=2, n_scat=12)
    ph = w["phantoms"][0]
    obs_ph = inputs.perturbed(ph, seed=1, sigma_pos=50e-6, sigma_R=0.1)
    su = oracle_setup(orc, w)
    x, y, z, R = (ph[k].astype(np.float64) for k in ("x", "y", "z", "R"))
    g = orc.grid(su, w["delays"], x, y, z)
    obs = orc.rf(su, g, w["delays"], w["apod"], obs_ph["x"], obs_ph["y"], obs_ph["z"], obs_ph["R"])
    L = lambda x_, z_, R_: 0.5 * np.sum((orc.rf(su, g, w["delays"], w["apod"], x_, y, z_, R_) - obs) ** 2)
    rho = orc.rf(su, g, w["delays"], w["apod"], x, y, z, R) - obs
    _, got = gpu_grads(S, w, rho[None].astype(np.float32))
    fd = {"refl": [], "x": [], "z": []}
    h = 1e-8
    for s in range(x.size):
        e = np.zeros_like(x)
        e[s] = h
        fd["x"].append((L(x + e, z, R) - L(x - e, z, R)) / (2 * h))
        fd["z"].append((L(x, z + e, R) - L(x, z - e, R)) / (2 * h))
        e[s] = 1e-3
        fd["refl"].append((L(x, z, R + e) - L(x, z, R - e)) / 2e-3)
    _check(got, {k: np.array(v) for k, v in fd.items()}, ["refl", "x", "z"])


def test_adjoint_full_size_sampled_scatterers(S, orc):
    """128 elements, 5 plane waves, 100,000 scatterers (the differentiable-RF
    workload) with a seeded random residual: gradients of 20 random
    scatterers per group against the oracle's adjoint."""
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128x5_s100k")
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    rho = np.random.default_rng(11).standard_normal((1, 5, 128, g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho)
    sel = np.random.default_rng(12).choice(x.size, 20, replace=False)
    ref = oracle_grads(orc, w, g, rho[0], sel=sel)
    _check({k: v[sel] for k, v in got.items()}, ref, ["refl", "x", "z"])


def test_adjoint_identities_full_size(S):
    """At the 100,000-scatterer size: the reflectivity gradient is the exact
    transpose of the forward map (<J v, rho> = <v, J^T rho>), and since RF is
    linear in R, sum_s R_s dL/dR_s = <rho, rf(R)>."""
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128x5_s100k")
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    dx, dz, dR = to_dev(x, z, R)
    v = torch.from_numpy(np.random.default_rng(3).standard_normal(x.size).astype(np.float32)).cuda()
    rho = torch.from_numpy(np.random.default_rng(4).standard_normal((1, 5, 128, g["n_t"])).astype(np.float32)).cuda()
    Jv = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, v)
    JT = S.rf_backward(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR, rho,
                       need=("refl",))["refl"]
    rfR = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
    torch.cuda.synchronize()
    lhs = float(torch.sum(Jv.double() * rho.double()))
    rhs = float(torch.sum(v.double() * JT.double()))
    print("dot test", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    e1 = float(torch.sum(dR.double() * JT.double()))
    e2 = float(torch.sum(rho.double() * rfR.double()))
    assert abs(e1 - e2) <= 1e-4 * abs(e2)


def test_autograd_function(S, orc):
    """torch.autograd through SimusRF gives the adjoint's gradients."""
    import torch
    from paper_2102_02738_amd.autograd import simus_rf_autograd
    w = small(n_scat=20)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    dx, dz, dR = (t.requires_grad_(True) for t in to_dev(x, z, R))
    obs = torch.zeros((1, 2, 8, g["n_t"]), device="cuda")
    rf = simus_rf_autograd(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
    loss = 0.5 * torch.sum((rf - obs) ** 2)
    loss.backward()
    rho = rf.detach().cpu().numpy()[0].astype(np.float64)
    ref = orc.adjoint(oracle_setup(orc, w), g, w["delays"], w["apod"], x, np.zeros_like(x), z, R, rho)
    ref["refl"] = ref.pop("R")
    _check({"refl": dR.grad.cpu().numpy(), "x": dx.grad.cpu().numpy(), "z": dz.grad.cpu().numpy()},
           ref, ["refl", "x", "z"])


def test_adjoint_empty_phantom(S):
    """No scatterers: the call succeeds and the gradients are empty."""
    import torch
    w = small()
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    e = torch.empty(0, device="cuda")
    rho = torch.ones((1, 2, 8, g["n_t"]), device="cuda")
    gr = S.rf_backward(w["probe"], w["medium"], o, w["delays"], w["apod"], e, None, e, e, rho)
    torch.cuda.synchronize()
    assert set(gr) >= {"refl", "x", "z"} and all(v.numel() == 0 for v in gr.values())


@pytest.mark.parametrize("path", PATHS)
def test_adjoint_single_scatterer(S, orc, path):
    """One scatterer: a single partial chunk on either kernel."""
    w = small(n_tx=3, n_scat=1, seed=5)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    rho = np.random.default_rng(5).standard_normal((1, 3, 8, g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho, flags=_path_flags(S, path))
    ref = oracle_grads(orc, w, g, rho[0])
    _check(got, ref, ["refl", "x", "z"])


def test_adjoint_600_sub_elements(S, orc):
    """300 elements with nu = 2: the vector adjoint over 600 sub-elements
    (the matrix-core adjoint serves up to 128 elements) against the
    oracle's adjoint."""
    w = small(n_el=300, n_tx=2, n_scat=50, seed=8)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g0 = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    assert g0["nu"] == 2
    rho = np.random.default_rng(8).standard_normal((1, 2, 300, g0["n_t"])).astype(np.float32)
    g, got = gpu_grads(S, w, rho)
    ref = oracle_grads(orc, w, g, rho[0])
    _check(got, ref, ["refl", "x", "z"])


@pytest.mark.parametrize("path", PATHS)
def test_adjoint_out_of_domain_scatterers(S, path):
    """Scatterers at z <= 0 before a linear array (G = 0 and dG = 0 on the
    device): appended to a phantom they get exactly zero gradients, and the
    other scatterers' gradients are bit for bit those without them."""
    import torch
    w = small(n_tx=3, n_scat=40, seed=13)
    ph = w["phantoms"][0]
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], ph["x"], None, ph["z"])
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"], flags=_path_flags(S, path))
    rng = np.random.default_rng(14)
    xo = np.concatenate([ph["x"], rng.uniform(-3e-3, 3e-3, 10)]).astype(np.float32)
    zo = np.concatenate([ph["z"], -rng.uniform(0, 2e-3, 10)]).astype(np.float32)
    Ro = np.concatenate([ph["R"], rng.standard_normal(10)]).astype(np.float32)
    (rho,) = to_dev(rng.standard_normal((1, 3, 8, g["n_t"])))
    a = S.rf_backward(w["probe"], w["medium"], o, w["delays"], w["apod"], *to_dev(ph["x"], None, ph["z"], ph["R"]), rho)
    b = S.rf_backward(w["probe"], w["medium"], o, w["delays"], w["apod"], *to_dev(xo, None, zo, Ro), rho)
    torch.cuda.synchronize()
    for k in ("refl", "x", "z"):
        assert torch.equal(a[k], b[k][:40]), k
        assert torch.all(b[k][40:] == 0), k
