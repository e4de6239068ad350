"""GPU parity of the forward path (spectra and RF) against the FP64 oracle.

Bar: relative L2 error <= 1e-4 (FP32 path vs FP64 oracle) on RF and on
spectra; bit-exact integers for the grid; bitwise-identical results for
repeated calls and for the persistent launch.
"""
import numpy as np
import pytest

from tests.helpers import (assert_grid_matches, band_peak_bin, concat_phantoms, oracle_setup,
                           oracle_spectrum_split, rel_l2, sample_bins, to_dev)

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2102_02738_amd as S
    S._lib.lib()
    return S


def _run(S, w, flags=0, with_y=False, spectrum=False, bins=None):
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, y if with_y else None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"], flags=flags)
    dx, dy, dz, dR = to_dev(x, y if with_y else None, z, R)
    offs = off if len(w["phantoms"]) > 1 else None
    if spectrum:
        out = S.rf_spectrum(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, dy, dz, dR,
                            offsets=offs, n_bins=g["n_bins"])
    else:
        out = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, dy, dz, dR, offsets=offs)
    import torch
    torch.cuda.synchronize()
    return g, out.cpu().numpy(), (x, y, z, R, off)


def _oracle_rf(orc, w, g, data, with_y=False):
    x, y, z, R, off = data
    su = oracle_setup(orc, w)
    out = []
    for p in range(len(off) - 1):
        sl = slice(off[p], off[p + 1])
        yy = y[sl] if with_y else np.zeros(off[p + 1] - off[p])
        out.append(orc.rf(su, g, w["delays"], w["apod"], x[sl], yy, z[sl], R[sl]))
    return np.stack(out)


def test_rf_pw32_s200_full(S, orc):
    """32 elements, 1 plane wave, 200 scatterers: full RF parity."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200")
    g, rf, data = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    print("pw32_s200 rel L2", rel_l2(rf, ref))
    assert rf.shape == ref.shape
    assert rel_l2(rf, ref) <= TOL


@pytest.mark.parametrize("direct", [False, True])
def test_rf_pw128_small_full(S, orc, direct):
    """128 elements, anechoic disks, attenuation, 50 mm depth, 1000 scatterers:
    full RF parity (several scatter tiles, ragged tail, n_t < nfft), with the
    tabulated and with the directly evaluated elevation term."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128_s50k", scale=0.02)
    g, rf, data = _run(S, w, flags=S.FLAG_NO_DELTA_TABLE if direct else 0)
    assert g["n_t"] == 1975
    ref = _oracle_rf(orc, w, g, data)
    print("pw128 1000 rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


def test_spectrum_pw128_s50k_full_size_sampled_bins(S, orc):
    """Full 50,000-scatterer workload in the benchmark's launch
    configuration; the oracle evaluates a spread of bins (band edges
    included) and the GPU spectra must match them."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128_s50k")
    g, spec, data = _run(S, w, spectrum=True)
    bins = sample_bins(g, 6)
    x, y, z, R, off = data
    assert_grid_matches(orc, w, g, x, None, z)
    ref = orc.spectrum(oracle_setup(orc, w), g["nfft"], w["delays"], w["apod"], x, y, z, R, bins)
    got = spec[0][:, :, bins - g["j_lo"]]
    print("pw128_s50k sampled bins rel L2", rel_l2(got, ref))
    assert rel_l2(got, ref) <= TOL
    # per-bin bound too (the band edges carry little energy)
    for k in range(bins.size):
        assert rel_l2(got[..., k], ref[..., k]) <= 3 * TOL


def test_general_y_path(S, orc):
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.5)
    rng = np.random.default_rng(4)
    w["phantoms"][0]["y"] = rng.uniform(-1.5e-3, 1.5e-3, w["phantoms"][0]["x"].size).astype(np.float32)
    g, rf, data = _run(S, w, with_y=True)
    ref = _oracle_rf(orc, w, g, data, with_y=True)
    print("y path rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


@pytest.mark.parametrize("baffle", [1, 2])
def test_rigid_and_impedance_baffles(S, orc, baffle):
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.5)
    w["probe"]["baffle"] = baffle
    g, rf, data = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    assert rel_l2(rf, ref) <= TOL


@pytest.mark.parametrize("n_tx", [2, 3, 5, 9])
def test_multi_transmit(S, orc, n_tx):
    """Steered plane waves with uneven apodisation; covers transmit groups
    and a ragged last group."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.5)
    ang = np.linspace(-12, 12, n_tx)
    w["delays"] = inputs.plane_wave_delays(w["probe"], ang)
    w["apod"] = np.random.default_rng(n_tx).uniform(0.2, 1.0, w["delays"].shape).astype(np.float32)
    g, rf, data = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    print(n_tx, "tx rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


def test_convex_diverging_waves_uneven_phantoms(S, orc):
    """Convex probe, 3 diverging waves, 4 phantoms of uneven size (one
    empty): the batched launch matches per-phantom oracle runs."""
    from paper_2102_02738_amd import inputs
    probe = inputs.convex_probe(48)
    rng = np.random.default_rng(9)
    phs = [inputs.sector_phantom(rng, n, probe["radius"], 60e-3, 30.0) for n in (37, 0, 120, 5)]
    dl = inputs.diverging_wave_delays(probe, [-10e-3, 0.0, 12e-3], -60e-3)
    w = dict(probe=probe, medium=dict(c=1540.0, alpha_db=0.5),
             options=dict(fs=4 * probe["fc"], n_cycles=1.0, nu=0, spectral_eps=1e-7, nfft=0, n_t=0),
             delays=dl, apod=np.ones(dl.shape, np.float32), phantoms=phs)
    g, rf, data = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    assert np.all(rf[1] == 0)
    print("convex rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL
    g2, rf2, _ = _run(S, w, flags=S.FLAG_STATIC)
    assert np.array_equal(rf, rf2)


def test_repeatable_and_persistent_bitwise(S):
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128_s50k", scale=0.1)
    _, a, _ = _run(S, w)
    _, b, _ = _run(S, w)
    _, c, _ = _run(S, w, flags=S.FLAG_STATIC)
    _, d, _ = _run(S, w, flags=S.FLAG_PERSISTENT)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    assert np.array_equal(a, d)


def test_inverse_transform_full_size(S, orc):
    """The inverse transform alone at the 128-element, 2400-point size, on a
    seeded random spectrum, against the oracle's explicit sum."""
    import torch
    rng = np.random.default_rng(0)
    nfft, n_t, j_lo, nb, nch = 2400, 1975, 120, 849, 128
    X = (rng.standard_normal((nch, nb)) + 1j * rng.standard_normal((nch, nb))).astype(np.complex64)
    bins = np.arange(j_lo, j_lo + nb)
    ref = orc.rf_from_spectrum(X.astype(np.complex128), bins, nfft, n_t)
    got = S.spectrum_to_rf(torch.from_numpy(X).cuda(), nfft, n_t, j_lo).cpu().numpy()
    print("idft rel L2", rel_l2(got, ref))
    assert rel_l2(got, ref) <= 1e-5


def test_empty_and_degenerate(S):
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.05)
    x, y, z, R, off = concat_phantoms(w["phantoms"])
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], x, None, z)
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"])
    e = torch.empty(0, device="cuda")
    rf = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], e, None, e, e, offsets=[0, 0])
    torch.cuda.synchronize()
    assert rf.shape == (1, 1, 32, g["n_t"]) and torch.all(rf == 0)
    # all-zero reflectivity gives exactly zero RF
    dx, dz, dR = to_dev(x, z, np.zeros_like(R))
    rf = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
    torch.cuda.synchronize()
    assert torch.all(rf == 0)


@pytest.mark.parametrize("n_tx,n_el,nu,with_y,no_mfma", [
    (21, 32, 0, False, False), (33, 32, 0, False, False), (6, 32, 0, True, False),
    (12, 64, 1, False, False), (5, 200, 1, False, False), (21, 32, 0, False, True),
    (11, 100, 0, False, False), (40, 128, 0, False, False), (70, 48, 1, False, False),
    (24, 100, 0, True, False), (20, 40, 1, True, False), (36, 40, 1, True, False),
    (45, 20, 2, False, False)])
def test_many_transmits(S, orc, n_tx, n_el, nu, with_y, no_mfma):
    """Many steered plane waves: the transmit contraction on the matrix cores
    (or, with the flag, on the VALU path) matches the oracle; covers the
    default kernels with 64 and 128 element slots: eight bins over groups of
    16 transmit columns up to 16 transmits, four bins over one to three
    groups of 32 above (of 64, two column tiles per wave, above 32 transmits
    on 64 slots: nu = 1 and 2, y != 0),
    several transmit groups with a ragged last one, y != 0, nu = 1 and 200
    elements (vector path)."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.3)
    w["probe"] = inputs.linear_probe(n_el)
    w["options"]["nu"] = nu
    w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-15, 15, n_tx))
    w["apod"] = np.random.default_rng(n_tx).uniform(0.2, 1.0, w["delays"].shape).astype(np.float32)
    if with_y:
        w["phantoms"][0]["y"] = np.random.default_rng(1).uniform(
            -1e-3, 1e-3, w["phantoms"][0]["x"].size).astype(np.float32)
    g, rf, data = _run(S, w, flags=S.FLAG_NO_MFMA if no_mfma else 0, with_y=with_y)
    ref = _oracle_rf(orc, w, g, data, with_y=with_y)
    print(n_tx, "tx", n_el, "el rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


@pytest.mark.parametrize("n_tx,n_el,nu,with_y,no_table", [
    (4, 128, 2, False, False), (16, 128, 1, False, False), (13, 96, 2, True, False),
    (7, 128, 1, True, False), (9, 72, 2, False, True), (15, 128, 1, False, True)])
def test_eight_bin_matrix_core_kernel(S, orc, n_tx, n_el, nu, with_y, no_table):
    """The default matrix-core kernel for more than 64 elements and at most 16
    transmits (eight bins per item, weights from the padded table): every
    compiled form (nu = 1 and 2; y != 0; the elevation term from the table or
    evaluated directly), from 4 to 16 transmits, element slots left empty
    (72, 96), ragged last bin tile and scatterer chunk; full RF against the
    oracle."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.43)
    w["probe"] = inputs.linear_probe(n_el)
    w["options"]["nu"] = nu
    w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-14, 14, n_tx))
    w["apod"] = np.random.default_rng(n_tx + n_el).uniform(0.2, 1.0, w["delays"].shape).astype(np.float32)
    if with_y:
        w["phantoms"][0]["y"] = np.random.default_rng(2).uniform(
            -1e-3, 1e-3, w["phantoms"][0]["x"].size).astype(np.float32)
    g, rf, data = _run(S, w, flags=S.FLAG_NO_DELTA_TABLE if no_table else 0, with_y=with_y)
    assert g["n_bins"] % 8 != 0 and data[0].size % 16 != 0, "ragged last bin tile and chunk"
    ref = _oracle_rf(orc, w, g, data, with_y=with_y)
    print(n_tx, "tx", n_el, "el nu", nu, "y" if with_y else "", "direct" if no_table else "",
          "bins", g["n_bins"], "rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


def test_many_transmits_full_size_sampled_bins(S, orc):
    """21 plane waves, 200,000 scatterers (the compounding workload) in the
    benchmark's launch configuration: sampled bins against the oracle."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw128x21_s200k")
    g, spec, data = _run(S, w, spectrum=True)
    bins = sample_bins(g, 3)
    x, y, z, R, off = data
    assert_grid_matches(orc, w, g, x, None, z)
    ref = orc.spectrum(oracle_setup(orc, w), g["nfft"], w["delays"], w["apod"], x, y, z, R, bins)
    got = spec[0][:, :, bins - g["j_lo"]]
    print("pw128x21_s200k sampled bins rel L2", rel_l2(got, ref))
    assert rel_l2(got, ref) <= TOL


def test_uneven_phantoms_full_size_sampled_bins(S, orc):
    """16 convex-probe phantoms of 10k-390k scatterers x 11 diverging waves
    (2.27 M scatterers, the uneven-batch workload) in one persistent launch
    on the matrix cores: the band's first and last bins, the bin of peak
    |S_P S_T| and the middle bin, for the smallest, a middle and the largest
    phantom, against the oracle.  The grid is the oracle's."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("cvx128x11_p16")
    g, spec, data = _run(S, w, flags=S.FLAG_PERSISTENT, spectrum=True)
    x, y, z, R, off = data
    assert_grid_matches(orc, w, g, x, None, z)
    sizes = np.diff(off)
    order = np.argsort(sizes)
    su = oracle_setup(orc, w)
    peak = band_peak_bin(orc, su, g)
    bins = np.unique(np.concatenate([sample_bins(g, 2), [peak, g["j_lo"] + g["n_bins"] // 2]]))
    assert bins.size == 4
    for p in (order[0], order[len(order) // 2], order[-1]):
        sl = slice(off[p], off[p + 1])
        ref = oracle_spectrum_split(orc, su, g["nfft"], w["delays"], w["apod"], x[sl], None, z[sl],
                                    R[sl], bins, parts=4)
        got = spec[p][:, :, bins - g["j_lo"]]
        e = rel_l2(got, ref)
        print("phantom", p, "scatterers", sizes[p], "bins", bins, "rel L2", e)
        assert e <= TOL
        for k in range(bins.size):
            assert rel_l2(got[..., k], ref[..., k]) <= 3 * TOL, (bins[k], rel_l2(got[..., k], ref[..., k]))


def test_large_t_focused_small_full_rf(S, orc):
    """Phased array, 128 focused transmits (two groups of 64 transmit
    columns on the matrix cores), 20 scatterers: full RF against the oracle."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("ph64x128_s40k", scale=0.0005)
    g, rf, data = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    print("128 tx, 20 scatterers rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


def test_large_t_focused_full_size_sampled_bins(S, orc):
    """The 128-transmit, 40,000-scatterer sequence in the benchmark's launch
    configuration: sampled bins against the oracle."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("ph64x128_s40k")
    g, spec, data = _run(S, w, spectrum=True)
    bins = sample_bins(g, 3)
    x, y, z, R, off = data
    assert_grid_matches(orc, w, g, x, None, z)
    ref = orc.spectrum(oracle_setup(orc, w), g["nfft"], w["delays"], w["apod"], x, y, z, R, bins)
    got = spec[0][:, :, bins - g["j_lo"]]
    print("ph64x128_s40k sampled bins rel L2", rel_l2(got, ref))
    assert rel_l2(got, ref) <= TOL


def test_coarse_grid_general_half_sinc(S, orc):
    """A grid so coarse that the half-angle sinc of the pair set-up reaches
    arguments above 1 (nu = 1, 0.9 mm elements, nfft = 10, so df b / c =
    0.35): the set-up's general sinc branch runs, and the matrix-core path
    declines the 5 transmits (the result equals the vector path's bit for
    bit).  RF against the oracle."""
    import torch
    from paper_2102_02738_amd import inputs
    probe = dict(inputs.linear_probe(8), pitch=1e-3, width=0.9e-3, fc=3e6)
    rng = np.random.default_rng(21)
    n = 40
    x = rng.uniform(-8e-3, 8e-3, n).astype(np.float32)
    z = rng.uniform(2e-3, 6e-3, n).astype(np.float32)
    R = rng.standard_normal(n).astype(np.float32)
    dl = inputs.plane_wave_delays(probe, [-10, -5, 0, 5, 10])
    ap = np.ones(dl.shape, np.float32)
    w = dict(probe=probe, medium=dict(c=1540.0, alpha_db=0.5),
             options=dict(fs=12e6, n_cycles=1.0, nu=1, spectral_eps=1e-7, nfft=10, n_t=10),
             delays=dl, apod=ap)
    g = S.grid(probe, w["medium"], w["options"], dl, x, None, z)
    assert g["nfft"] == 10 and g["n_t"] == 10
    assert g["df"] * 0.45e-3 / 1540.0 > 0.3
    dx, dz, dR = to_dev(x, z, R)
    got = S.rf(probe, w["medium"], w["options"], dl, ap, dx, None, dz, dR)
    vec = S.rf(probe, w["medium"], dict(w["options"], flags=S.FLAG_NO_MFMA), dl, ap, dx, None, dz, dR)
    torch.cuda.synchronize()
    assert torch.equal(got, vec)
    ref = orc.rf(oracle_setup(orc, w), g, dl, ap, x, np.zeros(n), z, R)
    e = rel_l2(got.cpu().numpy()[0], ref)
    print("coarse grid rel L2", e)
    assert e <= TOL


@pytest.mark.parametrize("n_tx,n_el,nu", [(21, 100, 0), (11, 128, 0), (11, 48, 0), (40, 48, 0), (5, 200, 0),
                                         (6, 64, 3)])
def test_alt_tile_shape(S, orc, n_tx, n_el, nu):
    """The alternative tile shape (SIMUS_FLAG_ALT_SHAPE: on the matrix cores
    the four-bin kernel with 32 transmit columns for 100 elements and 21
    transmits, with 16 for 128 elements and 11, the six-bin one with 32
    columns for 48 elements and 11 transmits, with 64 for 48 and 40, instead
    of the default split-bf16 kernels; on the vector path pairs instead of single
    transmits for 5, single instead of pairs for 6) matches the oracle and
    the default shape to rounding order."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.3)
    w["probe"] = inputs.linear_probe(n_el)
    w["options"]["nu"] = nu
    w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-12, 12, n_tx))
    w["apod"] = np.random.default_rng(n_tx).uniform(0.2, 1.0, w["delays"].shape).astype(np.float32)
    g, rf, data = _run(S, w, flags=S.FLAG_ALT_SHAPE)
    _, rf0, _ = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    print(n_tx, "tx", n_el, "el alternative shape rel L2", rel_l2(rf, ref), "vs default", rel_l2(rf, rf0))
    assert rel_l2(rf, ref) <= TOL
    assert rel_l2(rf, rf0) <= 3e-5


@pytest.mark.parametrize("n_tx,n_el,nu", [(21, 128, 0), (24, 48, 0), (40, 100, 1), (11, 128, 0), (7, 64, 2)])
def test_fp32_products_flag(S, orc, n_tx, n_el, nu):
    """SIMUS_FLAG_FP32_PRODUCTS: the eight-bin kernel with FP32 matrix-core
    products (k_synth_mq) instead of split-bf16 ones, over one to three
    groups of 16 columns (the last one ragged), 128 and 64 element slots,
    matches the oracle and the default (split-bf16) products to their
    rounding (about 2^-16 of each product)."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=0.3)
    w["probe"] = inputs.linear_probe(n_el)
    w["options"]["nu"] = nu
    w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-12, 12, n_tx))
    w["apod"] = np.random.default_rng(n_tx + 1).uniform(0.2, 1.0, w["delays"].shape).astype(np.float32)
    g, rf, data = _run(S, w, flags=S.FLAG_FP32_PRODUCTS)
    _, rf0, _ = _run(S, w)
    ref = _oracle_rf(orc, w, g, data)
    e_fp32, e_bf = rel_l2(rf, ref), rel_l2(rf0, ref)
    print(n_tx, "tx", n_el, "el FP32 products rel L2", e_fp32, "split bf16", e_bf, "between", rel_l2(rf, rf0))
    assert e_fp32 <= TOL and e_bf <= TOL
    assert rel_l2(rf, rf0) <= 3e-5


@pytest.mark.parametrize("kind,n", [("linear32", 613), ("linear64", 401), ("phased64_nu1", 577)])
def test_grouped_small_probes(S, orc, kind, n):
    """Probes of fewer than 256 sub-elements run several sub-element groups
    per 256-thread block (4 groups for 64 slots, 2 for 128), each on its own
    chunk of scatterers: full RF against the oracle, ragged super-chunks."""
    from paper_2102_02738_amd import inputs
    rng = np.random.default_rng(n)
    if kind == "phased64_nu1":
        w = inputs.workload("ph64x128_s40k", scale=n / 40000)
        w["delays"] = w["delays"][40:41]
        w["apod"] = w["apod"][40:41]
    else:
        w = inputs.workload("pw32_s200", scale=n / 200)
        w["probe"] = inputs.linear_probe(32 if kind == "linear32" else 64)
        w["delays"] = inputs.plane_wave_delays(w["probe"], [4.0])
        w["apod"] = rng.uniform(0.3, 1.0, w["delays"].shape).astype(np.float32)
    g, rf, data = _run(S, w)
    assert g["nu"] == (1 if kind == "phased64_nu1" else 2)
    ref = _oracle_rf(orc, w, g, data)
    print(kind, n, "scatterers rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL
    _, rf_static, _ = _run(S, w, flags=S.FLAG_STATIC)
    assert np.array_equal(rf, rf_static)


@pytest.mark.parametrize("n_tx", [1, 2])
def test_1024_thread_vector_kernel(S, orc, n_tx):
    """300 elements with nu = 2 (600 sub-elements) run the vector synthesis
    in 1024-thread blocks (6-bin tiles): full RF against the oracle, one
    transmit (8-scatterer chunks) and a pair of transmits (4-scatterer
    chunks), 300 scatterers (ragged last chunk)."""
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=1.5)
    w["probe"] = inputs.linear_probe(300)
    w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-6, 6, n_tx))
    w["apod"] = np.random.default_rng(n_tx).uniform(0.4, 1.0, w["delays"].shape).astype(np.float32)
    w["phantoms"][0]["x"] = (w["phantoms"][0]["x"] * 4).astype(np.float32)
    g, rf, data = _run(S, w)
    assert g["nu"] == 2
    ref = _oracle_rf(orc, w, g, data)
    print("300 elements,", n_tx, "tx rel L2", rel_l2(rf, ref))
    assert rel_l2(rf, ref) <= TOL


@pytest.mark.parametrize("kind", ["vector", "mfma"])
def test_out_of_domain_scatterers_add_nothing(S, orc, kind):
    """Scatterers at z <= 0 before a linear array lie behind every
    sub-element (G = 0 on the device, no EDOMAIN there): appended to a
    phantom, with the partition into work items fixed, they leave its RF
    bit for bit unchanged (on the vector path and on the matrix cores)."""
    import torch
    from paper_2102_02738_amd import inputs
    w = inputs.workload("pw32_s200", scale=1.28)            # 256 scatterers
    if kind == "mfma":
        w["delays"] = inputs.plane_wave_delays(w["probe"], np.linspace(-8, 8, 5))
        w["apod"] = np.ones(w["delays"].shape, np.float32)
    ph = w["phantoms"][0]
    n = ph["x"].size
    assert n == 256
    g = S.grid(w["probe"], w["medium"], w["options"], w["delays"], ph["x"], None, ph["z"])
    o = dict(w["options"], nfft=g["nfft"], n_t=g["n_t"], tile_scat=128)
    rng = np.random.default_rng(17)
    k = 128
    xo = np.concatenate([ph["x"], rng.uniform(-6e-3, 6e-3, k)]).astype(np.float32)
    zo = np.concatenate([ph["z"], -rng.uniform(0, 5e-3, k)]).astype(np.float32)
    zo[n] = 0.0
    Ro = np.concatenate([ph["R"], rng.standard_normal(k)]).astype(np.float32)
    dx, dz, dR = to_dev(ph["x"], ph["z"], ph["R"])
    ex, ez, eR = to_dev(xo, zo, Ro)
    a = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], dx, None, dz, dR)
    b = S.rf(w["probe"], w["medium"], o, w["delays"], w["apod"], ex, None, ez, eR)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = _oracle_rf(orc, w, g, (ph["x"], ph["y"], ph["z"], ph["R"], np.array([0, n])))
    assert rel_l2(b.cpu().numpy(), ref) <= TOL
