"""The seeded input generators: shapes, and the slicing of a batch into its
instances (data movement only)."""
import numpy as np

from paper_1311_0182_amd import inputs as I


def test_instances_partition_the_batch():
    cfg = I.batched(n_inst=5, side_lo=6, side_hi=10, n_ngb=32, n_steps=3)
    parts = [I.instance(cfg, k) for k in range(5)]
    for key in ("pos", "nH", "NH", "xHI", "T"):
        assert np.array_equal(np.concatenate([p[key] for p in parts]), cfg[key])
    for k, p in enumerate(parts):
        n = int(cfg["inst_off"][k + 1] - cfg["inst_off"][k])
        assert list(p["inst_off"]) == [0, n]
        assert np.array_equal(p["box"][0], cfg["box"][k])
        sel = cfg["sources"]["inst"] == k
        assert np.all(p["sources"]["inst"] == 0)
        assert np.array_equal(p["sources"]["pos"], cfg["sources"]["pos"][sel])
        assert np.array_equal(p["sources"]["rate"], cfg["sources"]["rate"][sel])
        assert p["params"] == cfg["params"]
        lo, hi = p["box"][0, :3], p["box"][0, 3:]
        assert np.all(p["pos"] >= lo) and np.all(p["pos"] <= hi)
    assert sum(len(p["sources"]["inst"]) for p in parts) == len(cfg["sources"]["inst"])


def test_verner_cross_section_and_grey_bins_against_the_paper():
    """The grey constants of the shadow set-up come from the Verner et al. (1996)
    hydrogen cross-section averaged over a 1e5 K blackbody (section 2.1).
    Pins: the cross-section at 13.6 eV is the paper's 6.3e-18 cm^2; all photons
    of 13.6-100 eV in one bin give section 4's printed 1.6e-18 cm^2 and 6.3 eV."""
    v, tol = _paper("sigma_13p6_cm2")
    assert abs(float(I.sigma_hi_verner(13.6)) / v - 1) < tol
    f1, s1, e1 = I.blackbody_grey_bins(1e5, (13.6, 100.0))
    v, tol = _paper("bb1e5_grey_sigma_cm2")
    assert abs(s1[0] / v - 1) < tol
    v, tol = _paper("bb1e5_grey_eps_ev")
    assert abs(e1[0] / v - 1) < tol
    # the three bins of the shadow set-up recombine into the single bin: the
    # photon-weighted cross-sections and the absorption-weighted energies add up
    f, sg, ep = I.BB1E5_FRAC, I.BB1E5_SIGMA, I.BB1E5_EPS_EV
    assert abs(sum(f) - 1) < 1e-12
    sbar = sum(a * b for a, b in zip(f, sg))
    assert abs(sbar / s1[0] - 1) < 1e-9
    assert abs(sum(a * b * c for a, b, c in zip(f, sg, ep)) / sbar / e1[0] - 1) < 1e-9
    # the cross-section falls steeply: the bins are ordered and separated
    assert sg[0] > 5 * sg[1] > 25 * sg[2]
    assert 0 < ep[0] < 11.0 < ep[1] < 40.8 < ep[2] < 86.4


def test_grey_bins_quadrature_against_adaptive_quadrature():
    """The Simpson quadrature of inputs.blackbody_grey_bins against scipy's
    adaptive quadrature of the same integrands (photon spectrum E^2/(e^(E/kT)-1)
    from B_nu/h nu; cross-section-weighted excess energy)."""
    from scipy.integrate import quad
    kT = 8.617333262e-5 * 1e5
    nph = lambda e: e * e / np.expm1(e / kT)
    sig = lambda e: float(I.sigma_hi_verner(e))
    edges = I.BB1E5_EDGES_EV
    tot = quad(nph, edges[0], edges[-1])[0]
    for b in range(3):
        a, c = edges[b], edges[b + 1]
        n = quad(nph, a, c)[0]
        sn = quad(lambda e: sig(e) * nph(e), a, c)[0]
        en = quad(lambda e: (e - 13.6) * sig(e) * nph(e), a, c)[0]
        assert abs(n / tot / I.BB1E5_FRAC[b] - 1) < 1e-8
        assert abs(sn / n / I.BB1E5_SIGMA[b] - 1) < 1e-8
        assert abs(en / sn / I.BB1E5_EPS_EV[b] - 1) < 1e-8


def test_shadow_layout():
    cfg = I.shadow(n_side=16, n_pp=8)
    p = cfg["params"]
    assert p["n_rc"] * p["n_freq"] == 64 and p["rr_bin"] == 3 and p["isothermal"] == 0
    nh = cfg["nH"]
    assert set(np.unique(nh)) == {2e-4, 0.04}
    assert 0 < np.sum(nh == 0.04) < nh.size // 10
    assert cfg["sources"]["kind"][0] == I.SRC_PLANE_XLO and cfg["sources"]["n_side"][0] == 8


def _paper(name):
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")
    for line in open(gold):
        f = line.split()
        if f and f[0] == name:
            return float(f[1]), float(f[2])
    raise KeyError(name)


def test_boundary_rr_intensity_appendix_b():
    from scipy.integrate import quad
    b = I.boundary_rr_intensity(1e6, 1e-3)
    # the appendix's mean free path for the section-4 flux and density
    v, tol = _paper("lambda_mfp_kpc")
    assert abs(b["mfp"] / I.KPC_CM / v - 1) < tol
    # ionization balance holds at the root taken
    x = b["x_HII"]
    assert abs(I.SIGMA_13P6 * 1e6 * (1 - x) / (b["alpha_B"] * 1e-3 * x * x) - 1) < 1e-9
    # the recombination coefficients are the Hui & Gnedin (1997) fits the
    # chemistry uses: inputs.py and the oracle code them independently
    from oracle import oracle as O
    r = O.rates(1e4)
    assert abs(b["alpha_A"] / r["alpha_A"] - 1) < 1e-12
    assert abs(b["alpha_B"] / r["alpha_B"] - 1) < 1e-12
    assert abs(b["emissivity"] / ((r["alpha_A"] - r["alpha_B"]) * 1e-6 * x * x) - 1) < 1e-12
    # the intensity is the integral over the sphere of radius lambda_mfp ...
    lam, E = b["mfp"], b["emissivity"]
    val, err = quad(lambda r: 4 * np.pi * E * np.exp(-r / lam) / (4 * np.pi * r * r) * r * r, 0.0, lam)
    assert abs(b["intensity"] / val - 1) < 1e-10
    # ... which the appendix prints as 0.63 lambda E
    v, tol = _paper("appB_intensity_factor")
    assert abs(b["intensity"] / (lam * E) / v - 1) < tol


def test_shadow_boundary_layout():
    cfg = I.shadow_boundary(n_side=8, n_pp=10, n_bd=5)
    p, L = cfg["params"], float(cfg["box"][0][3])
    assert p["n_rc"] * p["n_freq"] == 32 and p["rr_bin"] == 1 and p["n_em"] == 1
    b = cfg["boundary"]
    assert b["pos"].shape == (4 * 25, 3)
    on_face = np.isclose(b["pos"] % L, 0.0, atol=0.0) | np.isclose(b["pos"], L, rtol=0, atol=0)
    # every boundary source lies on exactly one y or z face, none on an x face
    assert np.all(on_face[:, 0] == False) and np.all(on_face[:, 1:].sum(1) == 1)
    for ax, side in I.BOUNDARY_FACES:
        sel = b["pos"][:, ax] == side * L
        assert sel.sum() == 25
        t = [k for k in range(3) if k != ax]
        for k in t:   # cell-centred 5 x 5 grid over the face
            assert np.allclose(np.unique(b["pos"][sel, k]) / L, (np.arange(5) + 0.5) / 5)
    assert np.all(b["rate"][:, [0, 1, 3]] == 0)
    assert np.isclose(b["rate"][:, 2].sum(), 4 * b["intensity"] * L * L)
    on = np.zeros(100, bool)
    on[[3, 50, 99]] = True
    s = I.boundary_sources(cfg, on)
    assert len(s["inst"]) == 4 and s["kind"][0] == I.SRC_PLANE_XLO and np.all(s["kind"][1:] == I.SRC_POINT)
    assert np.array_equal(s["pos"][1:], b["pos"][on])
    # the switch schedule follows the set-up's own front: twice the flux, twice as far
    t = 3 * cfg["params"]["dt"]
    x1 = b["pos"][I.boundary_schedule(cfg, t), 0].max()
    fast = I.shadow_boundary(n_side=8, n_pp=10, n_bd=5, flux=2e6)
    x2 = fast["boundary"]["pos"][I.boundary_schedule(fast, t), 0].max()
    assert x2 > x1 and abs(1e6 * t / 1e-3 - x1) < L / 5 and abs(2e6 * t / 1e-3 - x2) < L / 5


def test_clustered_field_recipe():
    # the lognormal recipe: g has the requested variance and a power spectrum
    # falling as k^-2.5; rho = exp(g - sigma^2/2) has mean 1 up to sampling;
    # cell counts by largest remainder give exactly N particles, each in its
    # cell, carrying that cell's density; the sources sit at the densest
    # particles with luminosities inside [1e48, 1e52]
    rng = np.random.default_rng(3)
    rho = I.lognormal_density(64, 1.5, -2.5, rng)
    g = np.log(rho) + 0.5 * 1.5 ** 2
    assert abs(g.std() - 1.5) < 1e-9
    assert abs(rho.mean() - 1.0) < 0.2
    fk = np.abs(np.fft.rfftn(g)) ** 2
    kx = np.fft.fftfreq(64)
    kz = np.fft.rfftfreq(64)
    k = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    sel1 = (k > 0.04) & (k < 0.06)
    sel2 = (k > 0.16) & (k < 0.24)
    slope = np.log(fk[sel2].mean() / fk[sel1].mean()) / np.log(k[sel2].mean() / k[sel1].mean())
    assert abs(slope + 2.5) < 0.15, slope
    cfg = I.clustered(n_side=24, n_src=32, box_mpc=1.0)
    N = 24 ** 3
    L = float(cfg["box"][0][3])
    assert cfg["pos"].shape == (N, 3)
    assert np.all((cfg["pos"] >= 0) & (cfg["pos"] < L))
    assert np.all(cfg["NH"] == cfg["NH"][0])
    assert abs(cfg["NH"][0] - 1e-3 * L ** 3 / N) <= 1e-12 * cfg["NH"][0]
    dens = np.sort(cfg["nH"])[::-1]
    src = cfg["sources"]
    assert np.all(np.sort(cfg["nH"][np.isin(np.arange(N), np.nonzero(np.isin(cfg["pos"], src["pos"]).all(1))[0])])[::-1] >= dens[31])
    tot = src["rate"][:, :4].sum(axis=1)
    assert np.all((tot >= 1e48 * (1 - 1e-12)) & (tot <= 1e52 * (1 + 1e-12)))
    assert cfg["params"]["n_rc"] * cfg["params"]["n_freq"] == 64
