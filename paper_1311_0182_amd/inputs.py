"""Seeded synthetic workloads for the TRAPHIC radiative-transfer step.

This module only builds input arrays and numerical parameters: particle
positions, densities, atom counts, initial ionization state and temperature,
sources and the per-bin grey constants.  It holds none of the transport,
chemistry or recombination arithmetic of the method, and it is the only code
shared by the CPU oracle and the HIP path (both take these arrays as inputs).
Three formulas size inputs only: the grey cross-sections and excess energies of
blackbody bins (a quadrature of the Verner et al. 1996 cross-section), the
recombination coefficients at 1e4 K that size the boundary sources of the
shadow test, and the appendix-B intensity those sources carry.

The shapes follow the paper's test set-ups:
  * Stromgren HII region (section 3): uniform hydrogen, n_H = 1e-3 cm^-3,
    T = 1e4 K, one source of 5e48 photons/s at the box centre, monochromatic
    13.6 eV photons with sigma = 6.3e-18 cm^2, N_EC = N_TC = N_RC = 8,
    dt = 0.1 Myr, emission sub-step dt_em = 0.01 Myr.
  * Recombination radiation in its own frequency bin with the 13.6 eV
    cross-section (section 2.2).
  * Plane-parallel front from one box face (section 4 and its footnote on the
    boundary emitters).
Particle sets are jittered lattices: x = (i + 1/2 + U(-0.3, 0.3)) dx per axis.
Every generator is seeded (numpy PCG64) so both sides see identical inputs.
"""
from __future__ import annotations

import math

import numpy as np

# Physical constants used only to express the recipes in cgs units.
KPC_CM = 3.0857e21
MYR_S = 3.1536e13
EV_ERG = 1.602176634e-12
K_BOLTZ = 1.380649e-16
SIGMA_13P6 = 6.3e-18          # cm^2, hydrogen cross-section at 13.6 eV (section 2.2)
ALPHA_B_1E4 = 2.59e-13        # cm^3/s, only to size batched boxes (R_S/L recipe)

# Enumerations mirrored from include/traphic_rt.h
CASE_B_OTS, CASE_A_NO_RR, RR_TRANSPORT, RR_ORIGINAL = 0, 1, 2, 3
FP64, FP32 = 0, 1
SRC_POINT, SRC_PLANE_XLO = 0, 1

BASE_SEED = 1311018200


def default_params(**kw):
    """Numerical parameters of one RT step (names follow the paper's notation)."""
    p = dict(
        n_ngb=32,          # SPH neighbours per particle
        n_tc=8,            # transmission cones: solid angle 4 pi / N_TC
        n_rc=8,            # reception cones
        n_ec=8,            # emission cones
        n_freq=1,          # grey frequency bins
        rr_bin=-1,         # bin that carries recombination photons (-1: none)
        recomb_mode=CASE_B_OTS,
        isothermal=1,
        freeze_chem=0,     # 1: skip the chemistry update (transport-only runs)
        precision=FP64,
        n_em=10,           # emission sub-steps per RT step (dt / dt_em)
        max_hops=4000,
        max_vip_depth=4,
        dt=0.1 * MYR_S,
        floor_rel=1e-20,   # packets below floor_rel * N_H of their particle are absorbed there
        chem_frac=0.1,     # sub-step = chem_frac * relaxation time
        seed=BASE_SEED,
    )
    p.update(kw)
    return p


def jittered_lattice(n_side, box_lo, box_len, rng, jitter=0.3):
    """Positions (i + 1/2 + U(-jitter, jitter)) * dx on an n_side^3 lattice, C order."""
    dx = box_len / n_side
    idx = np.arange(n_side, dtype=np.float64)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    lat = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    jit = rng.uniform(-jitter, jitter, size=lat.shape)
    return np.asarray(box_lo, dtype=np.float64)[None, :] + (lat + 0.5 + jit) * dx


def _uniform_gas(pos, n_h, box_len, x_hi0, t0):
    n = pos.shape[0]
    nh = np.full(n, n_h, dtype=np.float64)
    vol = box_len ** 3 / n
    NH = nh * vol
    return nh, NH, np.full(n, x_hi0, dtype=np.float64), np.full(n, t0, dtype=np.float64)


def _pack(name, params, sigma, eps, insts, sources, n_steps):
    """insts: list of dicts with pos, nH, NH, xHI, T, box_lo, box_hi."""
    pos = np.concatenate([d["pos"] for d in insts], axis=0)
    off = np.zeros(len(insts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([d["pos"].shape[0] for d in insts])
    box = np.array([list(d["box_lo"]) + list(d["box_hi"]) for d in insts], dtype=np.float64)
    cfg = dict(
        name=name,
        params=params,
        sigma=np.asarray(sigma, dtype=np.float64),
        eps=np.asarray(eps, dtype=np.float64),
        inst_off=off,
        box=box,
        pos=np.ascontiguousarray(pos),
        nH=np.concatenate([d["nH"] for d in insts]),
        NH=np.concatenate([d["NH"] for d in insts]),
        xHI=np.concatenate([d["xHI"] for d in insts]),
        T=np.concatenate([d["T"] for d in insts]),
        sources=sources,
        n_steps=n_steps,
    )
    return cfg


def _point_sources(inst, pos, rate):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    return dict(
        inst=np.asarray(inst, dtype=np.int32),
        kind=np.full(len(inst), SRC_POINT, dtype=np.int32),
        pos=np.ascontiguousarray(pos),
        rate=np.ascontiguousarray(np.asarray(rate, dtype=np.float64)),
        n_side=np.zeros(len(inst), dtype=np.int32),
    )


def stromgren(n_side=16, box_kpc=6.6, rr=False, n_ngb=32, ndot=5e48, n_h=1e-3,
              n_steps=100, seed_k=1, dt_myr=0.1, n_em=10, **pkw):
    """Stromgren HII region (section 3 set-up, scaled): uniform neutral hydrogen,
    one monochromatic 13.6 eV source at the exact box centre.  With rr=True a
    second bin carries recombination photons (case A + explicit transport);
    with rr="shared" they travel in the source's own bin (section 2.2's
    further saving, appropriate here since both are 13.6 eV photons)."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    L = box_kpc * KPC_CM
    lo = np.zeros(3)
    pos = jittered_lattice(n_side, lo, L, rng)
    nh, NH, xhi, T = _uniform_gas(pos, n_h, L, 1.0, 1e4)
    shared = rr == "shared"
    n_freq = 2 if (rr and not shared) else 1
    params = default_params(
        n_ngb=n_ngb, n_freq=n_freq, rr_bin=(0 if shared else 1 if rr else -1),
        recomb_mode=(RR_TRANSPORT if rr else CASE_B_OTS),
        dt=dt_myr * MYR_S, n_em=n_em, seed=BASE_SEED + seed_k)
    params.update(pkw)
    sigma = [SIGMA_13P6] * n_freq
    eps = [0.0] * n_freq          # 13.6 eV photons carry no excess energy; isothermal runs
    rate = np.zeros((1, n_freq))
    rate[0, 0] = ndot
    src = _point_sources([0], [L / 2, L / 2, L / 2], rate)
    inst = dict(pos=pos, nH=nh, NH=NH, xHI=xhi, T=T, box_lo=lo, box_hi=lo + L)
    return _pack(f"stromgren{n_side}{'_rr_shared' if shared else '_rr' if rr else ''}", params, sigma, eps, [inst], src,
                 n_steps)


def batched(n_inst=64, side_lo=8, side_hi=48, n_ngb=48, n_steps=100, seed_k=4, rr=True, **pkw):
    """Many independent HII regions of uneven size in one batch: n_side log-uniform
    in [side_lo, side_hi], n_H log-uniform in 1e-4..1e-1, Ndot log-uniform in
    1e47..1e50, box side L = R_S / U(0.2, 0.4)."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    insts = []
    rates = []
    spos = []
    x0 = 0.0
    n_freq = 2 if rr else 1
    for k in range(n_inst):
        ns = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        n_h = math.exp(rng.uniform(math.log(1e-4), math.log(1e-1)))
        ndot = math.exp(rng.uniform(math.log(1e47), math.log(1e50)))
        rs = (3.0 * ndot / (4.0 * math.pi * n_h * n_h * ALPHA_B_1E4)) ** (1.0 / 3.0)
        L = rs / rng.uniform(0.2, 0.4)
        lo = np.array([x0, 0.0, 0.0])
        x0 += 2.0 * L          # instances sit side by side; each keeps its own box
        pos = jittered_lattice(ns, lo, L, rng)
        nh, NH, xhi, T = _uniform_gas(pos, n_h, L, 1.0, 1e4)
        insts.append(dict(pos=pos, nH=nh, NH=NH, xHI=xhi, T=T, box_lo=lo, box_hi=lo + L))
        r = np.zeros(n_freq)
        r[0] = ndot
        rates.append(r)
        spos.append(lo + L / 2)
    params = default_params(
        n_ngb=n_ngb, n_freq=n_freq, rr_bin=(1 if rr else -1),
        recomb_mode=(RR_TRANSPORT if rr else CASE_B_OTS), seed=BASE_SEED + seed_k)
    params.update(pkw)
    src = _point_sources(list(range(n_inst)), np.array(spos), np.array(rates))
    return _pack(f"batched{n_inst}", params, [SIGMA_13P6] * n_freq, [0.0] * n_freq, insts, src, n_steps)


# Hydrogen photoionization cross-section: the analytic fit of Verner, Ferland,
# Korista & Yakovlev (1996, ApJ 465, 487), which section 2.1 cites for the
# frequency-dependent cross-sections.  For H I the fit's parameters are
# E_0 = 0.4298 eV, sigma_0 = 5.475e4 Mb, y_a = 32.88, P = 2.963 (y_w = y_0 =
# y_1 = 0): with x = y = E/E_0,
#   sigma(E) = sigma_0 (x - 1)^2 y^(P/2 - 5.5) (1 + sqrt(y/y_a))^-P  for E >= 13.6 eV.
VERNER_HI = dict(E0_ev=0.4298, sigma0_cm2=5.475e4 * 1e-18, ya=32.88, P=2.963)
E_HI_EV = 13.6


def sigma_hi_verner(e_ev):
    """Verner et al. (1996) hydrogen photoionization cross-section (cm^2) at photon energy e_ev."""
    v = VERNER_HI
    y = np.asarray(e_ev, dtype=np.float64) / v["E0_ev"]
    return v["sigma0_cm2"] * (y - 1.0) ** 2 * y ** (0.5 * v["P"] - 5.5) * (1.0 + np.sqrt(y / v["ya"])) ** (-v["P"])


def blackbody_grey_bins(t_bb, edges_ev, n_per_bin=4001):
    """Grey constants of a blackbody of temperature t_bb (K) in the photon-energy bins
    edges_ev (section 2.1's grey approximation: the spectral shape inside a bin
    enters as a cross-section averaged over the source spectrum): the fraction of
    the photons (between the first and last edge) in each bin, the photon-weighted
    cross-section <sigma> (cm^2), and the excess energy per absorption <eps> (eV),
    E - 13.6 eV weighted by sigma times the photon spectrum (the optically thin
    limit).  The photon spectrum is B_nu / h nu ~ E^2 / (exp(E / kT) - 1).
    Composite Simpson quadrature on n_per_bin points per bin, uniform in log E."""
    kt = K_BOLTZ * t_bb / EV_ERG
    frac, sig, eps, num = [], [], [], []
    for a, b in zip(edges_ev[:-1], edges_ev[1:]):
        u = np.linspace(math.log(a), math.log(b), n_per_bin)
        e = np.exp(u)
        w = np.full(n_per_bin, 2.0)
        w[1::2] = 4.0
        w[0] = w[-1] = 1.0
        w *= (u[1] - u[0]) / 3.0 * e           # dE = E du
        nph = e * e / (np.exp(e / kt) - 1.0)   # E / kT >= 1.5 here: no cancellation
        sg = sigma_hi_verner(e)
        n = np.sum(w * nph)
        sn = np.sum(w * sg * nph)
        num.append(n)
        sig.append(sn / n)
        eps.append(np.sum(w * (e - E_HI_EV) * sg * nph) / sn)
    tot = sum(num)
    frac = [n / tot for n in num]
    return tuple(frac), tuple(sig), tuple(eps)


# Grey bins of a 1e5 K blackbody between 13.6, 24.6, 54.4 and 100 eV (section 4
# uses this spectrum), from the Verner cross-section: the fraction of the
# photons in each bin, the photon-weighted cross-section and the
# cross-section-weighted excess energy per absorption.
BB1E5_EDGES_EV = (13.6, 24.6, 54.4, 100.0)
BB1E5_FRAC, BB1E5_SIGMA, BB1E5_EPS_EV = blackbody_grey_bins(1e5, BB1E5_EDGES_EV)
EPS_RR_EV = 2.327      # kT at 2.7e4 K: excess energy of a recombination photon (section 4)


def shadow(n_side=128, box_kpc=6.6, n_h=2e-4, clump_nh=0.04, clump_r_kpc=0.8,
           clump_c_kpc=(1.7, 3.3, 3.3), flux=1e6, n_pp=100, n_ngb=48, n_tc=16, n_rc=16,
           n_ec=16, t0=8000.0, n_steps=20, seed_k=3, dt_myr=0.1, **pkw):
    """Shadow set-up (section 4, scaled): a plane-parallel front from the x = 0
    face (n_pp^2 boundary emitters, flux in photons/s/cm^2) with a 1e5 K
    blackbody in three grey bins, a dense spherical clump in low-density gas,
    recombination radiation in a fourth bin, photoheating and cooling on.
    Particles are a jittered lattice; those inside the clump carry its density."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    L = box_kpc * KPC_CM
    lo = np.zeros(3)
    pos = jittered_lattice(n_side, lo, L, rng)
    c = np.asarray(clump_c_kpc, dtype=np.float64) * KPC_CM
    inside = np.sum((pos - c[None, :]) ** 2, axis=1) <= (clump_r_kpc * KPC_CM) ** 2
    nh = np.where(inside, clump_nh, n_h)
    NH = nh * (L ** 3 / pos.shape[0])
    xhi = np.ones(pos.shape[0])
    T = np.full(pos.shape[0], t0)
    n_freq = 4
    params = default_params(
        n_ngb=n_ngb, n_tc=n_tc, n_rc=n_rc, n_ec=n_ec, n_freq=n_freq, rr_bin=3,
        recomb_mode=RR_TRANSPORT, isothermal=0, dt=dt_myr * MYR_S, n_em=1,
        seed=BASE_SEED + seed_k)
    params.update(pkw)
    sigma = list(BB1E5_SIGMA) + [SIGMA_13P6]
    eps = [e * EV_ERG for e in BB1E5_EPS_EV] + [EPS_RR_EV * EV_ERG]
    rate = np.zeros((1, n_freq))
    rate[0, :3] = flux * np.asarray(BB1E5_FRAC)
    src = dict(inst=np.zeros(1, np.int32), kind=np.array([SRC_PLANE_XLO], np.int32),
               pos=np.zeros((1, 3)), rate=rate, n_side=np.array([n_pp], np.int32))
    inst = dict(pos=pos, nH=nh, NH=NH, xHI=xhi, T=T, box_lo=lo, box_hi=lo + L)
    return _pack(f"shadow{n_side}", params, sigma, eps, [inst], src, n_steps)


# Section 4 quotes one grey value pair for the 1e5 K blackbody when all its
# photons travel in one bin.
SIGMA_BB1E5_GREY = 1.6e-18     # cm^2
EPS_BB1E5_GREY_EV = 6.3        # eV


def alpha_hg97(t):
    """Case-A and case-B recombination coefficients of hydrogen (cm^3/s) at
    temperature t (K): the fits of Hui & Gnedin (1997) that section 2.1 adopts,
    with lambda = 2 T_HI / T and T_HI = 157807 K,
      alpha_A = 1.269e-13 lambda^1.503 / (1 + (lambda / 0.522)^0.470)^1.923,
      alpha_B = 2.753e-14 lambda^1.5 / (1 + (lambda / 2.740)^0.407)^2.242.
    Used here only to size the boundary sources of the recipe below."""
    lam = 2.0 * 157807.0 / t
    a_a = 1.269e-13 * lam ** 1.503 / (1.0 + (lam / 0.522) ** 0.470) ** 1.923
    a_b = 2.753e-14 * lam ** 1.5 / (1.0 + (lam / 2.740) ** 0.407) ** 2.242
    return a_a, a_b
# Boundary-source grid faces: (normal axis, side) for y = lo, y = hi, z = lo, z = hi.
BOUNDARY_FACES = ((1, 0), (1, 1), (2, 0), (2, 1))


def boundary_rr_intensity(flux, n_h, sigma=SIGMA_13P6):
    """Appendix B: recombination radiation reaching a point from uniformly
    ionized gas around it, for monochromatic radiation of cross-section sigma.
    Photoionization equilibrium with the front, sigma F (1 - x) = alpha_B n_H
    x^2 (x = x_HII), fixes the emissivity of ground-state recombinations,
    E = alpha_1 n_H^2 x^2 (alpha_1 = alpha_A - alpha_B), and the mean free path
    of their photons, lambda = 1 / (sigma n_H (1 - x)); integrating
    E e^{-r/lambda} / (4 pi r^2) over the sphere of radius lambda gives the
    intensity I = (1 - 1/e) lambda E (photons/s/cm^2), the appendix's 0.63 lambda E.
    Recombination coefficients at 1e4 K from alpha_hg97."""
    a_a, a_b = alpha_hg97(1e4)
    a = a_b * n_h / (sigma * flux)
    x = 2.0 / (1.0 + math.sqrt(1.0 + 4.0 * a))          # positive root of a x^2 + x - 1 = 0
    lam = 1.0 / (sigma * n_h * (1.0 - x))
    emis = (a_a - a_b) * n_h * n_h * x * x
    return dict(x_HII=x, mfp=lam, emissivity=emis, intensity=(1.0 - math.exp(-1.0)) * lam * emis,
                alpha_A=a_a, alpha_B=a_b)


def shadow_boundary(n_side=32, box_kpc=13.2, n_h=1e-3, clump_nh=1.0, clump_r=0.1,
                    clump_c=(0.27, 0.5, 0.5), flux=1e6, n_pp=100, n_bd=50, n_ngb=48, n_tc=16,
                    n_rc=8, n_ec=8, t0=1e4, n_steps=100, seed_k=4, dt_myr=0.1, barrier=False,
                    barrier_r=0.2, barrier_c=(0.27, 0.5, 0.5), **pkw):
    """Shadow set-up of section 4 with recombination radiation from outside the
    box (appendix B): 32^3 particles in a 13.2 kpc box at n_H = 1e-3, a plane
    front of 1e6 photons/s/cm^2 from the x = 0 face (n_pp^2 emitters) in one grey
    bin of the 1e5 K blackbody, a dense clump (radius clump_r L at clump_c L)
    casting the shadow, N_RC = 8, dt = dt_em = 0.1 Myr.  Bins: 0 source,
    1 recombination photons emitted in the box, 2 recombination photons from
    outside the box, 3 unused (no source: packet slots per particle, N_RC times
    the bins, must be a power of two).
    The outside-box photons come from n_bd^2 isotropic point sources on a
    regular grid on each of the four faces parallel to the front's direction,
    each emitting I L^2 / n_bd^2 photons/s in bin 2 (boundary_rr_intensity: the
    appendix's equilibrium estimate for monochromatic 13.6 eV photons).
    They start radiating once the I-front has passed them, which the caller
    decides between steps: cfg["boundary"] holds their positions and rates and
    boundary_sources(cfg, on) gives the source set with those switched on.
    barrier=True: section 4's own obstacle instead of the clump, uniform gas
    and an artificial disk of radius barrier_r L at barrier_c L in the plane
    parallel to the x = 0 face that removes every packet passing through it
    (cfg["barrier"]: instance, centre and radius in cm)."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    L = box_kpc * KPC_CM
    lo = np.zeros(3)
    pos = jittered_lattice(n_side, lo, L, rng)
    c = np.asarray(clump_c, dtype=np.float64) * L
    inside = np.sum((pos - c[None, :]) ** 2, axis=1) <= (clump_r * L) ** 2
    nh = np.full(pos.shape[0], float(n_h)) if barrier else np.where(inside, clump_nh, n_h)
    NH = nh * (L ** 3 / pos.shape[0])
    n_freq = 4
    params = default_params(
        n_ngb=n_ngb, n_tc=n_tc, n_rc=n_rc, n_ec=n_ec, n_freq=n_freq, rr_bin=1,
        recomb_mode=RR_TRANSPORT, isothermal=0, dt=dt_myr * MYR_S, n_em=1,
        seed=BASE_SEED + seed_k)
    params.update(pkw)
    sigma = [SIGMA_BB1E5_GREY, SIGMA_13P6, SIGMA_13P6, SIGMA_13P6]
    eps = [EPS_BB1E5_GREY_EV * EV_ERG] + [EPS_RR_EV * EV_ERG] * 3
    rate = np.zeros((1, n_freq))
    rate[0, 0] = flux
    src = dict(inst=np.zeros(1, np.int32), kind=np.array([SRC_PLANE_XLO], np.int32),
               pos=np.zeros((1, 3)), rate=rate, n_side=np.array([n_pp], np.int32))
    inst = dict(pos=pos, nH=nh, NH=NH, xHI=np.ones(pos.shape[0]), T=np.full(pos.shape[0], t0),
                box_lo=lo, box_hi=lo + L)
    cfg = _pack(f"shadow_{'barrier' if barrier else 'boundary'}{n_side}", params, sigma, eps, [inst], src, n_steps)
    if barrier:
        cfg["barrier"] = dict(inst=0, center=np.asarray(barrier_c, dtype=np.float64) * L + lo,
                              radius=float(barrier_r) * L)
    bi = boundary_rr_intensity(flux, n_h)
    g = (np.arange(n_bd) + 0.5) * (L / n_bd)
    bpos = []
    for ax, side in BOUNDARY_FACES:
        t1, t2 = [k for k in range(3) if k != ax]
        for u in g:
            for v in g:
                p = np.zeros(3)
                p[ax] = lo[ax] + side * L
                p[t1] = lo[t1] + u
                p[t2] = lo[t2] + v
                bpos.append(p)
    brate = np.zeros((len(bpos), n_freq))
    brate[:, 2] = bi["intensity"] * L * L / (n_bd * n_bd)
    cfg["boundary"] = dict(pos=np.array(bpos), rate=brate, flux=flux, n_h=n_h, **bi)
    return cfg


def shadow_barrier(n_side=32, n_tc=128, **kw):
    """Section 4's shadow test as the paper runs it: 32^3 particles in 13.2 kpc
    of uniform gas at n_H = 1e-3, the artificial barrier disk (radius 0.2 L at
    (0.27, 0.5, 0.5) L), the plane front, boundary recombination sources on the
    four faces parallel to it, N_TC = 128 and N_RC = 8.  At N_TC = 128 most
    transmission cones hold no neighbour, so virtual particles carry much of
    the transport; chains may run 15 deep (at depth 4 a fifth or more of the
    front's photons would end as removed)."""
    kw.setdefault("max_vip_depth", 15)
    return shadow_boundary(n_side=n_side, n_tc=n_tc, barrier=True, **kw)


def boundary_schedule(cfg, t):
    """Boundary sources of shadow_boundary the I-front has passed at time t (s),
    taking the front where it would be if no gas recombined: every photon of the
    flux ionizes one atom, so it advances at F / n_H (the Stromgren distance of
    the appendix, 1251 kpc, is far beyond the box).  A schedule for inputs only."""
    b = cfg["boundary"]
    lo = float(cfg["box"][0][0])
    return b["pos"][:, 0] - lo <= b["flux"] * t / b["n_h"]


def boundary_sources(cfg, on):
    """The front's sources plus the boundary sources of shadow_boundary whose
    entry in the boolean mask on[4 n_bd^2] is set."""
    on = np.asarray(on, dtype=bool)
    b, s = cfg["boundary"], cfg["sources"]
    n = int(on.sum())
    return dict(
        inst=np.concatenate([s["inst"], np.zeros(n, np.int32)]),
        kind=np.concatenate([s["kind"], np.full(n, SRC_POINT, np.int32)]),
        pos=np.ascontiguousarray(np.concatenate([s["pos"], b["pos"][on]])),
        rate=np.ascontiguousarray(np.concatenate([s["rate"], b["rate"][on]])),
        n_side=np.concatenate([s["n_side"], np.zeros(n, np.int32)]),
    )


def instance(cfg, k):
    """Instance k of a batch as a workload of its own (same particles, box,
    sources and parameters)."""
    lo, hi = int(cfg["inst_off"][k]), int(cfg["inst_off"][k + 1])
    src = cfg["sources"]
    sel = src["inst"] == k
    sources = dict(inst=np.zeros(int(sel.sum()), dtype=np.int32), kind=src["kind"][sel].copy(),
                   pos=np.ascontiguousarray(src["pos"][sel]), rate=np.ascontiguousarray(src["rate"][sel]),
                   n_side=src["n_side"][sel].copy())
    out = dict(cfg)
    out.update(name=f'{cfg["name"]}_{k}', inst_off=np.array([0, hi - lo], dtype=np.int64),
               box=np.ascontiguousarray(cfg["box"][k:k + 1]), sources=sources)
    for key in ("pos", "nH", "NH", "xHI", "T"):
        out[key] = np.ascontiguousarray(cfg[key][lo:hi])
    return out


def chain(n=12, spacing_kpc=0.1, n_h=1e-3, x_hi=1e-3, **pkw):
    """A 1-D chain of particles along x with two neighbours each and a plane
    front on the x = 0 face: used to check attenuation exp(-sigma n sum l)."""
    L = n * spacing_kpc * KPC_CM
    dxs = spacing_kpc * KPC_CM
    pos = np.zeros((n, 3))
    pos[:, 0] = (np.arange(n) + 0.5) * dxs
    pos[:, 1] = 0.5 * dxs
    pos[:, 2] = 0.5 * dxs
    nh = np.full(n, n_h)
    NH = nh * dxs ** 3
    params = default_params(n_ngb=2, n_freq=1, n_em=1, freeze_chem=1)
    params.update(pkw)
    src = dict(inst=np.zeros(1, np.int32), kind=np.array([SRC_PLANE_XLO], np.int32),
               pos=np.zeros((1, 3)), rate=np.array([[1e6]]), n_side=np.array([1], np.int32))
    inst = dict(pos=pos, nH=nh, NH=NH, xHI=np.full(n, x_hi), T=np.full(n, 1e4),
                box_lo=np.zeros(3), box_hi=np.array([L, dxs, dxs]))
    return _pack("chain", params, [SIGMA_13P6], [0.0], [inst], src, 1)


def lognormal_density(n_mesh, sigma_g, slope, rng):
    """A lognormal density on an n_mesh^3 periodic mesh: a Gaussian random
    field g with power spectrum P(k) ~ k^slope (the k = 0 mode removed), scaled
    to variance sigma_g^2, and rho = exp(g - sigma_g^2 / 2) (mean 1 in
    expectation)."""
    white = rng.standard_normal((n_mesh, n_mesh, n_mesh))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n_mesh)
    kz = np.fft.rfftfreq(n_mesh)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)    # sqrt(P(k)) = k^(slope / 2)
    g = np.fft.irfftn(fk * amp, s=(n_mesh, n_mesh, n_mesh), axes=(0, 1, 2))
    g *= sigma_g / g.std()
    return np.exp(g - 0.5 * sigma_g * sigma_g)


def clustered(n_side=256, box_mpc=10.0, n_h=1e-3, sigma_g=1.5, slope=-2.5, n_src=1024, ndot_lo=1e48,
              ndot_hi=1e52, n_ngb=48, n_tc=32, n_rc=8, n_ec=32, t0=100.0, n_steps=20, seed_k=5, dt_myr=0.1,
              vip_capacity=1 << 25, **pkw):
    """The large clustered field: n_side^3 equal-mass particles sampled from a
    lognormal density on an n_side^3 mesh in a box_mpc cube (cell counts N
    rho_c / sum rho by largest-remainder rounding, ties to the lower cell index;
    uniform within cells); a particle's n_H is that of its cell (mean n_h), its
    N_H the same for all.  n_src point sources at the densest particles (ties to
    the lower index) with Ndot drawn from dN/dNdot ~ Ndot^-2 between ndot_lo and
    ndot_hi; a 1e5 K blackbody in four grey bins (13.6-18-24.6-54.4-100 eV) and
    the recombination bin, padded with three empty bins so that a particle's
    packet slots (n_rc x 8) fill one wavefront: n_rc = 8, where the paper-scale
    recipe would use 32.  Photoheating and cooling from T0 = 100 K."""
    rng = np.random.default_rng(BASE_SEED + seed_k)
    L = box_mpc * 1e3 * KPC_CM
    n = n_side
    rho = lognormal_density(n, sigma_g, slope, rng)
    N = n ** 3
    q = N * rho.ravel() / rho.sum()
    cnt = np.floor(q).astype(np.int64)
    rest = N - int(cnt.sum())
    if rest > 0:
        order = np.argsort(-(q - cnt), kind="stable")
        cnt[order[:rest]] += 1
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), cnt)
    ijk = np.stack([cells // (n * n), (cells // n) % n, cells % n], axis=1).astype(np.float64)
    dx = L / n
    pos = (ijk + rng.random((N, 3))) * dx
    pos = np.minimum(pos, np.nextafter(L, 0.0))
    dens = rho.ravel() / rho.mean()
    nh = n_h * dens[cells]
    NH = np.full(N, n_h * L ** 3 / N)
    xhi = np.ones(N)
    T = np.full(N, t0)
    frac, sig, eps = blackbody_grey_bins(1e5, (13.6, 18.0, 24.6, 54.4, 100.0))
    n_freq = 8
    rr_bin = 4
    params = default_params(
        n_ngb=n_ngb, n_tc=n_tc, n_rc=n_rc, n_ec=n_ec, n_freq=n_freq, rr_bin=rr_bin,
        recomb_mode=RR_TRANSPORT, isothermal=0, dt=dt_myr * MYR_S, n_em=1,
        seed=BASE_SEED + seed_k, vip_capacity=vip_capacity)
    params.update(pkw)
    sigma = list(sig) + [SIGMA_13P6] * 4
    eps_erg = [e * EV_ERG for e in eps] + [EPS_RR_EV * EV_ERG] + [0.0] * 3
    dense = np.argsort(-nh, kind="stable")[:n_src]
    u = rng.random(n_src)
    ndot = 1.0 / (1.0 / ndot_lo - u * (1.0 / ndot_lo - 1.0 / ndot_hi))
    rate = np.zeros((n_src, n_freq))
    rate[:, :4] = ndot[:, None] * np.asarray(frac)[None, :]
    src = _point_sources(np.zeros(n_src, np.int32), pos[dense], rate)
    inst = dict(pos=pos, nH=nh, NH=NH, xHI=xhi, T=T, box_lo=np.zeros(3), box_hi=np.full(3, L))
    return _pack(f"clustered{n_side}", params, sigma, eps_erg, [inst], src, n_steps)


def config(k, **kw):
    """Named workloads: 1 = 16^3 Stromgren case B (FP64), 2 = 64^3 with recombination
    radiation (FP32 vs FP64), 3 = 128^3 shadow set-up (plane front, blackbody bins,
    clump, heating and cooling), 4 = 64 batched instances with recombination radiation,
    5 = 256^3 particles of a clustered (lognormal) field with 1024 sources."""
    if k == 1:
        return stromgren(16, rr=False, n_ngb=32, n_steps=100, seed_k=1, **kw)
    if k == 2:
        return stromgren(64, rr=True, n_ngb=48, n_steps=500, seed_k=2, **kw)
    if k == 3:
        return shadow(**kw)
    if k == 4:
        return batched(**kw)
    if k == 5:
        return clustered(**kw)
    raise ValueError(f"unknown workload {k}")


def n_particles(cfg):
    return int(cfg["pos"].shape[0])
