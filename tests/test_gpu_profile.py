"""Parity of the intensity profiles (sections 3 and 4) computed by the library
(rt_shell_profile, through the C ABI) with the oracle's.

Shell membership is an integer decided in FP64 with the same operations in the
same order on both sides, so the particle counts must agree bit for bit.  The
shell sums are sums of positive terms added in different orders (LDS and global
atomics on the GPU, particle order in the oracle); each side's relative error is
at most (n_s - 1) 2^-53 for n_s terms, so the bar is 2 n_s 2^-53 relative per
shell (plus one rounding for the mean and one for the normalisation).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_0182_amd import inputs as I

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(cfg, precision="fp64"):
    from paper_1311_0182_amd import traphic_rt as RT
    return RT.Context(cfg, precision=precision)


def _check(pg, cg, po, co):
    assert np.array_equal(cg, co)
    tol = (2.0 * np.maximum(co, 1) + 4.0) * U
    err = np.abs(pg - po) / np.maximum(np.abs(po), 1e-300)
    bad = (po != 0) & (err > tol[:, None])
    assert not bad.any(), (np.argwhere(bad)[:5], err[bad][:5])
    assert np.array_equal(pg == 0, po == 0)


def _passing(rng, n, nf):
    # photon counts spanning the range of a step: many zeros (no packet passed),
    # the rest log-uniform over 1e40 .. 1e56
    P = 10.0 ** rng.uniform(40, 56, size=(n, nf))
    P[rng.random((n, nf)) < 0.2] = 0.0
    return P


def _geometries(cfg, k):
    box = np.asarray(cfg["box"][k], dtype=float)
    lo, hi = box[:3], box[3:]
    L = float(np.max(hi - lo))
    mid = 0.5 * (lo + hi)
    own = np.flatnonzero(np.asarray(cfg["sources"]["inst"]) == k)
    src = np.asarray(cfg["sources"]["pos"][own[0]], dtype=float) if len(own) else mid
    return [
        ("sphere about the source, 128 shells", dict(center=src, r_max=0.5 * L, n_shells=128)),
        ("sphere about a corner, mean, normalised", dict(center=lo, r_max=1.8 * L, n_shells=37, mean=True,
                                                         norm=3.7e50)),
        ("cylinder along x through the centre, height cut", dict(center=mid, r_max=0.5 * L, n_shells=50,
                                                                axis=(1.0, 0.0, 0.0), half_height=0.25 * L,
                                                                mean=True)),
        ("tilted cylinder, no cut", dict(center=mid, r_max=0.7 * L, n_shells=19, axis=(0.3, -1.1, 0.4))),
    ]


def _oracle(cfg, k, P, g):
    j0, j1 = int(cfg["inst_off"][k]), int(cfg["inst_off"][k + 1])
    return O.shell_profile(cfg["pos"][j0:j1], P[j0:j1], cfg["params"]["dt"], g["center"], g["r_max"],
                           g["n_shells"], axis=g.get("axis"), half_height=g.get("half_height", 0.0),
                           mean=g.get("mean", False), norm=g.get("norm", 1.0))


@pytest.mark.parametrize("which", ["stromgren16", "stromgren64", "batched64"])
def test_shell_profile_given_passing(which):
    cfg = {"stromgren16": lambda: I.config(1), "stromgren64": lambda: I.config(2),
           "batched64": lambda: I.config(4)}[which]()
    n, nf = cfg["pos"].shape[0], int(cfg["params"]["n_freq"])
    say("shell profiles of seeded passing photons:", which, "N", n, "bins", nf)
    P = _passing(np.random.default_rng(11), n, nf)
    ctx = _ctx(cfg)
    insts = [0] if len(cfg["inst_off"]) == 2 else [0, 17, len(cfg["inst_off"]) - 2]
    for k in insts:
        for name, g in _geometries(cfg, k):
            say(" instance", k, name)
            pg, cg = ctx.shell_profile(inst=k, passing=P, **g)
            po, co = _oracle(cfg, k, P, g)
            _check(pg, cg, po, co)
            assert cg.sum() > 0
    ctx.close()


def test_shell_profile_of_last_step():
    # the library's own passing photons after a few FP64 steps against the
    # oracle's after the same steps (the transport itself agrees to 1e-6)
    cfg = I.stromgren(11, rr=True, n_ngb=32, dt_myr=0.5)
    steps = 6
    say("11^3 with RR,", steps, "steps, profile of the last step")
    s = O.OracleSim(cfg)
    s.step(steps)
    so = s.state()
    ctx = _ctx(cfg)
    ctx.step(steps)
    for name, g in _geometries(cfg, 0):
        pg, cg = ctx.shell_profile(**g)
        po, co = _oracle(cfg, 0, so["P"], g)
        assert np.array_equal(cg, co), name
        scale = np.max(np.abs(po), axis=0)
        assert np.all(np.abs(pg - po) <= 1e-6 * np.maximum(scale, 1e-300)), name
        assert np.all(po[:, 0] >= 0) and scale[0] > 0
    # source and diffuse columns: the RR bin carries photons once gas has recombined
    prof, _ = ctx.shell_profile(center=cfg["sources"]["pos"][0], r_max=0.5 * float(cfg["box"][0][3]), n_shells=8)
    assert prof[:, int(cfg["params"]["rr_bin"])].sum() > 0
    ctx.close()
    s.close()


def test_shell_profile_edge_cases():
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.config(2)
    n, nf = cfg["pos"].shape[0], int(cfg["params"]["n_freq"])
    P = _passing(np.random.default_rng(5), n, nf)
    ctx = _ctx(cfg)
    L = float(cfg["box"][0][3])
    src = cfg["sources"]["pos"][0]
    cases = [
        ("one shell holding everything", dict(center=src, r_max=2.0 * L, n_shells=1)),
        ("most shells (2048)", dict(center=src, r_max=0.9 * L, n_shells=2048)),
        ("all particles beyond r_max", dict(center=src, r_max=1e-3 * L / 64, n_shells=4)),
        ("centre far outside the box", dict(center=np.array([5.0, -3.0, 2.0]) * L, r_max=10.0 * L, n_shells=64)),
        ("height cut thinner than the spacing", dict(center=src, r_max=0.5 * L, n_shells=16, axis=(0, 0, 1.0),
                                                     half_height=1e-6 * L, mean=True)),
    ]
    for name, g in cases:
        say(" ", name)
        pg, cg = ctx.shell_profile(passing=P, **g)
        po, co = _oracle(cfg, 0, P, g)
        _check(pg, cg, po, co)
    pg, cg = ctx.shell_profile(passing=P, center=src, r_max=2.0 * L, n_shells=1)
    assert cg[0] == n
    # two calls in a row share the histograms: the second must not see the first
    a1, c1 = ctx.shell_profile(passing=P, center=src, r_max=0.5 * L, n_shells=64)
    a2, c2 = ctx.shell_profile(passing=P, center=src, r_max=0.5 * L, n_shells=64)
    _check(a2, c2, a1, c1)
    # a smaller call after a larger one
    a3, c3 = ctx.shell_profile(passing=P, center=src, r_max=0.5 * L, n_shells=3)
    p3, q3 = _oracle(cfg, 0, P, dict(center=src, r_max=0.5 * L, n_shells=3))
    _check(a3, c3, p3, q3)
    bad = [dict(n_shells=0), dict(n_shells=2049), dict(n_shells=2048, axis=(0, 0, 0)), dict(axis=(1e200, 0, 0)),
           dict(norm=0.0),
           dict(r_max=-1.0), dict(r_max=float("nan")), dict(inst=1), dict(inst=-1)]
    for b in bad:
        g = dict(center=src, r_max=0.5 * L, n_shells=8)
        g.update(b)
        with pytest.raises(RT.RTError) as e:
            ctx.shell_profile(**g)
        assert e.value.status == RT.RT_EINVAL
    with pytest.raises(ValueError):
        ctx.shell_profile(center=src, r_max=L, n_shells=8, passing=P[:-1])
    # the context still works after the rejected calls
    pg, cg = ctx.shell_profile(passing=P, center=src, r_max=2.0 * L, n_shells=1)
    assert cg[0] == n
    ctx.close()
