"""rt_shell_profile_noalloc (through the C ABI) against rt_shell_profile on the
same state and inputs.

The no-allocation variant bins into the library's static device scratch
instead of buffers the context allocates.  Shell counts must agree bit for bit;
shell sums are sums of positive terms whose order differs between two GPU runs
(LDS and global atomics), so they agree within 2 n_s 2^-53 relative per shell
(plus one rounding each for the mean and the normalisation), the bar of the
profile tests.  Two calls in a row, the second on a smaller input (a smaller
instance, fewer shells, a caller-given device array), must both agree: the
scratch keeps the first call's contents and must be cleared by the second.
"""
import sys

import numpy as np
import pytest

from paper_1311_0182_amd import inputs as I

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _agree(pa, ca, pb, cb):
    assert np.array_equal(ca, cb)
    tol = (2.0 * np.maximum(cb, 1) + 4.0) * U
    err = np.abs(pa - pb) / np.maximum(np.abs(pb), 1e-300)
    bad = (pb != 0) & (err > tol[:, None])
    assert not bad.any(), (np.argwhere(bad)[:5], err[bad][:5])
    assert np.array_equal(pa == 0, pb == 0)


def test_shell_profile_noalloc_matches_allocating_entry_point():
    import torch
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.batched(n_inst=3, side_lo=10, side_hi=18, n_ngb=32, n_steps=4)
    sizes = np.diff(cfg["inst_off"])
    big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
    assert sizes[small] < sizes[big]
    ctx = RT.Context(cfg, precision="fp64")
    ctx.step(3)
    n, nf = ctx.N, ctx.nf

    # call 1: the context's passing photons, the largest instance, many shells
    box = np.asarray(cfg["box"][big], dtype=float)
    L = float(box[3] - box[0])
    src = np.asarray(cfg["sources"]["pos"][big], dtype=float)
    g1 = dict(center=src, r_max=0.6 * L, n_shells=700, inst=big)
    say("call 1: instance", big, "particles", int(sizes[big]), "shells", g1["n_shells"])
    pa, ca = ctx.shell_profile_noalloc(**g1)
    pb, cb = ctx.shell_profile(**g1)
    assert ca.sum() > 0 and pa.max() > 0
    _agree(pa, ca, pb, cb)

    # call 2: a smaller instance, fewer shells, cylinders, a device array given
    rng = np.random.default_rng(1311018299)
    P = 10.0 ** rng.uniform(40, 56, size=(n, nf))
    P[rng.random((n, nf)) < 0.2] = 0.0
    Pd = torch.from_numpy(P.reshape(-1).copy()).to("cuda")
    box = np.asarray(cfg["box"][small], dtype=float)
    L = float(box[3] - box[0])
    mid = 0.5 * (box[:3] + box[3:])
    g2 = dict(center=mid, r_max=0.5 * L, n_shells=23, axis=(0.3, -1.1, 0.4), half_height=0.3 * L, mean=True,
              norm=2.5e49, inst=small)
    say("call 2: instance", small, "particles", int(sizes[small]), "shells", g2["n_shells"])
    pa, ca = ctx.shell_profile_noalloc(passing_dev=Pd, **g2)
    pb, cb = ctx.shell_profile(passing=P, **g2)
    assert ca.sum() > 0
    _agree(pa, ca, pb, cb)
    # the first call's histogram (700 shells) was cleared: nothing leaks into call 2
    assert pa.shape == (23, nf)

    # rejected: host memory for the passing photons, too many shells
    with pytest.raises(RT.RTError) as e:
        L_ = RT.load()
        c = np.asarray(mid, dtype=np.float64)
        prof = np.empty((4, nf))
        st = L_.rt_shell_profile_noalloc(ctx.h, 0, P.ctypes.data_as(RT.C.c_void_p), RT._p(c, RT.C.c_double), None,
                                         0.0, 1.0, 4, 0, 1.0, RT._p(prof, RT.C.c_double), None)
        ctx._check(st)
    assert e.value.status == RT.RT_EINVAL
    with pytest.raises(RT.RTError) as e:
        ctx.shell_profile_noalloc(center=mid, r_max=L, n_shells=2049)
    assert e.value.status == RT.RT_EINVAL
    ctx.close()
