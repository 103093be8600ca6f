"""Python binding of libtraphic_rt.so (include/traphic_rt.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies the HIP stream and, through the allocator callbacks,
the device memory (its caching allocator).  There is no CPU fallback: without
the built library or a GPU, creating a context raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtraphic_rt.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EHOPCAP, RT_ENONFINITE, RT_ESTATE, RT_EOVERFLOW, RT_EDRIFT = range(9)
STATUS = {0: "RT_OK", 1: "RT_EINVAL", 2: "RT_ENOMEM", 3: "RT_EDEVICE", 4: "RT_EHOPCAP",
          5: "RT_ENONFINITE", 6: "RT_ESTATE", 7: "RT_EOVERFLOW", 8: "RT_EDRIFT"}
RT_FP64, RT_FP32 = 0, 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

EXPORTS = ["rt_init", "rt_add_sources", "rt_step", "rt_get_state", "rt_get_bins", "rt_get_neighbours",
           "rt_n_emitters", "rt_get_emitter_neighbours", "rt_get_cone_masks", "rt_get_pending_rr",
           "rt_set_timing", "rt_get_timing", "rt_set_hop_shape", "rt_get_hop_shape", "rt_get_state_blob",
           "rt_set_state_blob", "rt_shell_profile", "rt_shell_profile_noalloc", "rt_set_barrier", "rt_set_step_graphs", "rt_destroy",
           "rt_last_error"]


class RTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("n_ngb", C.c_int32), ("n_tc", C.c_int32), ("n_rc", C.c_int32), ("n_ec", C.c_int32),
        ("n_freq", C.c_int32), ("rr_bin", C.c_int32), ("recomb_mode", C.c_int32),
        ("isothermal", C.c_int32), ("freeze_chem", C.c_int32), ("precision", C.c_int32),
        ("n_em", C.c_int32), ("max_hops", C.c_int32), ("max_vip_depth", C.c_int32),
        ("hop_batch", C.c_int32),
        ("dt", C.c_double), ("floor_rel", C.c_double), ("chem_frac", C.c_double),
        ("seed", C.c_uint64), ("vip_capacity", C.c_int64), ("record_capacity", C.c_int64),
        ("alloc", ALLOC_FN), ("dealloc", DEALLOC_FN), ("alloc_user", C.c_void_p),
    ]


_lib = None


def load():
    """Load the built library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1311_0182_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    dp, ip, i64p, u64p = P(C.c_double), P(C.c_int32), P(C.c_int64), P(C.c_uint64)
    vpp = P(C.c_void_p)
    L.rt_init.restype = C.c_int
    L.rt_init.argtypes = [vpp, P(Params), dp, dp, C.c_int32, i64p, dp, dp, dp, dp, dp, dp, C.c_void_p]
    L.rt_add_sources.restype = C.c_int
    L.rt_add_sources.argtypes = [C.c_void_p, C.c_int32, ip, ip, dp, dp, ip]
    L.rt_step.restype = C.c_int
    L.rt_step.argtypes = [C.c_void_p, C.c_int32]
    L.rt_get_state.restype = C.c_int
    L.rt_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, i64p]
    L.rt_get_bins.restype = C.c_int
    L.rt_get_bins.argtypes = [C.c_void_p, dp, dp, dp]
    L.rt_get_neighbours.restype = C.c_int
    L.rt_get_neighbours.argtypes = [C.c_void_p, ip, dp]
    L.rt_n_emitters.restype = C.c_int64
    L.rt_n_emitters.argtypes = [C.c_void_p]
    L.rt_get_emitter_neighbours.restype = C.c_int
    L.rt_get_emitter_neighbours.argtypes = [C.c_void_p, ip, dp]
    L.rt_get_cone_masks.restype = C.c_int
    L.rt_get_cone_masks.argtypes = [C.c_void_p, u64p]
    L.rt_get_pending_rr.restype = C.c_int
    L.rt_get_pending_rr.argtypes = [C.c_void_p, dp]
    L.rt_set_timing.restype = C.c_int
    L.rt_set_timing.argtypes = [C.c_void_p, C.c_int32]
    L.rt_get_timing.restype = C.c_int
    L.rt_get_timing.argtypes = [C.c_void_p, dp, C.c_int32]
    L.rt_set_hop_shape.restype = C.c_int
    L.rt_set_hop_shape.argtypes = [C.c_void_p, C.c_int32]
    L.rt_get_hop_shape.restype = C.c_int
    L.rt_get_hop_shape.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), dp]
    L.rt_get_state_blob.restype = C.c_int
    L.rt_get_state_blob.argtypes = [C.c_void_p, C.c_void_p, P(C.c_size_t)]
    L.rt_set_state_blob.restype = C.c_int
    L.rt_set_state_blob.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.rt_shell_profile.restype = C.c_int
    L.rt_shell_profile.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, C.c_double, C.c_double, C.c_int32,
                                   C.c_int32, C.c_double, dp, i64p]
    L.rt_shell_profile_noalloc.restype = C.c_int
    L.rt_shell_profile_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, dp, dp, C.c_double, C.c_double,
                                           C.c_int32, C.c_int32, C.c_double, dp, i64p]
    L.rt_set_step_graphs.restype = C.c_int
    L.rt_set_step_graphs.argtypes = [C.c_void_p, C.c_int32]
    L.rt_set_barrier.restype = C.c_int
    L.rt_set_barrier.argtypes = [C.c_void_p, C.c_int32, dp, C.c_double]
    L.rt_destroy.restype = None
    L.rt_destroy.argtypes = [C.c_void_p]
    L.rt_last_error.restype = C.c_char_p
    L.rt_last_error.argtypes = [C.c_void_p]
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params_struct(p, alloc_cb, dealloc_cb):
    """rt_params from a parameter dict of paper_1311_0182_amd.inputs."""
    return Params(
        int(p["n_ngb"]), int(p["n_tc"]), int(p["n_rc"]), int(p["n_ec"]), int(p["n_freq"]),
        int(p["rr_bin"]), int(p["recomb_mode"]), int(p["isothermal"]), int(p.get("freeze_chem", 0)),
        int(p.get("precision", RT_FP64)), int(p["n_em"]), int(p["max_hops"]), int(p["max_vip_depth"]),
        int(p.get("hop_batch", 0)), float(p["dt"]), float(p["floor_rel"]), float(p["chem_frac"]),
        int(p["seed"]) & 0xFFFFFFFFFFFFFFFF, int(p.get("vip_capacity", 0)),
        int(p.get("record_capacity", 0)), alloc_cb, dealloc_cb, None)


def init_call(handle, params, cfg, stream_ptr):
    """rt_init on a workload dict's arrays; returns the status."""
    keep = [_f64(cfg["sigma"]), _f64(cfg["eps"]), np.ascontiguousarray(cfg["inst_off"], dtype=np.int64),
            _f64(cfg["box"]), _f64(cfg["pos"]), _f64(cfg["nH"]), _f64(cfg["NH"]), _f64(cfg["xHI"]),
            _f64(cfg["T"])]
    n_inst = int(cfg["inst_off"].shape[0] - 1)
    return load().rt_init(C.byref(handle), C.byref(params), _p(keep[0], C.c_double), _p(keep[1], C.c_double),
                          n_inst, _p(keep[2], C.c_int64), _p(keep[3], C.c_double), _p(keep[4], C.c_double),
                          _p(keep[5], C.c_double), _p(keep[6], C.c_double), _p(keep[7], C.c_double),
                          _p(keep[8], C.c_double), C.c_void_p(stream_ptr))


class Context:
    """One library context built from a workload dict of paper_1311_0182_amd.inputs.

    precision: "fp64" or "fp32" (overrides the workload's); extra keyword
    arguments override rt_params fields."""

    def __init__(self, cfg, precision=None, torch_alloc=True, add_sources=True, **overrides):
        import torch  # device memory and stream come from PyTorch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the TRAPHIC library runs only on the GPU")
        L = load()
        self._torch = torch
        p = dict(cfg["params"])
        if precision is not None:
            p["precision"] = RT_FP32 if precision in ("fp32", RT_FP32) else RT_FP64
        p.update(overrides)
        self.p = p
        self.N = int(cfg["pos"].shape[0])
        self.nf = int(p["n_freq"])
        self.G = int(p["n_rc"]) * self.nf
        self.n_inst = int(cfg["inst_off"].shape[0] - 1)
        self._dev = torch.cuda.current_device()
        # a stream of its own (default priority): the library captures graphs on it
        self.stream = torch.cuda.Stream(device=self._dev)
        if torch_alloc:
            dev, strm = self._dev, self.stream

            def _alloc(user, nbytes):
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)

            def _dealloc(user, ptr):
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:       # interpreter shutdown: the allocator is gone
                    pass

            self._alloc_cb = ALLOC_FN(_alloc)
            self._dealloc_cb = DEALLOC_FN(_dealloc)
        else:
            self._alloc_cb = ALLOC_FN()
            self._dealloc_cb = DEALLOC_FN()
        self._params = params_struct(p, self._alloc_cb, self._dealloc_cb)
        h = C.c_void_p()
        st = init_call(h, self._params, cfg, self.stream.cuda_stream)
        if st != RT_OK:
            raise RTError(st, "rt_init failed")
        self.h = h
        if add_sources and cfg.get("sources") is not None:
            self.add_sources(cfg["sources"])
        if cfg.get("barrier") is not None:
            b = cfg["barrier"]
            self.set_barrier(b["inst"], b["center"], b["radius"])

    def _check(self, st, allow=()):
        if st != RT_OK and st not in allow:
            raise RTError(st, load().rt_last_error(self.h).decode())
        return st

    def add_sources(self, s):
        inst = np.ascontiguousarray(s["inst"], dtype=np.int32)
        kind = np.ascontiguousarray(s["kind"], dtype=np.int32)
        pos = _f64(s["pos"])
        rate = _f64(s["rate"])
        ns = np.ascontiguousarray(s["n_side"], dtype=np.int32)
        return self._check(load().rt_add_sources(self.h, len(inst), _p(inst, C.c_int32), _p(kind, C.c_int32),
                                                 _p(pos, C.c_double), _p(rate, C.c_double), _p(ns, C.c_int32)))

    def set_barrier(self, inst, center, radius):
        c = _f64(np.asarray(center, dtype=np.float64).reshape(3))
        return self._check(load().rt_set_barrier(self.h, int(inst), _p(c, C.c_double), float(radius)))

    def step(self, n=1, allow=(RT_EHOPCAP,)):
        return self._check(load().rt_step(self.h, int(n)), allow)

    def state(self):
        N, nf = self.N, self.nf
        x, T = np.empty(N), np.empty(N)
        A, P = np.empty(N * nf), np.empty(N * nf)
        led = np.empty(self.n_inst * nf * 5)
        cnt = np.empty(4, dtype=np.int64)
        self._check(load().rt_get_state(self.h, _p(x, C.c_double), _p(T, C.c_double), _p(A, C.c_double),
                                        _p(P, C.c_double), _p(led, C.c_double), _p(cnt, C.c_int64)))
        return dict(xHI=x, T=T, A=A.reshape(N, nf), P=P.reshape(N, nf),
                    ledger=led.reshape(self.n_inst, nf, 5), counters=cnt)

    def bins(self):
        B = self.N * self.G
        Nb, d, c = np.empty(B), np.empty(3 * B), np.empty(B)
        self._check(load().rt_get_bins(self.h, _p(Nb, C.c_double), _p(d, C.c_double), _p(c, C.c_double)))
        return Nb, d.reshape(B, 3), c

    def neighbours(self):
        k = int(self.p["n_ngb"])
        nb = np.empty(self.N * k, dtype=np.int32)
        h = np.empty(self.N)
        self._check(load().rt_get_neighbours(self.h, _p(nb, C.c_int32), _p(h, C.c_double)))
        return nb.reshape(self.N, k), h

    def emitter_neighbours(self):
        k = int(self.p["n_ngb"])
        m = int(load().rt_n_emitters(self.h))
        nb = np.empty(max(m, 1) * k, dtype=np.int32)
        h = np.empty(max(m, 1))
        self._check(load().rt_get_emitter_neighbours(self.h, _p(nb, C.c_int32), _p(h, C.c_double)))
        return nb[: m * k].reshape(m, k), h[:m]

    def cone_masks(self):
        m = np.empty(self.N * self.G, dtype=np.uint64)
        self._check(load().rt_get_cone_masks(self.h, _p(m, C.c_uint64)))
        return m

    def pending_rr(self):
        a = np.empty(self.N)
        self._check(load().rt_get_pending_rr(self.h, _p(a, C.c_double)))
        return a

    def set_timing(self, on=True):
        self._check(load().rt_set_timing(self.h, 1 if on else 0))

    def timing(self):
        out = np.zeros(9)
        self._check(load().rt_get_timing(self.h, _p(out, C.c_double), 9))
        keys = ["hop_ms", "hop_launches", "vip_ms", "chem_ms", "emit_ms", "ledger_ms", "hop_bytes_total",
                "hop_tiles_total", "dense_bytes_per_hop"]
        return {k: float(out[i]) for i, k in enumerate(keys)}

    def set_step_graphs(self, on=True):
        self._check(load().rt_set_step_graphs(self.h, 1 if on else 0))

    def set_hop_shape(self, shape=-1):
        self._check(load().rt_set_hop_shape(self.h, int(shape)))

    def hop_shape(self):
        sh, tu = C.c_int32(0), C.c_int32(0)
        ms = np.zeros(6)
        self._check(load().rt_get_hop_shape(self.h, C.byref(sh), C.byref(tu), _p(ms, C.c_double)))
        return dict(shape=int(sh.value), tuned=bool(tu.value), ms_per_launch=[float(x) for x in ms])

    def shell_profile(self, center, r_max, n_shells, axis=None, half_height=0.0, mean=False, norm=1.0,
                      inst=0, passing=None):
        """rt_shell_profile: (prof[n_shells, n_freq], count[n_shells])."""
        L = load()
        c = _f64(np.asarray(center).reshape(3))
        ap = None
        if axis is not None:
            a = _f64(np.asarray(axis).reshape(3))
            ap = _p(a, C.c_double)
        pp = None
        if passing is not None:
            ps = _f64(passing)
            if ps.size != self.N * self.nf:
                raise ValueError("passing must hold N * n_freq values")
            pp = _p(ps, C.c_double)
        prof = np.empty((int(n_shells), self.nf))
        cnt = np.empty(int(n_shells), dtype=np.int64)
        self._check(L.rt_shell_profile(self.h, int(inst), pp, _p(c, C.c_double), ap, float(half_height),
                                       float(r_max), int(n_shells), int(bool(mean)), float(norm),
                                       _p(prof, C.c_double), _p(cnt, C.c_int64)))
        return prof, cnt

    def shell_profile_noalloc(self, center, r_max, n_shells, axis=None, half_height=0.0, mean=False, norm=1.0,
                              inst=0, passing_dev=None):
        """rt_shell_profile_noalloc: passing_dev is None or a CUDA tensor of N * n_freq
        float64 values (device memory); returns (prof[n_shells, n_freq], count[n_shells])."""
        L = load()
        c = _f64(np.asarray(center).reshape(3))
        ap = None
        if axis is not None:
            a = _f64(np.asarray(axis).reshape(3))
            ap = _p(a, C.c_double)
        dptr = None
        if passing_dev is not None:
            if passing_dev.numel() != self.N * self.nf or not passing_dev.is_contiguous():
                raise ValueError("passing_dev must be a contiguous tensor of N * n_freq values")
            dptr = C.c_void_p(passing_dev.data_ptr())
        prof = np.empty((int(n_shells), self.nf))
        cnt = np.empty(int(n_shells), dtype=np.int64)
        self._check(L.rt_shell_profile_noalloc(self.h, int(inst), dptr, _p(c, C.c_double), ap, float(half_height),
                                               float(r_max), int(n_shells), int(bool(mean)), float(norm),
                                               _p(prof, C.c_double), _p(cnt, C.c_int64)))
        return prof, cnt

    def get_blob(self):
        n = C.c_size_t(0)
        self._check(load().rt_get_state_blob(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check(load().rt_get_state_blob(self.h, buf, C.byref(n)))
        return bytes(buf)

    def set_blob(self, blob):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(load().rt_set_state_blob(self.h, buf, len(blob)))

    def close(self):
        if getattr(self, "h", None):
            load().rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
