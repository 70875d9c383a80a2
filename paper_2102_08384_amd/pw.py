"""Thin ctypes binding of libpw (argument marshalling only; every step runs in libpw's kernels).

The library must be built in-tree (``python -m paper_2102_08384_amd.build``); importing this
module raises if ``libpw.so`` is missing.  Catalog arrays may be numpy arrays (host memory)
or torch tensors on the context's GPU (device memory), shaped [n, 4] = (x, y, z, w).
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PW_LIB names another build of the library (the host-only sanitized one, for CPU checks)
LIB_PATH = os.environ.get("PW_LIB") or os.path.join(HERE, "libpw.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pw.h")

PW_OK, PW_EINVAL, PW_ERANGE, PW_ENOMEM, PW_EDEVICE, PW_EBUSY, PW_EAGAIN, PW_ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
PW_PK, PW_XI = 0, 1
PW_MIDPOINT, PW_BISECTOR = 0, 1
PW_CIC, PW_TSC = 2, 3
PW_FP32, PW_FP64 = 0, 1
PW_PARITY_EVEN, PW_PARITY_ALL = 0, 1

_ERRNAMES = {PW_EINVAL: "PW_EINVAL", PW_ERANGE: "PW_ERANGE", PW_ENOMEM: "PW_ENOMEM",
             PW_EDEVICE: "PW_EDEVICE", PW_EBUSY: "PW_EBUSY", PW_EAGAIN: "PW_EAGAIN",
             PW_ECANCELED: "PW_ECANCELED"}


class PwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _Config(C.Structure):
    _fields_ = [("stat", C.c_int), ("los", C.c_int), ("assign", C.c_int), ("prec", C.c_int),
                ("n_mesh", C.c_int), ("box_len", C.c_double), ("box_origin", C.c_double * 3),
                ("ell_max", C.c_int), ("order", C.c_int), ("compensate", C.c_int),
                ("bin_lo", C.c_double), ("bin_width", C.c_double), ("n_bins", C.c_int),
                ("midpoint_parity", C.c_int), ("memory_lean", C.c_int)]


class _Catalog(C.Structure):
    _fields_ = [("xyzw", C.c_void_p), ("nbar", C.c_void_p), ("n", C.c_int64),
                ("dtype", C.c_int), ("on_device", C.c_int)]


class _Norm(C.Structure):
    _fields_ = [("alpha_r", C.c_double), ("I", C.c_double), ("S", C.c_double), ("use_given", C.c_int)]


def _load():
    # One HIP runtime per process: PyTorch-ROCm ships its own libamdhip64 (same soname as the
    # system one libpw links).  Loading torch first makes libpw bind to that same runtime; loading
    # libpw first would make torch load a second runtime, which then finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpw.so not built at {LIB_PATH}; run python -m paper_2102_08384_amd.build")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.pw_create.argtypes = [C.POINTER(P), C.c_int, C.c_size_t, P]
    lib.pw_destroy.argtypes = [P]
    lib.pw_estimate.argtypes = [P, C.POINTER(_Config), C.POINTER(_Catalog), C.POINTER(_Catalog),
                                C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_int64)]
    lib.pw_estimate_batch.argtypes = [P, C.POINTER(_Config), C.c_int, C.POINTER(_Catalog), C.POINTER(_Catalog),
                                      C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]
    lib.pw_serving_stats.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.pw_estimate_noalloc.argtypes = [P, C.POINTER(_Config), C.POINTER(_Catalog), C.POINTER(_Catalog),
                                        C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int64)]
    lib.pw_estimate_orders.argtypes = [P, C.POINTER(_Config), C.POINTER(_Catalog), C.POINTER(_Catalog),
                                       C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64)]
    lib.pw_estimate_xi_normalized.argtypes = [P, C.POINTER(_Config), C.POINTER(_Catalog), C.POINTER(_Catalog),
                                              C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                              C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_double),
                                              C.POINTER(C.c_int64)]
    lib.pw_submit.argtypes = [P, C.POINTER(_Config), C.POINTER(_Catalog), C.POINTER(_Catalog),
                              C.POINTER(_Norm), C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]
    lib.pw_poll.argtypes = [P, C.c_uint64]
    lib.pw_wait.argtypes = [P, C.c_uint64]
    lib.pw_cancel.argtypes = [P, C.c_uint64]
    lib.pw_set_lanes.argtypes = [P, C.c_int]
    lib.pw_set_queue_limit.argtypes = [P, C.c_int64]
    lib.pw_inspect.argtypes = [P, C.c_int, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.pw_set_timing.argtypes = [P, C.c_int]
    lib.pw_set_tuning.argtypes = [P, C.c_int]
    lib.pw_tune_entry.argtypes = [C.c_int, C.c_char_p, C.c_size_t, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    lib.pw_stage_info.argtypes = [P, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    lib.pw_last_error.argtypes = [P]
    lib.pw_last_error.restype = C.c_char_p
    lib.pw_footprint.argtypes = [C.POINTER(_Config), C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
    lib.pw_coupling_table.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                      C.c_int64, C.POINTER(C.c_int64)]
    return lib


_lib = _load()


def declared_symbols():
    """Names of every function declared in include/pw.h."""
    with open(HEADER) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(pw_[a-z_]+)\s*\(", txt, re.M)))


@dataclass
class Config:
    stat: int = PW_PK
    los: int = PW_BISECTOR
    assign: int = PW_TSC
    prec: int = PW_FP32
    n_mesh: int = 64
    box_len: float = 1000.0
    box_origin: tuple = (-500.0, -500.0, 500.0)
    ell_max: int = 4
    order: int = 4
    compensate: int = 1
    bin_lo: float = 0.01
    bin_width: float = 0.01
    n_bins: int = 20
    midpoint_parity: int = PW_PARITY_EVEN
    memory_lean: int = 0

    def _c(self):
        c = _Config()
        c.stat, c.los, c.assign, c.prec = self.stat, self.los, self.assign, self.prec
        c.n_mesh = self.n_mesh
        c.box_len = float(self.box_len)
        for i in range(3):
            c.box_origin[i] = float(self.box_origin[i])
        c.ell_max, c.order, c.compensate = self.ell_max, self.order, int(self.compensate)
        c.bin_lo, c.bin_width, c.n_bins = float(self.bin_lo), float(self.bin_width), self.n_bins
        c.midpoint_parity = int(self.midpoint_parity)
        c.memory_lean = int(self.memory_lean)
        return c

    @property
    def n_ell(self):
        return self.ell_max // 2 + 1


def _catalog(xyzw, nbar, keep):
    """Describe a catalog; keep references alive in `keep`."""
    cat = _Catalog()
    try:
        import torch
        is_torch = hasattr(xyzw, "data_ptr") and hasattr(xyzw, "is_cuda")
    except ImportError:
        is_torch = False
    if is_torch:
        t = xyzw.contiguous()
        if t.dim() != 2 or t.shape[1] != 4:
            raise ValueError("xyzw must be [n, 4]")
        keep.append(t)
        cat.xyzw = t.data_ptr() if t.numel() else None
        cat.n = t.shape[0]
        cat.dtype = PW_FP64 if str(t.dtype) == "torch.float64" else PW_FP32
        if str(t.dtype) not in ("torch.float32", "torch.float64"):
            raise ValueError("xyzw must be float32 or float64")
        cat.on_device = 1 if t.is_cuda else 0
        if nbar is not None:
            nb = nbar.to(dtype=t.dtype, device=t.device).contiguous()
            keep.append(nb)
            cat.nbar = nb.data_ptr()
        if t.is_cuda:
            # the library reads device inputs on its own streams: the copies and casts above
            # (and whatever produced the tensors) must be complete first
            torch.cuda.current_stream(t.device).synchronize()
        return cat
    a = np.ascontiguousarray(xyzw)
    if a.ndim != 2 or a.shape[1] != 4:
        raise ValueError("xyzw must be [n, 4]")
    if a.dtype not in (np.float32, np.float64):
        raise ValueError("xyzw must be float32 or float64")
    keep.append(a)
    cat.xyzw = a.ctypes.data if a.size else None
    cat.n = a.shape[0]
    cat.dtype = PW_FP64 if a.dtype == np.float64 else PW_FP32
    cat.on_device = 0
    if nbar is not None:
        nb = np.ascontiguousarray(nbar, dtype=a.dtype)
        keep.append(nb)
        cat.nbar = nb.ctypes.data
    return cat


class Context:
    """A libpw context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        self._h = C.c_void_p()
        rc = _lib.pw_create(C.byref(self._h), device, hbm_budget,
                            C.c_void_p(stream) if stream else None)
        if rc != PW_OK:
            raise PwError(rc, "pw_create failed")

    def close(self):
        if self._h:
            _lib.pw_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self):
        return _lib.pw_last_error(self._h).decode()

    def set_timing(self, on: bool):
        _lib.pw_set_timing(self._h, 1 if on else 0)

    def set_tuning(self, mode: int):
        """Launch shapes of the column passes: 1 autotuned (default), 0 defaults, 2 + i candidate i."""
        rc = _lib.pw_set_tuning(self._h, int(mode))
        if rc != PW_OK:
            raise PwError(rc, "pw_set_tuning: mode must be >= 0")

    def stages(self):
        """[(name, ms, algorithmic_bytes)] of the most recent estimate."""
        out = []
        i = 0
        while True:
            nm, ms, by = C.c_char_p(), C.c_double(), C.c_double()
            if _lib.pw_stage_info(self._h, i, C.byref(nm), C.byref(ms), C.byref(by)) != PW_OK:
                break
            out.append((nm.value.decode(), ms.value, by.value))
            i += 1
        return out

    def inspect(self, what: int, dtype=np.float32):
        """Copy an internal buffer of the last estimate (see pw_inspect in pw.h)."""
        need = C.c_size_t()
        rc = _lib.pw_inspect(self._h, what, None, 0, C.byref(need))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        out = np.empty(need.value, dtype=np.uint8)
        rc = _lib.pw_inspect(self._h, what, out.ctypes.data, need.value, C.byref(need))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        if what == 2:
            return out.view(np.uint32)
        return out.view(dtype)

    def estimate(self, cfg: Config, gal_xyzw, ran_xyzw, ran_nbar=None, norm=None):
        """Run one estimate.  norm = (alpha_r, I, S) to impose the normalisation."""
        return self._run(_lib.pw_estimate, (cfg.n_ell, cfg.n_bins), cfg, gal_xyzw, ran_xyzw, ran_nbar, norm)

    def estimate_batch(self, cfg: Config, cats):
        """pw_estimate_batch over cats = [(gal_xyzw, ran_xyzw, ran_nbar), ...] of one configuration;
        returns one result dict per catalog."""
        keep = []
        n = len(cats)
        gals = (_Catalog * n)()
        rans = (_Catalog * n)()
        for i, (g, r, nb) in enumerate(cats):
            gals[i] = _catalog(g, None, keep)
            rans[i] = _catalog(r, nb, keep)
        norms = (_Norm * n)()
        out = np.zeros((n, cfg.n_ell, cfg.n_bins))
        bm = np.zeros((n, cfg.n_bins))
        cnt = np.zeros((n, cfg.n_bins), dtype=np.int64)
        c = cfg._c()
        rc = _lib.pw_estimate_batch(self._h, C.byref(c), n, gals, rans, norms,
                                    out.ctypes.data_as(C.POINTER(C.c_double)),
                                    bm.ctypes.data_as(C.POINTER(C.c_double)),
                                    cnt.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        return [{"values": out[i], "bin_mean": bm[i], "counts": cnt[i],
                 "norm": (norms[i].alpha_r, norms[i].I, norms[i].S)} for i in range(n)]

    def serving_stats(self):
        """(launches, requests) of the serving loop so far."""
        a, b = C.c_uint64(), C.c_uint64()
        rc = _lib.pw_serving_stats(self._h, C.byref(a), C.byref(b))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        return a.value, b.value

    def estimate_noalloc(self, cfg: Config, gal_xyzw, ran_xyzw, ran_nbar=None, norm=None):
        """pw_estimate_noalloc: the estimate in the library's static device scratch (device
        tensors only; small configurations)."""
        return self._run(_lib.pw_estimate_noalloc, (cfg.n_ell, cfg.n_bins), cfg, gal_xyzw, ran_xyzw,
                         ran_nbar, norm)

    def estimate_orders(self, cfg: Config, gal_xyzw, ran_xyzw, ran_nbar=None, norm=None):
        """Each series order's contribution: values[o] holds the terms of order theta^(2o)
        (pw_estimate_orders); shape [order/2 + 1, n_ell, n_bins]."""
        step = 1 if (cfg.los == PW_MIDPOINT and cfg.midpoint_parity == PW_PARITY_ALL) else 2
        return self._run(_lib.pw_estimate_orders, (cfg.order // step + 1, cfg.n_ell, cfg.n_bins), cfg,
                         gal_xyzw, ran_xyzw, ran_nbar, norm)

    def estimate_xi_normalized(self, cfg: Config, gal_xyzw, ran_xyzw, ran_nbar=None, norm=None):
        """xi_l over the bins' random-pair counts (xi_rr), window-corrected (xi_edge), and the
        window multipoles f_L = R_L / R_0 (pw_estimate_xi_normalized)."""
        keep = []
        g = _catalog(gal_xyzw, None, keep)
        r = _catalog(ran_xyzw, ran_nbar, keep)
        nm = _Norm()
        if norm is not None:
            nm.alpha_r, nm.I, nm.S = (float(v) for v in norm)
            nm.use_given = 1
        rr = np.zeros((cfg.n_ell, cfg.n_bins))
        edge = np.zeros((cfg.n_ell, cfg.n_bins))
        win = np.zeros((5, cfg.n_bins))
        nw = C.c_int(0)
        bm = np.zeros(cfg.n_bins)
        cnt = np.zeros(cfg.n_bins, dtype=np.int64)
        c = cfg._c()
        dp = C.POINTER(C.c_double)
        rc = _lib.pw_estimate_xi_normalized(self._h, C.byref(c), C.byref(g), C.byref(r), C.byref(nm),
                                            rr.ctypes.data_as(dp), edge.ctypes.data_as(dp), win.ctypes.data_as(dp),
                                            C.byref(nw), bm.ctypes.data_as(dp),
                                            cnt.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        return {"xi_rr": rr, "xi_edge": edge, "window": win[:nw.value], "bin_mean": bm, "counts": cnt,
                "norm": (nm.alpha_r, nm.I, nm.S)}

    def _run(self, fn, shape, cfg, gal_xyzw, ran_xyzw, ran_nbar, norm):
        keep = []
        g = _catalog(gal_xyzw, None, keep)
        r = _catalog(ran_xyzw, ran_nbar, keep)
        nm = _Norm()
        if norm is not None:
            nm.alpha_r, nm.I, nm.S = (float(v) for v in norm)
            nm.use_given = 1
        out = np.zeros(shape)
        bm = np.zeros(cfg.n_bins)
        cnt = np.zeros(cfg.n_bins, dtype=np.int64)
        c = cfg._c()
        rc = fn(self._h, C.byref(c), C.byref(g), C.byref(r), C.byref(nm),
                out.ctypes.data_as(C.POINTER(C.c_double)),
                bm.ctypes.data_as(C.POINTER(C.c_double)),
                cnt.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        return {"values": out, "bin_mean": bm, "counts": cnt, "norm": (nm.alpha_r, nm.I, nm.S)}


    # ---------------------------------------------------------------- serving
    def set_lanes(self, n: int):
        rc = _lib.pw_set_lanes(self._h, n)
        if rc != PW_OK:
            raise PwError(rc, self.last_error())

    def set_queue_limit(self, n: int):
        """pw_submit raises PwError(PW_EBUSY) while n requests are pending or running."""
        rc = _lib.pw_set_queue_limit(self._h, int(n))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())

    def submit(self, cfg: Config, gal_xyzw, ran_xyzw, ran_nbar=None, norm=None):
        """Enqueue an estimate; returns a Ticket (inputs are kept alive by it)."""
        t = Ticket(self, cfg)
        g = _catalog(gal_xyzw, None, t._keep)
        r = _catalog(ran_xyzw, ran_nbar, t._keep)
        t._cats = (g, r)
        if norm is not None:
            t._norm.alpha_r, t._norm.I, t._norm.S = (float(v) for v in norm)
            t._norm.use_given = 1
        t._cfg_c = cfg._c()
        tk = C.c_uint64()
        rc = _lib.pw_submit(self._h, C.byref(t._cfg_c), C.byref(g), C.byref(r), C.byref(t._norm),
                            t.out.ctypes.data_as(C.POINTER(C.c_double)),
                            t.bin_mean.ctypes.data_as(C.POINTER(C.c_double)),
                            t.counts.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(tk))
        if rc != PW_OK:
            raise PwError(rc, self.last_error())
        t.id = tk.value
        return t


class Ticket:
    """A submitted request: its result buffers and the inputs they depend on."""

    def __init__(self, ctx: Context, cfg: Config):
        self._ctx = ctx
        self._keep = []
        self._norm = _Norm()
        self.id = 0
        self.status = PW_EAGAIN
        self.out = np.zeros((cfg.n_ell, cfg.n_bins))
        self.bin_mean = np.zeros(cfg.n_bins)
        self.counts = np.zeros(cfg.n_bins, dtype=np.int64)

    def __del__(self):
        # The worker writes a request's outputs into this ticket's arrays and reads its inputs
        # until the request is final: a ticket dropped while pending (an exception, interpreter
        # shutdown) waits for that before its buffers go.  After pw_destroy nothing is written.
        try:
            if self.status == PW_EAGAIN and self.id and self._ctx._h:
                _lib.pw_wait(self._ctx._h, self.id)
        except Exception:
            pass

    def _final(self, rc):
        self.status = rc
        if rc == PW_OK:
            self._keep = []
            return {"values": self.out, "bin_mean": self.bin_mean, "counts": self.counts,
                    "norm": (self._norm.alpha_r, self._norm.I, self._norm.S)}
        raise PwError(rc, self._ctx.last_error())

    def poll(self):
        """None while pending, else the result dict (raises PwError on failure)."""
        if self.status != PW_EAGAIN:
            return self._final(self.status)
        rc = _lib.pw_poll(self._ctx._h, self.id)
        if rc == PW_EAGAIN:
            return None
        return self._final(rc)

    def wait(self):
        if self.status != PW_EAGAIN:
            return self._final(self.status)
        return self._final(_lib.pw_wait(self._ctx._h, self.id))

    def cancel(self):
        rc = _lib.pw_cancel(self._ctx._h, self.id)
        if rc not in (PW_OK,):
            raise PwError(rc, self._ctx.last_error())


def tune_entries():
    """The process's autotuning table: [{key, choice, ms_best, ms_default}] (pw_tune_entry)."""
    out = []
    buf = C.create_string_buffer(256)
    ch, mb, md = C.c_int(), C.c_double(), C.c_double()
    i = 0
    while _lib.pw_tune_entry(i, buf, len(buf), C.byref(ch), C.byref(mb), C.byref(md)) == PW_OK:
        out.append({"key": buf.value.decode(), "choice": ch.value, "ms_best": mb.value, "ms_default": md.value})
        i += 1
    return out


def footprint(cfg: Config, n_gal: int, n_ran: int) -> int:
    b = C.c_size_t()
    c = cfg._c()
    rc = _lib.pw_footprint(C.byref(c), n_gal, n_ran, C.byref(b))
    if rc != PW_OK:
        raise PwError(rc, "pw_footprint failed")
    return b.value


def coupling_table(kind: int, ell_max: int, order: int, alpha: int = 0) -> np.ndarray:
    n = C.c_int64()
    rc = _lib.pw_coupling_table(kind, ell_max, order, alpha, None, 0, C.byref(n))
    if rc != PW_OK:
        raise PwError(rc, "pw_coupling_table failed")
    rows = np.zeros((n.value, 7))
    rc = _lib.pw_coupling_table(kind, ell_max, order, alpha, rows.ctypes.data_as(C.POINTER(C.c_double)),
                                n.value, C.byref(n))
    if rc != PW_OK:
        raise PwError(rc, "pw_coupling_table failed")
    return rows
