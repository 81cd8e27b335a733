"""ctypes binding of libnbs (include/nbs.h): argument marshalling only.

Every compute step runs in the HIP kernels of libnbs.so; if the library is
missing the import fails loudly (there is no host fallback).
"""
from __future__ import annotations

import ctypes
import os

from .channels import OPS

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libnbs.so")

NBS_FP64 = 0
NBS_FP32_MFMA = 1
STATUS = {0: "NBS_OK", 1: "NBS_ERR_INVALID", 2: "NBS_ERR_UNSUPPORTED", 3: "NBS_ERR_NOMEM",
          4: "NBS_ERR_DEVICE", 5: "NBS_ERR_STATE"}

# Every symbol include/nbs.h declares.
SYMBOLS = ("nbs_plan_create", "nbs_workspace_bytes", "nbs_build_blocks", "nbs_contract_channels",
           "nbs_relative_sum", "nbs_plan_destroy", "nbs_status_string", "nbs_last_error",
           "nbs_plan_info", "nbs_plan_diagrams", "nbs_plan_table", "nbs_plan_params", "nbs_run_graph",
           "nbs_plan_autotune", "nbs_plan_tuning", "nbs_plan_set_tuning", "nbs_two_point",
           "nbs_four_point_static", "nbs_static_last_error", "nbs_plan_nonfinite")


class NbsError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__("%s%s" % (STATUS.get(status, status), (": " + msg) if msg else ""))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 3), ("T", ctypes.c_int32), ("t0", ctypes.c_int32),
                ("t_begin", ctypes.c_int32), ("t_count", ctypes.c_int32)]


class Channel(ctypes.Structure):
    _fields_ = [("sink", ctypes.c_int32 * 2), ("src", ctypes.c_int32 * 2)]


class BaryonPair(ctypes.Structure):
    _fields_ = [("sink", ctypes.c_int32), ("src", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_channels", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("n_diagrams", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("n_products", ctypes.c_int32), ("sum_k", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("n_terms", ctypes.c_int64),
                ("n_wick_perms", ctypes.c_int64)]


class Diagram(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_int32), ("src_term", ctypes.c_int32),
                ("set1_mask", ctypes.c_int32), ("sign", ctypes.c_int32), ("k", ctypes.c_int32),
                ("labels1", ctypes.c_int32), ("open_mask", ctypes.c_int32), ("coef", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libnbs.so is not built (%s); run __graft_entry__.build()" % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        P, I32 = ctypes.c_void_p, ctypes.c_int32
        L.nbs_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Geometry), I32,
                                      ctypes.POINTER(Channel), I32, I32, I32]
        L.nbs_plan_create.restype = I32
        L.nbs_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.nbs_workspace_bytes.restype = I32
        L.nbs_build_blocks.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P]
        L.nbs_build_blocks.restype = I32
        L.nbs_contract_channels.argtypes = [P, P]
        L.nbs_contract_channels.restype = I32
        L.nbs_relative_sum.argtypes = [P, ctypes.POINTER(P), P]
        L.nbs_relative_sum.restype = I32
        L.nbs_plan_destroy.argtypes = [P]
        L.nbs_plan_destroy.restype = I32
        L.nbs_status_string.argtypes = [I32]
        L.nbs_status_string.restype = ctypes.c_char_p
        L.nbs_last_error.argtypes = [P]
        L.nbs_last_error.restype = ctypes.c_char_p
        L.nbs_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
        L.nbs_plan_info.restype = I32
        L.nbs_plan_diagrams.argtypes = [P, I32, ctypes.POINTER(Diagram), I32, ctypes.POINTER(I32)]
        L.nbs_plan_diagrams.restype = I32
        L.nbs_plan_table.argtypes = [P, ctypes.c_char_p, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.nbs_plan_table.restype = I32
        L.nbs_plan_params.argtypes = [P, ctypes.POINTER(I32)]
        L.nbs_plan_params.restype = I32
        L.nbs_run_graph.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P]
        L.nbs_run_graph.restype = I32
        L.nbs_plan_autotune.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P]
        L.nbs_plan_autotune.restype = I32
        L.nbs_two_point.argtypes = [P, ctypes.POINTER(BaryonPair), I32, ctypes.POINTER(P), P]
        L.nbs_two_point.restype = I32
        L.nbs_plan_tuning.argtypes = [P, ctypes.POINTER(I32)]
        L.nbs_plan_tuning.restype = I32
        L.nbs_plan_set_tuning.argtypes = [P, ctypes.POINTER(I32)]
        L.nbs_plan_set_tuning.restype = I32
        L.nbs_plan_nonfinite.argtypes = [P, ctypes.POINTER(I32)]
        L.nbs_plan_nonfinite.restype = I32
        L.nbs_four_point_static.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Channel), I32, I32, P, P, P,
                                            P, P]
        L.nbs_four_point_static.restype = I32
        L.nbs_static_last_error.argtypes = []
        L.nbs_static_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _op(x):
    return OPS[x] if isinstance(x, str) else int(x)


def make_geometry(L, T, t0=0, t_begin=0, t_count=None):
    g = Geometry()
    for k in range(3):
        g.L[k] = int(L[k])
    g.T = int(T)
    g.t0 = int(t0)
    g.t_begin = int(t_begin)
    g.t_count = int(T - t_begin if t_count is None else t_count)
    return g


def make_channels(chans):
    arr = (Channel * len(chans))()
    for i, (b1, b2, b3, b4) in enumerate(chans):
        arr[i].sink[0], arr[i].sink[1] = _op(b1), _op(b2)
        arr[i].src[0], arr[i].src[1] = _op(b3), _op(b4)
    return arr


def four_point_static(L, T, chans, prop_u, prop_d, prop_s, F_out, prec=NBS_FP64, t0=0, t_begin=0, t_count=None,
                      stream=0):
    """nbs_four_point_static: the whole path for one geometry with the
    library's static device workspace (no device allocation); arguments are
    device pointers."""
    g = make_geometry(L, T, t0, t_begin, t_count)
    ch = make_channels(chans)
    st = lib().nbs_four_point_static(ctypes.byref(g), ch, len(chans), int(prec), ctypes.c_void_p(prop_u),
                                     ctypes.c_void_p(prop_d), ctypes.c_void_p(prop_s), ctypes.c_void_p(F_out),
                                     ctypes.c_void_p(stream))
    if st != 0:
        raise NbsError(st, "nbs_four_point_static: %s" % lib().nbs_static_last_error().decode())


def _ptrs(x, n):
    xs = list(x) if isinstance(x, (list, tuple)) else [x]
    if len(xs) != n:
        raise ValueError("expected %d pointers, got %d" % (n, len(xs)))
    return (ctypes.c_void_p * n)(*xs)


class Plan:
    """Owner of an nbs_plan handle.  One geometry from (L, T, t0, t_begin,
    t_count), or several (the batching form) from geoms: a list of dicts
    with keys L, T and optionally t0, t_begin, t_count."""

    def __init__(self, L, T, chans, prec=NBS_FP64, device=0, t0=0, t_begin=0, t_count=None, geoms=None):
        self._h = ctypes.c_void_p()
        if geoms is None:
            geoms = [dict(L=L, T=T, t0=t0, t_begin=t_begin, t_count=t_count)]
        self.geoms = (Geometry * len(geoms))()
        for i, g in enumerate(geoms):
            self.geoms[i] = make_geometry(g["L"], g["T"], g.get("t0", 0), g.get("t_begin", 0), g.get("t_count"))
        self.geom = self.geoms[0]
        self.n_geom = len(geoms)
        self.chans = list(chans)
        self._ch = make_channels(self.chans)
        st = lib().nbs_plan_create(ctypes.byref(self._h), self.geoms, self.n_geom, self._ch,
                                   len(self.chans), int(prec), int(device))
        if st != 0:
            raise NbsError(st, "nbs_plan_create")
        self.prec = prec

    def _check(self, st, what):
        if st != 0:
            raise NbsError(st, "%s: %s" % (what, lib().nbs_last_error(self._h).decode()))

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self):
        n = ctypes.c_size_t()
        self._check(lib().nbs_workspace_bytes(self._h, ctypes.byref(n)), "nbs_workspace_bytes")
        return n.value

    def build_blocks(self, prop_u, prop_d, prop_s, stream=0):
        """Pointers (or, for several geometries, lists of pointers)."""
        n = self.n_geom
        self._check(lib().nbs_build_blocks(self._h, _ptrs(prop_u, n), _ptrs(prop_d, n), _ptrs(prop_s, n),
                                           ctypes.c_void_p(stream)), "nbs_build_blocks")

    def contract_channels(self, stream=0):
        self._check(lib().nbs_contract_channels(self._h, ctypes.c_void_p(stream)), "nbs_contract_channels")

    def two_point(self, pairs, C_out, stream=0):
        """Zero-momentum single-baryon two-point functions of (sink, source)
        operator pairs into C_out (one device pointer per geometry)."""
        arr = (BaryonPair * max(1, len(pairs)))()
        for i, (a, b) in enumerate(pairs):
            arr[i].sink, arr[i].src = _op(a), _op(b)
        self._check(lib().nbs_two_point(self._h, arr, len(pairs), _ptrs(C_out, self.n_geom), ctypes.c_void_p(stream)),
                    "nbs_two_point")

    def relative_sum(self, F_out, stream=0):
        self._check(lib().nbs_relative_sum(self._h, _ptrs(F_out, self.n_geom), ctypes.c_void_p(stream)),
                    "nbs_relative_sum")

    def run_graph(self, prop_u, prop_d, prop_s, F_out, stream=0):
        n = self.n_geom
        self._check(lib().nbs_run_graph(self._h, _ptrs(prop_u, n), _ptrs(prop_d, n), _ptrs(prop_s, n),
                                        _ptrs(F_out, n), ctypes.c_void_p(stream)), "nbs_run_graph")

    def autotune(self, prop_u, prop_d, prop_s, stream=0):
        n = self.n_geom
        self._check(lib().nbs_plan_autotune(self._h, _ptrs(prop_u, n), _ptrs(prop_d, n), _ptrs(prop_s, n),
                                            ctypes.c_void_p(stream)), "nbs_plan_autotune")

    def nonfinite(self):
        """True if the last build's propagators held a NaN or infinite entry."""
        f = ctypes.c_int32(0)
        self._check(lib().nbs_plan_nonfinite(self._h, ctypes.byref(f)), "nbs_plan_nonfinite")
        return bool(f.value)

    def tuning(self):
        out = (ctypes.c_int32 * 4)()
        self._check(lib().nbs_plan_tuning(self._h, out), "nbs_plan_tuning")
        return {"fft_line": out[0] & 1, "fft_plane": (out[0] >> 1) & 1, "fft_cube": (out[0] >> 2) & 1,
                "fft_tile": out[1], "waves": out[2],
                "split": out[3] & 1, "mfma": (out[3] >> 1) & 1, "gchunk": (out[3] >> 2) & 3,
                "engine": (out[3] >> 4) & 1, "persist": (out[3] >> 5) & 1}

    def set_tuning(self, **kw):
        """Change some launch shapes (keys as returned by tuning())."""
        t = self.tuning()
        t.update(kw)
        arr = (ctypes.c_int32 * 4)(int(t["fft_line"]) | (int(t["fft_plane"]) << 1) | (int(t["fft_cube"]) << 2),
                                   int(t["fft_tile"]),
                                   int(t["waves"]),
                                   int(t["split"]) | (int(t["mfma"]) << 1) | (int(t["gchunk"]) << 2)
                                   | (int(t["engine"]) << 4) | (int(t["persist"]) << 5))
        self._check(lib().nbs_plan_set_tuning(self._h, arr), "nbs_plan_set_tuning")

    def info(self):
        inf = PlanInfo()
        self._check(lib().nbs_plan_info(self._h, ctypes.byref(inf)), "nbs_plan_info")
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def diagrams(self, ch=-1):
        n = ctypes.c_int32()
        self._check(lib().nbs_plan_diagrams(self._h, ch, None, 0, ctypes.byref(n)), "nbs_plan_diagrams")
        arr = (Diagram * max(1, n.value))()
        self._check(lib().nbs_plan_diagrams(self._h, ch, arr, n.value, ctypes.byref(n)), "nbs_plan_diagrams")
        return [{k: getattr(arr[i], k) for k, _ in Diagram._fields_} for i in range(n.value)]

    def table(self, name):
        """One table of the compiled SoA program as a numpy array."""
        import numpy as np
        n = ctypes.c_int64()
        self._check(lib().nbs_plan_table(self._h, name.encode(), None, 0, ctypes.byref(n)), "nbs_plan_table")
        dbl = ("contrib_coef", "op_term_w", "op_alias_coef", "contrib_coef_iso")
        arr = np.zeros(max(1, n.value), dtype=np.float64 if name in dbl else np.int32)
        self._check(lib().nbs_plan_table(self._h, name.encode(), arr.ctypes.data_as(ctypes.c_void_p), n.value,
                                         ctypes.byref(n)), "nbs_plan_table")
        return arr[:n.value]

    def params(self):
        out = (ctypes.c_int32 * 4)()
        self._check(lib().nbs_plan_params(self._h, out), "nbs_plan_params")
        return {"prod_ints": out[0], "lanes_per_task": out[1], "max_group_products": out[2],
                "max_group_channels": out[3]}

    def close(self):
        if self._h:
            lib().nbs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
