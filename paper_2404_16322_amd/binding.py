"""ctypes binding of include/ddc.h (argument marshalling only; every step runs in libddc.so)."""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LOCK = threading.Lock()

DTYPE = {"f32": 0, "f16": 1, "bf16": 2}
ROT = {"f32": 0, "bf16": 1}
CORR = {"learned": 0, "lossless": 1, "none": 2, "ads": 3, "bsar": 4, "bsao": 5}
PROJ = {"pca": 0, "haar": 1}
EST = {"partial": 0, "residual": 1}
CALIB = {"joint": 0, "bonferroni": 1}
STATUS = {0: "DDC_OK", -1: "DDC_EINVAL", -2: "DDC_ENOMEM", -3: "DDC_EDEVICE", -4: "DDC_EIO",
          -5: "DDC_EBUSY", -6: "DDC_EUNSUP"}

SYMBOLS = ["ddc_fit_params_default", "ddc_fit", "ddc_import", "ddc_export", "ddc_index_get_info",
           "ddc_calibrate", "ddc_correction", "ddc_search", "ddc_search_var", "ddc_search_device",
           "ddc_debug_intermediates", "ddc_set_kernel_timing", "ddc_get_kernel_timing", "ddc_free",
           "ddc_last_error", "ddc_server_create", "ddc_server_submit", "ddc_server_poll",
           "ddc_server_get_stats", "ddc_server_destroy", "ddc_set_launch", "ddc_get_launch",
           "ddc_scan_variant", "ddc_save", "ddc_load", "ddc_set_ads_epsilon", "ddc_set_bsar_multiplier",
           "ddc_search_estimate", "ddc_correction_pq", "ddc_search_device_noalloc",
           "ddc_search_device_noalloc_bytes", "ddc_set_fault", "ddc_live_allocations"]


class FitParams(C.Structure):
    _fields_ = [("nlist", C.c_int32), ("delta_d", C.c_int32), ("block_b", C.c_int32),
                ("lag_l", C.c_int32), ("kmeans_iters", C.c_int32),
                ("kmeans_train_per_list", C.c_int32), ("calib_k", C.c_int32),
                ("calib_nprobe", C.c_int32), ("calib_max_neg", C.c_int32),
                ("calib_k_extra", C.c_int32 * 3), ("storage", C.c_int),
                ("rotation", C.c_int), ("projection", C.c_int), ("fp8_lead_dims", C.c_int32),
                ("pca_sample", C.c_int64),
                ("seed", C.c_uint64), ("pq_m", C.c_int32), ("pq_iters", C.c_int32),
                ("pq_train", C.c_int64)]


class Artifacts(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("nlist", C.c_int32), ("delta_d", C.c_int32),
                ("block_b", C.c_int32), ("lag_l", C.c_int32), ("storage", C.c_int),
                ("rotation", C.c_int), ("fp8_lead_dims", C.c_int32), ("mu", C.c_void_p),
                ("rot", C.c_void_p), ("lam", C.c_void_p), ("centroids", C.c_void_p),
                ("assign", C.c_void_p), ("y", C.c_void_p), ("n_tables", C.c_int32),
                ("table_k", C.c_int32 * 4), ("table_n0", C.c_int64 * 4), ("m", C.c_void_p),
                ("resid", C.c_void_p), ("codes8", C.c_void_p), ("scale8", C.c_void_p),
                ("pq_m", C.c_int32), ("pq_perm", C.c_void_p), ("pq_books", C.c_void_p),
                ("pq_codes", C.c_void_p), ("pq_m1", C.c_void_p), ("pq_m3", C.c_void_p),
                ("pq_resid", C.c_void_p)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("dim_padded", C.c_int32),
                ("nlist", C.c_int32), ("delta_d", C.c_int32), ("n_stages", C.c_int32),
                ("n_test_stages", C.c_int32), ("block_b", C.c_int32), ("lag_l", C.c_int32),
                ("storage", C.c_int), ("rotation", C.c_int), ("n0", C.c_int64),
                ("packed_bytes", C.c_int64), ("total_tiles", C.c_int64), ("fp8_lead_dims", C.c_int32),
                ("n_tables", C.c_int32), ("table_k", C.c_int32 * 4), ("pq_m", C.c_int32),
                ("pq_tables", C.c_int32)]


class SearchStats(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("refined", C.c_int64), ("stage_slices", C.c_int64),
                ("bytes_touched", C.c_int64), ("stage_stop", C.c_int64 * 64),
                ("prestage_reads", C.c_int64), ("prestage_pruned", C.c_int64),
                ("two_phase_sums", C.c_int64), ("two_phase_slices", C.c_int64)]

    def as_dict(self):
        return dict(candidates=self.candidates, refined=self.refined, stage_slices=self.stage_slices,
                    bytes_touched=self.bytes_touched, stage_stop=list(self.stage_stop),
                    prestage_reads=self.prestage_reads, prestage_pruned=self.prestage_pruned,
                    two_phase_sums=self.two_phase_sums, two_phase_slices=self.two_phase_slices)


class ServerParams(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch", C.c_int32), ("hbm_budget_bytes", C.c_int64),
                ("significance", C.c_double), ("mode", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("requests_done", C.c_int64), ("queries_done", C.c_int64), ("rejected", C.c_int64),
                ("qps", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("budget_peak_bytes", C.c_int64), ("max_concurrent", C.c_int32)]


class LaunchParams(C.Structure):
    _fields_ = [("waves_per_query", C.c_int32), ("lookahead", C.c_int32),
                ("query_order", C.c_int32), ("xcd_swizzle", C.c_int32), ("persistent", C.c_int32),
                ("two_phase", C.c_int32), ("full_d_matrix", C.c_int32), ("stage1_matrix", C.c_int32),
                ("waves_per_simd", C.c_int32)]


class DdcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib_path() -> str:
    return os.path.join(_HERE, "libddc.so")


def load_library():
    """Load libddc.so; raises if it is missing (there is no fallback path)."""
    global _LIB
    with _LOCK:
        if _LIB is not None:
            return _LIB
        p = lib_path()
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        lib = C.CDLL(p)
        vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        st = C.c_int
        lib.ddc_last_error.restype = C.c_char_p
        lib.ddc_fit_params_default.argtypes = [C.POINTER(FitParams)]
        lib.ddc_fit.argtypes = [vp, i64, i32, vp, i64, C.POINTER(FitParams), C.POINTER(vp)]
        lib.ddc_import.argtypes = [C.POINTER(Artifacts), C.POINTER(vp)]
        lib.ddc_export.argtypes = [vp, C.POINTER(Artifacts)]
        lib.ddc_index_get_info.argtypes = [vp, C.POINTER(IndexInfo)]
        lib.ddc_calibrate.argtypes = [vp, vp, i64, i32, i32, i32, C.c_uint64]
        lib.ddc_correction.argtypes = [vp, i32, f64, C.c_int, vp, vp]
        lib.ddc_search.argtypes = [vp, vp, i64, i32, i32, f64, C.c_int, vp, vp, C.POINTER(SearchStats)]
        lib.ddc_search_var.argtypes = [vp, vp, i64, vp, vp, f64, C.c_int, vp, vp, vp,
                                       C.POINTER(SearchStats)]
        lib.ddc_search_device.argtypes = [vp, vp, i64, vp, i32, i32, vp, i32, i32, f64, C.c_int, vp,
                                          vp, vp, vp, vp]
        lib.ddc_search_device_noalloc.argtypes = lib.ddc_search_device.argtypes
        lib.ddc_search_device_noalloc_bytes.argtypes = []
        lib.ddc_set_fault.argtypes = [C.c_char_p]
        lib.ddc_live_allocations.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.ddc_debug_intermediates.argtypes = [vp, vp, i64, i32, vp, vp]
        lib.ddc_search_estimate.argtypes = [vp, vp, i64, i32, i32, i32, C.c_int, vp, vp]
        lib.ddc_correction_pq.argtypes = [vp, i32, f64, vp, vp, vp]
        lib.ddc_set_kernel_timing.argtypes = [vp, C.c_int]
        lib.ddc_get_kernel_timing.argtypes = [vp, vp, vp, C.c_int]
        lib.ddc_set_ads_epsilon.argtypes = [vp, f64]
        lib.ddc_set_bsar_multiplier.argtypes = [vp, f64]
        lib.ddc_save.argtypes = [vp, C.c_char_p]
        lib.ddc_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        lib.ddc_set_launch.argtypes = [vp, C.POINTER(LaunchParams)]
        lib.ddc_get_launch.argtypes = [vp, C.POINTER(LaunchParams)]
        lib.ddc_scan_variant.argtypes = [vp, i64, i32, i32, C.c_int, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.ddc_server_create.argtypes = [vp, C.POINTER(ServerParams), C.POINTER(vp)]
        lib.ddc_server_submit.argtypes = [vp, vp, i32, vp, vp, C.POINTER(C.c_uint64)]
        lib.ddc_server_poll.argtypes = [vp, C.c_uint64, vp, vp, C.POINTER(C.c_int), C.POINTER(C.c_uint64)]
        lib.ddc_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        lib.ddc_server_destroy.argtypes = [vp]
        lib.ddc_server_destroy.restype = None
        lib.ddc_free.argtypes = [vp]
        lib.ddc_free.restype = None
        for name in SYMBOLS:
            if name not in ("ddc_free", "ddc_last_error", "ddc_server_destroy",
                            "ddc_search_device_noalloc_bytes"):
                getattr(lib, name).restype = st
        lib.ddc_search_device_noalloc_bytes.restype = C.c_size_t
        _LIB = lib
        return lib


def set_fault(spec: str):
    """Inject an allocation failure ("alloc:<n>": the n-th allocation from now fails; "alloc:0"
    turns it off) -- for tests of the error paths."""
    _check(load_library().ddc_set_fault(spec.encode()))


def live_allocations() -> tuple:
    """(count, device bytes) of the allocations the library holds now."""
    n, b = C.c_int64(), C.c_int64()
    _check(load_library().ddc_live_allocations(C.byref(n), C.byref(b)))
    return n.value, b.value


def _check(rc):
    if rc != 0:
        msg = load_library().ddc_last_error().decode(errors="replace")
        raise DdcError(rc, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def default_params(**kw) -> FitParams:
    p = FitParams()
    _check(load_library().ddc_fit_params_default(C.byref(p)))
    for k, v in kw.items():
        if k == "storage":
            v = DTYPE[v] if isinstance(v, str) else v
        if k == "rotation":
            v = ROT[v] if isinstance(v, str) else v
        if k == "projection":
            v = PROJ[v] if isinstance(v, str) else v
        if k == "calib_k_extra":
            v = (C.c_int32 * 3)(*(list(v) + [0, 0, 0])[:3])
        if not hasattr(p, k):
            raise TypeError(f"unknown fit parameter {k}")
        setattr(p, k, v)
    return p


class Index:
    """A fitted index living on the current GPU."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    # -- construction ------------------------------------------------------------------
    @classmethod
    def fit(cls, base, calib, **params) -> "Index":
        base, calib = _f32(base), _f32(calib)
        p = default_params(**params)
        h = C.c_void_p()
        _check(load_library().ddc_fit(_ptr(base), base.shape[0], base.shape[1], _ptr(calib),
                                      calib.shape[0], C.byref(p), C.byref(h)))
        return cls(h.value)

    @classmethod
    def from_artifacts(cls, art: dict) -> "Index":
        """art: mu, R (rows = eigenvectors), centroids, assign, y (stored rotated base), and
        optionally m, resid (label-0 residual matrix), lam, storage, rotation, delta_d, block_b,
        fp8_lead_dims (0 or 64; the codes are encoded from y on import), pq_perm (M, D/M) and
        pq_books (M, 256, D/M) of the quantization estimate (codes encoded on import), and per
        table pq_m1, pq_m3, pq_resid (the BSA-O classifier)."""
        mu = np.ascontiguousarray(art["mu"], np.float64)
        R = np.ascontiguousarray(art["R"], np.float64)
        cent = _f32(art["centroids"])
        assign = np.ascontiguousarray(art["assign"], np.int32)
        y = _f32(art["y"])
        a = Artifacts()
        a.n, a.dim = y.shape
        a.nlist = cent.shape[0]
        a.delta_d = int(art.get("delta_d", 32))
        a.block_b = int(art.get("block_b", 256))
        a.lag_l = int(art.get("lag_l", 0))
        st = art.get("storage", "f32")
        a.storage = DTYPE[st] if isinstance(st, str) else st
        rt = art.get("rotation", "f32")
        a.rotation = ROT[rt] if isinstance(rt, str) else rt
        a.fp8_lead_dims = int(art.get("fp8_lead_dims", 0))
        keep = [mu, R, cent, assign, y]
        a.mu, a.rot, a.centroids, a.assign, a.y = (_ptr(x) for x in keep)
        lam = art.get("lam")
        if lam is not None:
            lam = np.ascontiguousarray(lam, np.float64)
            keep.append(lam)
            a.lam = _ptr(lam)
        tabs = art.get("tables")
        if tabs is None and art.get("resid") is not None:
            tabs = [dict(kc=int(art.get("calib_k", 1)), m=art["m"], resid=art["resid"],
                         pq_m1=art.get("pq_m1"), pq_m3=art.get("pq_m3"), pq_resid=art.get("pq_resid"))]
        if art.get("pq_perm") is not None:
            perm = np.ascontiguousarray(np.asarray(art["pq_perm"]).reshape(-1), np.int32)
            books = _f32(art["pq_books"])
            keep += [perm, books]
            a.pq_m = int(np.asarray(art["pq_books"]).shape[0])
            a.pq_perm, a.pq_books = _ptr(perm), _ptr(books)
            if tabs and all(t.get("pq_resid") is not None for t in tabs):
                m1 = np.array([t["pq_m1"] for t in tabs], np.float64)
                m3 = np.array([t["pq_m3"] for t in tabs], np.float64)
                pr = np.ascontiguousarray(np.concatenate([np.reshape(t["pq_resid"], -1) for t in tabs]),
                                          np.float64)
                keep += [m1, m3, pr]
                a.pq_m1, a.pq_m3, a.pq_resid = _ptr(m1), _ptr(m3), _ptr(pr)
        if tabs:
            m = np.ascontiguousarray(np.vstack([np.atleast_2d(t["m"]) for t in tabs]), np.float64)
            G = np.ascontiguousarray(np.vstack([t["resid"] for t in tabs]), np.float64)
            keep += [m, G]
            a.m, a.resid, a.n_tables = _ptr(m), _ptr(G), len(tabs)
            for i, t in enumerate(tabs):
                a.table_k[i] = int(t["kc"])
                a.table_n0[i] = t["resid"].shape[0]
        h = C.c_void_p()
        _check(load_library().ddc_import(C.byref(a), C.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "Index":
        h = C.c_void_p()
        _check(load_library().ddc_load(os.fsencode(path), C.byref(h)))
        return cls(h.value)

    def save(self, path: str):
        _check(load_library().ddc_save(self._h, os.fsencode(path)))

    def close(self):
        if self._h is not None and self._h.value:
            load_library().ddc_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- inspection --------------------------------------------------------------------
    def info(self) -> dict:
        i = IndexInfo()
        _check(load_library().ddc_index_get_info(self._h, C.byref(i)))
        out = {f: getattr(i, f) for f, _ in IndexInfo._fields_}
        out["table_k"] = list(i.table_k)[:i.n_tables]
        return out

    def export(self, with_base: bool = True) -> dict:
        inf = self.info()
        n, D, nl, St, n0 = inf["n"], inf["dim"], inf["nlist"], inf["n_test_stages"], inf["n0"]
        out = dict(mu=np.zeros(D), R=np.zeros((D, D)), lam=np.full(D, np.nan),
                   centroids=np.zeros((nl, D), np.float32), assign=np.zeros(n, np.int32),
                   y=np.zeros((n, D), np.float32) if with_base else None,
                   m=np.zeros(St), resid=np.zeros((n0, St)))
        a = Artifacts()
        a.mu, a.rot, a.lam = _ptr(out["mu"]), _ptr(out["R"]), _ptr(out["lam"])
        a.centroids, a.assign, a.y = _ptr(out["centroids"]), _ptr(out["assign"]), _ptr(out["y"])
        nt = inf["n_tables"]
        m_all, r_all = np.zeros((max(nt, 1), St)), np.zeros((n0, St))
        a.m, a.resid = _ptr(m_all), _ptr(r_all)
        if inf["fp8_lead_dims"]:
            out["codes8"] = np.zeros((n, inf["fp8_lead_dims"]), np.uint8)
            out["scale8"] = np.zeros(n, np.float32)
            a.codes8, a.scale8 = _ptr(out["codes8"]), _ptr(out["scale8"])
        M = inf["pq_m"]
        if M:
            out["pq_perm"] = np.zeros((M, D // M), np.int32)
            out["pq_books"] = np.zeros((M, 256, D // M), np.float32)
            out["pq_codes"] = np.zeros((n, M), np.uint8)
            a.pq_perm, a.pq_books, a.pq_codes = _ptr(out["pq_perm"]), _ptr(out["pq_books"]), \
                _ptr(out["pq_codes"])
            pm1, pm3, pres = np.zeros(max(nt, 1)), np.zeros(max(nt, 1)), np.zeros(max(n0, 1))
            if inf["pq_tables"]:
                a.pq_m1, a.pq_m3, a.pq_resid = _ptr(pm1), _ptr(pm3), _ptr(pres)
        _check(load_library().ddc_export(self._h, C.byref(a)))
        tabs, r0 = [], 0
        for t in range(nt):
            n0t = a.table_n0[t]
            tabs.append(dict(kc=a.table_k[t], m=m_all[t].copy(), resid=r_all[r0:r0 + n0t].copy()))
            if M and inf["pq_tables"]:
                tabs[-1].update(pq_m1=float(pm1[t]), pq_m3=float(pm3[t]), pq_resid=pres[r0:r0 + n0t].copy())
            r0 += n0t
        if tabs:
            out["m"], out["resid"], out["calib_k"] = tabs[0]["m"], tabs[0]["resid"], tabs[0]["kc"]
        out.update(delta_d=a.delta_d, block_b=a.block_b, lag_l=a.lag_l, storage=a.storage, rotation=a.rotation,
                   fp8_lead_dims=a.fp8_lead_dims, tables=tabs)
        return out

    def correction(self, alpha: float, mode: str = "joint", k: int = 1):
        """(m, beta) of the correction table a search with this K uses."""
        St = self.info()["n_test_stages"]
        m, b = np.zeros(St), np.zeros(St)
        _check(load_library().ddc_correction(self._h, k, alpha, CALIB[mode], _ptr(m), _ptr(b)))
        return m, b

    def correction_pq(self, alpha: float, k: int = 1):
        """(m1, m3, beta) of the BSA-O classifier a search with this K uses."""
        m1, m3, b = C.c_double(), C.c_double(), C.c_double()
        _check(load_library().ddc_correction_pq(self._h, k, alpha, C.byref(m1), C.byref(m3), C.byref(b)))
        return m1.value, m3.value, b.value

    def calibrate(self, calib, calib_k=10, calib_nprobe=0, max_neg=50, seed=0):
        calib = _f32(calib)
        _check(load_library().ddc_calibrate(self._h, _ptr(calib), calib.shape[0], calib_k,
                                            calib_nprobe, max_neg, seed))

    # -- search ------------------------------------------------------------------------
    def search(self, queries, k: int, nprobe: int, alpha: float, mode: str = "learned"):
        q = _f32(queries)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int64)
        d = np.empty((nq, k), np.float32)
        st = SearchStats()
        _check(load_library().ddc_search(self._h, _ptr(q), nq, k, nprobe, alpha, CORR[mode],
                                         _ptr(ids), _ptr(d), C.byref(st)))
        return ids, d, st.as_dict()

    def search_estimate(self, queries, k: int, nprobe: int, dims: int, estimator: str = "partial"):
        """Top-k by an estimate over the leading `dims` rotated dims (no correction, no
        refinement): (ids [nq, k], estimates [nq, k])."""
        q = _f32(queries)
        ids = np.empty((q.shape[0], k), np.int64)
        d = np.empty((q.shape[0], k), np.float32)
        _check(load_library().ddc_search_estimate(self._h, _ptr(q), q.shape[0], k, nprobe, dims,
                                                  EST[estimator], _ptr(ids), _ptr(d)))
        return ids, d

    def search_var(self, queries, k, nprobe, alpha: float, mode: str = "learned"):
        q = _f32(queries)
        k = np.ascontiguousarray(k, np.int32)
        nprobe = np.ascontiguousarray(nprobe, np.int32)
        off = np.zeros(q.shape[0] + 1, np.int64)
        off[1:] = np.cumsum(k)
        ids = np.empty(off[-1], np.int64)
        d = np.empty(off[-1], np.float32)
        st = SearchStats()
        _check(load_library().ddc_search_var(self._h, _ptr(q), q.shape[0], _ptr(k), _ptr(nprobe),
                                             alpha, CORR[mode], _ptr(off), _ptr(ids), _ptr(d),
                                             C.byref(st)))
        return ids, d, off, st.as_dict()

    def search_device(self, d_queries, nq, k_all, nprobe_all, alpha, mode, d_ids, d_dists,
                      d_counters=0, stream=0, d_k=0, k_max=0, d_nprobe=0, nprobe_max=0,
                      d_offsets=0):
        """Device pointers (ints, e.g. torch tensors' data_ptr()) and a hipStream_t handle."""
        _check(load_library().ddc_search_device(
            self._h, d_queries, nq, d_k or None, k_all, k_max, d_nprobe or None, nprobe_all,
            nprobe_max, alpha, CORR[mode], d_offsets or None, d_ids, d_dists, d_counters or None,
            stream or None))

    def search_device_noalloc(self, d_queries, nq, k_all, nprobe_all, alpha, mode, d_ids, d_dists,
                              d_counters=0, stream=0, d_k=0, k_max=0, d_nprobe=0, nprobe_max=0,
                              d_offsets=0):
        """search_device with the library's fixed device scratch: allocates no device memory."""
        _check(load_library().ddc_search_device_noalloc(
            self._h, d_queries, nq, d_k or None, k_all, k_max, d_nprobe or None, nprobe_all,
            nprobe_max, alpha, CORR[mode], d_offsets or None, d_ids, d_dists, d_counters or None,
            stream or None))

    def set_bsar_multiplier(self, m: float):
        _check(load_library().ddc_set_bsar_multiplier(self._h, m))

    def set_ads_epsilon(self, eps0: float):
        _check(load_library().ddc_set_ads_epsilon(self._h, eps0))

    def set_launch(self, waves_per_query: int | None = None, lookahead: int | None = None,
                   query_order: int | None = None, xcd_swizzle: int | None = None,
                   persistent: int | None = None, two_phase: int | None = None,
                   full_d_matrix: int | None = None, stage1_matrix: int | None = None,
                   waves_per_simd: int | None = None):
        """Launch shape of the scan; None keeps the current value (waves_per_query 0,
        lookahead -1, persistent -1, two_phase -1 and waves_per_simd 0 mean tuned per size class).  Every knob
        but full_d_matrix and stage1_matrix=2 is result-invariant; those two take distances
        formed on the matrix cores in the expanded form as they are (results equal up to FP32
        rounding)."""
        cur = self.launch()
        lp = LaunchParams(*(cur[k] if v is None else int(v) for k, v in
                            (("waves_per_query", waves_per_query), ("lookahead", lookahead),
                             ("query_order", query_order), ("xcd_swizzle", xcd_swizzle),
                             ("persistent", persistent), ("two_phase", two_phase),
                             ("full_d_matrix", full_d_matrix), ("stage1_matrix", stage1_matrix),
                             ("waves_per_simd", waves_per_simd))))
        _check(load_library().ddc_set_launch(self._h, C.byref(lp)))

    def launch(self) -> dict:
        lp = LaunchParams()
        _check(load_library().ddc_get_launch(self._h, C.byref(lp)))
        return {k: getattr(lp, k) for k, _ in LaunchParams._fields_}

    def scan_variant(self, nq: int, k: int, nprobe: int, mode: str = "learned",
                     with_budget: bool = False) -> tuple:
        """(waves per query, lookahead, persistent, two-phase) a search of this shape runs
        (tuned or fixed rule); with_budget adds the kernel's waves per SIMD (4 or 5)."""
        w, la, pe, tp, ws = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load_library().ddc_scan_variant(self._h, nq, k, nprobe, CORR[mode], C.byref(w),
                                               C.byref(la), C.byref(pe), C.byref(tp), C.byref(ws)))
        v = (w.value, la.value, pe.value, tp.value)
        return v + (ws.value,) if with_budget else v

    def set_kernel_timing(self, enable: bool):
        _check(load_library().ddc_set_kernel_timing(self._h, int(enable)))

    def kernel_timing(self, reset: bool = True):
        """(ms_total[5], launches[5]) for rotation, coarse, select, scan and the two-phase
        scan's first phase since the last reset."""
        ms = np.zeros(5)
        n = np.zeros(5, np.int64)
        _check(load_library().ddc_get_kernel_timing(self._h, _ptr(ms), _ptr(n), int(reset)))
        return ms, n

    def debug_intermediates(self, queries, nprobe: int):
        q = _f32(queries)
        D = self.info()["dim"]
        qr = np.empty((q.shape[0], D), np.float32)
        pr = np.empty((q.shape[0], nprobe), np.int32)
        _check(load_library().ddc_debug_intermediates(self._h, _ptr(q), q.shape[0], nprobe,
                                                      _ptr(qr), _ptr(pr)))
        return qr, pr


class Server:
    """Continuous-batching search server on an index (the index must outlive it)."""

    def __init__(self, index: Index, n_streams=4, max_batch=1024, hbm_budget_bytes=2 << 30,
                 alpha=0.05, mode="learned"):
        p = ServerParams(n_streams, max_batch, hbm_budget_bytes, alpha, CORR[mode])
        h = C.c_void_p()
        _check(load_library().ddc_server_create(index.handle, C.byref(p), C.byref(h)))
        self._h = h
        self._index = index
        self._nres = {}

    def submit(self, queries, k, nprobe) -> int:
        q = _f32(queries)
        k = np.ascontiguousarray(k, np.int32)
        nprobe = np.ascontiguousarray(nprobe, np.int32)
        t = C.c_uint64()
        _check(load_library().ddc_server_submit(self._h, _ptr(q), q.shape[0], _ptr(k), _ptr(nprobe),
                                                C.byref(t)))
        self._nres[t.value] = (int(k.sum()), k.copy())
        return t.value

    def poll(self, ticket: int):
        """None while running, else (ids, dists, offsets, t_done_ns) for the request."""
        nres, k = self._nres[ticket]
        ids = np.empty(nres, np.int64)
        d = np.empty(nres, np.float32)
        done = C.c_int(0)
        tdone = C.c_uint64(0)
        _check(load_library().ddc_server_poll(self._h, ticket, _ptr(ids), _ptr(d), C.byref(done),
                                              C.byref(tdone)))
        if not done.value:
            return None
        del self._nres[ticket]
        off = np.zeros(k.shape[0] + 1, np.int64)
        off[1:] = np.cumsum(k)
        return ids, d, off, tdone.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().ddc_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            load_library().ddc_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
