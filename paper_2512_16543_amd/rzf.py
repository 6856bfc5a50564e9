"""Thin ctypes binding over the C ABI of librzf.so (declared in include/rzf.h).

Argument marshalling only: every step of the precoding path runs in the HIP
library.  PyTorch provides device memory (the arena, H and W tensors) and the
stream.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librzf.so")
TUNING_PATH = os.path.join(PKG, "tuning.json")

RZF_OK = 0
RZF_E_INVALID = 1
RZF_E_SHAPE = 2
RZF_E_NOMEM = 3
RZF_E_NOT_HPD = 4
RZF_E_NONFINITE = 5
RZF_E_DEVICE = 6

PATH_NOOP, PATH_WB, PATH_FULL_RANK, PATH_FULL_SINGULAR, PATH_RESET = 0, 1, 2, 3, 4
KINIT_FIXED, KINIT_WARM = 0, 1
PREC_FP32, PREC_BF16, PREC_BF16X3 = 0, 1, 2
KMAX = 256
NMAX = 4096


class Params(ctypes.Structure):
    _fields_ = [("k_init", ctypes.c_int), ("p", ctypes.c_int), ("i_max", ctypes.c_int),
                ("switch_ratio", ctypes.c_double), ("reset_period", ctypes.c_int),
                ("P", ctypes.c_double), ("seed", ctypes.c_uint64), ("track_id", ctypes.c_uint64),
                ("kinit_policy", ctypes.c_int), ("early_fallback", ctypes.c_int), ("precision", ctypes.c_int),
                ("error_feedback", ctypes.c_int)]


class UpdateInfo(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("iters", ctypes.c_int), ("path", ctypes.c_int),
                ("d", ctypes.c_int), ("dA_fro2", ctypes.c_double), ("captured", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class UpdateItem(ctypes.Structure):
    _fields_ = [("track", ctypes.c_void_p), ("H", ctypes.c_void_p), ("ldh", ctypes.c_int),
                ("W", ctypes.c_void_p), ("ldw", ctypes.c_int), ("info", ctypes.POINTER(UpdateInfo))]


class FullItem(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("N", ctypes.c_int), ("H", ctypes.c_void_p), ("ldh", ctypes.c_int),
                ("alpha", ctypes.c_double), ("P", ctypes.c_double), ("W", ctypes.c_void_p),
                ("ldw", ctypes.c_int), ("precision", ctypes.c_int)]


class RateItem(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("N", ctypes.c_int), ("H", ctypes.c_void_p), ("ldh", ctypes.c_int),
                ("W", ctypes.c_void_p), ("ldw", ctypes.c_int), ("rates", ctypes.c_void_p),
                ("sum_rate", ctypes.c_void_p), ("sigma2", ctypes.c_double)]


BATCH_MAX = 2048
SERVE_UPDATE, SERVE_FULL = 0, 1


class ServerParams(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int), ("max_wait_us", ctypes.c_double), ("tol", ctypes.c_double),
                ("mode", ctypes.c_int), ("max_inflight", ctypes.c_int)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("pad", ctypes.c_int),
                ("info", UpdateInfo), ("t_submit_us", ctypes.c_double), ("t_launch_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double)]


class ServeRequest(ctypes.Structure):
    _fields_ = [("track", ctypes.c_void_p), ("H", ctypes.c_void_p), ("ldh", ctypes.c_int),
                ("W", ctypes.c_void_p), ("ldw", ctypes.c_int), ("tag", ctypes.c_uint64),
                ("t_arrival_us", ctypes.c_double)]


class GraphRate(ctypes.Structure):
    _fields_ = [("P", ctypes.c_double), ("sigma2", ctypes.c_double), ("sums", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("N", ctypes.c_int), ("precoder_rows", ctypes.c_int),
                ("batch_precoder_rows", ctypes.c_int), ("rate_splits", ctypes.c_int)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("count", ctypes.c_int), ("total_ms", ctypes.c_double)]


class RzfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None

_SIGS = {
    "rzf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rzf_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "rzf_tune_switch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "rzf_track_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "rzf_params_check": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int]),
    "rzf_full_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_void_p]),
    "rzf_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_int, ctypes.c_double, ctypes.POINTER(Params),
                                ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(UpdateInfo)]),
    "rzf_full": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                ctypes.c_int]),
    "rzf_sum_rate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rzf_beamspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "rzf_get_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rzf_update_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(UpdateItem),
                                        ctypes.c_double]),
    "rzf_full_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(FullItem)]),
    "rzf_sum_rate_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(RateItem),
                                          ctypes.c_double, ctypes.c_double]),
    "rzf_track_query": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 5),
    "rzf_graph_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(UpdateItem), ctypes.c_double,
                                        ctypes.POINTER(GraphRate), ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_graph_full": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(FullItem),
                                      ctypes.POINTER(GraphRate), ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_graph_launch": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_tune_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(TuneEntry)]),
    "rzf_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_track_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_server_params_default": (ctypes.c_int, [ctypes.POINTER(ServerParams)]),
    "rzf_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerParams),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64]),
    "rzf_server_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ServeRequest)]),
    "rzf_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int)]),
    "rzf_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_server_now_us": (ctypes.c_double, [ctypes.c_void_p]),
    "rzf_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rzf_track_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "rzf_track_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "rzf_debug_sigma2": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "rzf_debug_counters": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "rzf_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "rzf_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ProfileEntry), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "rzf_debug_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p]),
}


def lib():
    """The loaded librzf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2512_16543_amd.build` (there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().rzf_status_string(st).decode()


def _check(st: int, where: str):
    if st != RZF_OK:
        raise RzfError(st, where)


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().rzf_params_default(ctypes.byref(p)), "rzf_params_default")
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def params_check(params: Params, K: int) -> int:
    """rzf_params_check: RZF_OK when `params` suit a K-user track."""
    return lib().rzf_params_check(ctypes.byref(params), int(K))


def full_noalloc(H, alpha: float, P: float, W, err=None, stream=None):
    """rzf_full_noalloc on H's device: W = full-inversion RZF of H, with the
    library's fixed device scratch (no context, no allocation).  err: an int32
    device tensor of one element, or None.  stream: a torch stream (None:
    the current one)."""
    import torch
    hp, ldh = _mat_args(H)
    wp, ldw = _mat_args(W)
    K, N = H.shape
    if tuple(W.shape) != (N, K):
        raise ValueError("shape mismatch")
    with torch.cuda.device(H.device):
        s = stream if stream is not None else torch.cuda.current_stream(H.device)
        ep = ctypes.c_void_p(err.data_ptr()) if err is not None else None
        _check(lib().rzf_full_noalloc(ctypes.c_void_p(s.cuda_stream), int(K), int(N), ctypes.c_void_p(hp), ldh,
                                      float(alpha), float(P), ctypes.c_void_p(wp), ldw, ep), "rzf_full_noalloc")


def load_tuning(path: str = TUNING_PATH):
    """The entries of an autotuner table (JSON)."""
    import json
    with open(path) as f:
        return json.load(f)["entries"]


def track_bytes(K: int, N: int) -> int:
    return int(lib().rzf_track_bytes(K, N))


def _dev_ptr(x) -> int:
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not x.is_cuda:
        raise ValueError("tensor must be on the GPU")
    return x.data_ptr()


def _mat_args(H, dtype_name="complex64"):
    import torch
    if H.dtype != torch.complex64:
        raise TypeError(f"expected {dtype_name}, got {H.dtype}")
    if H.dim() != 2 or H.stride(1) != 1:
        raise ValueError("expected a 2-D row-major matrix")
    return _dev_ptr(H), int(H.stride(0))


class Context:
    """rzf_ctx: one device, one stream, one arena (a torch uint8 tensor)."""

    def __init__(self, device: int = 0, arena_bytes: int = 64 << 20, stream=None, arena=None,
                 tuning: Optional[str] = TUNING_PATH):
        """arena: a caller's uint8 device tensor of arena_bytes (default: a new one).
        tuning: a launch-shape table written by the autotuner (default: the
        package's tuning.json when present; None: the library defaults)."""
        import torch
        self.device = device
        dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        if arena is not None and (arena.dtype != torch.uint8 or arena.numel() < arena_bytes):
            raise ValueError("arena must be a uint8 tensor of at least arena_bytes")
        self.arena = arena if arena is not None else torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        _check(lib().rzf_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.c_void_p(self.arena.data_ptr()), arena_bytes,
                                    ctypes.byref(h)), "rzf_ctx_create")
        self.h = h
        self._infos = []
        if tuning and os.path.exists(tuning):
            self.tune_table(load_tuning(tuning))

    def close(self):
        if self.h:
            lib().rzf_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(lib().rzf_sync(self.h), "rzf_sync")
        self._infos = []

    def sync_status(self) -> int:
        st = lib().rzf_sync(self.h)
        self._infos = []
        return st

    def import_track(self, blob: bytes) -> "Track":
        """A new track in this context from a checkpoint blob (rzf_track_import)."""
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().rzf_track_import(self.h, buf, len(blob), ctypes.byref(h)), "rzf_track_import")
        K, N = [ctypes.c_int() for _ in range(2)]
        _check(lib().rzf_track_query(h, ctypes.byref(K), ctypes.byref(N), None, None, None),
               "rzf_track_query")
        return Track(self, h, K.value, N.value)

    def init(self, H, alpha: float, params: Optional[Params] = None) -> "Track":
        ptr, ld = _mat_args(H)
        K, N = H.shape
        h = ctypes.c_void_p()
        _check(lib().rzf_init(self.h, K, N, ctypes.c_void_p(ptr), ld, float(alpha),
                              ctypes.byref(params) if params is not None else None,
                              ctypes.byref(h)), "rzf_init")
        return Track(self, h, K, N)

    def full(self, H, alpha: float, P: float, W):
        hp, ldh = _mat_args(H)
        wp, ldw = _mat_args(W)
        K, N = H.shape
        _check(lib().rzf_full(self.h, K, N, ctypes.c_void_p(hp), ldh, float(alpha), float(P),
                              ctypes.c_void_p(wp), ldw), "rzf_full")

    def sum_rate(self, H, W, P: float, sigma2: float, rates=None) -> float:
        hp, ldh = _mat_args(H)
        wp, ldw = _mat_args(W)
        K, N = H.shape
        rp = None
        if rates is not None:
            import torch
            if rates.dtype != torch.float32 or rates.numel() < K:
                raise ValueError("rates must be a float32 tensor of K entries")
            rp = ctypes.c_void_p(_dev_ptr(rates))
        out = ctypes.c_double()
        _check(lib().rzf_sum_rate(self.h, K, N, ctypes.c_void_p(hp), ldh, ctypes.c_void_p(wp), ldw,
                                  float(P), float(sigma2), rp, ctypes.byref(out)), "rzf_sum_rate")
        return out.value

    def sum_rate_async(self, H, W, P: float, sigma2: float, rates):
        hp, ldh = _mat_args(H)
        wp, ldw = _mat_args(W)
        K, N = H.shape
        _check(lib().rzf_sum_rate(self.h, K, N, ctypes.c_void_p(hp), ldh, ctypes.c_void_p(wp), ldw,
                                  float(P), float(sigma2), ctypes.c_void_p(_dev_ptr(rates)), None),
               "rzf_sum_rate")

    def beamspace(self, H, nx: int, ny: int, beams, H_eff, select: bool = True):
        """rzf_beamspace: H_eff = H F_RF over the DFT codebook of an nx x ny UPA.
        beams is a device int32 tensor of n_rf = H_eff.shape[1] entries, written
        when select is True and read otherwise (asynchronous)."""
        import torch
        hp, ldh = _mat_args(H)
        ep, lde = _mat_args(H_eff)
        K, n_rf = H_eff.shape
        if H.shape[0] != K:
            raise ValueError("H and H_eff must have the same number of rows")
        if beams.dtype != torch.int32 or not beams.is_contiguous() or beams.numel() != n_rf:
            raise ValueError("beams must be a contiguous int32 tensor of n_rf entries")
        _check(lib().rzf_beamspace(self.h, K, int(nx), int(ny), ctypes.c_void_p(hp), ldh, n_rf,
                                   1 if select else 0, ctypes.c_void_p(_dev_ptr(beams)),
                                   ctypes.c_void_p(ep), lde), "rzf_beamspace")

    def tune_switch(self, K: int, N: int, precision: int = 0) -> dict:
        """rzf_tune_switch: Alg. 2's switch ratio from measured branch costs on
        this device, with the cycle counts it was fitted from."""
        out = [ctypes.c_double() for _ in range(4)]
        _check(lib().rzf_tune_switch(self.h, int(K), int(N), int(precision),
                                     *[ctypes.byref(v) for v in out]), "rzf_tune_switch")
        return dict(zip(("switch_ratio", "direct_cycles", "wb_cycles_a", "wb_cycles_b"),
                        (v.value for v in out)))

    def update_batch(self, tracks, Hs, Ws, tol: float, want_info: bool = False):
        """rzf_update_batch over parallel lists of Track, H_t and W tensors."""
        n = len(tracks)
        arr = (UpdateItem * n)()
        infos = [UpdateInfo() for _ in range(n)] if want_info else None
        for i in range(n):
            hp, ldh = _mat_args(Hs[i])
            wp, ldw = _mat_args(Ws[i])
            it = arr[i]
            it.track = tracks[i].h
            it.H, it.ldh, it.W, it.ldw = hp, ldh, wp, ldw
            if want_info:
                it.info = ctypes.pointer(infos[i])
        _check(lib().rzf_update_batch(self.h, n, arr, float(tol)), "rzf_update_batch")
        if want_info:
            self._infos.extend(infos)
        return infos

    @staticmethod
    def update_items(tracks, Hs, Ws):
        """Prebuilt rzf_update_item array for update_batch_raw."""
        n = len(tracks)
        arr = (UpdateItem * n)()
        for i in range(n):
            hp, ldh = _mat_args(Hs[i])
            wp, ldw = _mat_args(Ws[i])
            arr[i].track = tracks[i].h
            arr[i].H, arr[i].ldh, arr[i].W, arr[i].ldw = hp, ldh, wp, ldw
        return arr

    def update_batch_raw(self, items, tol: float):
        _check(lib().rzf_update_batch(self.h, len(items), items, float(tol)), "rzf_update_batch")

    @staticmethod
    def full_items(Hs, alphas, P, Ws, precision: int = 0):
        n = len(Hs)
        arr = (FullItem * n)()
        for i in range(n):
            hp, ldh = _mat_args(Hs[i])
            wp, ldw = _mat_args(Ws[i])
            K, N = Hs[i].shape
            arr[i].K, arr[i].N, arr[i].H, arr[i].ldh = K, N, hp, ldh
            arr[i].alpha, arr[i].P, arr[i].W, arr[i].ldw = float(alphas[i]), float(P), wp, ldw
            arr[i].precision = int(precision)
        return arr

    def full_batch_raw(self, items):
        _check(lib().rzf_full_batch(self.h, len(items), items), "rzf_full_batch")

    @staticmethod
    def rate_items(Hs, Ws, rates=None, sums=None, sigma2s=None):
        """sigma2s: per-item noise powers (None: every item takes the call's)."""
        n = len(Hs)
        arr = (RateItem * n)()
        for i in range(n):
            hp, ldh = _mat_args(Hs[i])
            wp, ldw = _mat_args(Ws[i])
            K, N = Hs[i].shape
            it = arr[i]
            it.K, it.N, it.H, it.ldh, it.W, it.ldw = K, N, hp, ldh, wp, ldw
            it.rates = _dev_ptr(rates[i]) if rates is not None else None
            it.sum_rate = (_dev_ptr(sums) + 8 * i) if sums is not None else None
            it.sigma2 = float(sigma2s[i]) if sigma2s is not None else -1.0
        return arr

    def sum_rate_batch_raw(self, items, P: float, sigma2: float):
        _check(lib().rzf_sum_rate_batch(self.h, len(items), items, float(P), float(sigma2)),
               "rzf_sum_rate_batch")

    def tune_table(self, entries):
        """rzf_tune_table from dicts with K, N, precoder_rows, batch_precoder_rows, rate_splits."""
        n = len(entries)
        arr = (TuneEntry * max(n, 1))()
        for i, e in enumerate(entries):
            arr[i] = TuneEntry(int(e["K"]), int(e["N"]), int(e.get("precoder_rows", 0)),
                               int(e.get("batch_precoder_rows", 0)), int(e.get("rate_splits", 0)))
        _check(lib().rzf_tune_table(self.h, n, arr), "rzf_tune_table")

    def _graph_rate(self, rate):
        if rate is None:
            return None
        P, sigma2, sums = rate
        return ctypes.pointer(GraphRate(float(P), float(sigma2), _dev_ptr(sums)))

    def graph_update(self, tracks, Hs, Ws, tol: float, rate=None) -> "Graph":
        """Captured update step over fixed H / W tensors (rzf_graph_update);
        rate = (P, sigma2, sums) adds each item's sum rate into the float64
        device tensor sums."""
        items = self.update_items(tracks, Hs, Ws)
        out = ctypes.c_void_p()
        _check(lib().rzf_graph_update(self.h, len(tracks), items, float(tol), self._graph_rate(rate),
                                      ctypes.byref(out)), "rzf_graph_update")
        return Graph(self, out.value, (Hs, Ws, rate))

    def graph_full(self, Hs, alphas, P: float, Ws, precision: int = 0, rate=None) -> "Graph":
        """Captured full-inversion step over fixed H / W tensors (rzf_graph_full)."""
        items = self.full_items(Hs, alphas, P, Ws, precision)
        out = ctypes.c_void_p()
        _check(lib().rzf_graph_full(self.h, len(Hs), items, self._graph_rate(rate), ctypes.byref(out)),
               "rzf_graph_full")
        return Graph(self, out.value, (Hs, Ws, rate))

    def full_batch(self, Hs, alphas, P: float, Ws, precision: int = 0):
        arr = self.full_items(Hs, alphas, P, Ws, precision)
        _check(lib().rzf_full_batch(self.h, len(Hs), arr), "rzf_full_batch")

    def sum_rate_batch(self, Hs, Ws, P: float, sigma2: float, rates=None, sums=None, sigma2s=None):
        """rates: list of float32 device tensors (or None); sums: float64 device
        tensor of n; sigma2s: per-item noise powers (None: all take sigma2)."""
        arr = self.rate_items(Hs, Ws, rates, sums, sigma2s)
        _check(lib().rzf_sum_rate_batch(self.h, len(Hs), arr, float(P), float(sigma2)),
               "rzf_sum_rate_batch")

    def profile(self, enable: bool):
        _check(lib().rzf_profile(self.h, 1 if enable else 0), "rzf_profile")

    def profile_read(self):
        arr = (ProfileEntry * 16)()
        n = ctypes.c_int()
        _check(lib().rzf_profile_read(self.h, arr, 16, ctypes.byref(n)), "rzf_profile_read")
        return {arr[i].name.decode(): (arr[i].count, arr[i].total_ms) for i in range(min(n.value, 16))}

    def debug_sketch(self, seed: int, track: int, t: int, it: int, K: int, d: int):
        import torch
        dev = torch.device("cuda", self.device)
        om = torch.empty(d, K, dtype=torch.complex64, device=dev)      # column-major K x d
        words = torch.empty(K * d * 2, dtype=torch.int64, device=dev)
        _check(lib().rzf_debug_sketch(self.h, seed, track, t, it, K, d, ctypes.c_void_p(om.data_ptr()),
                                      ctypes.c_void_p(words.data_ptr())), "rzf_debug_sketch")
        return om.t(), words.view(K, d, 2)


class Graph:
    """A captured step (rzf_graph_*); keeps its buffers alive."""

    def __init__(self, ctx: Context, h, keep):
        self.ctx, self.h, self._keep = ctx, h, keep

    def launch(self):
        _check(lib().rzf_graph_launch(self.h), "rzf_graph_launch")

    def destroy(self):
        # a closed context has freed its graphs already
        if self.h and self.ctx.h:
            _check(lib().rzf_graph_destroy(self.h), "rzf_graph_destroy")
        self.h = None


class Track:
    """rzf_track: one channel track's resident state."""

    def __init__(self, ctx: Context, h, K: int, N: int):
        self.ctx, self.h, self.K, self.N = ctx, h, K, N

    def update(self, H_t, tol: float, W, want_info: bool = True) -> Optional[UpdateInfo]:
        hp, ldh = _mat_args(H_t)
        wp, ldw = _mat_args(W)
        if tuple(H_t.shape) != (self.K, self.N) or tuple(W.shape) != (self.N, self.K):
            raise ValueError("shape mismatch")
        info = UpdateInfo() if want_info else None
        _check(lib().rzf_update(self.h, ctypes.c_void_p(hp), ldh, float(tol), ctypes.c_void_p(wp), ldw,
                                ctypes.byref(info) if info is not None else None), "rzf_update")
        if info is not None:
            self.ctx._infos.append(info)   # keep alive until rzf_sync fills it
        return info

    def inverse(self):
        import torch
        out = torch.empty(self.K, self.K, dtype=torch.complex64, device=torch.device("cuda", self.ctx.device))
        _check(lib().rzf_get_inverse(self.h, ctypes.c_void_p(out.data_ptr())), "rzf_get_inverse")
        return out

    def query(self):
        vals = [ctypes.c_int() for _ in range(5)]
        _check(lib().rzf_track_query(self.h, *[ctypes.byref(v) for v in vals]), "rzf_track_query")
        return dict(zip(("K", "N", "t", "since_reset", "last_r"), (v.value for v in vals)))

    def counters(self):
        arr = (ctypes.c_int * 8)()
        _check(lib().rzf_debug_counters(self.h, arr, 8), "rzf_debug_counters")
        return {"jacobi_sweeps": arr[0], "jacobi_rounds": arr[1], "qr_columns": arr[2],
                "cyc_sketch": arr[3], "cyc_qr": arr[4], "cyc_jacobi": arr[5], "cyc_wb": arr[6],
                "realtime_ticks": arr[7]}

    def sigma2(self):
        arr = (ctypes.c_double * KMAX)()
        d = ctypes.c_int()
        _check(lib().rzf_debug_sigma2(self.h, arr, KMAX, ctypes.byref(d)), "rzf_debug_sigma2")
        return [arr[i] for i in range(d.value)]

    def export(self) -> bytes:
        """Checkpoint blob of the track (rzf_track_export)."""
        n = ctypes.c_size_t()
        _check(lib().rzf_track_export(self.h, None, ctypes.byref(n)), "rzf_track_export")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().rzf_track_export(self.h, buf, ctypes.byref(n)), "rzf_track_export")
        return buf.raw[:n.value]

    def residual(self):
        """The error-feedback residual R (K x K complex64 numpy array): the
        K*K entries of the checkpoint blob before its last 2 K*K (the two
        SVD bases)."""
        import numpy as np
        blob = self.export()
        n = self.K * self.K * 8
        return np.frombuffer(blob[len(blob) - 3 * n:len(blob) - 2 * n],
                             dtype=np.complex64).reshape(self.K, self.K).copy()

    def destroy(self):
        if self.h:
            _check(lib().rzf_track_destroy(self.h), "rzf_track_destroy")
            self.h = ctypes.c_void_p()


def server_params(**kw) -> ServerParams:
    p = ServerParams()
    _check(lib().rzf_server_params_default(ctypes.byref(p)), "rzf_server_params_default")
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Server:
    """rzf_server: batched serving of update (or full-inversion) requests."""

    def __init__(self, ctx: Context, params: Optional[ServerParams] = None):
        self.ctx = ctx
        h = ctypes.c_void_p()
        p = params if params is not None else server_params()
        _check(lib().rzf_server_create(ctx.h, ctypes.byref(p), ctypes.byref(h)), "rzf_server_create")
        self.h = h

    def submit(self, track: Track, H_t, W, tag: int = 0):
        hp, ldh = _mat_args(H_t)
        wp, ldw = _mat_args(W)
        _check(lib().rzf_server_submit(self.h, track.h, ctypes.c_void_p(hp), ldh, ctypes.c_void_p(wp), ldw,
                                       int(tag)), "rzf_server_submit")

    @staticmethod
    def requests(tracks, Hs, Ws, tags, t_arrival_us):
        """A ServeRequest array for replay (tracks, H_t and W tensors, tags, arrival offsets)."""
        n = len(tracks)
        arr = (ServeRequest * n)()
        for i in range(n):
            hp, ldh = _mat_args(Hs[i])
            wp, ldw = _mat_args(Ws[i])
            r = arr[i]
            r.track, r.H, r.ldh, r.W, r.ldw = tracks[i].h.value, hp, ldh, wp, ldw
            r.tag, r.t_arrival_us = int(tags[i]), float(t_arrival_us[i])
        return arr

    def replay(self, reqs):
        _check(lib().rzf_server_replay(self.h, len(reqs), reqs), "rzf_server_replay")

    def poll(self, max_n: int = 4096):
        arr = (Completion * max_n)()
        n = ctypes.c_int()
        _check(lib().rzf_server_poll(self.h, arr, max_n, ctypes.byref(n)), "rzf_server_poll")
        return [arr[i] for i in range(n.value)]

    def drain(self):
        _check(lib().rzf_server_drain(self.h), "rzf_server_drain")

    def now_us(self) -> float:
        return float(lib().rzf_server_now_us(self.h))

    def close(self):
        if self.h:
            _check(lib().rzf_server_destroy(self.h), "rzf_server_destroy")
            self.h = ctypes.c_void_p()
