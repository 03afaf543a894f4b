"""ctypes binding of libws.so (see include/ws.h for the contract of each call)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libws.so")

WS_OK, WS_EINVAL, WS_ENOMEM, WS_EDEVICE, WS_ENOCONV, WS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
WS_U8, WS_U16 = 1, 2
_STATUS = {WS_EINVAL: "WS_EINVAL", WS_ENOMEM: "WS_ENOMEM", WS_EDEVICE: "WS_EDEVICE",
           WS_ENOCONV: "WS_ENOCONV", WS_EUNSUPPORTED: "WS_EUNSUPPORTED"}

# Every symbol include/ws.h declares, with its ctypes signature.
_i64, _int, _ptr, _f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_float


class WsItem(ctypes.Structure):
    """ws_item of include/ws.h."""
    _fields_ = [("grad", ctypes.c_void_p), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("conn", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("nregions", ctypes.c_void_p)]


SIGNATURES = {
    "ws_create": (_int, [ctypes.POINTER(ctypes.c_void_p), _int, ctypes.c_size_t]),
    "ws_destroy": (None, [_ptr]),
    "ws_last_error": (ctypes.c_char_p, [_ptr]),
    "ws_sync": (_int, [_ptr, _ptr]),
    "ws_footprint_bytes": (ctypes.c_size_t, [_i64, _i64, _i64, _int, _int, _int]),
    "ws_gradient": (_int, [_ptr, _ptr, _i64, _i64, _i64, _f32, _int, _ptr, _ptr, _ptr]),
    "ws_watershed": (_int, [_ptr, _ptr, _int, _i64, _i64, _i64, _int, _ptr, _ptr]),
    "ws_watershed_noalloc": (_int, [_ptr, _ptr, _int, _i64, _i64, _i64, _int, _ptr, _ptr]),
    "ws_waterfall": (_int, [_ptr, _ptr, _ptr, _int, _i64, _i64, _i64, _int, _int, _ptr, _ptr, _ptr]),
    "ws_waterfall_recon": (_int, [_ptr, _ptr, _ptr, _int, _i64, _i64, _i64, _int, _int, _ptr, _ptr, _ptr]),
    "ws_rag": (_int, [_ptr, _ptr, _ptr, _int, _i64, _i64, _i64, _int, _i64, _ptr, _ptr, _ptr, _ptr, _ptr]),
    "ws_watershed_stages": (_int, [_ptr, _ptr, _int, _i64, _i64, _i64, _int, _ptr, _ptr, _ptr]),
    "ws_batch": (_int, [_ptr, ctypes.POINTER(WsItem), _int, _int, _int, _ptr]),
    "ws_set_option": (_int, [_ptr, ctypes.c_char_p, _i64]),
    "ws_get_stats": (_int, [_ptr, ctypes.POINTER(ctypes.c_int64), _int]),
    "ws_timing_read": (_int, [_ptr, ctypes.c_char_p, _int, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int64), _int]),
    "ws_timing_reset": (_int, [_ptr]),
}

_lib = None


class WSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "error"), code, msg))
        self.code = code


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads libws.so (no GPU call happens here). Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libws.so is not built (%s); run __graft_entry__.build() first" % _LIB_PATH)
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _dims(shape):
    if len(shape) == 1:
        return shape[0], 1, 1
    if len(shape) == 2:
        return shape[1], shape[0], 1
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    raise ValueError("images must be 1D, 2D or 3D")


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


def _grey_code(t):
    import torch
    if t.dtype == torch.uint8:
        return WS_U8
    if t.dtype == torch.uint16:
        return WS_U16
    raise TypeError("gradient must be uint8 or uint16")


class Context:
    """Owns a ws_ctx (device scratch memory) on one device; scratch_budget
    bounds the device scratch it may hold (bytes, 0 = no bound)."""

    def __init__(self, device: int = 0, scratch_budget: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        rc = self._lib.ws_create(ctypes.byref(h), int(device), int(scratch_budget))
        if rc != WS_OK:
            raise WSError(rc, self._lib.ws_last_error(None).decode())
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != WS_OK:
            raise WSError(rc, self._lib.ws_last_error(self._h).decode())

    # -- options and counters -------------------------------------------
    def set_option(self, name: str, value: int):
        self._check(self._lib.ws_set_option(self._h, name.encode(), int(value)))

    def stats(self):
        out = (ctypes.c_int64 * 7)()
        n = self._lib.ws_get_stats(self._h, out, 7)
        keys = ("sweeps_launched", "sweeps_changing", "step3_syncs", "tiles", "graph_replays", "allocations",
                "step4_passes")
        return {k: int(out[i]) for i, k in enumerate(keys[:n])}

    def timing_reset(self):
        self._check(self._lib.ws_timing_reset(self._h))

    def timing_read(self, cap: int = 64, name_len: int = 32):
        names = ctypes.create_string_buffer(cap * name_len)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = self._lib.ws_timing_read(self._h, names, name_len, ms, cnt, cap)
        if n < 0:
            self._check(n)
        out = {}
        for i in range(min(n, cap)):
            nm = names.raw[i * name_len:(i + 1) * name_len].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out

    def sync(self, stream=None):
        import torch
        s = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream)
        self._check(self._lib.ws_sync(self._h, s))

    # -- hot path ---------------------------------------------------------
    def gradient(self, img, sigma: float, dtype: str = "u8", out=None, mag=None):
        import torch
        if img.dtype != torch.float32:
            raise TypeError("image must be float32")
        nx, ny, nz = _dims(img.shape)
        if out is None:
            out = torch.empty(img.shape, dtype=torch.uint8 if dtype == "u8" else torch.uint16, device=img.device)
        code = WS_U8 if dtype == "u8" else WS_U16
        self._check(self._lib.ws_gradient(self._h, _dev(img, "image"), nx, ny, nz, float(sigma), code,
                                          _dev(out, "output"), _dev(mag, "mag") if mag is not None else None,
                                          _stream(img)))
        return out

    def watershed(self, grad, conn: int, out=None):
        import torch
        nx, ny, nz = _dims(grad.shape)
        if out is None:
            out = torch.empty(grad.shape, dtype=torch.int32, device=grad.device)
        self._check(self._lib.ws_watershed(self._h, _dev(grad, "gradient"), _grey_code(grad), nx, ny, nz, int(conn),
                                           _dev(out, "labels"), _stream(grad)))
        return out

    def watershed_noalloc(self, grad, conn: int, out):
        """ws_watershed_noalloc: the watershed into the caller's `out` (int32,
        the gradient's shape) using the library's fixed device scratch."""
        import torch
        nx, ny, nz = _dims(grad.shape)
        if out.shape != grad.shape or out.dtype != torch.int32:
            raise ValueError("out must be int32 with the gradient's shape")
        self._check(self._lib.ws_watershed_noalloc(self._h, _dev(grad, "gradient"), _grey_code(grad), nx, ny, nz,
                                                   int(conn), _dev(out, "labels"), _stream(grad)))
        return out

    def watershed_stages(self, grad, conn: int):
        import torch
        nx, ny, nz = _dims(grad.shape)
        bal = torch.empty(grad.shape, dtype=torch.int32, device=grad.device)
        arrow = torch.empty(grad.shape, dtype=torch.int32, device=grad.device)
        self._check(self._lib.ws_watershed_stages(self._h, _dev(grad, "gradient"), _grey_code(grad), nx, ny, nz,
                                                  int(conn), _dev(bal, "bal"), _dev(arrow, "arrow"), _stream(grad)))
        return bal, arrow

    def batch(self, grads, conn, NL: int, outs=None, nregions=None):
        """Watershed + NL-layer waterfall of a list of gradient tensors (same
        dtype; 2D and 3D may be mixed) in one batched call. `conn` is one
        connectivity for every image or a list with one per image. Returns
        (outs, nregions): per image an int32 [NL, *shape] tensor and an int64
        [NL] tensor."""
        import torch
        if not grads:
            raise ValueError("empty batch")
        conns = [int(conn)] * len(grads) if isinstance(conn, int) else [int(c) for c in conn]
        if len(conns) != len(grads):
            raise ValueError("one connectivity per image")
        code = _grey_code(grads[0])
        dev = grads[0].device
        if outs is None:
            outs = [torch.empty((int(NL),) + tuple(g.shape), dtype=torch.int32, device=dev) for g in grads]
        if nregions is None:
            nregions = [torch.zeros(int(NL), dtype=torch.int64, device=dev) for _ in grads]
        items = (WsItem * len(grads))()
        for i, g in enumerate(grads):
            if _grey_code(g) != code:
                raise TypeError("all gradients of a batch must share one dtype")
            nx, ny, nz = _dims(g.shape)
            items[i].grad = _dev(g, "gradient").value
            items[i].nx, items[i].ny, items[i].nz = nx, ny, nz
            items[i].conn = conns[i]
            items[i].out = _dev(outs[i], "out").value
            items[i].nregions = _dev(nregions[i], "nregions").value
        self._check(self._lib.ws_batch(self._h, items, len(grads), code, int(NL), _stream(grads[0])))
        return outs, nregions

    def waterfall(self, labels, grad, conn: int, NL: int, out=None, nregions=None):
        import torch
        nx, ny, nz = _dims(grad.shape)
        if labels.shape != grad.shape or labels.dtype != torch.int32:
            raise ValueError("labels must be int32 with the gradient's shape")
        if out is None:
            out = torch.empty((int(NL),) + tuple(grad.shape), dtype=torch.int32, device=grad.device)
        if nregions is None:
            nregions = torch.zeros(int(NL), dtype=torch.int64, device=grad.device)
        self._check(self._lib.ws_waterfall(self._h, _dev(labels, "labels"), _dev(grad, "gradient"), _grey_code(grad),
                                           nx, ny, nz, int(conn), int(NL), _dev(out, "out"),
                                           _dev(nregions, "nregions"), _stream(grad)))
        return out, nregions

    def rag(self, labels, grad, conn: int):
        """Region adjacency graph of `labels` (ws_rag): int32 tensors (a, b, h),
        a < b canonical labels of adjacent regions, h their lowest pass, sorted
        by (a, b). Two calls: the first returns the edge count only."""
        import torch
        nx, ny, nz = _dims(grad.shape)
        if labels.shape != grad.shape or labels.dtype != torch.int32:
            raise ValueError("labels must be int32 with the gradient's shape")
        n = torch.zeros(1, dtype=torch.int64, device=grad.device)
        args = (_dev(labels, "labels"), _dev(grad, "gradient"), _grey_code(grad), nx, ny, nz, int(conn))
        self._check(self._lib.ws_rag(self._h, *args, 0, None, None, None, _dev(n, "n_edges"), _stream(grad)))
        cnt = int(n.item())
        a, b, h = (torch.empty(max(cnt, 1), dtype=torch.int32, device=grad.device) for _ in range(3))
        self._check(self._lib.ws_rag(self._h, *args, cnt, _dev(a, "a"), _dev(b, "b"), _dev(h, "h"),
                                     _dev(n, "n_edges"), _stream(grad)))
        return a[:cnt], b[:cnt], h[:cnt]

    def waterfall_recon(self, labels, grad, conn: int, NL: int, out=None, nregions=None):
        """Reconstruction waterfall (ws_waterfall_recon): same arguments as waterfall."""
        import torch
        nx, ny, nz = _dims(grad.shape)
        if labels.shape != grad.shape or labels.dtype != torch.int32:
            raise ValueError("labels must be int32 with the gradient's shape")
        if out is None:
            out = torch.empty((int(NL),) + tuple(grad.shape), dtype=torch.int32, device=grad.device)
        if nregions is None:
            nregions = torch.zeros(int(NL), dtype=torch.int64, device=grad.device)
        self._check(self._lib.ws_waterfall_recon(self._h, _dev(labels, "labels"), _dev(grad, "gradient"),
                                                 _grey_code(grad), nx, ny, nz, int(conn), int(NL),
                                                 _dev(out, "out"), _dev(nregions, "nregions"), _stream(grad)))
        return out, nregions


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def ws_gradient(img, sigma, dtype="u8", out=None, mag=None):
    return default_context(img.device.index or 0).gradient(img, sigma, dtype, out=out, mag=mag)


def ws_watershed(grad, conn, out=None):
    return default_context(grad.device.index or 0).watershed(grad, conn, out=out)


def ws_waterfall(labels, grad, conn, NL, out=None, nregions=None):
    return default_context(grad.device.index or 0).waterfall(labels, grad, conn, NL, out=out, nregions=nregions)


def ws_waterfall_recon(labels, grad, conn, NL, out=None, nregions=None):
    return default_context(grad.device.index or 0).waterfall_recon(labels, grad, conn, NL, out=out, nregions=nregions)


def ws_rag(labels, grad, conn):
    return default_context(grad.device.index or 0).rag(labels, grad, conn)


def ws_batch(grads, conn, NL, outs=None, nregions=None):
    return default_context(grads[0].device.index or 0).batch(grads, conn, NL, outs=outs, nregions=nregions)


def ws_watershed_stages(grad, conn):
    return default_context(grad.device.index or 0).watershed_stages(grad, conn)
