"""ctypes binding of libccl's C ABI (argument marshalling only).

Every labeling step runs in the HIP kernels inside ``libccl.so``; torch is
used here only to own device memory and to name the current HIP stream.
If the library has not been built, every call raises ``CclError``.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(PKG, "libccl.so")
_lib = None
_lock = threading.Lock()

CCL_OK = 0


class CclError(RuntimeError):
    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("tile_h", ctypes.c_int32), ("waves", ctypes.c_int32)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("labels", ctypes.c_void_p), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("pitch", ctypes.c_int64)]


class CtxOpts(ctypes.Structure):
    _fields_ = [("max_images", ctypes.c_int32), ("max_pixels", ctypes.c_int64),
                ("cfg", Config), ("use_graph", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("n_workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("max_frame_pixels", ctypes.c_int64), ("max_batch_pixels", ctypes.c_int64),
                ("hbm_budget", ctypes.c_int64), ("connectivity", ctypes.c_int32),
                ("cfg", Config), ("use_graph", ctypes.c_int32), ("plain", ctypes.c_int32)]


class FrameResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("labels", ctypes.c_void_p), ("slot", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_launch_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

# name -> (restype, argtypes); every symbol include/ccl.h declares
SIGNATURES = {
    "ccl_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ccl_last_hip_error": (ctypes.c_int, []),
    "ccl_version": (ctypes.c_int, []),
    "ccl_label_2d": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, _P]),
    "ccl_workspace_size": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(Config),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "ccl_label_2d_ex": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, _P, ctypes.c_size_t,
                                       ctypes.POINTER(Config), _P]),
    "ccl_label_2d_noalloc": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, _P]),
    "ccl_label_2d_timed": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, ctypes.POINTER(Config), _P,
                                          ctypes.POINTER(ctypes.c_float)]),
    "ccl_label_2d_equal": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, ctypes.POINTER(Config), _P]),
    "ccl_component_stats": (ctypes.c_int, [_P, _I32, _I32, _P, _I64, _P, _P]),
    "ccl_label_2d_stats": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, _P, _I64, _P,
                                          ctypes.POINTER(Config), _P]),
    "ccl_label_3d": (ctypes.c_int, [_P, _I32, _I32, _I32, _I64, _I64, _I32, _P, _P]),
    "ccl_shutdown": (None, []),
    "ccl_ctx_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(CtxOpts)]),
    "ccl_ctx_destroy": (ctypes.c_int, [_P]),
    "ccl_label_batch": (ctypes.c_int, [_P, ctypes.POINTER(ImageDesc), _I32, _I32, _P]),
    "ccl_ctx_config": (ctypes.c_int, [_P, _I32, ctypes.POINTER(Config)]),
    "ccl_ctx_autotune": (ctypes.c_int, [_P, ctypes.POINTER(ImageDesc), _I32, _I32, _I32, _P,
                                        ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_float)]),
    "ccl_autotune": (ctypes.c_int, [_P, _I32, _I32, _I64, _I32, _P, _I32, _P, ctypes.POINTER(Config),
                                    ctypes.POINTER(ctypes.c_float)]),
    "ccl_tuning_get": (ctypes.c_int, [_I32, _I32, _I32, ctypes.POINTER(Config)]),
    "ccl_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
    "ccl_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "ccl_tuning_clear": (None, []),
    "ccl_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ServerOpts)]),
    "ccl_server_slots": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "ccl_server_submit": (ctypes.c_int, [_P, _P, _I32, _I32, _I64, ctypes.c_uint64]),
    "ccl_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(FrameResult), _I32, ctypes.POINTER(ctypes.c_int32)]),
    "ccl_server_release": (ctypes.c_int, [_P, _I32]),
    "ccl_server_pending": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "ccl_server_destroy": (ctypes.c_int, [_P]),
}


def library_path() -> str:
    return _LIB_PATH


_hip_rt = None


def _load_hip_runtime():
    """Make a HIP runtime's symbols global before libccl.so is loaded.

    libccl.so does not link a HIP runtime of its own.  When torch is present
    its bundled runtime is the one that owns the tensors and streams handed to
    the library, so that one is used; otherwise the ROCm installation's."""
    global _hip_rt
    if _hip_rt is not None:
        return _hip_rt
    candidates = []
    try:
        import torch

        candidates.append(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    except ImportError:
        pass
    candidates += ["libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"]
    for c in candidates:
        if os.path.sep in c and not os.path.exists(c):
            continue
        try:
            _hip_rt = ctypes.CDLL(c, mode=ctypes.RTLD_GLOBAL)
            return _hip_rt
        except OSError:
            continue
    raise CclError("no HIP runtime (libamdhip64.so) could be loaded")


def load_library():
    """Load libccl.so once; raise CclError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise CclError("libccl.so is not built (expected at %s); run __graft_entry__.build()"
                           % _LIB_PATH)
        _load_hip_runtime()
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != CCL_OK:
        lib = load_library()
        msg = lib.ccl_status_string(rc).decode()
        if rc == 4:
            msg += " (hipError %d)" % lib.ccl_last_hip_error()
        raise CclError("%s failed: %s" % (what, msg), rc)


def _torch():
    import torch

    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _pitch(img) -> int:
    H, W = img.shape
    return int(img.stride(0)) if H > 1 else int(W)


def _check_image(img):
    torch = _torch()
    if not isinstance(img, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if img.dim() != 2:
        raise ValueError("expected a 2D image, got shape %s" % (tuple(img.shape),))
    if img.dtype != torch.uint8:
        raise ValueError("expected uint8 pixels, got %s" % img.dtype)
    if not img.is_cuda:
        raise ValueError("image must be a device (cuda) tensor")
    if img.shape[1] > 1 and img.stride(1) != 1:
        raise ValueError("image rows must be contiguous (stride(1) == 1)")


def _check_out(out, img, shape=None):
    """An output tensor the kernels may write: int32, contiguous, of the
    input's shape and on the input's device.  Returns `out`, or a new tensor
    when it is None."""
    torch = _torch()
    shape = tuple(img.shape) if shape is None else tuple(shape)
    if out is None:
        return torch.empty(shape, dtype=torch.int32, device=img.device)
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a torch.Tensor")
    if tuple(out.shape) != shape or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of shape %s" % (shape,))
    if not out.is_cuda or out.device != img.device:
        raise ValueError("out must be a device tensor on the input's device (%s)" % img.device)
    return out


def label(img, conn: int = 8, out=None, config=None, stream=None, workspace=None):
    """Label a 2D uint8 device image; returns an int32 tensor holding the
    uint32 labels bit for bit (0 = background, else 1 + min raster index)."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    cfg = None
    if config is not None:
        cfg = ctypes.byref(Config(int(config[0]), int(config[1])))
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        if not workspace.is_cuda or workspace.device != img.device or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous device tensor on the input's device")
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    with torch.cuda.device(img.device):
        rc = lib.ccl_label_2d_ex(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                 ws_ptr, ws_bytes, cfg, _stream_handle(stream))
    _check(rc, "ccl_label_2d_ex")
    return out


def label_plain(img, conn: int = 8, out=None, stream=None):
    """The plain ccl_label_2d entry point (library-owned workspace, default tiles)."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    with torch.cuda.device(img.device):
        rc = lib.ccl_label_2d(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                              _stream_handle(stream))
    _check(rc, "ccl_label_2d")
    return out


def label_noalloc(img, conn: int = 8, out=None, stream=None):
    """The ccl_label_2d_noalloc entry point: default tiles, workspace in the
    library's fixed device array (no allocation by the library).  Calls
    whose work overlaps on one device race on that array."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    with torch.cuda.device(img.device):
        rc = lib.ccl_label_2d_noalloc(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                      _stream_handle(stream))
    _check(rc, "ccl_label_2d_noalloc")
    return out


def label_equal(img, conn: int = 8, out=None, config=None, stream=None):
    """Equal-value labeling of a 2D uint8 CUDA tensor (every value class,
    background included): int32 tensor of 1 + the smallest raster index of
    each pixel's equal-valued component."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    cfg = ctypes.byref(Config(int(config[0]), int(config[1]))) if config else None
    with torch.cuda.device(img.device):
        rc = lib.ccl_label_2d_equal(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                    cfg, _stream_handle(stream))
    _check(rc, "ccl_label_2d_equal")
    return out


# Layout of struct ccl_component (include/ccl.h).
COMPONENT_DTYPE = [("label", "<u4"), ("area", "<u4"), ("x_min", "<u4"), ("y_min", "<u4"),
                   ("x_max", "<u4"), ("y_max", "<u4"), ("sum_x", "<u8"), ("sum_y", "<u8")]
COMPONENT_BYTES = 40


def component_stats(labels, capacity: int = None, stream=None):
    """Per-component statistics of a canonical label tensor (int32 CUDA,
    H x W, from label / label_equal): a numpy structured array, one record
    per component in increasing label order.  With capacity None the
    components are counted first (one synchronization) and all returned."""
    import numpy as np

    torch = _torch()
    if not isinstance(labels, torch.Tensor) or labels.dim() != 2 or labels.dtype != torch.int32 \
            or not labels.is_contiguous() or not labels.is_cuda:
        raise ValueError("labels must be a contiguous 2D int32 CUDA tensor")
    H, W = labels.shape
    lib = load_library()
    n_dev = torch.zeros(1, dtype=torch.int32, device=labels.device)
    with torch.cuda.device(labels.device):
        if capacity is None:
            _check(lib.ccl_component_stats(labels.data_ptr(), H, W, None, 0, n_dev.data_ptr(),
                                           _stream_handle(stream)), "ccl_component_stats")
            capacity = int(n_dev.cpu().numpy().view(np.uint32)[0])
        out = torch.empty(max(1, capacity) * COMPONENT_BYTES, dtype=torch.uint8, device=labels.device)
        _check(lib.ccl_component_stats(labels.data_ptr(), H, W, out.data_ptr() if capacity else None,
                                       int(capacity), n_dev.data_ptr(), _stream_handle(stream)),
               "ccl_component_stats")
    n = int(n_dev.cpu().numpy().view(np.uint32)[0])
    rec = out.cpu().numpy()[:min(n, capacity) * COMPONENT_BYTES].view(np.dtype(COMPONENT_DTYPE))
    return rec


def label_stats(img, conn: int = 8, capacity: int = None, out=None, config=None, stream=None):
    """Labels and per-component statistics of a 2D uint8 device image in
    one call (ccl_label_2d_stats): returns (labels int32 tensor, numpy
    structured array of records in increasing label order).  With capacity
    None the image is labeled once to count the components (one
    synchronization), then again with room for all of them."""
    import numpy as np

    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    cfg = ctypes.byref(Config(int(config[0]), int(config[1]))) if config else None
    n_dev = torch.zeros(1, dtype=torch.int32, device=img.device)
    with torch.cuda.device(img.device):
        if capacity is None:
            _check(lib.ccl_label_2d_stats(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                          None, 0, n_dev.data_ptr(), cfg, _stream_handle(stream)),
                   "ccl_label_2d_stats")
            capacity = int(n_dev.cpu().numpy().view(np.uint32)[0])
        recs = torch.empty(max(1, capacity) * COMPONENT_BYTES, dtype=torch.uint8, device=img.device)
        _check(lib.ccl_label_2d_stats(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                      recs.data_ptr() if capacity else None, int(capacity),
                                      n_dev.data_ptr(), cfg, _stream_handle(stream)), "ccl_label_2d_stats")
    n = int(n_dev.cpu().numpy().view(np.uint32)[0])
    rec = recs.cpu().numpy()[:min(n, capacity) * COMPONENT_BYTES].view(np.dtype(COMPONENT_DTYPE))
    return out, rec


def label3d(vol, conn: int = 26, out=None, stream=None):
    """Label a 3D uint8 CUDA tensor (D, H, W) with unit stride along W;
    returns an int32 tensor of 1 + the smallest raster index of each voxel's
    component (0 for background)."""
    torch = _torch()
    if vol.dim() != 3 or vol.dtype != torch.uint8 or not vol.is_cuda or vol.stride(2) != 1:
        raise ValueError("vol must be a 3D uint8 CUDA tensor with unit stride along W")
    D, H, W = vol.shape
    out = _check_out(out, vol)
    pitch_y = vol.stride(1) if H > 1 else W
    pitch_z = vol.stride(0) if D > 1 else H * pitch_y
    lib = load_library()
    with torch.cuda.device(vol.device):
        rc = lib.ccl_label_3d(vol.data_ptr(), D, H, W, pitch_y, pitch_z, int(conn), out.data_ptr(),
                              _stream_handle(stream))
    _check(rc, "ccl_label_3d")
    return out


def label_timed(img, conn: int = 8, out=None, config=None, stream=None):
    """Label and return (labels, [ms_phase1, ms_phase2, ms_phase3]); blocks."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = _check_out(out, img)
    lib = load_library()
    cfg = ctypes.byref(Config(int(config[0]), int(config[1]))) if config else None
    ms = (ctypes.c_float * 3)()
    with torch.cuda.device(img.device):
        rc = lib.ccl_label_2d_timed(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(),
                                    cfg, _stream_handle(stream), ms)
    _check(rc, "ccl_label_2d_timed")
    return out, [float(ms[0]), float(ms[1]), float(ms[2])]


def workspace_size(H: int, W: int, config=None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    cfg = ctypes.byref(Config(int(config[0]), int(config[1]))) if config else None
    _check(lib.ccl_workspace_size(int(H), int(W), cfg, ctypes.byref(n)), "ccl_workspace_size")
    return int(n.value)


def shutdown():
    load_library().ccl_shutdown()


class BatchContext:
    """Owns a ccl_ctx (fixed capacity, device buffers, batch graphs)."""

    def __init__(self, max_images: int, max_pixels: int, config=None, use_graph: bool = True):
        lib = load_library()
        opts = CtxOpts(int(max_images), int(max_pixels),
                       Config(*(config if config else (0, 0))), 1 if use_graph else 0)
        h = ctypes.c_void_p()
        _check(lib.ccl_ctx_create(ctypes.byref(h), ctypes.byref(opts)), "ccl_ctx_create")
        self._h = h
        self.max_images = int(max_images)
        self.max_pixels = int(max_pixels)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(load_library().ccl_ctx_destroy(self._h), "ccl_ctx_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def descs(self, images, outs):
        arr = (ImageDesc * len(images))()
        for k, (img, out) in enumerate(zip(images, outs)):
            _check_image(img)
            H, W = img.shape
            try:
                _check_out(out, img)
            except (TypeError, ValueError) as e:
                raise ValueError("out[%d]: %s" % (k, e)) from None
            arr[k] = ImageDesc(img.data_ptr(), out.data_ptr(), H, W, _pitch(img))
        return arr

    def label(self, images, conn: int = 8, outs=None, stream=None, descs=None):
        """Label a list of 2D uint8 device images in one call; returns the list
        of int32 label tensors (uint32 bits).  `descs` may be a prebuilt
        descriptor array from ``descs()`` for the same tensors."""
        torch = _torch()
        if outs is None:
            outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in images]
        if descs is None:
            descs = self.descs(images, outs)
        rc = load_library().ccl_label_batch(self._h, descs, len(images), int(conn),
                                             _stream_handle(stream))
        _check(rc, "ccl_label_batch")
        return outs

    def config(self, conn: int = 8):
        """(tile_h, waves) the context uses for this connectivity."""
        cfg = Config()
        _check(load_library().ccl_ctx_config(self._h, int(conn), ctypes.byref(cfg)), "ccl_ctx_config")
        return (cfg.tile_h, cfg.waves)

    def autotune(self, images, conn: int = 8, reps: int = 3, outs=None, stream=None):
        """Time every tile configuration on this batch and keep the fastest
        for `conn` (ccl_ctx_autotune); returns ((tile_h, waves), ms per call)."""
        torch = _torch()
        if outs is None:
            outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in images]
        descs = self.descs(images, outs)
        best, ms = Config(), ctypes.c_float()
        _check(load_library().ccl_ctx_autotune(self._h, descs, len(images), int(conn), int(reps),
                                               _stream_handle(stream), ctypes.byref(best), ctypes.byref(ms)),
               "ccl_ctx_autotune")
        return (best.tile_h, best.waves), float(ms.value)


def label_batch(images, conn: int = 8, ctx: BatchContext = None, stream=None):
    """Label several images with one batched call (a context is created when
    none is given)."""
    if ctx is None:
        px = sum(int(im.shape[0]) * int(im.shape[1]) for im in images)
        ctx = BatchContext(max(1, len(images)), max(1, px))
    return ctx.label(images, conn, stream=stream)


def autotune(img, conn: int = 8, reps: int = 5, stream=None):
    """Time every tile configuration on `img`, record the fastest for its size
    class; returns ((tile_h, waves), ms_per_call)."""
    torch = _torch()
    _check_image(img)
    H, W = img.shape
    out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    best = Config(0, 0)
    ms = ctypes.c_float(0.0)
    lib = load_library()
    with torch.cuda.device(img.device):
        rc = lib.ccl_autotune(img.data_ptr(), H, W, _pitch(img), int(conn), out.data_ptr(), int(reps),
                              _stream_handle(stream), ctypes.byref(best), ctypes.byref(ms))
    _check(rc, "ccl_autotune")
    return (best.tile_h, best.waves), float(ms.value)


def tuning_get(H: int, W: int, conn: int = 8):
    c = Config(0, 0)
    _check(load_library().ccl_tuning_get(int(H), int(W), int(conn), ctypes.byref(c)), "ccl_tuning_get")
    return (c.tile_h, c.waves)


def tuning_save(path: str):
    _check(load_library().ccl_tuning_save(os.fsencode(path)), "ccl_tuning_save")


def tuning_load(path: str):
    _check(load_library().ccl_tuning_load(os.fsencode(path)), "ccl_tuning_load")


def tuning_clear():
    load_library().ccl_tuning_clear()


class Server:
    """Owns a ccl_server (request loop with HBM-budget admission and
    continuous batching over several worker streams).  Workers launch their
    batches directly by default: for the few-frame batches a server forms,
    a graph replay measured several microseconds slower per batch."""

    def __init__(self, max_frame_pixels: int, hbm_budget: int, n_workers: int = 2,
                 max_batch: int = 8, max_batch_pixels: int = None, conn: int = 8, config=None,
                 use_graph: bool = False, plain: bool = False):
        lib = load_library()
        if plain:
            n_workers, max_batch = 1, 1
        if max_batch_pixels is None:
            max_batch_pixels = max_frame_pixels * max_batch
        opts = ServerOpts(int(n_workers), int(max_batch), int(max_frame_pixels), int(max_batch_pixels),
                          int(hbm_budget), int(conn), Config(*(config if config else (0, 0))),
                          1 if use_graph else 0, 1 if plain else 0)
        h = ctypes.c_void_p()
        _check(lib.ccl_server_create(ctypes.byref(h), ctypes.byref(opts)), "ccl_server_create")
        self._h = h
        self._buf = (FrameResult * 4096)()
        n = ctypes.c_int32(0)
        _check(lib.ccl_server_slots(self._h, ctypes.byref(n)), "ccl_server_slots")
        self.n_slots = int(n.value)

    def submit(self, img, tag: int):
        """Submit a 2D uint8 device tensor (must stay unchanged until done)."""
        _check_image(img)
        H, W = img.shape
        return load_library().ccl_server_submit(self._h, img.data_ptr(), H, W, _pitch(img), int(tag))

    def poll(self):
        """Finished frames as tuples (tag, labels_ptr, slot, t_submit, t_admit, t_launch, t_done)."""
        n = ctypes.c_int32(0)
        rc = load_library().ccl_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(n))
        out = [(r.tag, r.labels, r.slot, r.t_submit_ns, r.t_admit_ns, r.t_launch_ns, r.t_done_ns)
               for r in self._buf[:n.value]]
        _check(rc, "ccl_server_poll")
        return out

    def release(self, slot: int):
        _check(load_library().ccl_server_release(self._h, int(slot)), "ccl_server_release")

    def pending(self) -> int:
        v = ctypes.c_int64(0)
        _check(load_library().ccl_server_pending(self._h, ctypes.byref(v)), "ccl_server_pending")
        return int(v.value)

    def close(self):
        if self._h:
            rc = load_library().ccl_server_destroy(self._h)
            self._h = None
            _check(rc, "ccl_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
