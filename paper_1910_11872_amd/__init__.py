"""Python binding of libbosmusic (sliding-window root-MUSIC demodulation).

Thin ctypes marshalling over the C ABI declared in ``include/bosmusic.h``:
the functions below carry the ABI's names and pass plain device pointers,
sizes and a HIP stream.  PyTorch is used only for device memory and the
current stream; every step of the computation runs in the HIP kernels of
``libbosmusic.so``.  There is no CPU fallback: if the library cannot be
loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_uint32, c_uint64, c_void_p
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbosmusic.so")

BM_OK, BM_E_INVALID_ARG, BM_E_UNSUPPORTED, BM_E_NOMEM, BM_E_DEVICE = 0, -1, -2, -3, -4
BM_F16, BM_F32, BM_F64, BM_C32, BM_U8 = 1, 2, 3, 4, 5
BM_DIR_X, BM_DIR_Y, BM_BLOCK = 1, 2, 4
BM_PLAIN, BM_SURROGATE = 0, 1
BM_OPT_STATS = 1
BM_OPT_TIMING = 2
BM_OPT_JACOBI = 4
BM_OPT_GRAPH = 8
BM_OPT_FULL_ROOTS = 16
BM_FLAG_UNDEFINED, BM_FLAG_NO_POLISH, BM_FLAG_DEGENERATE = 1, 2, 4

ABI_FUNCTIONS = ("bosmusic_create", "bosmusic_destroy", "bosmusic_demodulate", "bosmusic_integrate",
                 "bosmusic_autotune", "bosmusic_get_stats", "bosmusic_status_string", "bosmusic_last_error",
                 "bosmusic_version", "bosmusic_surrogate_load", "bosmusic_surrogate_save",
                 "bosmusic_surrogate_config", "bosmusic_surrogate_forward", "bosmusic_surrogate_dataset",
                 "bosmusic_surrogate_grad", "bosmusic_surrogate_step", "bosmusic_surrogate_train",
                 "bosmusic_integrate_many", "bosmusic_integrate_noalloc", "bosmusic_surrogate_get_state",
                 "bosmusic_surrogate_set_state")
MLP_PARAMS = 6402


class bosmusic_config(ctypes.Structure):
    _fields_ = [("device", c_int32), ("max_width", c_int32), ("max_height", c_int32), ("options", c_uint32),
                ("max_batch_pixels", c_int64), ("tune_cache", c_char_p)]


class bosmusic_frame(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("dtype", c_int32), ("width", c_int32), ("height", c_int32),
                ("row_stride", c_int64), ("L", c_int32), ("N", c_int32), ("dirs", c_uint32),
                ("omega_x", c_void_p), ("omega_y", c_void_p), ("flags", c_void_p), ("phase", c_void_p),
                ("prev_omega_x", c_void_p), ("prev_omega_y", c_void_p)]


class bosmusic_integrate_job(ctypes.Structure):
    _fields_ = [("omega_x", c_void_p), ("omega_y", c_void_p), ("width", c_int32), ("height", c_int32),
                ("Nx", c_int32), ("Ny", c_int32), ("carrier_x", c_double), ("carrier_y", c_double),
                ("phi", c_void_p)]


class bosmusic_stats(ctypes.Structure):
    _fields_ = [("windows", c_uint64), ("eig_iters", c_uint64), ("root_iters", c_uint64),
                ("polish_fail", c_uint64), ("sur_accepted", c_uint64), ("sur_rejected", c_uint64),
                ("pair_iters", c_uint64), ("rm_launches", c_uint64), ("rm_time_ns", c_uint64),
                ("pair_iters32", c_uint64), ("power_windows", c_uint64)]


class BosmusicError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"bosmusic status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """Load libbosmusic.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1910_11872_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.bosmusic_create.argtypes = [POINTER(bosmusic_config), POINTER(c_void_p)]
        L.bosmusic_create.restype = c_int32
        L.bosmusic_destroy.argtypes = [c_void_p]
        L.bosmusic_destroy.restype = c_int32
        L.bosmusic_demodulate.argtypes = [c_void_p, POINTER(bosmusic_frame), c_int32, c_int32, c_void_p]
        L.bosmusic_demodulate.restype = c_int32
        L.bosmusic_integrate.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                         c_double, c_double, c_void_p, c_void_p]
        L.bosmusic_integrate.restype = c_int32
        L.bosmusic_autotune.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, POINTER(c_double), c_void_p]
        L.bosmusic_autotune.restype = c_int32
        L.bosmusic_get_stats.argtypes = [c_void_p, POINTER(bosmusic_stats), c_int32, c_void_p]
        L.bosmusic_get_stats.restype = c_int32
        L.bosmusic_surrogate_load.argtypes = [c_void_p, c_void_p, c_int64]
        L.bosmusic_surrogate_load.restype = c_int32
        L.bosmusic_surrogate_save.argtypes = [c_void_p, c_void_p, c_int64]
        L.bosmusic_surrogate_save.restype = c_int32
        L.bosmusic_surrogate_get_state.argtypes = [c_void_p, c_void_p, c_int64, POINTER(c_int64)]
        L.bosmusic_surrogate_get_state.restype = c_int32
        L.bosmusic_surrogate_set_state.argtypes = [c_void_p, c_void_p, c_int64, c_int64]
        L.bosmusic_surrogate_set_state.restype = c_int32
        L.bosmusic_surrogate_config.argtypes = [c_void_p, ctypes.c_float, c_int32]
        L.bosmusic_surrogate_config.restype = c_int32
        L.bosmusic_surrogate_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
        L.bosmusic_surrogate_forward.restype = c_int32
        L.bosmusic_integrate_noalloc.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                                 c_double, c_double, c_void_p, c_void_p]
        L.bosmusic_integrate_noalloc.restype = c_int32
        L.bosmusic_integrate_many.argtypes = [c_void_p, POINTER(bosmusic_integrate_job), c_int32, c_void_p]
        L.bosmusic_integrate_many.restype = c_int32
        L.bosmusic_surrogate_dataset.argtypes = [c_void_p, c_int64, c_int64, ctypes.c_uint64, c_void_p, c_void_p,
                                                 c_void_p, c_void_p]
        L.bosmusic_surrogate_dataset.restype = c_int32
        L.bosmusic_surrogate_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
        L.bosmusic_surrogate_grad.restype = c_int32
        L.bosmusic_surrogate_step.argtypes = [c_void_p, c_void_p, ctypes.c_float, c_void_p]
        L.bosmusic_surrogate_step.restype = c_int32
        L.bosmusic_surrogate_train.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int32,
                                               ctypes.c_float, c_void_p, c_void_p]
        L.bosmusic_surrogate_train.restype = c_int32
        L.bosmusic_status_string.argtypes = [c_int32]
        L.bosmusic_status_string.restype = c_char_p
        L.bosmusic_last_error.argtypes = [c_void_p]
        L.bosmusic_last_error.restype = c_char_p
        L.bosmusic_version.argtypes = []
        L.bosmusic_version.restype = c_int32
        _lib = L
    return _lib


def _check(st, h=None):
    if st != BM_OK:
        detail = lib().bosmusic_last_error(h).decode()
        raise BosmusicError(st, f"{lib().bosmusic_status_string(st).decode()}: {detail}")


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    m = {torch.float16: BM_F16, torch.float32: BM_F32, torch.float64: BM_F64, torch.complex64: BM_C32,
         torch.uint8: BM_U8}
    if t.dtype not in m:
        raise TypeError(f"unsupported frame dtype {t.dtype}")
    return m[t.dtype]


# ----------------------------------------------------------------------------
# ABI-named wrappers
# ----------------------------------------------------------------------------
def bosmusic_version() -> int:
    return lib().bosmusic_version()


def bosmusic_status_string(st: int) -> str:
    return lib().bosmusic_status_string(st).decode()


def bosmusic_last_error(h=None) -> str:
    return lib().bosmusic_last_error(h).decode()


def bosmusic_create(device: int = 0, max_width: int = 4096, max_height: int = 4096, options: int = 0,
                    max_batch_pixels: int = 0, tune_cache: str | None = None):
    cfg = bosmusic_config(device, max_width, max_height, options, max_batch_pixels,
                          tune_cache.encode() if tune_cache else None)
    h = c_void_p()
    _check(lib().bosmusic_create(byref(cfg), byref(h)), None)
    return h


def bosmusic_destroy(h) -> None:
    _check(lib().bosmusic_destroy(h), None)


@dataclass
class FrameSpec:
    """One frame: a (H, W) device tensor and its outputs (device tensors or None)."""
    data: object
    L: int
    N: int
    dirs: int
    omega_x: object = None
    omega_y: object = None
    flags: object = None
    phase: object = None
    prev_omega_x: object = None   # temporal warm start: the previous frame's maps
    prev_omega_y: object = None


def _device_check(tensors, device) -> None:
    """Every buffer the C ABI touches is device memory of the handle's GPU: refuse host
    tensors and tensors on another device (a kernel would fault or read the wrong memory)."""
    for t, name in tensors:
        if t is None:
            continue
        if t.device.type != "cuda":
            raise ValueError(f"{name}: need a GPU (cuda) tensor, got one on {t.device}")
        if device is not None and t.device != device:
            raise ValueError(f"{name}: on {t.device}, the frame is on {device}")


def _marshal(f: FrameSpec) -> bosmusic_frame:
    """Frame descriptor of the C ABI.  The kernels store 4-byte omega and phase values and
    1-byte flags row-major with row stride = width, so any other dtype, shape, layout or
    device is refused here (a float16 map would take out-of-bounds stores)."""
    import torch
    d = f.data
    if d.dim() != 2 or d.stride(1) != 1:
        raise ValueError("frame must be a 2-D tensor with unit column stride")
    code = _dtype_code(d)
    H, W = d.shape
    for out, name, dt in ((f.omega_x, "omega_x", torch.float32), (f.omega_y, "omega_y", torch.float32),
                          (f.flags, "flags", torch.uint8), (f.phase, "phase", torch.float32),
                          (f.prev_omega_x, "prev_omega_x", torch.float32),
                          (f.prev_omega_y, "prev_omega_y", torch.float32)):
        if out is None:
            continue
        if tuple(out.shape) != (H, W) or out.dtype != dt or not out.is_contiguous():
            raise ValueError(f"{name}: need a contiguous {dt} tensor of shape {(H, W)}, "
                             f"got {out.dtype} {tuple(out.shape)} strides {out.stride()}")
    _device_check([(d, "frame")], None)
    _device_check([(f.omega_x, "omega_x"), (f.omega_y, "omega_y"), (f.flags, "flags"), (f.phase, "phase"),
                   (f.prev_omega_x, "prev_omega_x"), (f.prev_omega_y, "prev_omega_y")], d.device)
    ptr = lambda t: c_void_p(t.data_ptr()) if t is not None else c_void_p()
    return bosmusic_frame(c_void_p(d.data_ptr()), code, W, H, d.stride(0), f.L, f.N, f.dirs,
                          ptr(f.omega_x), ptr(f.omega_y), ptr(f.flags), ptr(f.phase),
                          ptr(f.prev_omega_x), ptr(f.prev_omega_y))


def bosmusic_demodulate(h, frames, mode: int = BM_PLAIN, stream=None) -> None:
    arr = (bosmusic_frame * len(frames))(*[_marshal(f) for f in frames])
    _check(lib().bosmusic_demodulate(h, arr, len(frames), mode, _stream_ptr(stream)), h)


def _map_check(omega_x, omega_y, phi) -> None:
    """The C ABI reads and writes the maps row-major with row stride = width: refuse
    tensors laid out otherwise (a transposed view would be read in the wrong order)."""
    import torch
    H, W = omega_x.shape
    for t, name, dt in ((omega_x, "omega_x", torch.float32), (omega_y, "omega_y", torch.float32),
                        (phi, "phi", torch.float64)):
        if t is None:
            continue
        if tuple(t.shape) != (H, W) or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous {dt} tensor of shape {(H, W)}, "
                             f"got {t.dtype} {tuple(t.shape)} strides {t.stride()}")
    _device_check([(omega_x, "omega_x")], None)
    _device_check([(omega_y, "omega_y"), (phi, "phi")], omega_x.device)


def bosmusic_integrate(h, omega_x, omega_y, Nx: int, Ny: int, carrier_x: float, carrier_y: float, phi,
                       stream=None) -> None:
    _map_check(omega_x, omega_y, phi)
    H, W = omega_x.shape
    wy = c_void_p(omega_y.data_ptr()) if omega_y is not None else c_void_p()
    _check(lib().bosmusic_integrate(h, c_void_p(omega_x.data_ptr()), wy, W, H, Nx, Ny, carrier_x, carrier_y,
                                    c_void_p(phi.data_ptr()), _stream_ptr(stream)), h)


def bosmusic_integrate_noalloc(omega_x, omega_y, Nx: int, Ny: int, carrier_x: float, carrier_y: float, phi,
                               stream=None) -> None:
    """bosmusic_integrate without a handle and without any allocation, on the current device
    (the maps' device must be current); height <= BOSMUSIC_NOALLOC_MAX_HEIGHT."""
    _map_check(omega_x, omega_y, phi)
    H, W = omega_x.shape
    wy = c_void_p(omega_y.data_ptr()) if omega_y is not None else c_void_p()
    _check(lib().bosmusic_integrate_noalloc(c_void_p(omega_x.data_ptr()), wy, W, H, Nx, Ny, carrier_x, carrier_y,
                                            c_void_p(phi.data_ptr()), _stream_ptr(stream)), None)


def bosmusic_autotune(h, L: int, N: int, width: int = 1024, lines: int = 512, stream=None) -> float:
    """Tune the root-MUSIC launch for (L, N); returns the best time in microseconds."""
    us = c_double(0.0)
    _check(lib().bosmusic_autotune(h, L, N, width, lines, byref(us), _stream_ptr(stream)), h)
    return us.value


def init_params(seed: int = 0):
    """Seeded starting weights for training: W ~ N(0, 1/fan_in), b ~ N(0, 0.01), flat FP32."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((32, (32, 64)), (0, (64,)), (64, (64, 64)), (0, (64,)), (64, (64, 2)), (0, (2,))):
        z = rng.standard_normal(shape)
        parts.append((z / np.sqrt(fan_in) if fan_in else 0.1 * z).astype(np.float32).reshape(-1))
    return np.concatenate(parts)


def _flat_params(params):
    import numpy as np
    if isinstance(params, dict):
        params = np.concatenate([np.asarray(params[k], np.float32).reshape(-1)
                                 for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    a = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if a.size != MLP_PARAMS:
        raise ValueError(f"need {MLP_PARAMS} parameters, got {a.size}")
    return a


def bosmusic_surrogate_load(h, params) -> None:
    """params: flat FP32 array (W1, b1, W2, b2, W3, b3 row-major) or a dict of them."""
    a = _flat_params(params)
    _check(lib().bosmusic_surrogate_load(h, a.ctypes.data_as(c_void_p), a.size), h)


def bosmusic_surrogate_save(h):
    import numpy as np
    a = np.empty(MLP_PARAMS, np.float32)
    _check(lib().bosmusic_surrogate_save(h, a.ctypes.data_as(c_void_p), a.size), h)
    return a


def bosmusic_surrogate_get_state(h):
    """(state, adam_step): FP32 parameters, Adam first and second moments (3 x MLP_PARAMS)."""
    import numpy as np
    a = np.empty(3 * MLP_PARAMS, np.float32)
    step = c_int64(0)
    _check(lib().bosmusic_surrogate_get_state(h, a.ctypes.data_as(c_void_p), a.size, byref(step)), h)
    return a, int(step.value)


def bosmusic_surrogate_set_state(h, state, adam_step: int) -> None:
    import numpy as np
    a = np.ascontiguousarray(state, dtype=np.float32).reshape(-1)
    if a.size != 3 * MLP_PARAMS:
        raise ValueError(f"need {3 * MLP_PARAMS} state values, got {a.size}")
    _check(lib().bosmusic_surrogate_set_state(h, a.ctypes.data_as(c_void_p), a.size, int(adam_step)), h)


def bosmusic_surrogate_config(h, tau: float = 0.25, predictor: int = 0) -> None:
    _check(lib().bosmusic_surrogate_config(h, tau, predictor), h)


def bosmusic_surrogate_forward(h, X, Y, stream=None) -> None:
    """Y[M, 2] = MLP(X[M, 32]); X, Y contiguous FP32 device tensors."""
    _buf_check([(X, "X", (X.shape[0], 32)), (Y, "Y", (X.shape[0], 2))])
    _check(lib().bosmusic_surrogate_forward(h, c_void_p(X.data_ptr()), c_void_p(Y.data_ptr()), X.shape[0],
                                            _stream_ptr(stream)), h)


def bosmusic_integrate_many(h, maps, stream=None) -> None:
    """maps: iterable of (omega_x, omega_y or None, Nx, Ny, carrier_x, carrier_y, phi) device tensors."""
    items = list(maps)
    arr = (bosmusic_integrate_job * max(1, len(items)))()
    for i, (wx, wy, nx, ny, cx, cy, phi) in enumerate(items):
        _map_check(wx, wy, phi)
        H, W = wx.shape
        arr[i] = bosmusic_integrate_job(c_void_p(wx.data_ptr()), c_void_p(wy.data_ptr() if wy is not None else None),
                                        W, H, nx, ny, cx, cy, c_void_p(phi.data_ptr()))
    _check(lib().bosmusic_integrate_many(h, arr, len(items), _stream_ptr(stream)), h)


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(None)


def _buf_check(items) -> None:
    """Surrogate buffers: contiguous FP32 device tensors of the stated shapes, all on
    the first one's device (None entries are optional buffers left out)."""
    import torch
    dev = None
    for t, name, shape in items:
        if t is None:
            continue
        if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: need a contiguous torch.float32 tensor of shape {tuple(shape)}, "
                             f"got {t.dtype} {tuple(t.shape)} strides {t.stride()}")
        _device_check([(t, name)], dev)
        dev = t.device


def bosmusic_surrogate_dataset(h, first_line: int, X, T, omega=None, seed: int = 0, stream=None) -> None:
    """Fill X[M, 32], T[M, 2] (and omega[M]) with training lines first_line .. first_line+M-1."""
    M = X.shape[0]
    _buf_check([(X, "X", (M, 32)), (T, "T", (M, 2)), (omega, "omega", (M,))])
    _check(lib().bosmusic_surrogate_dataset(h, first_line, X.shape[0], seed, _ptr(X), _ptr(T), _ptr(omega),
                                            _stream_ptr(stream)), h)


def bosmusic_surrogate_grad(h, X, T, grad, loss=None, stream=None) -> None:
    M = X.shape[0]
    _buf_check([(X, "X", (M, 32)), (T, "T", (M, 2)), (grad, "grad", (MLP_PARAMS,)), (loss, "loss", (1,))])
    _check(lib().bosmusic_surrogate_grad(h, _ptr(X), _ptr(T), X.shape[0], _ptr(grad), _ptr(loss),
                                         _stream_ptr(stream)), h)


def bosmusic_surrogate_step(h, grad, lr: float, stream=None) -> None:
    _buf_check([(grad, "grad", (MLP_PARAMS,))])
    _check(lib().bosmusic_surrogate_step(h, _ptr(grad), lr, _stream_ptr(stream)), h)


def bosmusic_surrogate_train(h, X, T, batch: int, steps: int, lr: float, want_losses: bool = True, stream=None):
    """Minibatch Adam over (X, T); returns the per-step losses (host) when want_losses."""
    import numpy as np
    _buf_check([(X, "X", (X.shape[0], 32)), (T, "T", (X.shape[0], 2))])
    losses = np.empty(max(steps, 1), np.float32) if want_losses else None
    _check(lib().bosmusic_surrogate_train(h, _ptr(X), _ptr(T), X.shape[0], batch, steps, lr,
                                          losses.ctypes.data_as(c_void_p) if want_losses else c_void_p(None),
                                          _stream_ptr(stream)), h)
    return losses[:steps] if want_losses else None


def bosmusic_get_stats(h, reset: bool = False, stream=None) -> dict:
    s = bosmusic_stats()
    _check(lib().bosmusic_get_stats(h, byref(s), int(reset), _stream_ptr(stream)), h)
    return {k: getattr(s, k) for k, _ in bosmusic_stats._fields_}


# ----------------------------------------------------------------------------
# Convenience wrapper: owns a handle, allocates output maps
# ----------------------------------------------------------------------------
class Demodulator:
    def __init__(self, device: int = 0, max_width: int = 4096, max_height: int = 4096, stats: bool = False,
                 timing: bool = False, jacobi: bool = False, graph: bool = False, max_batch_pixels: int = 0,
                 tune_cache: str | None = None, full_roots: bool = False):
        self.device = device
        self.h = bosmusic_create(device, max_width, max_height,
                                 (BM_OPT_STATS if stats else 0) | (BM_OPT_TIMING if timing else 0) |
                                 (BM_OPT_JACOBI if jacobi else 0) | (BM_OPT_GRAPH if graph else 0) |
                                 (BM_OPT_FULL_ROOTS if full_roots else 0),
                                 max_batch_pixels, tune_cache)

    def close(self):
        if self.h is not None and self.h.value:
            bosmusic_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def demodulate(self, frame, L: int, N: int, dirs: str = "xy", flags: bool = False, stream=None,
                   mode: int = BM_PLAIN, block: bool = False, phase: bool = False):
        """Returns (omega_x or None, omega_y or None[, flags][, phase]) for one device frame.

        block=True: the paper's L x L block window (N must equal L); phase=True
        (block windows, both directions) also returns the wrapped block phase."""
        import torch
        H, W = frame.shape
        d = (BM_DIR_X if "x" in dirs else 0) | (BM_DIR_Y if "y" in dirs else 0) | (BM_BLOCK if block else 0)
        wx = torch.empty((H, W), dtype=torch.float32, device=frame.device) if "x" in dirs else None
        wy = torch.empty((H, W), dtype=torch.float32, device=frame.device) if "y" in dirs else None
        fl = torch.empty((H, W), dtype=torch.uint8, device=frame.device) if flags else None
        ph = torch.empty((H, W), dtype=torch.float32, device=frame.device) if phase else None
        bosmusic_demodulate(self.h, [FrameSpec(frame, L, N, d, wx, wy, fl, ph)], mode, stream)
        out = (wx, wy)
        if flags:
            out += (fl,)
        if phase:
            out += (ph,)
        return out

    def demodulate_many(self, specs, stream=None):
        bosmusic_demodulate(self.h, specs, BM_PLAIN, stream)

    def integrate(self, omega_x, omega_y, Nx: int, Ny: int = 0, carrier_x: float = 0.0, carrier_y: float = 0.0,
                  stream=None):
        import torch
        H, W = omega_x.shape
        phi = torch.empty((H, W), dtype=torch.float64, device=omega_x.device)
        bosmusic_integrate(self.h, omega_x, omega_y, Nx, Ny, carrier_x, carrier_y, phi, stream)
        return phi

    def stats(self, reset: bool = False, stream=None) -> dict:
        return bosmusic_get_stats(self.h, reset, stream)

    def autotune(self, L: int, N: int, width: int = 1024, lines: int = 512, stream=None) -> float:
        return bosmusic_autotune(self.h, L, N, width, lines, stream)
