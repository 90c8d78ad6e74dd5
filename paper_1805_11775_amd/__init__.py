"""Python binding of ``libhos.so``, the gfx950 higher-order-spectra library.

Argument marshalling only: every step of the estimator runs in the HIP
kernels behind the C ABI declared in ``include/hos.h``.  PyTorch provides
device memory (tensors) and the stream; nothing here computes on the CPU,
and there is no fallback -- importing fails loudly when the library is not
built, and every non-OK status raises ``HosError``.

Two layers:

* the raw C entry points under their C names (the library is loaded on
  first use, so building never needs an already-built copy) (``hos_bispectrum``, ...),
  taking integer device addresses;
* ``bispectrum(x, M, ...)`` / ``trispectrum(x, M, ...)``: allocate the
  outputs and the workspace as torch tensors on ``x.device`` and call
  ``hos_bispectrum`` / ``hos_trispectrum`` on the current stream.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HOS_LIB_PATH selects another build of the library (e.g. a variant under test).
LIB_PATH = os.environ.get("HOS_LIB_PATH", os.path.join(_HERE, "libhos.so"))

HOS_OK = 0
HOS_EINVAL = -1
HOS_EWORKSPACE = -2
HOS_EDEVICE = -3
HOS_ENODEVICE = -4
HOS_EUNSUPPORTED = -5

HOS_F32 = 0
HOS_F64 = 1
HOS_WIN_NONE = 0
HOS_WIN_PARZEN = 1
HOS_PATH_FP32 = 0
HOS_PATH_SPLIT_FP16 = 1
HOS_PATH_SPLIT_BF16 = 2
HOS_NO_CENTER = 1

PATHS = {"fp32": HOS_PATH_FP32, "split_fp16": HOS_PATH_SPLIT_FP16,
         "split_bf16": HOS_PATH_SPLIT_BF16}
WINDOWS = {"none": HOS_WIN_NONE, "parzen": HOS_WIN_PARZEN}


class HosError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, hos_strerror(status), status))


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libhos.so is not built (%s); run `python -m paper_1805_11775_amd.build`"
            % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    p64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "hos_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "hos_version": (ctypes.c_int, []),
        "hos_device_check": (ctypes.c_int, []),
        "hos_bispectrum_workspace": (ctypes.c_int, [i64, i32, i32, i32, u32,
                                                    ctypes.POINTER(sz)]),
        "hos_bispectrum": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                          vp, vp, vp, sz, vp]),
        "hos_bispectrum_timed": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                                vp, vp, vp, sz, vp,
                                                ctypes.POINTER(ctypes.c_float)]),
        "hos_c3_plan_info": (ctypes.c_int, [i64, i32, i32, p64, i32]),
        "hos_trispectrum_workspace": (ctypes.c_int, [i64, i32, i32, i32, u32,
                                                     ctypes.POINTER(sz)]),
        "hos_trispectrum": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                           vp, vp, vp, sz, vp]),
        "hos_trispectrum_timed": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                                 vp, vp, vp, sz, vp,
                                                 ctypes.POINTER(ctypes.c_float)]),
        "hos_c4_plan_info": (ctypes.c_int, [i64, i32, i32, p64, i32]),
        "hos_c3_schedule": (ctypes.c_int, [i64, i32, i32, p64, p64, p64, i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    """The loaded libhos.so (loaded on first use; raises if missing/stale)."""
    global _lib
    if _lib is None:
        _lib = _load_lib()
    return _lib


# ---------------------------------------------------------------- raw C ABI
def hos_strerror(status: int) -> str:
    return lib().hos_strerror(int(status)).decode()


def hos_version() -> int:
    return lib().hos_version()


def hos_device_check() -> int:
    return lib().hos_device_check()


def hos_bispectrum_workspace(n, M, nfft, path, flags=0) -> int:
    out = ctypes.c_size_t(0)
    st = lib().hos_bispectrum_workspace(int(n), int(M), int(nfft), int(path), int(flags),
                                       ctypes.byref(out))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_workspace")
    return out.value


def hos_bispectrum(x_ptr, dtype, n, M, window, nfft, path, flags, c3_ptr, B_ptr,
                   ws_ptr, ws_bytes, stream) -> int:
    """Raw call; returns the status code (does not raise)."""
    return lib().hos_bispectrum(x_ptr, int(dtype), int(n), int(M), int(window), int(nfft),
                               int(path), int(flags), c3_ptr, B_ptr, ws_ptr,
                               int(ws_bytes), stream)


STAGES = ("moments", "prep", "contract", "diag_dot", "reduce", "finish", "dft", "total")


def hos_bispectrum_timed(x_ptr, dtype, n, M, window, nfft, path, flags, c3_ptr, B_ptr,
                         ws_ptr, ws_bytes, stream):
    """Raw timed call; returns (status, {stage: milliseconds})."""
    ms = (ctypes.c_float * 8)()
    st = lib().hos_bispectrum_timed(x_ptr, int(dtype), int(n), int(M), int(window),
                                   int(nfft), int(path), int(flags), c3_ptr, B_ptr, ws_ptr,
                                   int(ws_bytes), stream, ms)
    return st, dict(zip(STAGES, list(ms)))


def hos_c3_plan_info(n, M, path) -> dict:
    buf = (ctypes.c_int64 * 10)()
    st = lib().hos_c3_plan_info(int(n), int(M), int(path), buf, 10)
    if st != HOS_OK:
        raise HosError(st, "hos_c3_plan_info")
    keys = ("G", "smax", "TR", "C", "NB", "NBR", "nleft", "npad", "ctot", "ws_bytes")
    return dict(zip(keys, list(buf)))


def hos_c3_schedule(n, M, path):
    """(owner, slot, rslot) lists over every (tile, chunk) of the plan."""
    info = hos_c3_plan_info(n, M, path)
    cap = info["TR"] * (info["TR"] + 1) // 2 * info["C"]
    arrs = [(ctypes.c_int64 * max(cap, 1))() for _ in range(3)]
    st = lib().hos_c3_schedule(int(n), int(M), int(path), arrs[0], arrs[1], arrs[2], cap)
    if st != HOS_OK:
        raise HosError(st, "hos_c3_schedule")
    return tuple(list(a)[:cap] for a in arrs)


def hos_trispectrum_workspace(n, M, nfft, path, flags=0) -> int:
    out = ctypes.c_size_t(0)
    st = lib().hos_trispectrum_workspace(int(n), int(M), int(nfft), int(path), int(flags),
                                        ctypes.byref(out))
    if st != HOS_OK:
        raise HosError(st, "hos_trispectrum_workspace")
    return out.value


def hos_trispectrum(x_ptr, dtype, n, M, window, nfft, path, flags, c4_ptr, T_ptr,
                    ws_ptr, ws_bytes, stream) -> int:
    """Raw call; returns the status code (does not raise)."""
    return lib().hos_trispectrum(x_ptr, int(dtype), int(n), int(M), int(window), int(nfft),
                                int(path), int(flags), c4_ptr, T_ptr, ws_ptr,
                                int(ws_bytes), stream)


STAGES4 = ("moments", "prep", "contract", "reduce", "finish", "dft", "total")


def hos_trispectrum_timed(x_ptr, dtype, n, M, window, nfft, path, flags, c4_ptr, T_ptr,
                          ws_ptr, ws_bytes, stream):
    """Raw timed call; returns (status, {stage: milliseconds})."""
    ms = (ctypes.c_float * 7)()
    st = lib().hos_trispectrum_timed(x_ptr, int(dtype), int(n), int(M), int(window),
                                    int(nfft), int(path), int(flags), c4_ptr, T_ptr, ws_ptr,
                                    int(ws_bytes), stream, ms)
    return st, dict(zip(STAGES4, list(ms)))


def hos_c4_plan_info(n, M, path) -> dict:
    buf = (ctypes.c_int64 * 8)()
    st = lib().hos_c4_plan_info(int(n), int(M), int(path), buf, 8)
    if st != HOS_OK:
        raise HosError(st, "hos_c4_plan_info")
    keys = ("P", "RB", "NCB", "WX", "S", "CPS", "C", "ws_bytes")
    return dict(zip(keys, list(buf)))


# ------------------------------------------------------------- torch layer
def _next_fft_size(m: int) -> int:
    k = max(2, int(m))
    while True:
        r = k
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return k
        k += 1


def default_nfft(M: int, window: str = "parzen") -> int:
    need = 2 * M if window == "parzen" else 2 * M + 1
    return _next_fft_size(max(need, 2))


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def bispectrum(x, M: int, nfft: int | None = None, window: str = "parzen",
               path: str = "fp32", center: bool = True, return_c3: bool = True,
               return_B: bool = True, workspace=None):
    """c3 over |w| <= M ((2M+1)^2 float64) and the windowed 2D DFT B
    (nfft x nfft complex128) of a 1-D float32/float64 CUDA tensor.

    Returns (c3 or None, B or None).  ``workspace`` may be a uint8 CUDA
    tensor of at least ``hos_bispectrum_workspace`` bytes to reuse.
    """
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    n = x.numel()
    pth = PATHS[path]
    win = WINDOWS[window]
    if nfft is None:
        nfft = default_nfft(M, window)
    flags = 0 if center else HOS_NO_CENTER
    ws_bytes = hos_bispectrum_workspace(n, M, nfft if return_B else 0, pth, flags)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
    c3 = torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64,
                     device=x.device) if return_c3 else None
    B = torch.empty((nfft, nfft), dtype=torch.complex128,
                    device=x.device) if return_B else None
    st = hos_bispectrum(x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32,
                        n, M, win, nfft if return_B else 0, pth, flags,
                        c3.data_ptr() if c3 is not None else None,
                        B.data_ptr() if B is not None else None,
                        workspace.data_ptr(), workspace.numel(), _stream_handle(x.device))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum")
    return c3, B


def trispectrum(x, M: int, nfft: int | None = None, window: str = "parzen",
                path: str = "fp32", center: bool = True, return_c4: bool = True,
                return_T: bool = True, workspace=None):
    """c4 over |t| <= M ((2M+1)^3 float64) and the windowed 3D DFT T
    (nfft^3 complex128) of a 1-D float32/float64 CUDA tensor.

    Returns (c4 or None, T or None).  ``workspace`` may be a uint8 CUDA
    tensor of at least ``hos_trispectrum_workspace`` bytes to reuse.
    """
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    n = x.numel()
    pth = PATHS[path]
    win = WINDOWS[window]
    if nfft is None:
        nfft = default_nfft(M, window)
    flags = 0 if center else HOS_NO_CENTER
    ws_bytes = hos_trispectrum_workspace(n, M, nfft if return_T else 0, pth, flags)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
    S = 2 * M + 1
    c4 = torch.empty((S, S, S), dtype=torch.float64,
                     device=x.device) if return_c4 else None
    T = torch.empty((nfft, nfft, nfft), dtype=torch.complex128,
                    device=x.device) if return_T else None
    st = hos_trispectrum(x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32,
                         n, M, win, nfft if return_T else 0, pth, flags,
                         c4.data_ptr() if c4 is not None else None,
                         T.data_ptr() if T is not None else None,
                         workspace.data_ptr(), workspace.numel(), _stream_handle(x.device))
    if st != HOS_OK:
        raise HosError(st, "hos_trispectrum")
    return c4, T
