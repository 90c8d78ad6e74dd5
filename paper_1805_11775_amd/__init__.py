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
HOS_ESCRATCH = -6
HOS_NOALLOC_SCRATCH_BYTES = 128 << 20

HOS_F32 = 0
HOS_F64 = 1
HOS_WIN_NONE = 0
HOS_WIN_PARZEN = 1
HOS_WIN_PARZEN_SEPARABLE = 2
HOS_PATH_FP32 = 0
HOS_PATH_SPLIT_FP16 = 1
HOS_PATH_SPLIT_BF16 = 2
HOS_NO_CENTER = 1
HOS_FULL_SQUARE = 2
HOS_PD_ONLY = 4
HOS_PLAN_ADJOINT = 16
HOS_PLAN_SEGMENTS = 32

PATHS = {"fp32": HOS_PATH_FP32, "split_fp16": HOS_PATH_SPLIT_FP16,
         "split_bf16": HOS_PATH_SPLIT_BF16}
WINDOWS = {"none": HOS_WIN_NONE, "parzen": HOS_WIN_PARZEN,
           "separable": HOS_WIN_PARZEN_SEPARABLE}


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
        "hos_bispectrum_noalloc": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                                  vp, vp, vp]),
        "hos_c3_plan_info": (ctypes.c_int, [i64, i32, i32, p64, i32]),
        "hos_trispectrum_workspace": (ctypes.c_int, [i64, i32, i32, i32, u32,
                                                     ctypes.POINTER(sz)]),
        "hos_trispectrum": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                           vp, vp, vp, sz, vp]),
        "hos_trispectrum_timed": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                                 vp, vp, vp, sz, vp,
                                                 ctypes.POINTER(ctypes.c_float)]),
        "hos_c4_plan_info": (ctypes.c_int, [i64, i32, i32, p64, i32]),
        "hos_c5_plan_info": (ctypes.c_int, [i64, i32, i32, p64, i32]),
        "hos_bispectrum_streamed_workspace": (ctypes.c_int, [i64, i32, i32, i32, i32, i64,
                                                             ctypes.POINTER(sz)]),
        "hos_bispectrum_streamed": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32, i64,
                                                   vp, vp, vp, sz, vp]),
        "hos_cumulant5_workspace": (ctypes.c_int, [i64, i32, i32, i32, u32,
                                                   ctypes.POINTER(sz)]),
        "hos_cumulant5": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                         vp, vp, vp, sz, vp]),
        "hos_cumulant5_timed": (ctypes.c_int, [vp, i32, i64, i32, i32, i32, i32, u32,
                                               vp, vp, vp, sz, vp,
                                               ctypes.POINTER(ctypes.c_float)]),
        "hos_batch_plan_size": (ctypes.c_int, [i32, p64, ctypes.POINTER(ctypes.c_int32), i32,
                                               i32, u32, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "hos_batch_plan": (ctypes.c_int, [i32, p64, ctypes.POINTER(ctypes.c_int32), i32, i32,
                                          u32, ctypes.POINTER(ctypes.c_int32), vp, sz]),
        "hos_batch_plan_info": (ctypes.c_int, [vp, p64, i32]),
        "hos_tune_workspace": (ctypes.c_int, [i32, ctypes.POINTER(ctypes.c_int32), i32, p64, i32,
                                              i32, ctypes.POINTER(sz)]),
        "hos_tune": (ctypes.c_int, [i32, ctypes.POINTER(ctypes.c_int32), i32, p64, i32, i32, i32,
                                    vp, sz, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_float), vp]),
        "hos_mfma_rate": (ctypes.c_int, [i32, i32, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_double), vp]),
        "hos_batch_series": (ctypes.c_int, [vp, p64, i64]),
        "hos_batch_items": (ctypes.c_int, [vp, i32, p64, i64]),
        "hos_bispectrum_batched": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "hos_bispectrum_batched_timed": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, sz, vp,
                                                        ctypes.POINTER(ctypes.c_float)]),
        "hos_bispectrum_loss_fwd": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "hos_bispectrum_segments": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "hos_bispectrum_loss_bwd": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, sz,
                                                   vp]),
        "hos_c3_schedule": (ctypes.c_int, [i64, i32, i32, p64, p64, p64, i64]),
        "hos_dbs_workspace": (ctypes.c_int, [i64, i32, i32, ctypes.POINTER(sz)]),
        "hos_dbs": (ctypes.c_int, [vp, i32, i64, i32, i32, u32, vp, vp, sz, vp]),
        "hos_dbs_timed": (ctypes.c_int, [vp, i32, i64, i32, i32, u32, vp, vp, sz, vp, i32,
                                         i32, ctypes.POINTER(ctypes.c_float)]),
        "hos_dbs_plan_info": (ctypes.c_int, [i64, i32, i32, i32, i32, p64, i32]),
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


def hos_bispectrum_noalloc(x_ptr, dtype, n, M, window, nfft, path, flags, c3_ptr, B_ptr,
                           stream) -> int:
    """Raw call of the non-allocating entry point (the library's fixed
    per-device scratch is the workspace); returns the status code."""
    return lib().hos_bispectrum_noalloc(x_ptr, int(dtype), int(n), int(M), int(window),
                                        int(nfft), int(path), int(flags), c3_ptr, B_ptr,
                                        stream)


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


DBS_INFO_KEYS = ("K", "mode", "P1", "P2", "W", "TW", "NS", "R", "NWG", "SR", "SC", "G",
                 "Kg", "npd", "ws_bytes", "rows")
DBS_STAGES = ("dft", "part_sums", "smooth", "total")


def hos_dbs_plan_info(n, P, M3, seg_rows=0, strip_w=0) -> dict:
    buf = (ctypes.c_int64 * 16)()
    st = lib().hos_dbs_plan_info(int(n), int(P), int(M3), int(seg_rows), int(strip_w), buf, 16)
    if st != HOS_OK:
        raise HosError(st, "hos_dbs_plan_info")
    return dict(zip(DBS_INFO_KEYS, list(buf)))


def hos_dbs_workspace(n, P, M3) -> int:
    out = ctypes.c_size_t(0)
    st = lib().hos_dbs_workspace(int(n), int(P), int(M3), ctypes.byref(out))
    if st != HOS_OK:
        raise HosError(st, "hos_dbs_workspace")
    return out.value


def hos_dbs(x_ptr, dtype, n, P, M3, flags, B_ptr, ws_ptr, ws_bytes, stream) -> int:
    """Raw call; returns the status code (does not raise)."""
    return lib().hos_dbs(x_ptr, int(dtype), int(n), int(P), int(M3), int(flags), B_ptr,
                         ws_ptr, int(ws_bytes), stream)


def hos_dbs_timed(x_ptr, dtype, n, P, M3, flags, B_ptr, ws_ptr, ws_bytes, stream,
                  seg_rows=0, strip_w=0):
    """Raw timed call; returns (status, {stage: milliseconds})."""
    ms = (ctypes.c_float * 4)()
    st = lib().hos_dbs_timed(x_ptr, int(dtype), int(n), int(P), int(M3), int(flags), B_ptr,
                             ws_ptr, int(ws_bytes), stream, int(seg_rows), int(strip_w), ms)
    return st, dict(zip(DBS_STAGES, list(ms)))


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


def pd_count(N: int) -> int:
    """Points of the principal domain 0 <= k2 <= k1, k1 + k2 < N/2."""
    H = (N - 1) // 2
    return sum(min(k1, H - k1) + 1 for k1 in range(H + 1))


def default_nfft(M: int, window: str = "parzen") -> int:
    need = 2 * M if window != "none" else 2 * M + 1
    return _next_fft_size(max(need, 2))


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def mfma_rate(path: str = "split_fp16", iters: int = 1 << 19, device="cuda") -> dict:
    """``hos_mfma_rate``: the matrix cores' attainable rate on ``device``
    (independent 32 x 32 ops, one wave per SIMD; a measurement helper, not a
    step of the estimator).  Returns {"ms", "flops", "tflops"}."""
    import torch
    ms = ctypes.c_float(0.0)
    fl = ctypes.c_double(0.0)
    st = lib().hos_mfma_rate(PATHS[path], int(iters), ctypes.byref(ms), ctypes.byref(fl),
                             _stream_handle(torch.device(device)))
    if st != HOS_OK:
        raise HosError(st, "hos_mfma_rate")
    return {"ms": float(ms.value), "flops": float(fl.value),
            "tflops": float(fl.value) / (float(ms.value) * 1e-3) / 1e12}


def bispectrum(x, M: int, nfft: int | None = None, window: str = "parzen",
               path: str = "fp32", center: bool = True, return_c3: bool = True,
               return_B: bool = True, workspace=None, full_square: bool = False,
               pd_only: bool = False):
    """c3 over |w| <= M ((2M+1)^2 float64; the hexagon, or with
    ``full_square`` every lag of the square) and the windowed 2D DFT B
    (nfft x nfft complex128, or with ``pd_only`` the principal domain,
    packed) of a 1-D float32/float64 CUDA tensor.

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
    flags = (0 if center else HOS_NO_CENTER) | (HOS_FULL_SQUARE if full_square else 0) | \
        (HOS_PD_ONLY if pd_only else 0)
    ws_bytes = hos_bispectrum_workspace(n, M, nfft if return_B else 0, pth, flags)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
    c3 = torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64,
                     device=x.device) if return_c3 else None
    if not return_B:
        B = None
    elif pd_only:
        B = torch.empty(pd_count(nfft), dtype=torch.complex128, device=x.device)
    else:
        B = torch.empty((nfft, nfft), dtype=torch.complex128, device=x.device)
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


def dbs(x, P: int, M3: int, center: bool = True, workspace=None, timed: bool = False,
        seg_rows: int = 0, strip_w: int = 0):
    """The direct method (``hos_dbs``): parts of P samples, an M3 x M3 box.
    Returns the principal domain of the P grid (complex128, row-major in
    (k1, k2)); with ``timed`` also the stage times in ms.  ``seg_rows`` and
    ``strip_w`` are the tuning arguments of ``hos_dbs_timed``."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    n = x.numel()
    info = hos_dbs_plan_info(n, P, M3, seg_rows, strip_w)
    ws_bytes = info["ws_bytes"]
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
    B = torch.empty(info["npd"], dtype=torch.complex128, device=x.device)
    args = (x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32, n, P, M3,
            0 if center else HOS_NO_CENTER, B.data_ptr(), workspace.data_ptr(),
            workspace.numel(), _stream_handle(x.device))
    if timed:
        st, ms = hos_dbs_timed(*args, seg_rows=seg_rows, strip_w=strip_w)
        if st != HOS_OK:
            raise HosError(st, "hos_dbs_timed")
        return B, ms
    if seg_rows or strip_w:
        st, _ = hos_dbs_timed(*args, seg_rows=seg_rows, strip_w=strip_w)
    else:
        st = hos_dbs(*args)
    if st != HOS_OK:
        raise HosError(st, "hos_dbs")
    return B


def hos_bispectrum_streamed_workspace(n, M, nfft, path, dtype, piece) -> int:
    out = ctypes.c_size_t(0)
    st = lib().hos_bispectrum_streamed_workspace(int(n), int(M), int(nfft), int(path),
                                                int(dtype), int(piece), ctypes.byref(out))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_streamed_workspace")
    return out.value


def bispectrum_streamed(x, M: int, piece: int = 1 << 22, nfft: int | None = None,
                        window: str = "parzen", path: str = "fp32", center: bool = True,
                        device="cuda", return_c3: bool = True, return_B: bool = True,
                        workspace=None, full_square: bool = False):
    """``hos_bispectrum_streamed``: c3 and B of a record held in host memory
    (a CPU torch tensor, ideally pinned, or a numpy array), streamed in
    pieces of ``piece`` samples through a device workspace independent of
    n.  Outputs are CUDA tensors on ``device``.  A pinned record is still
    being read by the library's copies when the call returns, so for a
    pinned ``x`` this waits for the stream before returning (the caller's
    tensor may be freed, and its block reused, as soon as it returns)."""
    import numpy as np
    import torch
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    if not isinstance(x, torch.Tensor) or x.is_cuda:
        raise TypeError("x must be a host (CPU) tensor or a numpy array")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    n = x.numel()
    dtype = HOS_F64 if x.dtype == torch.float64 else HOS_F32
    pth, win = PATHS[path], WINDOWS[window]
    if nfft is None:
        nfft = default_nfft(M, window)
    nf = nfft if return_B else 0
    ws_bytes = hos_bispectrum_streamed_workspace(n, M, nf, pth, dtype, piece)
    dev = torch.device(device)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    c3 = torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64,
                     device=dev) if return_c3 else None
    B = torch.empty((nfft, nfft), dtype=torch.complex128, device=dev) if return_B else None
    flags = (0 if center else HOS_NO_CENTER) | (HOS_FULL_SQUARE if full_square else 0)
    st = lib().hos_bispectrum_streamed(
        x.data_ptr(), dtype, n, M, win, nf, pth, flags, int(piece),
        c3.data_ptr() if c3 is not None else None, B.data_ptr() if B is not None else None,
        workspace.data_ptr(), workspace.numel(), _stream_handle(dev))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_streamed")
    if x.is_pinned():
        torch.cuda.current_stream(dev).synchronize()
    return c3, B


STAGES5 = ("prep", "contract", "reduce_fold", "dft", "total")


def hos_c5_plan_info(n, M, path) -> dict:
    buf = (ctypes.c_int64 * 8)()
    st = lib().hos_c5_plan_info(int(n), int(M), int(path), buf, 8)
    if st != HOS_OK:
        raise HosError(st, "hos_c5_plan_info")
    keys = ("P", "RB", "NCB", "WX", "S", "CPS", "C", "ws_bytes")
    return dict(zip(keys, list(buf)))


def cumulant5(x, M: int, nfft: int | None = None, window: str = "parzen", path: str = "fp32",
              center: bool = True, return_c5: bool = True, return_Q: bool = True,
              workspace=None, timed: bool = False):
    """Order five (``hos_cumulant5``): c5 over |t| <= M ((2M+1)^4 float64)
    and its windowed 4-D DFT Q (nfft^4 complex128).  Returns (c5 or None,
    Q or None), and the stage times in ms with ``timed``."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    n = x.numel()
    pth, win = PATHS[path], WINDOWS[window]
    if nfft is None:
        nfft = default_nfft(M, window)
    flags = 0 if center else HOS_NO_CENTER
    out = ctypes.c_size_t(0)
    st = lib().hos_cumulant5_workspace(n, M, nfft if return_Q else 0, pth, flags,
                                      ctypes.byref(out))
    if st != HOS_OK:
        raise HosError(st, "hos_cumulant5_workspace")
    if workspace is None or workspace.numel() < out.value:
        workspace = torch.empty(out.value, dtype=torch.uint8, device=x.device)
    S = 2 * M + 1
    c5 = torch.empty((S, S, S, S), dtype=torch.float64, device=x.device) if return_c5 else None
    Q = torch.empty((nfft,) * 4, dtype=torch.complex128, device=x.device) if return_Q else None
    args = (x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32, n, M, win,
            nfft if return_Q else 0, pth, flags, c5.data_ptr() if c5 is not None else None,
            Q.data_ptr() if Q is not None else None, workspace.data_ptr(), workspace.numel(),
            _stream_handle(x.device))
    if timed:
        ms = (ctypes.c_float * 5)()
        st = lib().hos_cumulant5_timed(*args, ms)
        if st != HOS_OK:
            raise HosError(st, "hos_cumulant5_timed")
        return c5, Q, dict(zip(STAGES5, list(ms)))
    st = lib().hos_cumulant5(*args)
    if st != HOS_OK:
        raise HosError(st, "hos_cumulant5")
    return c5, Q


# ------------------------------------------------------------------ batches
def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


BATCH_INFO_KEYS = ("batch", "c3_elems", "pd_elems", "x_elems", "ws_bytes", "plan_bytes",
                   "items0", "items1", "G0", "G1", "uniform_M", "max_npd")


class BatchPlan:
    """A host-built plan for a batch of series (see ``hos_batch_plan``):
    lengths ``n``, maximum lags ``M``.  Holds the host bytes and, once
    ``to(device)`` has run, an identical device copy."""

    def __init__(self, n, M, window="parzen", path="fp32", center=True, adjoint=False,
                 tile=None, segments=False):
        """``tile``: None (built-in rule), a mapping M -> tile choice (0, 2 or 4,
        e.g. the output of ``tune.tune``), or one choice per series.
        ``segments``: also lay out the buffers of ``bispectrum_segments``."""
        import numpy as np
        self.n = np.ascontiguousarray(np.asarray(n, dtype=np.int64).ravel())
        self.M = np.ascontiguousarray(np.asarray(M, dtype=np.int32).ravel())
        if self.n.size != self.M.size or self.n.size == 0:
            raise ValueError("n and M must be non-empty and of equal length")
        self.window, self.path = window, path
        self.flags = ((0 if center else HOS_NO_CENTER) | (HOS_PLAN_ADJOINT if adjoint else 0) |
                      (HOS_PLAN_SEGMENTS if segments else 0))
        if tile is None:
            self.tile = None
        elif isinstance(tile, dict):
            self.tile = np.ascontiguousarray(
                [int(tile.get(int(m), tile.get(str(int(m)), 0))) for m in self.M], dtype=np.int32)
        else:
            self.tile = np.ascontiguousarray(np.asarray(tile, dtype=np.int32).ravel())
            if self.tile.size != self.n.size:
                raise ValueError("one tile choice per series")
        tp = _i32p(self.tile) if self.tile is not None else None
        pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        st = lib().hos_batch_plan_size(self.n.size, _i64p(self.n), _i32p(self.M),
                                       WINDOWS[window], PATHS[path], self.flags, tp,
                                       ctypes.byref(pb), ctypes.byref(wb))
        if st != HOS_OK:
            raise HosError(st, "hos_batch_plan_size")
        self.host = np.zeros((pb.value + 7) // 8, dtype=np.int64)   # 8-byte aligned bytes
        st = lib().hos_batch_plan(self.n.size, _i64p(self.n), _i32p(self.M), WINDOWS[window],
                                  PATHS[path], self.flags, tp, self.host.ctypes.data, pb.value)
        if st != HOS_OK:
            raise HosError(st, "hos_batch_plan")
        info = np.zeros(12, dtype=np.int64)
        st = lib().hos_batch_plan_info(self.host.ctypes.data, _i64p(info), 12)
        if st != HOS_OK:
            raise HosError(st, "hos_batch_plan_info")
        self.info = dict(zip(BATCH_INFO_KEYS, [int(v) for v in info]))
        self.dev = None
        self._ws = None

    def series(self):
        """Per-series rows: n, M, N, npd, x offset, c3 offset, B offset, class."""
        import numpy as np
        out = np.zeros((self.n.size, 8), dtype=np.int64)
        st = lib().hos_batch_series(self.host.ctypes.data, _i64p(out), out.size)
        if st != HOS_OK:
            raise HosError(st, "hos_batch_series")
        return out

    def items(self, cls):
        """Work items of tile class cls (0: 2 x 2 blocks, 1: 4 x 4 blocks, -1:
        all) in launch order, 8 columns (see hos_batch_items)."""
        import numpy as np
        k = (self.info["items0"] + self.info["items1"]) if cls < 0 else \
            self.info["items%d" % cls]
        out = np.zeros((max(k, 1), 8), dtype=np.int64)
        st = lib().hos_batch_items(self.host.ctypes.data, int(cls), _i64p(out), out.size)
        if st != HOS_OK:
            raise HosError(st, "hos_batch_items")
        return out[:k]

    def to(self, device):
        import torch
        if self.dev is None or self.dev.device != torch.device(device):
            h = torch.from_numpy(self.host.view("uint8"))
            self.dev = h.to(device)
            self._ws = None
        return self

    def workspace(self, device):
        import torch
        if self._ws is None or self._ws.device != torch.device(device):
            self._ws = torch.empty(self.info["ws_bytes"], dtype=torch.uint8, device=device)
        return self._ws


def _check_packed(x, plan):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    if x.numel() != plan.info["x_elems"]:
        raise ValueError("x holds %d samples, the plan %d" % (x.numel(), plan.info["x_elems"]))
    return x


def bispectrum_batched(x, plan: BatchPlan, return_c3=True, return_B=True):
    """Packed c3 blocks and principal-domain spectra of every series of
    ``plan`` (``x`` packed in series order).  Returns (c3 or None, B_pd or
    None) as flat float64 / complex128 tensors."""
    import torch
    x = _check_packed(x, plan)
    plan.to(x.device)
    ws = plan.workspace(x.device)
    c3 = torch.empty(plan.info["c3_elems"], dtype=torch.float64,
                     device=x.device) if return_c3 else None
    B = torch.empty(plan.info["pd_elems"], dtype=torch.complex128,
                    device=x.device) if return_B else None
    st = lib().hos_bispectrum_batched(
        x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32,
        plan.host.ctypes.data, plan.dev.data_ptr(),
        c3.data_ptr() if c3 is not None else None, B.data_ptr() if B is not None else None,
        ws.data_ptr(), ws.numel(), _stream_handle(x.device))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_batched")
    return c3, B


def bispectrum_segments(x, P: int, M: int, window: str = "parzen", path: str = "fp32",
                        center: bool = True, return_c3: bool = True, return_B: bool = True,
                        tile=None, plan: "BatchPlan | None" = None):
    """Segment averaging (``hos_bispectrum_segments``): the first K = n // P
    segments of P samples of a 1-D CUDA tensor, each centred on its own mean,
    their c3 averaged, then windowed and transformed on the N x N grid of the
    plan (N as for ``default_nfft(M, window)``).  Returns (c3 or None, B or
    None).  A ``plan`` from an earlier call with the same arguments may be
    passed back in."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("x must be a CUDA tensor")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    x = x.contiguous().view(-1)
    K = x.numel() // int(P)
    if K < 1:
        raise ValueError("fewer than P samples")
    if plan is None:
        plan = BatchPlan([P] * K, [M] * K, window=window, path=path, center=center, tile=tile,
                         segments=True)
    plan.to(x.device)
    ws = plan.workspace(x.device)
    N = int(plan.series()[0, 2])
    c3 = torch.empty((2 * M + 1, 2 * M + 1), dtype=torch.float64,
                     device=x.device) if return_c3 else None
    B = torch.empty((N, N), dtype=torch.complex128, device=x.device) if return_B else None
    st = lib().hos_bispectrum_segments(
        x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32,
        plan.host.ctypes.data, plan.dev.data_ptr(),
        c3.data_ptr() if c3 is not None else None, B.data_ptr() if B is not None else None,
        ws.data_ptr(), ws.numel(), _stream_handle(x.device))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_segments")
    return c3, B


BATCH_STAGES = ("prep", "contract", "reduce", "spectra", "total")


def bispectrum_batched_timed(x, plan: BatchPlan, return_c3=False):
    """Like ``bispectrum_batched`` (principal-domain spectra always); also
    returns {stage: milliseconds} measured with HIP events (waits)."""
    import torch
    x = _check_packed(x, plan)
    plan.to(x.device)
    ws = plan.workspace(x.device)
    c3 = torch.empty(plan.info["c3_elems"], dtype=torch.float64,
                     device=x.device) if return_c3 else None
    B = torch.empty(plan.info["pd_elems"], dtype=torch.complex128, device=x.device)
    ms = (ctypes.c_float * 5)()
    st = lib().hos_bispectrum_batched_timed(
        x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32,
        plan.host.ctypes.data, plan.dev.data_ptr(),
        c3.data_ptr() if c3 is not None else None, B.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream_handle(x.device), ms)
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_batched_timed")
    return c3, B, dict(zip(BATCH_STAGES, list(ms)))


def bispectrum_loss_fwd(x, target_pd, plan: BatchPlan):
    """(loss as a 0-d float64 tensor, B_pd) for packed x."""
    import torch
    x = _check_packed(x, plan)
    plan.to(x.device)
    ws = plan.workspace(x.device)
    target_pd = target_pd.to(device=x.device, dtype=torch.complex128).contiguous()
    B = torch.empty(plan.info["pd_elems"], dtype=torch.complex128, device=x.device)
    loss = torch.empty((), dtype=torch.float64, device=x.device)
    st = lib().hos_bispectrum_loss_fwd(
        x.data_ptr(), HOS_F64 if x.dtype == torch.float64 else HOS_F32, plan.host.ctypes.data,
        plan.dev.data_ptr(), target_pd.data_ptr(), B.data_ptr(), loss.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream_handle(x.device))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_loss_fwd")
    return loss, B


def bispectrum_loss_bwd(x, target_pd, B_pd, dL, plan: BatchPlan):
    """dL * dLoss/dx for packed x (same dtype and shape as x)."""
    import torch
    xf = _check_packed(x, plan)
    plan.to(xf.device)
    ws = plan.workspace(xf.device)
    target_pd = target_pd.to(device=xf.device, dtype=torch.complex128).contiguous()
    dL = dL.to(device=xf.device, dtype=torch.float64).contiguous().reshape(())
    dx = torch.empty_like(xf)
    st = lib().hos_bispectrum_loss_bwd(
        xf.data_ptr(), HOS_F64 if xf.dtype == torch.float64 else HOS_F32,
        plan.host.ctypes.data, plan.dev.data_ptr(), B_pd.data_ptr(), target_pd.data_ptr(),
        dL.data_ptr(), dx.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(xf.device))
    if st != HOS_OK:
        raise HosError(st, "hos_bispectrum_loss_bwd")
    return dx.view_as(x)


def _loss_function():
    import torch

    class BispectrumLoss(torch.autograd.Function):
        """L(x) = sum over series and principal-domain frequencies of
        |B(x_s) - target|^2, with the hand-written adjoint as backward."""

        @staticmethod
        def forward(ctx, x, target_pd, plan):
            loss, B = bispectrum_loss_fwd(x, target_pd, plan)
            ctx.save_for_backward(x, target_pd, B)
            ctx.plan = plan
            return loss

        @staticmethod
        def backward(ctx, grad):
            x, target_pd, B = ctx.saved_tensors
            return bispectrum_loss_bwd(x, target_pd, B, grad, ctx.plan), None, None

    return BispectrumLoss


_LOSS_FN = None


def bispectrum_loss(x, target_pd, plan: BatchPlan):
    """Differentiable loss of a (batch, n) or packed tensor ``x`` (plan made
    with ``adjoint=True``)."""
    global _LOSS_FN
    if _LOSS_FN is None:
        _LOSS_FN = _loss_function()
    return _LOSS_FN.apply(x, target_pd, plan)
