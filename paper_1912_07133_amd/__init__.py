"""MI355X (gfx950) blob-detection filter bank of Kennedy, "Digital filters with
vanishing moments for shape analysis" (arXiv:1912.07133).

Thin Python binding of the C ABI in include/fdvm.h (libfdvm.so, built in-tree
by ``paper_1912_07133_amd.build``).  Every step of the filter bank runs in the
library's HIP kernels; this module only marshals arguments: PyTorch provides
device memory and the current stream.  There is no CPU fallback -- importing
works without the library, but every call raises if it is not built.
"""

from __future__ import annotations

import ctypes
import functools
import os
import re
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdvm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fdvm.h")

# enums (include/fdvm.h)
OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EOVERFLOW, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
IIR_REPEATED_POLE, FIR_COLORED_SG, FIR_GAUSSIAN, IIR_REPEATED_POLE_DSIGMA, IIR_BUTTERWORTH = 0, 1, 2, 3, 4
FIR_COLORED_SG_DSIGMA, FIR_GAUSSIAN_DSIGMA = 5, 6
# `order` of the IIR calls: 2 or 3 (repeated pole, Filter D) or BUTTERWORTH
# (the L_B = 4 Butterworth blur, Filter E)
BUTTERWORTH = "butterworth"
BC_REPLICATE, BC_ZERO = 0, 1
U16, F32, F16, BF16 = 0, 1, 2, 3
FIR_DIRECT, FIR_TOEPLITZ_MFMA, FIR_TOEPLITZ_MFMA_HALF = 0, 1, 2
HP_LAPLACIAN, HP_D20, HP_D02, HP_D11, HP_D10, HP_D01 = 1, 2, 4, 8, 16, 32
(OP_BLUR_IIR, OP_BLUR_FIR, OP_DETECT, OP_IIR_LAPLACIAN, OP_BLUR_IIR_ADJOINT, OP_PLANE_DOTS, OP_IIR_HESSIAN,
 OP_FIR_LAPLACIAN, OP_IIR_LAPLACIAN_BACKWARD, OP_FIR_LAPLACIAN_BACKWARD, OP_FIR_LAPLACIAN_MFMA) = range(11)
MAX_FIR_LAP_MFMA_HALF = 511
GRAD_X, GRAD_SIGMA = 1, 2
MAX_SCALES = 16
MAX_FIR_HALF = 512

KINDS = {"iir": IIR_REPEATED_POLE, "butterworth": IIR_BUTTERWORTH, "sg": FIR_COLORED_SG,
         "colored_sg": FIR_COLORED_SG, "gaussian": FIR_GAUSSIAN}
# the sigma derivative of each FIR design
FIR_DSIGMA = {FIR_COLORED_SG: FIR_COLORED_SG_DSIGMA, FIR_GAUSSIAN: FIR_GAUSSIAN_DSIGMA}
BOUNDARIES = {"replicate": BC_REPLICATE, "zero": BC_ZERO}


class FdvmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Filter(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("p", ctypes.c_double), ("b0", ctypes.c_double), ("bp", ctypes.c_double * 4),
                ("ap", ctypes.c_double * 4), ("side_gain", ctypes.c_double),
                ("omega_c", ctypes.c_double), ("ntaps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Blob(ctypes.Structure):
    _fields_ = [("y", ctypes.c_int32), ("x", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("polarity", ctypes.c_int32), ("value", ctypes.c_float)]


class Frame(ctypes.Structure):
    """fdvm_frame: one frame of a batch (device pointers)."""
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("row_chunk", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("count", ctypes.c_void_p), ("cap", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


BLOB_BYTES = ctypes.sizeof(Blob)
MAX_LANES = 16
BLOB_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32), ("polarity", np.int32),
                       ("value", np.float32)])
_lib = None


def library_available() -> bool:
    return os.path.exists(LIB_PATH)


def lib() -> ctypes.CDLL:
    """The loaded libfdvm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_1912_07133_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.fdvm_status_string.restype = ctypes.c_char_p
        L.fdvm_status_string.argtypes = [ctypes.c_int]
        L.fdvm_filter_design.restype = ctypes.c_int
        L.fdvm_filter_design.argtypes = [ctypes.c_int, ctypes.c_int, dbl, ctypes.c_int,
                                         ctypes.POINTER(Filter), ctypes.POINTER(dbl), ctypes.c_int]
        L.fdvm_workspace_bytes.restype = ctypes.c_size_t
        L.fdvm_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, ctypes.c_int, ctypes.c_int]
        L.fdvm_blur_iir.restype = ctypes.c_int
        L.fdvm_blur_iir.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64,
                                    ctypes.POINTER(Filter), ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fdvm_iir_laplacian.restype = ctypes.c_int
        L.fdvm_iir_laplacian.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64,
                                         ctypes.POINTER(Filter), ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fdvm_iir_pass.restype = ctypes.c_int
        L.fdvm_iir_pass.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, vp, i64, i64,
                                    ctypes.POINTER(Filter), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                    ctypes.c_size_t, vp]
        L.fdvm_blur_fir.restype = ctypes.c_int
        L.fdvm_blur_fir.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64,
                                    ctypes.POINTER(dbl), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fdvm_fir_laplacian.restype = ctypes.c_int
        L.fdvm_fir_laplacian.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64, vp, ctypes.POINTER(i32),
                                         ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.c_int, ctypes.c_int, vp,
                                         ctypes.c_size_t, vp]
        L.fdvm_fir_laplacian_mfma.restype = ctypes.c_int
        L.fdvm_fir_laplacian_mfma.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64, ctypes.POINTER(dbl),
                                              ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                              ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fdvm_highpass.restype = ctypes.c_int
        L.fdvm_highpass.argtypes = [vp, i64, i64, i64, i64, ctypes.c_int, ctypes.POINTER(dbl),
                                    ctypes.c_uint, ctypes.c_int, vp, i64, vp]
        L.fdvm_detect_blobs.restype = ctypes.c_int
        L.fdvm_detect_blobs.argtypes = [vp, i64, i64, i64, i64, ctypes.c_int, ctypes.c_float,
                                        ctypes.c_int, vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.fdvm_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.fdvm_noalloc_scratch_bytes.argtypes = []
        L.fdvm_detect_blobs_noalloc.restype = ctypes.c_int
        L.fdvm_detect_blobs_noalloc.argtypes = [vp, i64, i64, i64, i64, ctypes.c_int, ctypes.c_float,
                                                ctypes.c_int, vp, i32, vp, vp]
        L.fdvm_iir_hessian.restype = ctypes.c_int
        L.fdvm_iir_hessian.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64, ctypes.POINTER(Filter),
                                       ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_int, vp,
                                       i32, vp, vp, ctypes.c_size_t, vp]
        L.fdvm_blur_iir_adjoint.restype = ctypes.c_int
        L.fdvm_blur_iir_adjoint.argtypes = [vp, i64, i64, i64, i64, vp, i64, i64, ctypes.POINTER(Filter),
                                            ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fdvm_laplacian_adjoint.restype = ctypes.c_int
        L.fdvm_laplacian_adjoint.argtypes = [vp, i64, i64, i64, i64, ctypes.c_int, ctypes.POINTER(dbl), vp, i64,
                                             i64, vp]
        L.fdvm_plane_dots.restype = ctypes.c_int
        L.fdvm_plane_dots.argtypes = [vp, vp, i64, i64, i64, i64, ctypes.c_int, vp, vp, ctypes.c_size_t, vp]
        bwd = [vp, ctypes.c_int, i64, i64, i64, i64, vp, vp, i64, i64, i64, ctypes.c_int]
        tail = [ctypes.c_int, ctypes.c_uint, vp, i64, i64, vp, vp, ctypes.c_size_t, vp]
        L.fdvm_iir_laplacian_backward.restype = ctypes.c_int
        L.fdvm_iir_laplacian_backward.argtypes = bwd + [ctypes.POINTER(Filter), ctypes.c_int] + tail
        L.fdvm_fir_laplacian_backward.restype = ctypes.c_int
        L.fdvm_fir_laplacian_backward.argtypes = bwd + [ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                                        ctypes.POINTER(i32), ctypes.POINTER(i32),
                                                        ctypes.POINTER(dbl), ctypes.c_int] + tail
        L.fdvm_batch_workspace_bytes.restype = ctypes.c_size_t
        L.fdvm_batch_workspace_bytes.argtypes = [ctypes.POINTER(Frame), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.fdvm_batch_detect.restype = ctypes.c_int
        L.fdvm_batch_detect.argtypes = [ctypes.POINTER(Frame), ctypes.c_int, ctypes.POINTER(Filter), ctypes.c_int,
                                        ctypes.c_int, ctypes.c_float, ctypes.c_int, ctypes.c_int, vp,
                                        ctypes.c_size_t, vp]
        _lib = L
    return _lib


def header_symbols() -> list:
    """Entry points declared in include/fdvm.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(fdvm_[a-z_]+)\s*\(", text)))


def status_string(status: int) -> str:
    if _lib is None and not library_available():
        return "library not built"
    return lib().fdvm_status_string(status).decode()


def _check(status: int, what: str):
    if status != OK:
        raise FdvmError(status, what)


# ------------------------------------------------------------------ design

def filter_design(kind: str | int, sigma: float, order: int = 3, fir_half_len: int = 0) -> dict:
    """fdvm_filter_design.  Returns a dict with the DE coefficients (IIR) or the
    taps h(-K..K) (FIR) as float64."""
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    f = Filter()
    cap = 2 * MAX_FIR_HALF + 1
    taps = (ctypes.c_double * cap)()
    _check(lib().fdvm_filter_design(k, order, float(sigma), int(fir_half_len), ctypes.byref(f), taps, cap),
           "fdvm_filter_design")
    out = {"kind": f.kind, "order": f.order, "sigma": f.sigma, "p": f.p, "b0": f.b0,
           "bp": list(f.bp), "ap": list(f.ap), "side_gain": f.side_gain, "omega_c": f.omega_c,
           "ntaps": f.ntaps, "_struct": f}
    if f.ntaps:
        out["taps"] = np.array(taps[: f.ntaps], dtype=np.float64)
    return out


def workspace_bytes(op: int, H: int, W: int, nscales: int, max_half_len: int = 0) -> int:
    return int(lib().fdvm_workspace_bytes(op, H, W, nscales, max_half_len))


# ------------------------------------------------------------------ device calls

def _torch():
    import torch
    return torch


def _stream_ptr(device) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype in (torch.uint16, torch.int16):
        return U16
    if t.dtype == torch.float16:
        return F16
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported image dtype {t.dtype}")


def _frame(x):
    torch = _torch()
    if not x.is_cuda:
        raise ValueError("frame must be a CUDA (HIP) tensor")
    if x.dim() != 2:
        raise ValueError("frame must be [H, W]")
    if x.stride(1) != 1:
        x = x.contiguous()
    return x


def _workspace(op, H, W, S, device, workspace=None, max_half=0):
    torch = _torch()
    need = workspace_bytes(op, H, W, S, max_half)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    return workspace


def blur_iir(x, sigmas: Sequence[float], order: int = 3, boundary: str = "replicate", out=None, workspace=None):
    """Repeated-pole IIR blur (fdvm_blur_iir): [H, W] -> float32 [S, H, W]."""
    torch = _torch()
    x = _frame(x)
    H, W = x.shape
    S = len(sigmas)
    filt = iir_designs(sigmas, order)
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    ws = _workspace(OP_BLUR_IIR, H, W, S, x.device, workspace)
    _check(lib().fdvm_blur_iir(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(), out.stride(1),
                               out.stride(0), filt, S, BOUNDARIES[boundary], ws.data_ptr(), ws.numel(),
                               _stream_ptr(x.device)), "fdvm_blur_iir")
    return out


def iir_laplacian(x, sigmas: Sequence[float], order: int = 3, boundary: str = "replicate", out=None,
                  workspace=None):
    """Blur + normalised Laplacian in one call (fdvm_iir_laplacian):
    [H, W] -> float32 V [S, H, W]."""
    torch = _torch()
    x = _frame(x)
    H, W = x.shape
    S = len(sigmas)
    filt = iir_designs(sigmas, order)
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    ws = _workspace(OP_IIR_LAPLACIAN, H, W, S, x.device, workspace)
    _check(lib().fdvm_iir_laplacian(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(),
                                    out.stride(1), out.stride(0), filt, S, BOUNDARIES[boundary], ws.data_ptr(),
                                    ws.numel(), _stream_ptr(x.device)), "fdvm_iir_laplacian")
    return out


def iir_designs(sigmas: Sequence[float], order: int = 3, dsigma: bool = False):
    """ctypes array of fdvm_filter designs, one per scale (fdvm_filter_design);
    order 2 or 3: repeated pole; BUTTERWORTH: the L_B = 4 Butterworth blur;
    dsigma: the sigma derivatives of the (repeated-pole) blurs instead.
    Designs are pure functions of their arguments and the library only reads
    them, so the arrays are memoised (callers must not modify them)."""
    return _iir_designs_cached(tuple(float(s) for s in sigmas), order, bool(dsigma))


@functools.lru_cache(maxsize=128)
def _iir_designs_cached(sigmas, order, dsigma):
    if order == BUTTERWORTH:
        if dsigma:
            raise FdvmError(EUNSUPPORTED, "sigma derivative of the Butterworth blur")
        kind, order = IIR_BUTTERWORTH, 4
    else:
        kind = IIR_REPEATED_POLE_DSIGMA if dsigma else IIR_REPEATED_POLE
    filt = (Filter * len(sigmas))()
    for i, s in enumerate(sigmas):
        _check(lib().fdvm_filter_design(kind, order, s, 0, ctypes.byref(filt[i]), None, 0), "fdvm_filter_design")
    return filt


def iir_pass(x, sigmas: Sequence[float], axis: int, order: int = 3, boundary: str = "replicate", out=None,
             workspace=None, dsigma: bool = False):
    """One pass of the IIR blur (fdvm_iir_pass).  axis 0: frame [H, W] ->
    [S, H, W] filtered along x; axis 1: planes [S, H, W] (float32) filtered
    along y (out may be the input itself); axis 2: as 1, then the normalised
    Laplacian.  dsigma (axes 0, 1): apply d h / d sigma instead of h."""
    torch = _torch()
    S = len(sigmas)
    filt = iir_designs(sigmas, order, dsigma)
    if axis == 0:
        x = _frame(x)
        H, W = x.shape
        in_plane = 0
        dt = _dtype_code(x)
        pitch = x.stride(0)
    else:
        if x.dtype != torch.float32 or x.dim() != 3 or x.stride(2) != 1:
            raise ValueError("axes 1, 2 need float32 planes [S, H, W] with unit x stride")
        _, H, W = x.shape
        in_plane, pitch, dt = x.stride(0), x.stride(1), F32
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    ws = _workspace(OP_BLUR_IIR, H, W, S, x.device, workspace)
    _check(lib().fdvm_iir_pass(x.data_ptr(), dt, H, W, pitch, in_plane, out.data_ptr(), out.stride(1),
                               out.stride(0), filt, S, BOUNDARIES[boundary], axis, ws.data_ptr(), ws.numel(),
                               _stream_ptr(x.device)), "fdvm_iir_pass")
    return out


def fir_taps(kind: str, sigmas: Sequence[float], half_lens: Sequence[int] | None = None):
    """Designs for fdvm_blur_fir: (taps float64 concatenated, half_len, offsets)."""
    taps, half, off = [], [], []
    pos = 0
    for i, s in enumerate(sigmas):
        K = 0 if half_lens is None else int(half_lens[i])
        d = filter_design(kind, s, fir_half_len=K)
        taps.append(d["taps"])
        half.append(d["order"])
        off.append(pos)
        pos += d["ntaps"]
    return np.concatenate(taps), np.array(half, dtype=np.int32), np.array(off, dtype=np.int32)


def blur_fir(x, sigmas: Sequence[float], kind: str = "sg", half_lens: Sequence[int] | None = None,
             boundary: str = "replicate", algo: int = FIR_DIRECT, out=None, workspace=None, taps=None):
    """FIR blur (fdvm_blur_fir): [H, W] -> float32 [S, H, W].  `taps` may be a
    precomputed (taps, half_len, offsets) triple (e.g. from fir_taps)."""
    torch = _torch()
    x = _frame(x)
    H, W = x.shape
    S = len(sigmas)
    t, half, off = taps if taps is not None else fir_taps(kind, sigmas, half_lens)
    t = np.ascontiguousarray(t, dtype=np.float64)
    half = np.ascontiguousarray(half, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.int32)
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    need = workspace_bytes(OP_BLUR_FIR, H, W, S, int(half.max()))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    _check(lib().fdvm_blur_fir(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(), out.stride(1),
                               out.stride(0), t.ctypes.data_as(dp), half.ctypes.data_as(ip),
                               off.ctypes.data_as(ip), S, BOUNDARIES[boundary], algo, workspace.data_ptr(),
                               workspace.numel(), _stream_ptr(x.device)), "fdvm_blur_fir")
    return out


def fir_taps_device(kind: str, sigmas: Sequence[float], half_lens: Sequence[int] | None, device):
    """(taps on `device` as float64, half_len, offsets) for fdvm_fir_laplacian;
    designs are pure functions of their arguments, so the device copies are
    memoised per device (callers must not modify them)."""
    key = (kind, tuple(float(s) for s in sigmas), None if half_lens is None else tuple(int(k) for k in half_lens),
           str(device))
    hit = _DEVICE_TAPS.get(key)
    if hit is None:
        torch = _torch()
        t, half, off = fir_taps(kind, sigmas, half_lens)
        hit = (torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(device),
               np.ascontiguousarray(half, dtype=np.int32), np.ascontiguousarray(off, dtype=np.int32))
        _DEVICE_TAPS[key] = hit
    return hit


_DEVICE_TAPS: dict = {}


def fir_laplacian(x, sigmas: Sequence[float], kind: str = "sg", half_lens: Sequence[int] | None = None,
                  boundary: str = "replicate", out=None, workspace=None, algo: int = FIR_DIRECT, taps=None):
    """FIR blur + normalised Laplacian in one call: [H, W] -> float32 V [S, H, W].
    algo FIR_DIRECT: fdvm_fir_laplacian (float64 passes); FIR_TOEPLITZ_MFMA_HALF:
    fdvm_fir_laplacian_mfma (matrix cores, half-precision operand pairs; float16,
    bfloat16 or uint16 frames), `taps` optionally a precomputed fir_taps triple."""
    torch = _torch()
    x = _frame(x)
    H, W = x.shape
    S = len(sigmas)
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    sig = (ctypes.c_double * S)(*[float(s) for s in sigmas])
    ip = ctypes.POINTER(ctypes.c_int32)
    if algo == FIR_TOEPLITZ_MFMA_HALF:
        t, half, off = taps if taps is not None else fir_taps(kind, sigmas, half_lens)
        t = np.ascontiguousarray(t, dtype=np.float64)
        half = np.ascontiguousarray(half, dtype=np.int32)
        off = np.ascontiguousarray(off, dtype=np.int32)
        ws = _workspace(OP_FIR_LAPLACIAN_MFMA, H, W, S, x.device, workspace)
        _check(lib().fdvm_fir_laplacian_mfma(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(),
                                             out.stride(1), out.stride(0),
                                             t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             half.ctypes.data_as(ip), off.ctypes.data_as(ip), sig, S,
                                             BOUNDARIES[boundary], ws.data_ptr(), ws.numel(),
                                             _stream_ptr(x.device)), "fdvm_fir_laplacian_mfma")
        return out
    if algo != FIR_DIRECT:
        raise ValueError("fir_laplacian: algo FIR_DIRECT or FIR_TOEPLITZ_MFMA_HALF")
    taps, half, off = fir_taps_device(kind, sigmas, half_lens, x.device)
    ws = _workspace(OP_FIR_LAPLACIAN, H, W, S, x.device, workspace)
    _check(lib().fdvm_fir_laplacian(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(), out.stride(1),
                                    out.stride(0), taps.data_ptr(), half.ctypes.data_as(ip), off.ctypes.data_as(ip),
                                    sig, S, BOUNDARIES[boundary], ws.data_ptr(), ws.numel(), _stream_ptr(x.device)),
           "fdvm_fir_laplacian")
    return out


def highpass(blur, sigmas: Sequence[float], what: int = HP_LAPLACIAN, normalize: bool = True, out=None):
    """fdvm_highpass on float32 planes [S, H, W] -> [S, nout, H, W] (nout =
    number of bits in `what`; squeezed to [S, H, W] when nout == 1)."""
    torch = _torch()
    if blur.dim() == 2:
        blur = blur[None]
    blur = blur.contiguous()  # output planes share the input pitch
    S, H, W = blur.shape
    nout = bin(what).count("1")
    if out is None:
        out = torch.empty((S, nout, H, W), dtype=torch.float32, device=blur.device)
    sig = (ctypes.c_double * S)(*[float(s) for s in sigmas])
    _check(lib().fdvm_highpass(blur.data_ptr(), H, W, blur.stride(1), blur.stride(0), S, sig, what,
                               1 if normalize else 0, out.data_ptr(), out.stride(1), _stream_ptr(blur.device)),
           "fdvm_highpass")
    return out[:, 0] if nout == 1 else out


def detect_blobs(resp, tau: float, border: int = 1, cap: int = 1 << 20, workspace=None, count_only=False):
    """fdvm_detect_blobs on float32 planes [S, H, W].  Returns an int/float
    numpy structured array (y, x, scale, polarity, value) in (scale, y, x)
    order.  Raises FdvmError(EOVERFLOW) if more than `cap` detections."""
    torch = _torch()
    if resp.dim() == 2:
        resp = resp[None]
    resp = resp.contiguous()
    S, H, W = resp.shape
    dev = resp.device
    buf = torch.empty(max(cap, 1) * BLOB_BYTES, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_bytes(OP_DETECT, H, W, S)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().fdvm_detect_blobs(resp.data_ptr(), H, W, resp.stride(1), resp.stride(0), S, float(tau),
                                   int(border), buf.data_ptr(), int(cap), cnt.data_ptr(), workspace.data_ptr(),
                                   workspace.numel(), _stream_ptr(dev)), "fdvm_detect_blobs")
    n = int(cnt.item())
    if n > cap:
        raise FdvmError(EOVERFLOW, f"fdvm_detect_blobs: {n} detections > cap {cap}")
    if count_only:
        return n
    raw = buf[: n * BLOB_BYTES].cpu().numpy()
    dt = np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32), ("polarity", np.int32),
                   ("value", np.float32)])
    return raw.view(dt).copy()


def detect(frame, sigmas: Sequence[float], tau: float, kind: str = "iir", order: int = 3,
           boundary: str = "replicate", border: int = 1, cap: int = 1 << 20):
    """The whole filter bank: blur (IIR or FIR) fused with the normalised
    Laplacian -> multi-scale extrema.  Returns (blob list, Laplacian planes)."""
    if kind == "iir":
        V = iir_laplacian(frame, sigmas, order=order, boundary=boundary)
    else:
        V = fir_laplacian(frame, sigmas, kind=kind, boundary=boundary)
    return detect_blobs(V, tau, border, cap), V


def iir_hessian(x, sigmas: Sequence[float], t1: float, t2: float | None = None, border: int = 1, order: int = 3,
                boundary: str = "replicate", cap: int = 1 << 20):
    """The Hessian blob detector (fdvm_iir_hessian): returns (blob list,
    sigma^4 |H| planes [S, H, W]).  t2 None disables Threshold #2."""
    torch = _torch()
    x = _frame(x)
    H, W = x.shape
    S = len(sigmas)
    out = torch.empty((S, H, W), dtype=torch.float32, device=x.device)
    filt = iir_designs(sigmas, order)
    ws = _workspace(OP_IIR_HESSIAN, H, W, S, x.device)
    buf = torch.empty(max(cap, 1) * BLOB_BYTES, dtype=torch.uint8, device=x.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=x.device)
    _check(lib().fdvm_iir_hessian(x.data_ptr(), _dtype_code(x), H, W, x.stride(0), out.data_ptr(), out.stride(1),
                                  out.stride(0), filt, S, BOUNDARIES[boundary], float(t1),
                                  float(t2) if t2 is not None else 0.0, int(border), buf.data_ptr(), int(cap),
                                  cnt.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(x.device)),
           "fdvm_iir_hessian")
    n = int(cnt.item())
    if n > cap:
        raise FdvmError(EOVERFLOW, f"fdvm_iir_hessian: {n} detections > cap {cap}")
    return buf[: n * BLOB_BYTES].cpu().numpy().view(BLOB_DTYPE).copy(), out


# ------------------------------------------------------------------ gradients
def _planes(t):
    torch = _torch()
    if t.dtype != torch.float32 or t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("expected float32 planes [S, H, W] with unit x stride")
    return t


def blur_iir_adjoint(g, sigmas: Sequence[float], order: int = 3, boundary: str = "replicate", out=None):
    """fdvm_blur_iir_adjoint: planes [S, H, W] -> G_s^T g_s, the transpose of
    the replicate (or zero) extension blur of blur_iir."""
    torch = _torch()
    g = _planes(g.contiguous())
    S, H, W = g.shape
    if out is None:
        out = torch.empty_like(g)
    filt = iir_designs(sigmas, order)
    ws = _workspace(OP_BLUR_IIR_ADJOINT, H, W, S, g.device)
    _check(lib().fdvm_blur_iir_adjoint(g.data_ptr(), H, W, g.stride(1), g.stride(0), out.data_ptr(), out.stride(1),
                                       out.stride(0), filt, S, BOUNDARIES[boundary], ws.data_ptr(), ws.numel(),
                                       _stream_ptr(g.device)), "fdvm_blur_iir_adjoint")
    return out


def laplacian_adjoint(g, sigmas: Sequence[float], out=None):
    """fdvm_laplacian_adjoint: planes [S, H, W] -> sigma_s^2 Lap^T g_s."""
    torch = _torch()
    g = _planes(g.contiguous())
    S, H, W = g.shape
    if out is None:
        out = torch.empty_like(g)
    sig = (ctypes.c_double * S)(*[float(x) for x in sigmas])
    _check(lib().fdvm_laplacian_adjoint(g.data_ptr(), H, W, g.stride(1), g.stride(0), S, sig, out.data_ptr(),
                                        out.stride(1), out.stride(0), _stream_ptr(g.device)), "fdvm_laplacian_adjoint")
    return out


def plane_dots(a, b):
    """fdvm_plane_dots: per-plane float64 inner products of two [S, H, W]
    float32 stacks with the same layout -> float64 device tensor [S]."""
    torch = _torch()
    a = _planes(a.contiguous())
    b = _planes(b.contiguous())
    if a.shape != b.shape:
        raise ValueError("shapes differ")
    S, H, W = a.shape
    out = torch.empty(S, dtype=torch.float64, device=a.device)
    ws = _workspace(OP_PLANE_DOTS, H, W, S, a.device)
    _check(lib().fdvm_plane_dots(a.data_ptr(), b.data_ptr(), H, W, a.stride(1), a.stride(0), S, out.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream_ptr(a.device)), "fdvm_plane_dots")
    return out


def dblur_dsigma_parts(x, sigmas: Sequence[float], order: int = 3, boundary: str = "replicate"):
    """d B_s / d sigma_s of blur_iir as two stacks whose sum it is:
    (d/dsigma along x, blur along y) and (blur along x, d/dsigma along y)."""
    R = iir_pass(x, sigmas, 0, order, boundary)
    Rd = iir_pass(x, sigmas, 0, order, boundary, dsigma=True)
    D1 = iir_pass(Rd, sigmas, 1, order, boundary, out=Rd)
    D2 = iir_pass(R, sigmas, 1, order, boundary, out=R, dsigma=True)
    return D1, D2


def _frames3(x):
    """A frame [H, W] or a batch [N, H, W] (CUDA, unit column stride) as
    ([N, H, W] view, whether a single frame was given)."""
    if not x.is_cuda:
        raise ValueError("frames must be CUDA (HIP) tensors")
    single = x.dim() == 2
    x3 = x.unsqueeze(0) if single else x
    if x3.dim() != 3:
        raise ValueError("frames must be [H, W] or [N, H, W]")
    if x3.stride(2) != 1:
        x3 = x3.contiguous()
    return x3, single


def _response_frames(fwd, x3, S, op):
    """V [N, S, H, W]: the forward call frame after frame, one workspace."""
    torch = _torch()
    N, H, W = x3.shape
    V = torch.empty((N, S, H, W), dtype=torch.float32, device=x3.device)
    ws = _workspace(op, H, W, S, x3.device)
    for f in range(N):
        fwd(x3[f], out=V[f], workspace=ws)
    return V


def _backward(ctx, gV, call, op, extra):
    """Marshals one fdvm_*_laplacian_backward call for the whole batch."""
    torch = _torch()
    x3, V = ctx.saved_tensors[0], ctx.saved_tensors[1]
    N, H, W = x3.shape
    S = V.shape[1]
    what = (GRAD_X if ctx.needs_input_grad[0] else 0) | (GRAD_SIGMA if ctx.needs_input_grad[1] else 0)
    if what == 0:
        return None, None
    gV = gV.reshape(N, S, H, W).float().contiguous()
    gx = torch.empty((N, H, W), dtype=torch.float32, device=V.device) if what & GRAD_X else None
    gs = torch.empty(S, dtype=torch.float64, device=V.device) if what & GRAD_SIGMA else None
    ws = torch.empty(max(workspace_bytes(op, H, W, S), 1), dtype=torch.uint8, device=V.device)
    _check(call(x3.data_ptr(), _dtype_code(x3), H, W, x3.stride(1), x3.stride(0), V.data_ptr(), gV.data_ptr(), W,
                H * W, S * H * W, N, *extra, S, BOUNDARIES[ctx.boundary], what,
                gx.data_ptr() if gx is not None else None, W, H * W,
                gs.data_ptr() if gs is not None else None, ws.data_ptr(), ws.numel(), _stream_ptr(V.device)),
           call.__name__)
    if gx is not None and ctx.single:
        gx = gx[0]
    return gx, gs


def _make_grad_fns():
    torch = _torch()

    class IirLaplacianFn(torch.autograd.Function):
        """V_s = sigma_s^2 (D20 + D02)(B_s), B_s the repeated-pole blur of x
        (iir_laplacian, frame after frame), differentiable in x (float32
        frames) and sigma (float64 tensor [S]).  The backward is one call of
        fdvm_iir_laplacian_backward for the batch (transposed Laplacian,
        transposed blurs summed over the scales, the sigma-derivative
        recursions and the inner products of dL/dsigma, all on the device)."""

        @staticmethod
        def forward(ctx, x, sigma, order=3, boundary="replicate"):
            sig = _host_values(sigma)
            x3, single = _frames3(x.detach())
            V = _response_frames(lambda xf, out, workspace: iir_laplacian(xf, sig, order=order, boundary=boundary,
                                                                          out=out, workspace=workspace),
                                 x3, len(sig), OP_IIR_LAPLACIAN)
            ctx.save_for_backward(x3, V)
            ctx.sig, ctx.boundary, ctx.single = sig, boundary, single
            ctx.filters = iir_designs(sig, order)
            ctx.sigma_device, ctx.sigma_dtype = sigma.device, sigma.dtype
            return V[0] if single else V

        @staticmethod
        def backward(ctx, gV):
            gx, gs = _backward(ctx, gV, lib().fdvm_iir_laplacian_backward, OP_IIR_LAPLACIAN_BACKWARD,
                               (ctx.filters,))
            if gs is not None:
                gs = gs.to(device=ctx.sigma_device, dtype=ctx.sigma_dtype)
            return gx, gs, None, None

    class FirLaplacianFn(torch.autograd.Function):
        """The FIR form (fir_laplacian: the taps of `kind` at the half-lengths
        half_lens, or K = ceil(3 sigma)); the sigma gradient differentiates the
        taps at fixed K (fdvm_filter_design's *_DSIGMA kinds).  Backward: one
        call of fdvm_fir_laplacian_backward for the batch."""

        @staticmethod
        def forward(ctx, x, sigma, kind="sg", half_lens=None, boundary="replicate"):
            sig = _host_values(sigma)
            x3, single = _frames3(x.detach())
            taps, half, off = fir_taps(kind, sig, half_lens)
            V = _response_frames(lambda xf, out, workspace: fir_laplacian(xf, sig, kind=kind, half_lens=half,
                                                                          boundary=boundary, out=out,
                                                                          workspace=workspace),
                                 x3, len(sig), OP_FIR_LAPLACIAN)
            ctx.save_for_backward(x3, V)
            ctx.sig, ctx.boundary, ctx.single = sig, boundary, single
            ctx.kind, ctx.taps, ctx.half, ctx.off = kind, np.ascontiguousarray(taps), half, off
            ctx.sigma_device, ctx.sigma_dtype = sigma.device, sigma.dtype
            return V[0] if single else V

        @staticmethod
        def backward(ctx, gV):
            dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
            dtaps = None
            if ctx.needs_input_grad[1]:
                dkind = FIR_DSIGMA[KINDS[ctx.kind] if isinstance(ctx.kind, str) else int(ctx.kind)]
                dtaps = np.ascontiguousarray(fir_taps(dkind, ctx.sig, ctx.half)[0])
            sig = (ctypes.c_double * len(ctx.sig))(*ctx.sig)
            extra = (ctx.taps.ctypes.data_as(dp), dtaps.ctypes.data_as(dp) if dtaps is not None else None,
                     ctx.half.ctypes.data_as(ip), ctx.off.ctypes.data_as(ip), sig)
            gx, gs = _backward(ctx, gV, lib().fdvm_fir_laplacian_backward, OP_FIR_LAPLACIAN_BACKWARD, extra)
            if gs is not None:
                gs = gs.to(device=ctx.sigma_device, dtype=ctx.sigma_dtype)
            return gx, gs, None, None, None

    return IirLaplacianFn, FirLaplacianFn


_iir_lap_fn = None
_sigma_cache = None


def _host_values(sigma):
    """The scales as Python floats (they become kernel arguments).  A device
    tensor is copied to the host once per object and in-place version, so a
    loop over frames with the same scales does not synchronise per frame."""
    global _sigma_cache
    import weakref
    if _sigma_cache is None:
        _sigma_cache = {}
    hit = _sigma_cache.get(id(sigma))
    if hit is not None and hit[0]() is sigma and hit[1] == sigma._version:
        return hit[2]
    vals = [float(v) for v in sigma.detach().cpu().tolist()]
    if len(_sigma_cache) > 64:
        _sigma_cache = {k: v for k, v in _sigma_cache.items() if v[0]() is not None}
    _sigma_cache[id(sigma)] = (weakref.ref(sigma), sigma._version, vals)
    return vals


def _grad_fns():
    global _iir_lap_fn
    if _iir_lap_fn is None:
        _iir_lap_fn = _make_grad_fns()
    return _iir_lap_fn


def iir_laplacian_grad(x, sigma, order: int = 3, boundary: str = "replicate"):
    """Differentiable iir_laplacian: x float32 [H, W] or a batch [N, H, W]
    (requires_grad allowed), sigma float64 tensor [S] (requires_grad allowed)
    -> V [S, H, W] or [N, S, H, W]."""
    return _grad_fns()[0].apply(x, sigma, order, boundary)


def fir_laplacian_grad(x, sigma, kind: str = "sg", half_lens: Sequence[int] | None = None,
                       boundary: str = "replicate"):
    """Differentiable fir_laplacian (same shapes as iir_laplacian_grad); the
    sigma gradient is taken at fixed half-lengths."""
    return _grad_fns()[1].apply(x, sigma, kind, half_lens, boundary)


# ------------------------------------------------------------------ batch
class Batch:
    """Many frames of uneven size through fdvm_batch_detect: per frame the
    fused IIR blur + normalised Laplacian and the multi-scale extrema, spread
    over `nlanes` internal streams.  Owns the per-frame outputs and the
    workspace, so run() allocates nothing and can be captured into a graph
    (torch.cuda.graph) and replayed.  row_chunks: per frame 0 (default) or the
    row-pass samples per lane (8, 16, 32), e.g. from autotune_batch()."""

    def __init__(self, frames, sigmas: Sequence[float], tau: float, order: int = 3, boundary: str = "replicate",
                 border: int = 1, nlanes: int = 4, cap: int = 1 << 16, row_chunks=None):
        torch = _torch()
        self.frames = [_frame(f) for f in frames]
        dev = self.frames[0].device
        n = len(self.frames)
        self.sigmas = list(sigmas)
        self.filters = iir_designs(self.sigmas, order)
        self.tau, self.border, self.boundary = float(tau), int(border), boundary
        self.nlanes = int(max(1, min(nlanes, MAX_LANES)))
        self.cap = int(cap)
        self.out = torch.empty((n, max(self.cap, 1) * BLOB_BYTES), dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(n, dtype=torch.int32, device=dev)
        self.desc = (Frame * n)()
        chunks = row_chunks if row_chunks is not None else [0] * n
        for i, f in enumerate(self.frames):
            H, W = f.shape
            self.desc[i] = Frame(f.data_ptr(), _dtype_code(f), H, W, int(chunks[i]), f.stride(0),
                                 self.out[i].data_ptr(), self.counts[i:].data_ptr(), self.cap, 0)
        need = int(lib().fdvm_batch_workspace_bytes(self.desc, n, len(self.sigmas), self.nlanes))
        if need == 0:
            raise FdvmError(EINVAL, "fdvm_batch_workspace_bytes")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.device = dev

    def run(self):
        """Enqueue the batch on the current stream (asynchronous)."""
        _check(lib().fdvm_batch_detect(self.desc, len(self.frames), self.filters, len(self.sigmas),
                                       BOUNDARIES[self.boundary], self.tau, self.border, self.nlanes,
                                       self.ws.data_ptr(), self.ws.numel(), _stream_ptr(self.device)),
               "fdvm_batch_detect")

    def results(self):
        """Per frame, the blob list as a structured numpy array (synchronises)."""
        counts = self.counts.cpu().numpy()
        out = []
        for i, n in enumerate(counts):
            if n > self.cap:
                raise FdvmError(EOVERFLOW, f"frame {i}: {n} detections > cap {self.cap}")
            raw = self.out[i, : int(n) * BLOB_BYTES].cpu().numpy()
            out.append(raw.view(BLOB_DTYPE).copy())
        return out


def row_chunk_choices(W: int):
    """Row-pass samples per lane that can cover a row of W samples."""
    return [c for c in (8, 16, 32) if W <= 8 * 64 * c]


def autotune_batch(frames, sigmas: Sequence[float], tau: float, lanes=(1, 2, 4, 8), reps: int = 3, **kw):
    """Pick the lane count and, per distinct frame width, the row-pass chunk by
    timing the batch on the device.  Returns (nlanes, row_chunks, timings)."""
    torch = _torch()
    frames = [_frame(f) for f in frames]
    widths = sorted({int(f.shape[1]) for f in frames})

    def time_batch(nl, chunk_of):
        b = Batch(frames, sigmas, tau, nlanes=nl, row_chunks=[chunk_of[int(f.shape[1])] for f in frames], **kw)
        b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    chunk_of = {w: 0 for w in widths}
    timings = {}
    best_nl, best_t = None, None
    for nl in lanes:
        t = time_batch(nl, chunk_of)
        timings[("lanes", nl)] = t
        if best_t is None or t < best_t:
            best_nl, best_t = nl, t
    for w in widths:   # one width at a time, the others at their current choice
        for c in row_chunk_choices(w):
            trial = dict(chunk_of)
            trial[w] = c
            t = time_batch(best_nl, trial)
            timings[("chunk", w, c)] = t
            if t < best_t:
                best_t, chunk_of = t, trial
    return best_nl, [chunk_of[int(f.shape[1])] for f in frames], timings


__all__ = ["filter_design", "iir_designs", "iir_pass", "blur_iir", "iir_laplacian", "blur_fir", "highpass", "detect_blobs", "detect", "fir_taps",
           "workspace_bytes", "header_symbols", "lib", "library_available", "FdvmError",
           "Batch", "autotune_batch", "row_chunk_choices", "Frame", "blur_iir_adjoint", "laplacian_adjoint",
           "plane_dots", "dblur_dsigma_parts", "iir_laplacian_grad", "fir_laplacian_grad", "iir_hessian"]
