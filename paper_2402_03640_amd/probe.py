"""ctypes binding of ``libhipmsat_probe.so`` (``include/hipmsat_probe.h``):
the streaming-copy and random-row gather probes that give the memory-system
ceilings the solve loop's kernels are measured against.  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhipmsat_probe.so")
EXPORTS = ["hmsp_copy", "hmsp_gather", "hmsp_grid_barrier", "hmsp_launch_gap", "hmsp_last_error"]
# (floats per lane, rows per output) shapes of the gather probe; a ceiling is
# the best of them
GATHER_SHAPES = [(1, 16), (2, 8), (2, 16), (4, 8), (4, 16)]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_03640_amd.build`")
        import torch  # noqa: F401  (its HIP runtime first, as for the solver library)
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.hmsp_copy.argtypes = [P, P, I64, I32, P, P]
        L.hmsp_copy.restype = I32
        L.hmsp_gather.argtypes = [P, I64, I32, P, I64, I32, I32, P, I32, P, P]
        L.hmsp_gather.restype = I32
        L.hmsp_grid_barrier.argtypes = [I32, I32, P, P, P]
        L.hmsp_grid_barrier.restype = I32
        L.hmsp_launch_gap.argtypes = [I32, I32, I32, P, P]
        L.hmsp_launch_gap.restype = I32
        L.hmsp_last_error.argtypes = []
        L.hmsp_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"probe error {rc}: {lib().hmsp_last_error().decode()}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def copy_ms(src, dst, iters: int = 20) -> float:
    """Average ms of one streaming copy of src (a contiguous device tensor) into dst."""
    ms = C.c_double()
    nbytes = src.numel() * src.element_size()
    _check(lib().hmsp_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, int(iters), _stream(),
                           C.byref(ms)))
    return ms.value


def gather_ms(src, idx, out, deg: int = 16, vec: int = 2, iters: int = 20) -> float:
    """Average ms of one gather-sum launch: src [rows][W] float32, idx n
    int32 row indices (n a multiple of 16, values below rows), out
    [n / deg][W] float32; `vec` floats per lane."""
    ms = C.c_double()
    rows, W = src.shape
    _check(lib().hmsp_gather(C.c_void_p(src.data_ptr()), rows, W, C.c_void_p(idx.data_ptr()), idx.numel(),
                             int(deg), int(vec), C.c_void_p(out.data_ptr()), int(iters), _stream(), C.byref(ms)))
    return ms.value


def grid_barrier_us(blocks: int, rounds: int = 2000):
    """(average microseconds per grid-barrier round, whether a bounded wait gave up)."""
    us, gave = C.c_double(), C.c_int32()
    _check(lib().hmsp_grid_barrier(int(blocks), int(rounds), _stream(), C.byref(us), C.byref(gave)))
    return us.value, bool(gave.value)


def launch_gap_us(blocks: int, kernels: int = 2000, graph: bool = True) -> float:
    """Average microseconds per launch of dependent do-nothing kernels."""
    us = C.c_double()
    _check(lib().hmsp_launch_gap(int(blocks), int(kernels), int(bool(graph)), _stream(), C.byref(us)))
    return us.value
