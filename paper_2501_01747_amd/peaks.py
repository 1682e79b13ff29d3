"""ctypes binding of libadg_peaks.so (include/adg_peaks.h): measured copy bandwidth and FP64
vector rate of the device, the ceilings the stage kernels are compared with next to the
published ones.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libadg_peaks.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)
_sig = {
    "adg_peak_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_double)]),
    "adg_peak_fp64_out_bytes": (C.c_size_t, []),
    "adg_peak_fp64": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    "adg_peak_fp64_fmas": (C.c_double, []),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

EXPORTED = tuple(_sig)


def fp64_rate(n_reps: int = 20) -> float:
    """FP64 FMA rate (TFLOP/s) of the FMA-chain kernel on torch's current stream."""
    import torch

    out = torch.empty(adg_peak_fp64_out_bytes() // 8, dtype=torch.float64, device="cuda")
    tf = C.c_double()
    rc = adg_peak_fp64(out.data_ptr(), n_reps, torch.cuda.current_stream().cuda_stream, C.byref(tf))
    if rc:
        raise RuntimeError(f"adg_peak_fp64 failed ({rc})")
    return tf.value


def measure(copy_bytes: int = 1 << 30, n_reps: int = 20) -> dict:
    """Copy bandwidth (GB/s, read + write) over copy_bytes and the FP64 FMA rate (TFLOP/s),
    on torch's current stream of the current device."""
    import torch

    src = torch.ones(copy_bytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    gbs = C.c_double()
    rc = adg_peak_copy(src.data_ptr(), dst.data_ptr(), copy_bytes, n_reps, stream, C.byref(gbs))
    if rc:
        raise RuntimeError(f"adg_peak_copy failed ({rc})")
    if not torch.equal(dst[:1024], src[:1024]):
        raise RuntimeError("copy probe produced wrong data")
    del src, dst
    tf = fp64_rate(n_reps)
    torch.cuda.empty_cache()
    return {"copy_GBps": gbs.value, "fp64_vector_TFLOPs": tf, "copy_bytes": copy_bytes}
