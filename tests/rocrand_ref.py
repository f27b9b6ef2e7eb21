"""rocRAND's Philox4x32-10, compiled on the host from its public header, as
an independent reference for the oracle's generator (tests only)."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "helpers", "rocrand_philox_ref.cpp")
_lib = None


def lib():
    global _lib
    if _lib is None:
        out = os.path.join(tempfile.gettempdir(), "srm_rocrand_ref_%d.so" % os.getpid())
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-fPIC", "-shared",
                               "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", _SRC, "-o", out])
        L = C.CDLL(out)
        up = C.POINTER(C.c_uint32)
        L.ref_philox4x32.argtypes = [up, up, up, C.c_int64]
        _lib = L
    return _lib


def philox4x32(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr (n, 4), key (n, 2) uint32 -> (n, 4) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    up = C.POINTER(C.c_uint32)
    lib().ref_philox4x32(ctr.ctypes.data_as(up), key.ctypes.data_as(up), out.ctypes.data_as(up),
                         ctr.shape[0])
    return out
