"""Build + ctypes driver of tests/devprims/devprims.hip (GPU unit tests of the
team primitives; tests only)."""
import ctypes as C
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "libdevprims.so")
_CSRC = os.path.join(_HERE, "..", "..", "paper_1908_09378_amd", "csrc")


def build():
    srcs = [os.path.join(_HERE, "devprims.hip")] + [os.path.join(_CSRC, f) for f in ("pbh_core.h", "pbh_team.h")]
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(s) for s in srcs):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           srcs[0], "-o", tmp], stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} not built")
        _lib = C.CDLL(LIB)
        _lib.dp_run.restype = C.c_int
        _lib.dp_run.argtypes = [C.c_int, C.c_int] + [C.c_void_p, C.c_void_p, C.c_uint32] * 2 + [C.c_void_p] * 8
    return _lib
