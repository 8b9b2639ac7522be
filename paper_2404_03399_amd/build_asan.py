"""Host-side AddressSanitizer build of libadg.so (device code unchanged).

    python -m paper_2404_03399_amd.build_asan

writes paper_2404_03399_amd/_lib_asan/libadg.so.  The Python interpreter is
not instrumented, so load the library with the sanitizer runtime preloaded
and point the binding at it:

    ADG_LIBRARY=$PWD/paper_2404_03399_amd/_lib_asan/libadg.so \
    LD_PRELOAD=$(/opt/rocm/llvm/bin/clang++ --print-file-name=libclang_rt.asan-x86_64.so) \
    ASAN_OPTIONS=detect_leaks=0 python -m pytest tests/test_library_host.py

Every sanitizer option applies to the host compilation only (-Xarch_host).
"""
from __future__ import annotations

import os

from . import build as _b

LIBDIR = os.path.join(_b.PKG, "_lib_asan")
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False) -> str:
    return _b.build(verbose=verbose, extra=HOST_ASAN, libdir=LIBDIR)


if __name__ == "__main__":
    print(build(verbose=True))
