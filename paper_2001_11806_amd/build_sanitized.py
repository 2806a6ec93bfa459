"""Host-sanitizer build of the library, for CPU-only checks of the host code.

``runtime.hip`` (context creation, argument validation, the tape and step
bookkeeping) is compiled with AddressSanitizer and UndefinedBehaviorSanitizer
on its host pass only (device code is built as usual) and linked with the
ordinary objects of ``build.py`` into ``_build/liblbm_mi355x_san.so``.
Loading it needs the clang ASan runtime preloaded; ``tests/test_host_sanitizers.py``
runs the C ABI tests against it.  Never used on a GPU.
"""

import glob
import os
import subprocess

from paper_2001_11806_amd import build as B

SAN_LIB = os.path.join(B.OBJ, "liblbm_mi355x_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]


def asan_runtime():
    """Path of clang's shared ASan runtime shipped with ROCm's LLVM."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang ASan runtime not found")
    return hits[-1]


def build():
    """Compile runtime.hip with host sanitizers; link with the other objects
    (built first by ``build.build`` if they are missing)."""
    src = os.path.join(B.CSRC, "runtime.hip")
    others = [os.path.join(B.OBJ, f + ".o") for f in sorted(os.listdir(B.CSRC))
              if f.endswith(".hip") and f != "runtime.hip"]
    if not all(os.path.exists(o) for o in others):
        B.build(verbose=False)
    obj = os.path.join(B.OBJ, "runtime.hip.san.o")
    subprocess.run(["hipcc", *B.FLAGS, *SAN_FLAGS, "-c", src, "-o", obj], check=True, capture_output=True)
    subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=" + B.ARCH, "-Xarch_host", "-fsanitize=address,undefined",
                    obj, *others, "-o", SAN_LIB], check=True, capture_output=True)
    return SAN_LIB


if __name__ == "__main__":
    print(build())
