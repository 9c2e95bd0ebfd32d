"""Kernel names of the built library as profiler summaries print them.

The gfx950 code objects are extracted from the shared library (a copy, in
a temporary directory) with llvm-objdump, their kernel symbols (functions
that have a `.kd` kernel descriptor) demangled
with c++filt and shortened the way the profile summaries shorten
rocprofv3's names.  Used by tests to check the names the library gives
its profiled launches."""

import os
import shutil
import subprocess
import tempfile

from paper_2507_21791_amd import bcgs
from paper_2507_21791_amd.prof_summary import short_name

LLVM = "/opt/rocm/llvm/bin"


def library_kernel_names():
    out = set()
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "lib.so")
        shutil.copy(bcgs.LIB_PATH, lib)
        subprocess.run([os.path.join(LLVM, "llvm-objdump"), "--offloading",
                        lib], check=True, capture_output=True, cwd=d)
        mangled, descriptors = set(), set()
        for f in os.listdir(d):
            if "amdgcn" not in f:
                continue
            r = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "-sW",
                                os.path.join(d, f)], check=True,
                               capture_output=True, text=True)
            for line in r.stdout.splitlines():
                parts = line.split()
                if len(parts) >= 8 and parts[7].startswith("_Z"):
                    if parts[3] == "FUNC":
                        mangled.add(parts[7])
                    elif parts[7].endswith(".kd"):
                        descriptors.add(parts[7][:-3])
        # kernels are the functions with a kernel descriptor; the rest are
        # non-inlined device functions
        mangled &= descriptors
        dem = subprocess.run(["c++filt"], input="\n".join(sorted(mangled)),
                             capture_output=True, text=True, check=True)
        for n in dem.stdout.splitlines():
            if "bcgs::" in n:
                out.add(short_name(n))
    return out
