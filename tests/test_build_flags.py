"""The library's hipcc flags keep packed FP32 instructions out of device code.

``paper_1801_00338_amd/build.py`` passes ``-Xclang -target-feature -Xclang
-packed-fp32-ops``.  hipcc's host (x86) pass does not know that feature and
warns; the device (gfx950) pass honours it.  This test compiles a small float2
kernel to gfx950 assembly with and without the flag: without it the compiler
forms ``v_pk_fma_f32``, with the library's flags it forms none.  CPU only
(hipcc cross-compiles).
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1801_00338_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KERNEL = r"""
#include <hip/hip_runtime.h>
__global__ void k(const float2 *a, const float2 *b, float2 *c, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float2 x = a[i], y = b[i];
        c[i] = make_float2(x.x * y.x + x.y, x.y * y.y + x.x);
    }
}
"""
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def _asm(tmp_path, flags):
    src = tmp_path / "k.hip"
    src.write_text(KERNEL)
    out = tmp_path / "k.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
           *flags, str(src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC),
                    reason="hipcc not installed")
def test_library_flags_keep_packed_fp32_out(tmp_path):
    lib_flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")
                 and not f.startswith("-I")]
    assert "-packed-fp32-ops" in lib_flags
    plain = _asm(tmp_path, [])
    assert PACKED.search(plain), "the probe kernel no longer forms packed FP32 without the flag"
    assert not PACKED.search(_asm(tmp_path, lib_flags))
