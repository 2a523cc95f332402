"""The build's code-generation guarantees, checked without a GPU.

The HIP library is compiled with -ffp-contract=off (no fused multiply-add in
the method's arithmetic) and with the device target feature that disables
packed binary32 instructions (v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32).  The
host pass of hipcc warns that x86 does not know that feature; the device pass
honours it.  These tests show it on a small kernel the compiler would
otherwise pack, and check the device code of the built library itself.
"""

import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1612_01395_amd import build

PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")
LLVM = "/opt/rocm/llvm/bin"

KERNEL = r"""
#include <hip/hip_runtime.h>
__global__ void axpy2(float2* a, const float2* b, float s) {
  const int i = threadIdx.x;
  float2 x = a[i], y = b[i];
  x.x = x.x + y.x * s;
  x.y = x.y + y.y * s;
  a[i] = x;
}
"""


def _device_asm(flags, tmp):
    src = os.path.join(tmp, "k.hip")
    with open(src, "w") as f:
        f.write(KERNEL)
    out = os.path.join(tmp, "k.s")
    cmd = [build.HIPCC, f"--offload-arch={build.ARCH}", "-O3", "--cuda-device-only", "-S", "-o", out, src] + flags
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read()


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not installed")
def test_packed_fp32_feature_is_honoured_by_the_device_pass():
    feature = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    assert all(f in build.FLAGS for f in feature)
    with tempfile.TemporaryDirectory() as tmp:
        assert PACKED.search(_device_asm([], tmp)), "the probe kernel no longer packs: choose another"
        assert not PACKED.search(_device_asm(feature, tmp))


@pytest.mark.skipif(not os.path.exists(build.LIB) or not os.path.exists(os.path.join(LLVM, "llvm-objdump")),
                    reason="library not built or LLVM tools missing")
def test_built_library_holds_no_packed_fp32_instructions():
    with tempfile.TemporaryDirectory() as tmp:
        fat = os.path.join(tmp, "fatbin.bin")
        co = os.path.join(tmp, "dev.co")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", build.LIB],
                       check=True, capture_output=True)
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fat}",
                        f"--targets=hipv4-amdgcn-amd-amdhsa--{build.ARCH}", f"--output={co}"],
                       check=True, capture_output=True)
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", f"--mcpu={build.ARCH}", co],
                             check=True, capture_output=True, text=True).stdout
    assert "k_pb" in dis  # the fused kernels are there
    assert not PACKED.search(dis)
