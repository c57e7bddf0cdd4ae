"""Why the library has no BF16 tap mode: gfx950 has packed FP16 arithmetic but
no packed BF16 arithmetic. The assembler for gfx950 accepts the packed FP16
fused multiply-add and rejects packed BF16 multiply, add and fused
multiply-add; BF16 math therefore runs as FP32 instructions plus conversions,
so a BF16 tap path would cost as much as the FP32 one and only add rounding.
(The one packed BF16 instruction with FP32 accumulation, a two-term dot
product, cannot carry the per-tap polynomial of the FP16 path within its
error budget: 8-bit mantissas put the tap error near the 2e-3 tolerance.)"""
import os
import shutil
import subprocess

import pytest

LLVM_MC = "/opt/rocm/llvm/bin/llvm-mc"


def _assembles(line: str) -> bool:
    r = subprocess.run([LLVM_MC, "-arch=amdgcn", "-mcpu=gfx950", "-show-encoding"], input=line + "\n",
                       capture_output=True, text=True, timeout=60)
    return r.returncode == 0 and "error" not in r.stderr


@pytest.mark.skipif(not os.path.exists(LLVM_MC) and shutil.which("llvm-mc") is None, reason="llvm-mc not installed")
def test_gfx950_has_packed_fp16_but_no_packed_bf16_arithmetic():
    assert _assembles("v_pk_fma_f16 v0, v1, v2, v3")
    assert _assembles("v_pk_mul_f16 v0, v1, v2")
    for ins in ("v_pk_fma_bf16 v0, v1, v2, v3", "v_pk_mul_bf16 v0, v1, v2", "v_pk_add_bf16 v0, v1, v2"):
        assert not _assembles(ins), ins
    assert _assembles("v_dot2_f32_bf16 v0, v1, v2, v3")
