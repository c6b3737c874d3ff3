"""The built library's gfx950 code object: every block kernel keeps its
state in registers and LDS.

A private (scratch) segment on k_block means the compiler spilled or
outlined one of the per-workgroup work functions (heads, tier passes, tail
multiply-accumulate) into a call with a stack frame; both put scratch
traffic on the streaming path.  Read from the kernel metadata notes of the
library built in-tree (no GPU needed); skipped where the ROCm LLVM tools or
the library are missing.
"""
import os
import re
import subprocess

import pytest

LLVM = "/opt/rocm/llvm/bin"
LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2509_04390_amd", "librta.so")


def _kernel_notes(tmp_path):
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(os.path.exists(t) for t in tools) or not os.path.exists(LIB):
        pytest.skip("needs the ROCm LLVM tools and the built library")
    objcopy, bundler, readelf = tools
    fb = str(tmp_path / "fatbin.bin")
    co = str(tmp_path / "gfx950.co")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fb}", LIB], check=True)
    subprocess.run([bundler, "--type=o", f"--input={fb}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}", "--unbundle"],
                   check=True)
    notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
    kernels = {}
    name = None
    for line in notes.splitlines():
        m = re.match(r"\s*\.name:\s+(\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.match(r"\s*\.(private_segment_fixed_size|vgpr_count|vgpr_spill_count|uses_dynamic_stack):\s+(\S+)",
                     line)
        if m and name is not None:
            kernels[name][m.group(1)] = m.group(2)
    return kernels


def test_block_kernels_use_no_scratch(tmp_path):
    kernels = _kernel_notes(tmp_path)
    blocks = {k: v for k, v in kernels.items() if "k_block" in k}
    # three spectrum types x G in {1, 2, 4} x two load kinds
    assert len(blocks) == 18, sorted(kernels)
    for name, meta in blocks.items():
        assert meta.get("private_segment_fixed_size") == "0", (name, meta)
        assert meta.get("vgpr_spill_count", "0") == "0", (name, meta)
        assert meta.get("uses_dynamic_stack", "false") == "false", (name, meta)
        assert int(meta["vgpr_count"]) <= 168, (name, meta)  # at least 3 waves per SIMD
