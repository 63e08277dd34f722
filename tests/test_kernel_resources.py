"""Register and private-memory use of the diagnostic kernels, read on the host from the kernel
metadata of a gfx950 compile of their source (no GPU needed). A node's populations held in a
local array that is indexed at run time end up in per-thread private memory; that made the FP16
reductions six to ten times slower than the FP32 ones, so the reductions and node fields must
keep them in registers."""

import os
import re
import shutil
import subprocess

import pytest

from paper_2212_11024_amd import build as B


def _kernel_metadata(src, tmp_path):
    out = tmp_path / "k.s"
    cmd = [B.hipcc(), "-O3", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", "--cuda-device-only", "-S",
           os.path.join(B.CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    meta = {}
    for block in out.read_text().split("\n  - "):
        name = re.search(r"\.name:\s+(\S+)", block)
        priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
        if name and priv and vgpr:
            meta[name.group(1)] = (int(priv.group(1)), int(vgpr.group(1)))
    return meta


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is not installed")
def test_reductions_and_node_fields_keep_the_node_in_registers(tmp_path):
    meta = _kernel_metadata("flame_api.hip", tmp_path)
    checked = [k for k in meta if "reduce_kernel" in k or "moments_kernel" in k]
    # three storage types each
    assert len(checked) == 6, checked
    for k in checked:
        priv, vgpr = meta[k]
        if "reduce_kernelId" in k:
            # FP64: a few spilled registers under the two-waves-per-SIMD bound, nothing more
            assert priv <= 64 and vgpr <= 256, (k, priv, vgpr)
        else:
            assert priv == 0, (k, priv)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is not installed")
def test_lattice_variant_node_fields_keep_the_node_in_registers(tmp_path):
    meta = _kernel_metadata("flame_lattice.hip", tmp_path)
    checked = [k for k in meta if "variant_moments" in k or "variant_component" in k or "variant_reduce" in k]
    assert len(checked) >= 18, checked
    for k in checked:
        assert meta[k][0] == 0, (k, meta[k])
