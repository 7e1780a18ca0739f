"""Register-resident kernels stay in registers (hipcc resource-usage remarks; no GPU needed).

The wavefront-level kernels keep per-lane state in registers by design: the wave kernel's
mirror of reached-vertex ids and its seed-quad cache, the packed kernel's seed cache. A
private array that the compiler indexes at run time, or a spill, moves such state into
scratch memory, where every access is a memory round trip; nothing fails, it only gets
slower. This test compiles the two sources for gfx950 with the build's flags and checks
that those kernels use no scratch and keep the occupancy their launch shapes assume.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2302_13529_amd import build

HIPCC = build.HIPCC


def _resources(source, tmp_path):
    """{kernel symbol: {field: value}} from hipcc's kernel-resource-usage remarks."""
    out = tmp_path / (os.path.basename(source) + ".o")
    flags = [f for f in build.FLAGS if f != "-shared"]
    cmd = [HIPCC, *flags, "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC,
           "--offload-device-only", "-c", source, "-o", str(out),
           "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-2000:]
    kernels, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark: (.*?) \[-Rpass-analysis", line)
        if not m:
            continue
        text = m.group(1).strip()
        if text.startswith("Function Name:"):
            cur = text.split(":", 1)[1].strip()
            kernels[cur] = {}
        elif cur is not None and ":" in text:
            k, v = text.rsplit(":", 1)
            kernels[cur][k.strip()] = v.strip()
    return kernels


needs_hipcc = pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")),
                                 reason="hipcc not available")


@needs_hipcc
@pytest.mark.parametrize("source, kernel, min_waves", [
    ("small.hip", "decrease_small_kernel", 4),
    ("pack.hip", "decrease_pack_kernel", 4),
])
def test_wavefront_kernels_use_no_scratch(tmp_path, source, kernel, min_waves):
    ks = _resources(os.path.join(build.CSRC, source), tmp_path)
    found = {name: f for name, f in ks.items() if kernel in name}
    assert found, f"no {kernel} in {source}: {sorted(ks)}"
    for name, f in found.items():
        assert int(f["ScratchSize [bytes/lane]"]) == 0, (name, f)
        assert int(f["VGPRs Spill"]) == 0, (name, f)
        assert f["Dynamic Stack"] == "False", (name, f)
        assert int(f["Occupancy [waves/SIMD]"]) >= min_waves, (name, f)
