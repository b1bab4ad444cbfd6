"""The built library's gfx950 kernels (CPU only): read each code object's
metadata notes and check that no kernel keeps per-lane scratch memory (a
private segment, or vector registers spilled to memory).  A kernel argument
whose address is taken, or a lane state too large for the registers, lands
there and multiplies the kernel's time; the metadata shows it without a GPU.
Spills of scalar registers into vector-register lanes use no memory and are
allowed."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_27193_amd", "libaeb.so")
LLVM = "/opt/rocm/llvm/bin"
TOOLS = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

pytestmark = pytest.mark.skipif(not all(os.path.exists(t) for t in TOOLS),
                                reason="ROCm LLVM tools not installed")


def kernels(tmp):
    """(name, private segment bytes, VGPR spills) of every kernel in every
    device bundle of the library's fat-binary section."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    fat = os.path.join(tmp, "fat.bin")
    subprocess.run([TOOLS[0], f"--dump-section=.hip_fatbin={fat}", LIB, os.path.join(tmp, "x")],
                   check=True, capture_output=True)
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    out = []
    for k, s in enumerate(starts):
        e = starts[k + 1] if k + 1 < len(starts) else len(data)
        bundle, co = os.path.join(tmp, f"b{k}.bin"), os.path.join(tmp, f"b{k}.co")
        with open(bundle, "wb") as f:
            f.write(data[s:e])
        subprocess.run([TOOLS[1], "--unbundle", "--type=o", f"--input={bundle}",
                        f"--targets={TARGET}", f"--output={co}"], check=True, capture_output=True)
        notes = subprocess.run([TOOLS[2], "--notes", co], check=True, capture_output=True,
                               text=True).stdout
        # one metadata map per kernel: split at each kernel's name
        for part in notes.split(".name:")[1:]:
            name = part.split()[0]
            priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", part)
            vsp = re.search(r"\.vgpr_spill_count:\s+(\d+)", part)
            out.append((name, int(priv.group(1)) if priv else None,
                        int(vsp.group(1)) if vsp else None))
    return out


def test_no_kernel_uses_scratch(tmp_path):
    ks = kernels(str(tmp_path))
    names = {n for n, _, _ in ks}
    # the integration, preparation and reduction kernels are all there
    for want in ("k_roll_fp64", "k_roll_fp32c", "k_prep", "k_pass1", "k_collect", "k_sample"):
        assert any(want in n for n in names), want
    bad = [(n, p, v) for n, p, v in ks if p is None or v is None or p != 0 or v != 0]
    assert not bad, bad[:10]
