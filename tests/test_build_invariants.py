"""CPU checks of properties of the compiled gfx950 code that the kernels rely on."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_00276_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_particle_kernel_dynamic_lds_is_16_byte_aligned(tmp_path):
    """The int64 current tile lives in dynamic LDS right after the static LDS;
    its 8-byte LDS atomics need the dynamic base (= the static segment size)
    to be a multiple of 8, which the aligned extern declaration guarantees."""
    out = tmp_path / "gpd.s"
    subprocess.check_call(["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
                           "-munsafe-fp-atomics", os.path.join(CSRC, "gpd.hip"), "-o", str(out)],
                          stderr=subprocess.DEVNULL)
    sizes = [int(v) for v in re.findall(r"amdhsa_group_segment_fixed_size (\d+)", out.read_text())]
    # 2 dims x 3 orders x (periodic, moving window) + 3 orders x (r-z, r-z with window)
    # + 3 orders x periodic 3D in two phases (int64 tile; 32-bit tile with compile-time
    # and with runtime LDS strides) + 3 orders x periodic 2D in two phases
    assert len(sizes) == 30
    assert all(v % 16 == 0 for v in sizes), sizes


def test_counter_records_match_the_kernel_source():
    """The committed rocprofv3 counter records (profiles/*_counters.json) were
    taken on the particle kernel's current source: bench.py reports their
    traffic only when the SHA-256 of gpd.hip + pic_dev.h matches, so a stale
    record would leave the measured traffic out silently."""
    import glob
    import hashlib
    import json

    h = hashlib.sha256()
    for fn in ("gpd.hip", "pic_dev.h"):
        with open(os.path.join(CSRC, fn), "rb") as f:
            h.update(f.read())
    recs = glob.glob(os.path.join(ROOT, "profiles", "*_counters.json"))
    assert recs
    for p in recs:
        with open(p) as f:
            rec = json.load(f)
        assert rec["source_sha256"] == h.hexdigest(), os.path.basename(p)
        assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
