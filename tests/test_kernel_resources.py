"""Register and scratch budget of every HIP kernel, from the compiler's
resource report that the build keeps beside each object file.

No kernel may use scratch memory or spill vector registers (a spill turns
register-resident tiles into per-lane memory traffic), and the kernels whose
occupancy the design relies on keep it: five waves per SIMD for the
complex64 tile pass and the 5-qubit complex64 matrix-core block, four for
the 5-qubit complex128 block.
"""
import glob
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "qsv")


def _reports():
    files = sorted(glob.glob(os.path.join(BUILD, "*.resources.txt")))
    if not files:
        pytest.skip("no build resource reports (run the build first)")
    rows = {}
    for fn in files:
        for line in open(fn):
            parts = line.split()
            if not parts:
                continue
            rows[parts[0]] = dict(p.split("=", 1) for p in parts[1:])
    return rows


def test_every_device_source_reported():
    srcs = glob.glob(os.path.join(ROOT, "paper_2502_11385_amd", "csrc",
                                  "*.hip"))
    names = {os.path.splitext(os.path.basename(s))[0] for s in srcs}
    have = {os.path.basename(f)[:-len(".resources.txt")]
            for f in glob.glob(os.path.join(BUILD, "*.resources.txt"))}
    if not have:
        pytest.skip("no build resource reports (run the build first)")
    assert names <= have, names - have


def test_no_scratch_and_no_vector_spills():
    rows = _reports()
    assert len(rows) >= 60
    bad = {k: v for k, v in rows.items()
           if v.get("ScratchSize") != "0" or v.get("VGPRs_Spill") != "0"}
    assert not bad, bad


@pytest.mark.parametrize("fragment,min_waves", [
    ("tile_kernel_c64_rb4", 5),
    ("fused_mfma_c64_kernelILi5", 5),
    ("fused_mfma_c64_kernelILi4", 8),
    ("fused_mfma_c128_kernelILi5", 4),
])
def test_occupancy_of_the_hot_kernels(fragment, min_waves):
    rows = _reports()
    hits = {k: v for k, v in rows.items() if fragment in k}
    assert hits, fragment
    for k, v in hits.items():
        assert int(v["Occupancy"]) >= min_waves, (k, v)
