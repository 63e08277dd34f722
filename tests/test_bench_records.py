"""Host checks of bench.py's bookkeeping: every measured-traffic record names a committed
rocprofv3 summary that states the same kernel-source fingerprint and the same measured bytes
per launch, and the algorithmic bytes per node are the stated sums."""

import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_records_match_their_profiles():
    assert bench.TRAFFIC_RECORDS, "no traffic record"
    for (storage, jmode, layout), rec in bench.TRAFFIC_RECORDS.items():
        path = os.path.join(ROOT, rec["profile"])
        text = open(path).read()
        assert f"{storage.upper().replace('F', 'FP')}, {jmode} J, {layout.upper()} layout" in text, (storage, jmode, path)
        fp = re.search(r"first\s+16 hex\): `([0-9a-f]{16})`", text)
        assert fp and fp.group(1) == rec["fingerprint"], path
        gb = re.search(r"Measured \([^)]*\): ([0-9.]+) GB per launch", text)
        assert gb and round(float(gb.group(1)), 1) == rec["GB_per_launch"], path
        # the measured traffic of a fused step is at least its algorithmic bytes
        n = 512 ** 3
        assert rec["GB_per_launch"] >= bench.bytes_per_node(storage) * n / 1e9 * 0.999, (storage, jmode, layout)


def test_bytes_per_node():
    # read and write 27 + 21 populations, plus 3 + 3 forcing values in the arithmetic type
    assert bench.bytes_per_node("f32") == 2 * 48 * 4 + 6 * 4 == 408
    assert bench.bytes_per_node("f64") == 2 * 48 * 8 + 6 * 8 == 816
    assert bench.bytes_per_node("f16") == 2 * 48 * 2 + 6 * 4 == 216
    assert bench.bytes_per_node("f32", forced=False) == 384


def test_kernel_fingerprint_is_stable():
    assert re.fullmatch(r"[0-9a-f]{16}", bench.kernel_fingerprint())
    assert bench.kernel_fingerprint() == bench.kernel_fingerprint()
