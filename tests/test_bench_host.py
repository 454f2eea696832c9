"""Host-side logic of bench.py (no GPU): the algorithmic byte counts behind
the roofline, the kernel-name shortening of the profiler summaries, and the
traffic lookup, which must refuse a counter summary taken on other kernel
sources."""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N, L, E = 187500, 21, 4
LAT = [(5, 13051), (2, 24540)]   # (d, M) of the 500x375 image's lattices


def test_class_bytes_per_pixel_figures():
    verts = sum(M for _, M in LAT) * L * E
    # k_fw_lmo_rows: y, P_y, P_s, c in; y, P_y out; two label arrays
    assert bench.class_bytes("k_fw_lmo_rows", N, L, E, LAT) == N * 512
    # k_fw_slice_rows: 248 B per pixel plus the vertex rows once
    assert bench.class_bytes("k_fw_slice_rows", N, L, E, LAT) == N * 248 + verts
    # one-hot splat: label + 9 (id, weight) pairs per pixel, vertex rows out
    for k in ("k_splat_labels_lds", "k_splat_labels_chunks"):
        assert bench.class_bytes(k, N, L, E, LAT) == N * 76 + verts


def test_class_bytes_blur_is_per_launch():
    # G = 2: the 6 bilateral directions take 3 launches, the 3 spatial 2
    per_row = 2 * L * E + 9 * 4
    total = 3 * 13051 * per_row + 2 * 24540 * per_row
    assert bench.class_bytes("k_blur_group", N, L, E, LAT) == pytest.approx(total / 3)
    per_row1 = 2 * L * E + 3 * 4
    total1 = 6 * 13051 * per_row1 + 3 * 24540 * per_row1
    assert bench.class_bytes("k_blur_pass", N, L, E, LAT) == pytest.approx(total1 / 6)


def test_lattice_bytes_matches_the_documented_total():
    assert bench.lattice_bytes(N, L, E, LAT) == 91554264


def test_short_kernel_names_keep_template_arguments():
    name = ("void dcrf::(anonymous namespace)::k_fw_slice_rows<float, 24, true>"
            "(dcrf::(anonymous namespace)::FWSliceArgs<float>, dcrf::LatSet<float>)")
    assert bench._short(name) == "k_fw_slice_rows<float, 24, true>"
    assert bench._short("dcrf::(anonymous namespace)::k_scan_tiles(int*, int)") == \
        "k_scan_tiles"


def test_traffic_lookup_requires_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("\n".join([
        "# test summary",
        f"source_sha256 {bench.source_digest()}",
        "calib FETCH_SIZE measured_kib 131072.0 expected_kib 262144.0 dispatches 5",
        "calib WRITE_SIZE measured_kib 262144.0 expected_kib 262144.0 dispatches 5",
        "kernel k_fw_slice_rows<float,24,true> fetch_kib 100.0 write_kib 50.0 dispatches 9",
        "kernel k_fw_slice_rows<float,24,false> fetch_kib 999.0 write_kib 999.0 dispatches 1",
    ]) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    # FETCH scaled by 2 (calibration), WRITE by 1; the instantiation with the
    # most dispatches wins
    assert bench.traffic_bytes("k_fw_slice_rows") == pytest.approx((200.0 + 50.0) * 1024)
    assert bench.traffic_bytes("k_fw_lmo_rows") is None
    f.write_text(f.read_text().replace(bench.source_digest(), "0" * 64))
    assert bench.traffic_bytes("k_fw_slice_rows") is None
