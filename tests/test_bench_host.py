"""Host logic of bench.py (no device work): the one-GPU guard, the instruction-mix
peaks and the HBM traffic lookup in the committed counter profile."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_mix_peak_of_the_pure_sine_cosine_pair_is_the_transcendental_bound():
    # 2 transcendentals and no other work: 256 CUs x 2.4 GHz x 32 lanes / 2
    assert bench.alu_peak(0.0, 2.0) == pytest.approx(bench.PEAK_SINCOS_PAIRS)
    # adding VALU work lowers the peak by its issue time
    assert bench.alu_peak(3.25, 2.0) == pytest.approx(256 * 2.4e9 / (3.25 / 128 + 2 / 32))


def test_per_pair_mixes_of_the_row_and_general_forms():
    # planar row form at 4 pixels per lane: 1 FMA phase + the q_y term per 4 pixels + 2 FMA sums
    assert bench.pair_mix("forward_fp32c", False, 4, True, rows=True) == (3.25, 2.0, 0.0)
    assert bench.pair_mix("forward_fp32c", False, 4, False, rows=True) == (4.25, 2.0, 0.0)
    assert bench.pair_mix("forward_fp32c", False, 4, True) == (4, 2.0, 0.0)
    # adjoint: one sine per pair; row groups drop the y term
    assert bench.pair_mix("adjoint_fp32c", False, 2, True, rows=True) == (4, 1.0, 0.0)
    assert bench.pair_mix("adjoint_fp32c", False, 2, True) == (5, 1.0, 0.0)


def test_traffic_lookup_needs_the_profiled_source_and_shape(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2204_13241_amd", "csrc", "k_fp32c.hip")
    prof = json.load(open(os.path.join(ROOT, "profiles", "pair_kernels_pmc_grad65536.json")))
    rec = prof["kernels"]["forward_fp32c"]
    shape = rec["tile_shape"]
    if prof["source_sha256_16"] == bench.source_hash(src):
        assert bench.traffic_from_profile(src, "forward_fp32c", shape) == rec["hbm_bytes_per_launch"]
    other = dict(shape, atom_split=shape["atom_split"] * 2)
    assert bench.traffic_from_profile(src, "forward_fp32c", other) is None
    # a changed device part of the source invalidates the profile
    changed = tmp_path / "k.hip"
    changed.write_bytes(open(src, "rb").read().replace(bench.DEVICE_END, b"// x\n" + bench.DEVICE_END, 1))
    assert bench.traffic_from_profile(str(changed), "forward_fp32c", shape) is None

