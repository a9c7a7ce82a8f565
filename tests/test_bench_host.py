"""Host-side figures of bench.py (CPU): the algorithmic work per launch that the
roofline divides by, and the validity rule of the committed traffic counters."""

import json
import os

import pytest

import bench
from synth import make_system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def molecule():
    return make_system(1, with_start=False)


def test_stage_work_of_the_molecule_workload(molecule):
    # box 29 x 29 x 29 (|g| <= 14), rebuild grid 64^3, N_aux = 64
    b = bench.stage_bytes(molecule, 64, 29, 29, (64, 64, 64), 16)
    slab = 29 * 64 * 29 * 64 * 16
    assert b["xz_planes"] == 2 * slab + 64 ** 3 * 8 == 112_328_704
    assert b["y_lines"] == slab + 12000 * 64 * 16 + 12000 * 8
    f = bench.stage_flops(molecule, 64, 29, 29, (64, 64, 64))
    # per column and plane: 2 x 29 x-transforms, 64 z-transform pairs and products
    per = 2 * 29 * 5 * 64 * 6 + 64 * (2 * 5 * 64 * 6 + 2 * 64)
    assert f["xz_planes"] == pytest.approx(64 * 64 * per)
    assert f["xz_planes"] == pytest.approx(1_496_317_952)
    # complex64 slabs halve the bytes of the slab terms
    b32 = bench.stage_bytes(molecule, 64, 29, 29, (64, 64, 64), 8)
    assert b32["xz_planes"] == slab + 64 ** 3 * 4


def test_traffic_counters_apply_only_to_their_own_source_and_workload():
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    recs = json.load(open(path))
    assert isinstance(recs, list) and recs
    rec = recs[0]
    cur = bench.traffic_from_profiles("fft.hip", rec["stage"], rec["precision"], rec["config"])
    import hashlib

    src = open(os.path.join(ROOT, "paper_2403_04351_amd", "csrc", "fft.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() == rec["source_sha256"]:
        assert cur == rec["bytes_per_launch"]
    else:
        assert cur is None
    other = "fp32" if rec["precision"] == "fp64" else "fp64"
    assert bench.traffic_from_profiles("fft.hip", rec["stage"], other, rec["config"]) is None
    assert bench.traffic_from_profiles("fft.hip", rec["stage"], rec["precision"], rec["config"] + 1) is None
    assert bench.traffic_from_profiles("fft.hip", "y_lines", rec["precision"], rec["config"]) is None
    assert bench.traffic_from_profiles("api.hip", rec["stage"], rec["precision"], rec["config"]) is None
