"""Host-side logic of bench.py (no GPU): the committed profile summaries
are used only while the kernel sources hash to the profiled ones and the
launch settings match."""
import hashlib
import os

import bench

LAUNCH = {"tile_variant": 2, "tile_block": 256, "bank_align": 1, "sort_every": 4}


def _write(tmp_path, sha, config="tile_variant 2, tile_block 256, bank_align 1, sort_every 4", extra=()):
    p = tmp_path / "profile.md"
    p.write_text("\n".join(["# summary", "", "config: " + config, *extra, "kernel_source_sha256: " + sha]) + "\n")
    return str(p)


def _sha():
    return hashlib.sha256(b"".join(open(os.path.join(bench.HERE, f), "rb").read()
                                   for f in bench.KERNEL_SOURCES)).hexdigest()


def test_profile_fields_need_matching_sources_and_launch(tmp_path):
    good = _write(tmp_path, _sha(), extra=("traffic_bytes_per_launch: 123",))
    assert bench._profile_fields(good, LAUNCH)["traffic_bytes_per_launch"] == "123"
    assert bench._profile_fields(_write(tmp_path, "0" * 64), LAUNCH) is None
    assert bench._profile_fields(good, dict(LAUNCH, tile_block=512)) is None
    assert bench._profile_fields(str(tmp_path / "missing.md"), LAUNCH) is None


def test_valu_ceiling_from_the_sq_summary(tmp_path, monkeypatch):
    path = _write(tmp_path, _sha(), extra=("valu_per_particle_wave: 833.0", "valu_issue_us_per_pass: 355.4"))
    os.rename(path, path + ".f32")
    monkeypatch.setattr(bench, "SQ_PROFILE", path + ".{}")
    c = bench.valu_ceiling(LAUNCH, "f32", 899678208.0)
    assert c["valu_per_particle_wave"] == 833.0
    assert abs(c["valu_issue_ms_per_pass"] - 0.3554) < 1e-12
    # 899.7 MB in 355.4 us is 2.53 TB/s: 0.316 of 8 TB/s
    assert abs(c["hbm_frac_at_valu_issue"] - 899678208.0 / 355.4e-6 / 8e12) < 1e-12


def test_algorithmic_bytes_per_pass():
    # one FP32 species of the 128x64x32 box: 16,777,216 particles, 262,144 nodes
    assert bench.algorithmic_bytes(16777216, 262144, 4, 4) == 899678208
    assert bench.algorithmic_bytes(16777216, 262144, 8, 8) == 1778384896
