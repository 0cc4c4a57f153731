"""bench.py reports measured HBM traffic only while the committed counter
record still applies: a change to any kernel source or included header named
in the record voids it (the field becomes null)."""
import json
import os
import shutil

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _tree(tmp_path, tag):
    rec = json.load(open(os.path.join(ROOT, "profiles", "counters_%s.json" % tag)))
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "counters_%s.json" % tag), tmp_path / "profiles")
    csrc = tmp_path / "paper_2309_05331_amd" / "csrc"
    csrc.mkdir(parents=True)
    for nm in rec["sources"]:
        shutil.copy(os.path.join(ROOT, "paper_2309_05331_amd", "csrc", nm), csrc / nm)
    return rec, csrc


def test_committed_records_apply_to_the_current_sources():
    for tag in ("D6_gs512-dp5", "ens_kernel_ens512-dp5"):
        v = bench.traffic_from_profiles(tag)
        assert isinstance(v, int) and v > 0, tag
    assert bench.traffic_from_profiles("no_such_kernel") is None


def test_a_changed_header_voids_the_record(tmp_path, monkeypatch):
    rec, csrc = _tree(tmp_path, "D6_gs512-dp5")
    assert "hode_dev.h" in rec["sources"]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("D6_gs512-dp5") == rec["hbm_bytes_per_launch"]
    with open(csrc / "hode_dev.h", "a") as f:
        f.write("\n// changed\n")
    assert bench.traffic_from_profiles("D6_gs512-dp5") is None
