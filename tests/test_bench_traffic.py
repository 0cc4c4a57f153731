"""bench.py reports measured HBM traffic only while a counter record still
applies: a change to any kernel source or included header named in the
record voids it (the field becomes null)."""
import glob
import hashlib
import json
import os
import shutil

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2309_05331_amd", "csrc")


def test_committed_records_are_well_formed():
    recs = sorted(glob.glob(os.path.join(ROOT, "profiles", "counters_*.json")))
    assert recs
    for path in recs:
        rec = json.load(open(path))
        assert rec["sources"] and all(os.path.exists(os.path.join(CSRC, nm)) for nm in rec["sources"]), path
        assert len(rec["sources_sha256"]) == 64
        v = rec.get("hbm_bytes_per_launch", rec.get("hbm_bytes_per_run"))
        assert isinstance(v, int) and v > 0, path
        # FETCH_SIZE and WRITE_SIZE in KiB, scaled by the copy calibration
        assert v == round((rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024) \
            or abs(v - (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024) <= 1024
        tag = os.path.basename(path)[len("counters_"):-len(".json")]
        # applies exactly when the named sources are unchanged
        h = hashlib.sha256()
        for nm in rec["sources"]:
            h.update(open(os.path.join(CSRC, nm), "rb").read())
        expect = v if h.hexdigest() == rec["sources_sha256"] else None
        assert bench.traffic_from_profiles(tag) == expect, tag
    assert bench.traffic_from_profiles("no_such_kernel") is None


def test_a_changed_header_voids_the_record(tmp_path, monkeypatch):
    sources = ["stage.h", "gs.hip", "hode_dev.h", "hode_internal.h"]
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_2309_05331_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for nm in sources:
        shutil.copy(os.path.join(CSRC, nm), csrc / nm)
        h.update(open(csrc / nm, "rb").read())
    rec = {"kernel": "D6", "workload": "w", "sources": sources, "sources_sha256": h.hexdigest(),
           "fetch_kib": 1.0, "write_kib": 1.0, "fetch_scale": 2.0, "write_scale": 1.0,
           "hbm_bytes_per_launch": 3072}
    json.dump(rec, open(tmp_path / "profiles" / "counters_D6_w.json", "w"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("D6_w") == 3072
    with open(csrc / "hode_dev.h", "a") as f:
        f.write("\n// changed\n")
    assert bench.traffic_from_profiles("D6_w") is None
