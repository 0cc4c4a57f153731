"""The profile summary tool: counter means and records are taken over real
dispatches only (graph-chunk launches that return at once are left out), and
kernel names are shortened to the stage kinds the bench reports."""
import csv
import json

from paper_2309_05331_amd import prof_summary as ps

D6 = "void hode::(anonymous namespace)::gs_stage<float, 8, 1, 4>(hode::GSLaunch, hode::DevCtrl*)"
EW = "void hode::(anonymous namespace)::ew_step<double, 1, 3>(hode::DevCtrl*, double*, double*, long)"


def _csv(path, counter, rows):
    cols = ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        t = 1000
        for name, value, us in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
                        "Start_Timestamp": t, "End_Timestamp": t + int(us * 1000)})
            t += int(us * 1000) + 500


def test_short_names():
    assert ps.short(D6) == "gs_stage D6 float ry=1 vw=4"
    assert ps.short(D6.replace("1, 4>", "1, 4, 8>")) == "gs_stage D6 float ry=1 vw=4 nw=8"
    assert ps.short(D6.replace("1, 4>", "1, 4, 4>")) == "gs_stage D6 float ry=1 vw=4"
    assert ps.short(EW) == "ew_step double rhs=1 mode=3"
    assert ps.short("void hode::ew_ab<float, 2, 4>(x)") == "ew_ab float rhs=2 s=4"
    assert ps.short("void hode::(anonymous namespace)::ens_kernel<float>(x)") == "ens_kernel float"


def test_counter_means_skip_empty_dispatches(tmp_path):
    fe, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    # three real launches and two empty ones (the run had already finished)
    _csv(fe, "FETCH_SIZE", [(D6, 3000.0, 1500), (D6, 3100.0, 1490), (D6, 18.0, 3), (D6, 2900.0, 1510),
                            (D6, 18.0, 2)])
    _csv(wr, "WRITE_SIZE", [(D6, 2048.0, 1500), (D6, 0.0, 3), (D6, 2048.0, 1495), (D6, 2048.0, 1505),
                            (D6, 0.0, 2)])
    rec = ps.counters_record(str(fe), str(wr), 2.0, 1.0, "gs_stage D6 float ry=1 vw=4", "D6", "w", "stage.h")
    assert rec["dispatches"] == 3
    assert rec["fetch_kib"] == 3000.0 and rec["write_kib"] == 2048.0
    assert rec["hbm_bytes_per_launch"] == (3000 * 2 + 2048) * 1024
    table = ps.counters(str(fe), str(wr), 2.0, 1.0)
    row = [ln for ln in table.splitlines() if ln.startswith("gs_stage D6")][0].split()
    assert row[-4:] == ["3", "3000.0", "2048.0", "%.4g" % ((3000 * 2 + 2048) * 1024)]
    # per run: the sum over the real launches
    run = ps.counters_record(str(fe), str(wr), 2.0, 1.0, "gs_stage D6 float ry=1 vw=4", "D6", "w", "stage.h",
                             per="run")
    assert run["hbm_bytes_per_run"] == (9000 * 2 + 3 * 2048) * 1024
    json.dumps(rec)


def test_early_exit_launch_above_the_absolute_cut_is_still_empty(tmp_path):
    # a graph-chunk launch that returns at once can take a little over 20 us
    # on a large grid; next to 1.5 ms launches of the same kernel it is
    # empty all the same (below 5% of the median of the longer ones), while a
    # kernel whose every launch is short keeps them all
    fe, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    short_k = D6.replace("1, 4>", "2, 4>")
    _csv(fe, "FETCH_SIZE", [(D6, 3000.0, 1500), (D6, 40.0, 20.5), (D6, 3000.0, 1490), (short_k, 100.0, 45),
                            (short_k, 100.0, 44)])
    _csv(wr, "WRITE_SIZE", [(D6, 2048.0, 1500), (D6, 0.0, 20.5), (D6, 2048.0, 1495), (short_k, 50.0, 45),
                            (short_k, 50.0, 44)])
    rec = ps.counters_record(str(fe), str(wr), 2.0, 1.0, "gs_stage D6 float ry=1 vw=4", "D6", "w", "stage.h")
    assert rec["dispatches"] == 2 and rec["fetch_kib"] == 3000.0 and rec["write_kib"] == 2048.0
    rec2 = ps.counters_record(str(fe), str(wr), 2.0, 1.0, "gs_stage D6 float ry=2 vw=4", "D6", "w", "stage.h")
    assert rec2["dispatches"] == 2 and rec2["fetch_kib"] == 100.0
    assert ps._split_empty([1500.0, 20.5, 1490.0, 3.0], 20.0) == [True, False, True, False]
    assert ps._split_empty([45.0, 44.0, 21.0], 20.0) == [True, True, True]
