"""Host logic of bench.py (CPU): the HBM counter summary and the roofline
entries it feeds.  Synthetic rocprofv3 counter files stand in for a run."""
import csv
import os

import pytest

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": f"void cpic::{name}(int, int)", "Counter_Name": counter,
                        "Counter_Value": value})


def make_runs(tmp_path):
    copy_kib = (256 << 20) / 1024
    write_counters(tmp_path / "cf", "FETCH_SIZE", [(1, "copy_kernel", copy_kib / 2)])   # reads half: factor 2
    write_counters(tmp_path / "cw", "WRITE_SIZE", [(1, "copy_kernel", copy_kib)])
    a, b = "field_ctile_kernel<double, 64, 8, 2>", "field_ctile_kernel<double, 64, 4, 2>"
    # run 1: 64x8 throughout (40 dispatches); run 2: 64x8 for a 20-dispatch warm-up, then 64x4
    for c, scale in (("FETCH_SIZE", 1.0), ("WRITE_SIZE", 2.0)):
        r1 = [(i, a, scale * (100.0 if i >= 24 else 1.0)) for i in range(40)]
        r1 += [(100 + i, "push_kernel<double, 4, false>", scale * 7.0) for i in range(40)]
        r2 = [(i, a, scale * 3.0) for i in range(20)] + [(20 + i, b, scale * 50.0) for i in range(20)]
        write_counters(tmp_path / f"r1_{c}", c, r1)
        write_counters(tmp_path / f"r2_{c}", c, r2)
    return a, b


def test_summary_takes_each_kernel_from_its_own_run(tmp_path):
    a, b = make_runs(tmp_path)
    out = tmp_path / "pmc.txt"
    t = str(tmp_path)
    bench.pmc_summary(str(out), f"{t}/r1_FETCH_SIZE,{t}/r2_FETCH_SIZE", f"{t}/r1_WRITE_SIZE,{t}/r2_WRITE_SIZE",
                      f"{t}/cf", f"{t}/cw", "cmd one; cmd two", "a test workload")
    text = out.read_text()
    assert "a test workload" in text and "#   cmd two" in text
    got = bench.read_pmc_summary(str(out))
    # the 64x8 kernel from run 1 (its last 16 dispatches), not from run 2's warm-up
    assert got[a] == (pytest.approx(100 * 1024 * 2), pytest.approx(200 * 1024))
    assert got[b] == (pytest.approx(50 * 1024 * 2), pytest.approx(100 * 1024))
    assert got["push_kernel<double, 4, false>"] == (pytest.approx(7 * 1024 * 2), pytest.approx(14 * 1024))


def test_summary_of_other_sources_is_ignored(tmp_path):
    make_runs(tmp_path)
    out = tmp_path / "pmc.txt"
    t = str(tmp_path)
    bench.pmc_summary(str(out), f"{t}/r1_FETCH_SIZE", f"{t}/r1_WRITE_SIZE", f"{t}/cf", f"{t}/cw", "c", "w")
    out.write_text(out.read_text().replace(bench.kernel_source_hash(), "0" * 64))
    assert bench.read_pmc_summary(str(out)) is None
    assert bench.read_pmc_summary(str(tmp_path / "missing.txt")) is None


def test_rooflines_attach_traffic_by_kernel_name(tmp_path, monkeypatch):
    make_runs(tmp_path)
    out = tmp_path / "pmc.txt"
    t = str(tmp_path)
    bench.pmc_summary(str(out), f"{t}/r1_FETCH_SIZE", f"{t}/r1_WRITE_SIZE", f"{t}/cf", f"{t}/cw", "c", "w")
    monkeypatch.setitem(bench.PMC_SUMMARIES, "512_fp64", str(out))
    res = {"timing": {"field_ms": 7.5, "n_field": 100, "push_ms": 4.4, "n_push": 100},
           "launch": {"variant": 3, "bx": 64, "by": 8, "nt_store": 1, "push_lanes": 4, "push_mode": "gather"}}
    V = 512 * 512
    k = bench.rooflines(res, "fp64", 10**5, V)
    f = k["field"]
    assert f["kernel"] == "field_ctile_kernel<double, 64, 8, 2>"
    assert f["traffic"] == pytest.approx(100 * 1024 * 2 + 200 * 1024)
    assert f["traffic_read"] == pytest.approx(100 * 1024 * 2) and f["traffic_written"] == pytest.approx(200 * 1024)
    # a site-update is priced at 68 reals read and written (full links), the
    # two-row figure (56 + 56 reals) beside it
    assert f["bytes_per_unit"] == 1088 and f["bytes_per_unit_two_row_links"] == 896
    assert f["frac"] == pytest.approx(1088 * V / 75e-6 / 8e12)
    assert f["frac_two_row_links"] == pytest.approx(896 * V / 75e-6 / 8e12)
    assert k["push"]["traffic"] == pytest.approx(7 * 1024 * 2 + 14 * 1024)
    # another tile than the one counted, or a two-kernel push not counted: no traffic
    res["launch"].update(by=4, push_mode="table")
    k = bench.rooflines(res, "fp64", 10**5, V)
    assert k["field"]["traffic"] is None and k["push"]["traffic"] is None
    assert k["push"]["kernel"] == "force_table_kernel<double> + push_table_kernel<double>"


def test_step_plan_reaches_formation_and_fits_the_run():
    # the driver's short run: the warm-up is extended past the formation step
    w, kt = bench.plan_steps(20, 5, 69)
    assert w == 70 and kt == 128
    assert w + kt + 48 + 20 <= 1024
    w, kt = bench.plan_steps(512, 96, 69)
    assert w == 96 and w + kt + 48 + 512 <= 1024
    assert bench.formation_step(bench.charm()) == 69
    assert bench.formation_step(bench.jet_quarks()) == 0
    with pytest.raises(SystemExit):
        bench.plan_steps(1000, 5, 69)
