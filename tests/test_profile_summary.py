"""Host logic of the rocprofv3 summaries that the committed profiles and the
bench line's counter-based figures come from, on small hand-made databases
in the layout rocprofv3 writes (a counters_collection table per run)."""
import os
import sqlite3

import pytest

from paper_2403_09990_amd import profile_summary as S


def _db(tmp_path, name, rows):
    d = tmp_path / name
    d.mkdir()
    con = sqlite3.connect(str(d / "run_results.db"))
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, "
                "value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(d)


def _dispatch(did, kernel, **vals):
    # every counter split over two hardware instances, as the per-XCD rows are
    out = []
    for k, v in vals.items():
        out += [(did, kernel, k, v / 2.0), (did, kernel, k, v / 2.0)]
    return out


def test_counters_keep_only_the_dispatches_that_carry_the_workload(tmp_path):
    # a warm-up launch of 4 iterations, two timed launches, and a launch group
    # with no instances (same kernel prefix, its waves exit at once)
    rows = (_dispatch(1, "k_sample<1, 0>", SQ_WAVES=8192, SQ_INSTS_VALU=4 * 100.0)
            + _dispatch(2, "k_sample<1, 0>", SQ_WAVES=8192, SQ_INSTS_VALU=10000 * 100.0)
            + _dispatch(3, "k_sample<1, 0>", SQ_WAVES=8192, SQ_INSTS_VALU=10002 * 100.0)
            + _dispatch(4, "k_sample<0, 0>", SQ_WAVES=8192, SQ_INSTS_VALU=50.0)
            + _dispatch(5, "k_prologue", SQ_WAVES=2, SQ_INSTS_VALU=1e9))
    c = S.counters(_db(tmp_path, "p", rows), "k_sample")
    assert c["dispatches"] == 2 and c["dispatches_dropped"] == 2
    assert c["SQ_INSTS_VALU"] == pytest.approx(10001 * 100.0)
    assert c["SQ_WAVES"] == 8192


def test_counters_without_an_instruction_counter_weigh_by_the_sum(tmp_path):
    rows = (_dispatch(1, "k_x", FETCH_SIZE=10.0) + _dispatch(2, "k_x", FETCH_SIZE=1000.0)
            + _dispatch(3, "k_x", FETCH_SIZE=900.0))
    c = S.counters(_db(tmp_path, "p", rows), "k_x")
    assert c["dispatches"] == 2 and c["FETCH_SIZE"] == pytest.approx(950.0)


def test_valu_counts_64_lanes_and_two_operations_per_fma(tmp_path):
    rows = _dispatch(7, "k_sample<1, 0>", SQ_INSTS_VALU=100.0, SQ_INSTS_VALU_FMA_F32=10.0,
                     SQ_INSTS_VALU_MUL_F32=3.0, SQ_INSTS_VALU_ADD_F32=2.0, SQ_INSTS_VALU_TRANS_F32=1.0,
                     SQ_ACTIVE_INST_VALU=30.0, SQ_WAVE_CYCLES=60.0)
    out = str(tmp_path / "v.json")
    r = S.valu(_db(tmp_path, "p", rows), "k_sample", out, "cmd")
    assert r["f32_flops_per_dispatch"] == 64 * (2 * 10 + 3 + 2 + 1)
    assert r["valu_active_per_wave_cycle"] == pytest.approx(0.5)
    assert r["source_hash"] == S.source_hash("k_sample") == S.source_hash("k_sample<1, 0>")
    assert os.path.exists(out)


def test_valu_refuses_a_run_without_the_f32_counters(tmp_path):
    rows = _dispatch(1, "k_sample<1, 0>", SQ_INSTS_VALU=100.0)
    with pytest.raises(RuntimeError):
        S.valu(_db(tmp_path, "p", rows), "k_sample")


def test_traffic_scales_each_counter_by_the_calibration_copy(tmp_path):
    mib = 1 << 20
    fetch = (_dispatch(1, "k_sample<1, 0>", FETCH_SIZE=100.0) + _dispatch(2, "k_sample<0, 0>", FETCH_SIZE=1.0)
             + _dispatch(3, "__amd_rocclr_copyBuffer", FETCH_SIZE=512.0))      # reads half of 1 MiB
    write = (_dispatch(1, "k_sample<1, 0>", WRITE_SIZE=2048.0)
             + _dispatch(3, "__amd_rocclr_copyBuffer", WRITE_SIZE=1024.0))
    r = S.traffic(_db(tmp_path, "f", fetch), _db(tmp_path, "w", write), "k_sample", mib,
                  str(tmp_path / "t.json"))
    assert r["fetch"]["factor"] == pytest.approx(0.5) and r["write"]["factor"] == pytest.approx(1.0)
    assert r["bytes_per_launch"] == pytest.approx(100 * 1024 / 0.5 + 2048 * 1024)
