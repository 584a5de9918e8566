"""The request loop's scheduling policy on the CPU (simulated time; no device).

tests/sched_driver.cpp links only paper_1005_5198_amd/csrc/rs_sched.h (pure host
logic) and prints the outcomes checked here.
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def res(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_1005_5198_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sched_driver.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return json.loads(out)


def test_admission_by_footprint_fifo(res):
    assert res["admit1"] == [1, 2]          # 600 + 300 fit 1000; 200 does not
    assert res["done1"] == [1, 2]           # both finished in one big step
    assert res["admit2"] == [3, 4]          # then 3 (not overtaken by 4) and 4
    assert res["rejected"] == [5]           # larger than the whole budget
    assert res["plan1_rows_quantum"]


def test_slot_limit(res):
    assert res["slots_admit"] == [1, 2] and res["slots_waiting"] == 3


def test_shortest_remaining_first(res):
    step1 = res["srpt_step1"]
    # the small job (2: 70 rows) takes its whole remainder first; the large one still gets one band
    assert step1[0] == [2, 0, 70, 1]
    assert step1[1] == [1, 0, 32, 1]
    assert res["srpt_done1"] == [2]
    # then job 1 alone: 968 rows left at 128 per step
    assert res["srpt_total_steps"] == 1 + -(-(1000 - 32) // 128)


def test_starvation_guard(res):
    # the big job has waited past starve_s: it takes the whole budget (128 rows); the small one
    # waits for the next step (only the first job may go past the budget)
    assert res["starve_step1"] == [[1, 0, 128]]
    # neither has waited that long: least remaining work first, as before
    assert res["starve_none"] == [[2, 0, 70], [1, 0, 32]]


def test_cancellation(res):
    assert res["cancel_dropped"] == [2]
    assert res["cancel_plan_after"] == 0    # a cancelled job gets no more slices
    assert res["cancel_reaped"] == 1 and res["cancel_reaped_flag"]
    assert res["cancel_active_left"] == 0


def test_arena(res):
    assert res["arena_three"] and not res["arena_full"]
    assert res["arena_hole"] == 1024        # 4096 - 3*1024 = 1024 tail; hole of 1024
    assert res["arena_coalesced"] == 2048
    assert res["arena_empty"] == 4096 and res["arena_in_use"] == 0 and res["arena_peak"] == 3072


def test_percentiles(res):
    assert float(res["p50"]) == 50.0 and float(res["p99"]) == 99.0 and float(res["p100"]) == 100.0
