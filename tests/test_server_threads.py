"""The request loop's threads (paper_1005_5198_amd/csrc/rs_server_core.h) on the CPU, over a
simulated device (tests/server_driver.cpp), under ThreadSanitizer and under
AddressSanitizer + UndefinedBehaviorSanitizer: four clients submit, poll, wait and cancel at
once while a fifth reads the statistics; a bounded waiting queue refuses with RS_EBUSY; a
device error fails every unfinished request. No GPU.

ThreadSanitizer needs clang (ROCm's): GCC 11's runtime does not intercept the clocked
condition-variable wait of libstdc++ and reports false double locks.
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "server_driver.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1005_5198_amd", "csrc")]
CLANG = shutil.which("clang++", path="/opt/rocm/llvm/bin") or shutil.which("clang++")

RS_EBUSY, RS_EHIP = -4, -3


def run(cmd_compile, exe, env=None):
    subprocess.run(cmd_compile + [SRC, "-o", exe, "-lpthread"], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    return json.loads(p.stdout)


@pytest.fixture(scope="module", params=["tsan", "asan_ubsan"])
def res(request, tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("srv") / f"server_{request.param}")
    if request.param == "tsan":
        if CLANG is None:
            pytest.skip("clang++ not found")
        cmd = [CLANG, "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=thread", *INC]
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    else:
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", *INC]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    return run(cmd, exe, env)


def test_concurrent_clients_get_exact_maps(res):
    assert res["mix_bad"] == 0 and res["mix_other"] == 0
    # 120 requests: 8 larger than the pool, up to 6 cancelled, the rest exact
    assert res["mix_nomem"] == 8
    assert res["mix_ok"] + res["mix_canceled"] == 112
    assert res["mix_completed"] == res["mix_ok"]
    assert res["mix_in_use_after"] == 0


def test_bounded_queue_refuses_with_ebusy(res):
    assert res["busy_refused"] >= 1
    assert res["busy_refused"] + res["busy_accepted"] == 12
    assert res["busy_accepted_ok"] == res["busy_accepted"]
    assert res["busy_counter"] == res["busy_refused"]


def test_device_error_fails_unfinished_requests(res):
    assert res["err_first"] == 0
    assert res["err_failed"] == res["err_submitted"] == 6
    assert res["err_after"] == RS_EHIP
