"""The library's plan, graph and event bookkeeping under the host sanitizers
(CPU only): flame_api.hip built for the host with AddressSanitizer and
UndefinedBehaviorSanitizer against a checked model of the HIP calls it makes
(tests/native/hipstub), driven through long sequences of graph builds,
replays, drops and rebuilds, timing sessions and autotuning."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-I", os.path.join(NATIVE, "hipstub"),
         "-I", os.path.join(ROOT, "paper_0911_2889_amd", "csrc"), "-I", os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def drive(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("g++ is not available")
    out = tmp_path_factory.mktemp("sanitize")
    api = out / "flame_api.o"
    subprocess.run([cxx] + FLAGS + ["-x", "c++", "-c", os.path.join(ROOT, "paper_0911_2889_amd", "csrc",
                                                                     "flame_api.hip"), "-o", str(api)],
                   check=True, capture_output=True)
    exe = out / "plan_bookkeeping_check"
    subprocess.run([cxx] + FLAGS + [os.path.join(NATIVE, "hipstub", "hip_stub.cpp"),
                                    os.path.join(NATIVE, "plan_bookkeeping_check.cpp"), str(api), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def test_bookkeeping_is_clean_under_sanitizers(drive):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([str(drive)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "ALL OK" in res.stdout
    assert "graph launches" in res.stdout and " 0, " not in res.stdout.split("graph launches")[1][:4]


def test_the_model_reports_a_graph_destroyed_with_a_queued_launch(drive):
    """The stub's lifetime model catches the pattern of destroying a graph exec
    while a launch of it is still queued on a stream (what drop_graph avoids
    by draining the plan's stream first)."""
    res = subprocess.run([str(drive), "control"], capture_output=True, text=True, timeout=60)
    assert res.returncode != 0
    assert "graph exec destroyed while a launch of it is still queued" in res.stderr
