"""Host model of the persistent batched launch's scheduling loop (CPU).

tests/persist_model.cpp runs the loop of csrc/tnrd_persist.hpp, the source the
GPU kernel k_batched_persist runs, with threads standing for waves, real
barriers and std::atomic flags, and replaces each stage's work by the reads
and writes it makes in the exchange form (u planes, slab sets) on plain
words.  Under ThreadSanitizer every such read and overwrite must be ordered
by the loop's synchronisation, and every stamp read must be the one the stage
before wrote.  The checks: every item runs once, every flag ends at T + 1,
every output holds u_T, no wait gives up; with far more workgroups than tiles
per stage (most items wait on neighbours); and a launch whose waits give up
(after one poll, or once the workgroup's clock budget is spent) still ends
with the abort flag raised (the path that keeps a GPU launch finite).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "persist_model.cpp")
INC = os.path.join(ROOT, "paper_1702_07482_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build(tmp_path, tsan):
    exe = str(tmp_path / ("pm_tsan" if tsan else "pm"))
    flags = ["-std=c++20", "-pthread", "-Wall", "-Wno-unknown-pragmas", "-I", INC]
    flags += ["-O1", "-g", "-fsanitize=thread"] if tsan else ["-O2"]
    subprocess.check_call(["g++", *flags, SRC, "-o", exe])
    return exe


@pytest.fixture(scope="module")
def model_tsan(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("pm"), True)


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("pm"), False)


# (seed, workgroups, waves per workgroup, stages)
CASES = [(1, 4, 4, 6), (2, 4, 4, 8), (3, 16, 2, 5), (4, 40, 2, 6), (5, 2, 8, 3), (6, 1, 4, 4)]


@pytest.mark.parametrize("seed,wgs,waves,stages", CASES)
def test_schedule_is_race_free_and_complete(model_tsan, seed, wgs, waves, stages):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([model_tsan, str(seed), str(wgs), str(waves), str(stages), "100000000",
                        "100000000000", "0"],
                       capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "stamps off 0" in r.stdout and "abort 0" in r.stdout


# (spin limit, clock budget in ns): give up after one poll; after 1 ms with
# unbounded polls
@pytest.mark.parametrize("seed,limits", [(1, ("1", "100000000000")), (2, ("1", "100000000000")),
                                         (3, ("2000000000", "1000000")), (4, ("2000000000", "1000000"))])
def test_waits_that_give_up_still_end_the_launch(model, seed, limits):
    r = subprocess.run([model, str(seed), "48", "2", "5", *limits, "1"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "ended; abort flag 1" in r.stdout
