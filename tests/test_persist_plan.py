"""CPU checks of the persistent factorisation's task plan and queue protocol
(paper_1805_00569_amd/csrc/persist_plan.hpp), by an event simulation in
tests/persist_sim.cpp: every task taken once, no deadlock under random task
times with own-queue-first dispatch, a task starts only after its system's
earlier stages, every system runs on the one XCD that owns its queue (also
when only some XCDs hold workers and the others' queues are claimed), and
the tasks of each system cover its blocked factorisation exactly (one column
per stage, or the column-pair stages).  Batches: the balanced workload (96 systems of 64
tile rows), ragged K-means-sized batches (sizes up to 219 tile rows, i.e.
m = 14,000), one very large system, and tiny or degenerate shapes."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("psim") / "persist_sim")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "persist_sim.cpp")], check=True,
                   capture_output=True)
    return exe


def _run(sim, seed, workers, packed, wp, sizes):
    r = subprocess.run([sim, str(seed), str(workers), str(int(packed)), str(wp)] + [str(int(t)) for t in sizes],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
    return r.stdout.split()


def _ragged_tiles(seed, n_sys=32):
    """Tile rows of a K-means-like ragged batch: sizes 512..14,000 points."""
    g = np.random.default_rng(seed)
    m = np.clip(np.round(131072 * g.dirichlet(np.full(n_sys, 0.8))), 512, 14000)
    return np.ceil(m / 64).astype(int)


# packed: 0 the FP32/FP64 matrix-core path, 1 the BF16 packed path, 2 the
# packed path with column-pair stages
@pytest.mark.parametrize("packed", [1, 0, 2])
def test_balanced_batch(sim, packed):
    out = _run(sim, 1, 512, packed, 16, [64] * 96)
    assert out[3] == "8"   # one queue per XCD


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("packed", [1, 0, 2])
def test_ragged_batches(sim, seed, packed):
    _run(sim, 10 + seed, 512, packed, 16, _ragged_tiles(seed))


@pytest.mark.parametrize("workers", [1, 3, 64])
def test_few_workers_and_odd_panels(sim, workers):
    _run(sim, 5, workers, True, 5, [13, 1, 2, 40, 7, 7, 9, 3, 64])
    _run(sim, 6, workers, False, 3, [13, 1, 2, 40, 7])
    _run(sim, 7, workers, 2, 5, [13, 1, 2, 40, 7, 7, 9, 3, 64])
    _run(sim, 8, workers, 2, 2, [13, 1, 2, 3, 4, 40])


def test_one_large_system(sim):
    out = _run(sim, 7, 512, True, 16, [256])
    assert out[3] == "1"   # fewer systems than XCDs: one shared queue
    out = _run(sim, 7, 512, 2, 24, [256])
    assert out[3] == "1"


def test_single_tiles(sim):
    _run(sim, 8, 8, True, 16, [1] * 9)
    _run(sim, 9, 8, False, 16, [1, 1])
    _run(sim, 10, 8, 2, 16, [1] * 9 + [2, 3])


@pytest.mark.parametrize("packed", [1, 0, 2])
def test_per_system_panel_widths(sim, packed):
    """Each system with its own panel width (as the autotuner may choose)."""
    _run(sim, 21, 256, packed, 0, _ragged_tiles(4, n_sys=24))
    _run(sim, 22, 16, packed, 0, [5, 64, 1, 17, 33, 2, 9, 64, 40])
