"""Host code built with sanitizers by g++:
the ordering code (the plan's step a0) on random, tied, duplicated and
degenerate inputs, whose permutations must equal the oracle's (brute-force
definitions), and the serving loop's first-fit arena against a brute-force
model, under AddressSanitizer and UndefinedBehaviorSanitizer; the serving
loop's scheduler (submit, poll, grouping, retirement, shutdown) with many
client threads against a simulated device, under ThreadSanitizer and under
AddressSanitizer. The sanitizers must stay silent. Host code only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ordering

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_15195_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "order_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "order_check.cpp"), os.path.join(CSRC, "host_order.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    return exe


def _run(exe, locs):
    text = f"{len(locs)}\n" + "\n".join(f"{float(x)!r} {float(y)!r}" for x, y in locs) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    lines = r.stdout.strip().splitlines()
    return np.array(lines[0].split(), dtype=np.int64), np.array(lines[1].split(), dtype=np.int64)


def _cases():
    rng = np.random.default_rng(11)
    yield rng.random((1, 2))
    yield rng.random((2, 2))
    yield rng.random((777, 2))
    g = np.array([(a / 9.0, b / 9.0) for a in range(10) for b in range(10)])   # ties everywhere
    yield g
    d = rng.random((50, 2))
    yield np.concatenate([d, d[:20], d[:5]])                                     # duplicates
    yield np.column_stack([rng.random(200), np.full(200, 0.5)])                  # collinear, zero y-range
    yield np.full((7, 2), 3.25)                                                  # one point seven times
    yield rng.normal(0.0, 1e6, size=(300, 2))                                    # wide coordinates


def test_orderings_under_sanitizers(checker):
    for locs in _cases():
        coord, maxmin = _run(checker, locs)
        assert np.array_equal(coord, ordering.coord_order(locs))
        assert np.array_equal(maxmin, ordering.maxmin_order(locs))


def test_serving_arena_against_a_brute_force_model(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "arena_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "arena_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-500:], r.stderr[-2000:])


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_serving_scheduler_under_sanitizers(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitizer}", "-I", CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "sched_check.cpp"), "-o", exe, "-lpthread"]
    if "undefined" in sanitizer:
        cmd.insert(5, "-fno-sanitize-recover=undefined")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-1500:], r.stderr[-3000:])
    assert "ThreadSanitizer" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
