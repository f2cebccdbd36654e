"""The request loop's memory-based admission (paper_2212_09807_amd/csrc/admission.hpp) under fake budgets, on the CPU:
batches are halved until they fit the lane's share and the free device memory, the events cut off go back to the
queue front in order, an event that alone exceeds the share is rejected, and every event is run or rejected exactly
once, in queue order."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MB = 1 << 20


@pytest.fixture(scope="module")
def scenarios(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("adm") / "admission_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-I",
                           os.path.join(ROOT, "paper_2212_09807_amd", "csrc"),
                           os.path.join(ROOT, "tests", "admission_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.strip().splitlines():
        name, *steps = line.split()
        parsed = []
        for s in steps:
            if s.startswith("run:"):
                ids, total = s[4:].split("@")
                parsed.append(("run", [int(x) for x in ids.split(",")], int(total)))
            elif s.startswith("released:"):
                parsed.append(("released", [], int(s.split(":")[1])))
            else:
                parsed.append(("reject", [int(s.split(":")[1])], 0))
        res[name] = parsed
    return res


def _order(steps):
    return [e for kind, ids, _ in steps if kind != "released" for e in ids]


def test_everything_fits_in_one_batch_of_16(scenarios):
    s = scenarios["all_fit"]
    assert [len(ids) for _, ids, _ in s] == [16, 4] and _order(s) == list(range(20))


def test_budget_halves_batches_until_they_fit(scenarios):
    s = scenarios["budget_5"]               # 50 + 100 k MB within 560 MB: k <= 5
    assert all(kind == "run" and total <= 560 * MB for kind, _, total in s)
    # each tentative batch is the queue head (up to 16), halved until it fits: 16 -> 8 -> 4, then 12 -> 6 -> 3,
    # 9 -> 4, and the last 5 fit as they are
    assert [len(ids) for _, ids, _ in s] == [4, 4, 3, 4, 5]
    assert _order(s) == list(range(20))     # FIFO kept: cut-off events went back to the queue front


def test_free_device_memory_limits_growth(scenarios):
    s = scenarios["free_memory_3"]          # growth <= 1360 - 1000 MB: 50 + 100 k <= 360 -> k <= 3
    assert all(kind == "run" and total <= 360 * MB for kind, _, total in s)
    assert max(len(ids) for _, ids, _ in s) == 3 and _order(s) == list(range(20))


def test_event_larger_than_the_share_is_rejected_alone(scenarios):
    s = scenarios["big_events"]
    rejected = [ids[0] for kind, ids, _ in s if kind == "reject"]
    assert rejected == [0, 7]
    ran = [e for kind, ids, _ in s if kind == "run" for e in ids]
    assert sorted(ran) == [e for e in range(20) if e not in (0, 7)]
    assert _order(s) == list(range(20))
    assert all(total <= 4000 * MB for kind, _, total in s if kind == "run")


def test_mixed_sizes_every_event_exactly_once(scenarios):
    s = scenarios["mixed"]
    assert sorted(_order(s)) == list(range(12)) and _order(s) == list(range(12))
    assert [ids for kind, ids, _ in s if kind == "reject"] == [[7]]       # 1500 MB > 1000 MB share
    assert all(total <= 1000 * MB for kind, _, total in s if kind == "run")


def test_nothing_fits(scenarios):
    s = scenarios["nothing_fits"]
    assert [kind for kind, _, _ in s] == ["reject"] * 20 and _order(s) == list(range(20))


def test_pool_release_admits_an_event_the_grown_pool_refused(scenarios):
    """A lane's pool keeps every buffer at its largest size; a single event refused because of that pool is sized
    again after the lane releases it, and only an event that alone exceeds the share is rejected."""
    MB = 1 << 20
    steps = scenarios["pool_release"]
    assert steps[0] == ("run", list(range(16)), 50 * MB + 3200 * MB)
    assert steps[1] == ("run", [16], 50 * MB + 2000 * MB)      # only after the pool was released
    assert steps[2] == ("reject", [17], 0)
    assert steps[3] == ("released", [], 2)
