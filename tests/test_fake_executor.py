"""The server's admission control (paper_2302_05002_amd/csrc/fpo_sched.h, the
code the request server runs) driven by a simulated executor on the CPU:
requests with Poisson arrivals, workspace sizes up to the whole budget,
simulated build durations, results held by the client for a while, and
cancellations.  Checked: every request is admitted or cancelled (no
starvation), admissions follow arrival order, no more builds than slots run
at once, the arena never holds more than the budget and its blocks never
overlap, a cancelled request was never admitted, and everything is free at
the end.  Built with AddressSanitizer and UBSan (host code only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fake_executor.cpp")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("sim") / "fake_executor")
    subprocess.check_call([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", SRC, "-o", exe])
    return exe


def run(sim, seed, requests, slots, budget, cancel_every=0):
    out = subprocess.run([sim, str(seed), str(requests), str(slots), str(budget), str(cancel_every)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    ev = [line.split() for line in out.stdout.splitlines()]
    return ev


def check_trace(ev, requests, slots, budget):
    submit = {}
    admit = {}
    cancelled = set()
    running = 0
    used = 0
    live = {}
    order = []
    for e in ev:
        kind = e[0]
        if kind == "submit":
            submit[int(e[1])] = float(e[2])
        elif kind == "admit":
            i, off, size = int(e[1]), int(e[3]), int(e[4])
            assert i not in admit and i not in cancelled
            admit[i] = float(e[2])
            order.append(i)
            running += 1
            used += size
            assert running <= slots
            assert used <= budget
            for j, (o, s) in live.items():   # disjoint from every live block
                assert off + size <= o or o + s <= off, (i, j)
            assert off + size <= budget
            live[i] = (off, size)
        elif kind == "finish":
            running -= 1
        elif kind == "release":
            i = int(e[1])
            used -= live.pop(i)[1]
        elif kind == "cancel":
            if e[3] == "1":
                cancelled.add(int(e[1]))
        elif kind == "summary":
            assert int(e[1]) == len(admit) and int(e[2]) == len(cancelled)
    assert set(admit) | cancelled == set(range(requests)), "a request was neither admitted nor cancelled"
    assert not (set(admit) & cancelled)
    # first come, first served: admission order is arrival order
    assert order == sorted(order, key=lambda i: (submit[i], i))
    assert used == 0 and running == 0 and not live
    return admit, cancelled


@pytest.mark.parametrize("seed,requests,slots,budget_mb", [(1, 400, 4, 1000), (2, 400, 1, 1000), (3, 800, 8, 50),
                                                          (4, 300, 64, 100_000), (5, 500, 3, 7)])
def test_admission_invariants(sim, seed, requests, slots, budget_mb):
    budget = budget_mb << 20
    check_trace(run(sim, seed, requests, slots, budget), requests, slots, budget)


def test_cancellation_while_waiting(sim):
    budget = 64 << 20
    ev = run(sim, 11, 600, 2, budget, cancel_every=3)
    admit, cancelled = check_trace(ev, 600, 2, budget)
    assert cancelled, "the scenario should cancel some waiting requests"


def test_no_overtaking_by_small_requests(sim):
    """A request that needs the whole budget is admitted once everything
    before it has released, and no later (smaller) request starts before it."""
    budget = 256 << 20
    ev = run(sim, 21, 300, 4, budget)
    admit, _ = check_trace(ev, 300, 4, budget)
    sizes = {int(e[1]): int(e[4]) for e in ev if e[0] == "admit"}
    big = [i for i, s in sizes.items() if s > budget // 2]
    assert big, "the scenario should hold requests above half the budget"
    for i in big:
        assert all(admit[j] >= admit[i] for j in admit if j > i)
