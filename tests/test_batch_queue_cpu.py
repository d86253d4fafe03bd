"""CPU model of the persistent batch's work-queue protocol (no GPU): a ring of tickets with
per-slot sequence numbers, workgroups that take tickets in order, per-problem phase counters
whose last finisher enqueues the next phase, and the exit once no problem is left.

Workgroups are simulated as generators advanced one atomic step at a time in a seeded random
order (every interleaving the steps allow is possible), with problems of uneven item counts
and iteration counts.  The checks: every problem runs its phases in order and finishes, every
item of every phase is executed exactly once, no producer ever finds its slot still unread,
the ring never holds more than half its capacity, and every workgroup returns."""
import os
import random
import re

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2101_07249_amd", "csrc",
                   "bpcg.hip")


def kernel_phase_graph():
    """The phase list, the successor of each phase and the phases the transition handles, as
    the persistent kernel's source defines them."""
    src = open(SRC).read()
    enum = re.search(r"enum Phase \{([^}]*)\}", src).group(1)
    phases = [t.strip().split("=")[0].strip()[3:] for t in enum.split(",") if t.strip()]
    phases = [ph for ph in phases if ph != "NPHASE"]
    body = re.search(r"constexpr int next_phase\(int ph\) \{(.*?)\n\}", src, re.S).group(1)
    nxt = {a: b for a, b in re.findall(r"case PH_(\w+): return PH_(\w+);", body)}
    tr = re.search(r"__device__ (?:__noinline__ )?bool transition\((.*?)\n\}\n", src, re.S).group(1)
    handled = set(re.findall(r"case PH_(\w+):", tr))
    return phases, nxt, handled


PHASES, NEXT, HANDLED = kernel_phase_graph()


def test_kernel_phase_graph_is_complete():
    """Every phase has a successor and a transition case; the successors form the start
    chain C1 -> C4 and the iteration cycle D1 -> ... -> P -> D1."""
    assert PHASES == ["C1", "C2", "C3", "C4", "D1", "FW", "BW", "D2", "T", "UP", "P"]
    assert set(NEXT) == set(PHASES) and set(PHASES) <= HANDLED
    chain, ph = [], "C1"
    while ph not in chain:
        chain.append(ph)
        ph = NEXT[ph]
    assert chain == PHASES and ph == "D1"


def phase_items(prob, ph):
    if ph in ("D1", "D2"):
        return prob["tiles"]
    if ph in ("FW", "BW"):
        return 1
    return prob["rows"]


def simulate(n_problems, n_wg, ring, seed):
    rnd = random.Random(seed)
    probs = []
    for p in range(n_problems):
        probs.append({"tiles": rnd.randint(1, 12), "rows": rnd.randint(1, 9), "iters": rnd.randint(0, 6),
                      "pending": 0, "done": False, "trace": []})
    seq = list(range(ring))
    items = [None] * ring
    head = 0
    tail = 0
    left = n_problems
    executed = {}
    max_outstanding = 0

    # host fill: the first phase of every problem
    for p, pr in enumerate(probs):
        pr["pending"] = phase_items(pr, "C1")
        for j in range(pr["pending"]):
            items[tail % ring] = (p, "C1", j, 0)
            seq[tail % ring] = tail + 1
            tail += 1

    state = {"head": head, "tail": tail, "left": left}

    def enqueue(p, ph, it):
        pr = probs[p]
        cnt = phase_items(pr, ph)
        pr["pending"] = cnt
        t0 = state["tail"]
        state["tail"] += cnt
        yield
        for j in range(cnt):
            t = t0 + j
            slot = t % ring
            # a producer never waits on an unread slot when the ring is at most half full
            assert seq[slot] == t, "producer found its slot still unread"
            items[slot] = (p, ph, j, it)
            seq[slot] = t + 1
            yield

    def transition(p, ph, it):
        pr = probs[p]
        pr["trace"].append(ph)
        if ph == "C4":
            if pr["iters"] == 0:
                pr["done"] = True
                state["left"] -= 1
                return
            yield from enqueue(p, "D1", 1)
        elif ph == "UP":
            if it >= pr["iters"]:
                pr["done"] = True
                state["left"] -= 1
                return
            yield from enqueue(p, "P", it)
        elif ph == "P":
            yield from enqueue(p, "D1", it + 1)
        else:
            yield from enqueue(p, NEXT[ph], it)

    def workgroup():
        while True:
            ticket = state["head"]
            state["head"] += 1
            yield
            slot = ticket % ring
            while seq[slot] != ticket + 1:
                if state["left"] <= 0:
                    return
                yield
            p, ph, j, it = items[slot]
            seq[slot] = ticket + ring
            yield
            key = (p, ph, j, it)
            assert key not in executed, f"item executed twice: {key}"
            executed[key] = True
            for _ in range(rnd.randint(0, 3)):   # the item's work
                yield
            probs[p]["pending"] -= 1
            last = probs[p]["pending"] == 0
            yield
            if last:
                yield from transition(p, ph, it)

    wgs = [workgroup() for _ in range(n_wg)]
    live = list(range(n_wg))
    steps = 0
    while live:
        w = rnd.choice(live)
        try:
            next(wgs[w])
        except StopIteration:
            live.remove(w)
        max_outstanding = max(max_outstanding, state["tail"] - state["head"])
        steps += 1
        assert steps < 5_000_000, "no progress (deadlock)"
    return probs, executed, max_outstanding


@pytest.mark.parametrize("seed", range(12))
def test_queue_protocol_drains_and_runs_every_item_once(seed):
    n_problems, n_wg = 7, 5
    # ring at least twice the largest sum of one phase per problem (the library's condition)
    ring = 2 * n_problems * 12
    probs, executed, max_out = simulate(n_problems, n_wg, ring, seed)
    for p, pr in enumerate(probs):
        assert pr["done"], p
        it = pr["iters"]
        expect = ["C1", "C2", "C3", "C4"] + ["D1", "FW", "BW", "D2", "T", "UP", "P"] * it
        if it:
            expect = expect[:-1]   # the last iteration ends at UP
        assert pr["trace"] == expect, (p, pr["trace"])
        for ph in PHASES:
            for i in range(1, it + 1) if ph not in ("C1", "C2", "C3", "C4") else [0]:
                if ph == "P" and i == it:
                    continue
                for j in range(phase_items(pr, ph)):
                    assert (p, ph, j, i) in executed, (p, ph, j, i)
    total = sum(4 * pr["rows"] + pr["iters"] * (2 * pr["tiles"] + 2 + 3 * pr["rows"]) - (pr["rows"] if pr["iters"] else 0)
                for pr in probs)
    assert len(executed) == total
    assert max_out <= ring // 2


def test_queue_protocol_with_more_workgroups_than_items():
    probs, executed, _ = simulate(2, 40, 48, 99)
    assert all(pr["done"] for pr in probs)
