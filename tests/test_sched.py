"""The serving scheduler on the CPU, driven by a fake executor that completes
planned steps on command: admission by memory and slots, full coverage of
every request's work items, continuous batching, cancellation, refusal."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
QUEUED, ACTIVE, DONE, CANCELLED = 0, 1, 2, 3


@pytest.fixture(scope="module")
def lib():
    from paper_2609_35619_amd import build as b
    path = b.build_sched_test_lib()
    L = ctypes.CDLL(path)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    L.sched_new.restype = P
    L.sched_new.argtypes = [U64, U64, I32, I64, I64]
    L.sched_free.argtypes = [P]
    L.sched_set_min_items.argtypes = [P, I64]
    L.sched_submit.restype = I64
    L.sched_submit.argtypes = [P, I32, I32, I32, I64, U64, U64, D]
    L.sched_admit.restype = I32
    L.sched_admit.argtypes = [P, D, P, I32]
    L.sched_plan.restype = I64
    L.sched_plan.argtypes = [P, P, I32, P, I32, P, P, P]
    L.sched_step_done.restype = I32
    L.sched_step_done.argtypes = [P, I64, D, P, I32]
    for f in ("sched_cancel",):
        getattr(L, f).restype = I32
        getattr(L, f).argtypes = [P, I64, D]
    for f in ("sched_finish", "sched_state", "sched_slot"):
        getattr(L, f).restype = I32
        getattr(L, f).argtypes = [P, I64]
    for f in ("sched_active", "sched_queued"):
        getattr(L, f).restype = I32
        getattr(L, f).argtypes = [P]
    for f in ("sched_dev_free", "sched_host_free", "sched_dev_largest"):
        getattr(L, f).restype = U64
        getattr(L, f).argtypes = [P]
    return L


class Fake:
    """Fake executor: plans steps and completes them in order."""

    def __init__(self, lib, dev=1 << 30, host=1 << 30, slots=4, step_pairs=1000, max_items=64):
        self.L = lib
        self.s = lib.sched_new(dev, host, slots, step_pairs, max_items)
        self.t = 0.0
        self.issued = {}      # ticket -> list of (tile, split)
        self.slot_of = {}
        self.inflight = []    # (step, items, completing)

    def close(self):
        self.L.sched_free(self.s)

    def submit(self, tiles, splits, pairs=10, dev=1000, host=1000, variant=0):
        return self.L.sched_submit(self.s, tiles, splits, variant, pairs, dev, host, self.t)

    def admit(self):
        out = (ctypes.c_int64 * 64)()
        n = self.L.sched_admit(self.s, self.t, out, 64)
        for t in out[:n]:
            self.slot_of[self.L.sched_slot(self.s, t)] = t
        return list(out[:n])

    def plan(self):
        items = (ctypes.c_int32 * (4 * 4096))()
        comp = (ctypes.c_int32 * 64)()
        ni, nc, pairs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        step = self.L.sched_plan(self.s, items, 4096, comp, 64, ctypes.byref(ni), ctypes.byref(nc),
                                 ctypes.byref(pairs))
        if step == 0:
            return None
        arr = np.frombuffer(items, np.int32)[:4 * ni.value].reshape(-1, 4)
        for slot, tile, split, _ in arr:
            self.issued.setdefault(self.slot_of[int(slot)], []).append((int(tile), int(split)))
        self.inflight.append((step, arr.copy(), list(comp[:nc.value]), pairs.value))
        return step, arr, list(comp[:nc.value]), pairs.value

    def complete_oldest(self):
        step = self.inflight.pop(0)[0]
        self.t += 1.0
        out = (ctypes.c_int64 * 64)()
        n = self.L.sched_step_done(self.s, step, self.t, out, 64)
        return list(out[:n])

    def state(self, t):
        return self.L.sched_state(self.s, t)


def test_every_item_issued_once_and_requests_complete(lib):
    f = Fake(lib, slots=3, step_pairs=50, max_items=16)
    reqs = {f.submit(tiles=7, splits=3): (7, 3), f.submit(tiles=1, splits=1): (1, 1),
            f.submit(tiles=20, splits=2): (20, 2), f.submit(tiles=4, splits=5): (4, 5)}
    done = set()
    for _ in range(200):
        f.admit()
        p = f.plan()
        if p is None and not f.inflight:
            break
        if f.inflight:
            done |= set(f.complete_oldest())
    assert done == set(reqs)
    for t, (tiles, splits) in reqs.items():
        got = sorted(f.issued[t])
        assert got == sorted((a, b) for b in range(splits) for a in range(tiles)), t
        assert f.state(t) == DONE
    assert lib.sched_active(f.s) == 0
    for t in reqs:
        assert lib.sched_finish(f.s, t) == 1
    assert lib.sched_dev_free(f.s) == 1 << 30 and lib.sched_host_free(f.s) == 1 << 30
    f.close()


def test_step_budget_and_round_robin(lib):
    f = Fake(lib, slots=4, step_pairs=40, max_items=1000)
    a = f.submit(tiles=100, splits=1, pairs=10)
    b = f.submit(tiles=100, splits=1, pairs=10)
    f.admit()
    step, items, comp, pairs = f.plan()
    assert pairs == 40 and len(items) == 4
    # both requests progress in the same step (continuous batching, fair share)
    assert set(items[:, 0].tolist()) == {lib.sched_slot(f.s, a), lib.sched_slot(f.s, b)}
    f.close()


def test_new_request_joins_while_others_run(lib):
    """A small request that arrives while a large one is on the device is
    admitted at once and finishes long before the large one."""
    f = Fake(lib, slots=4, step_pairs=100, max_items=1000)
    big = f.submit(tiles=500, splits=2, pairs=10)
    f.admit()
    f.plan()
    f.plan()            # two steps of the big request in flight
    small = f.submit(tiles=2, splits=1, pairs=10)
    assert f.admit() == [small]
    done_at = {}
    for step in range(200):
        for t in f.complete_oldest() if f.inflight else []:
            done_at[t] = step
        f.admit()
        f.plan()
        if not f.inflight:
            break
    assert done_at[small] < 4 < done_at[big]
    f.close()


def test_admission_by_memory_and_slots(lib):
    f = Fake(lib, dev=10_000, host=10_000, slots=2, step_pairs=1000)
    a = f.submit(1, 1, dev=6000)
    b = f.submit(1, 1, dev=6000)      # does not fit next to a
    c = f.submit(1, 1, dev=3000)      # fits: smaller requests are not blocked behind b
    assert f.admit() == [a, c]
    assert f.state(b) == QUEUED
    d = f.submit(1, 1, dev=100)       # no free slot
    assert f.admit() == [] and f.state(d) == QUEUED
    # never fits: refused at submit
    assert f.submit(1, 1, dev=20_000) == -1 and f.submit(1, 1, host=20_000) == -1
    f.plan()
    f.complete_oldest()
    assert f.state(a) == DONE and f.state(c) == DONE
    assert set(f.admit()) == {b, d}
    f.close()


def test_cancel_queued_active_and_inflight(lib):
    f = Fake(lib, slots=1, step_pairs=10, max_items=100)
    a = f.submit(tiles=50, splits=1, pairs=10)
    b = f.submit(tiles=5, splits=1, pairs=10)
    f.admit()
    assert lib.sched_cancel(f.s, b, 0.0) == 1 and f.state(b) == CANCELLED   # queued: dropped
    f.plan()                                   # one item of a in flight
    assert lib.sched_cancel(f.s, a, 0.0) == 1
    assert f.state(a) == ACTIVE                # in-flight item still on the device
    assert f.plan() is None                    # nothing more is issued for a
    assert f.complete_oldest() == [a] and f.state(a) == CANCELLED
    assert lib.sched_finish(f.s, a) == 1 and lib.sched_finish(f.s, b) == 1
    assert lib.sched_dev_free(f.s) == 1 << 30
    f.close()


def test_zero_item_request_gets_a_combine_only_step(lib):
    f = Fake(lib, slots=2)
    t = f.submit(tiles=3, splits=0)   # empty scene: nothing to evaluate, outputs still written
    f.admit()
    step, items, comp, pairs = f.plan()
    assert len(items) == 0 and comp == [lib.sched_slot(f.s, t)]
    assert f.complete_oldest() == [t] and f.state(t) == DONE
    f.close()


def test_arena_coalesces(lib):
    f = Fake(lib, dev=1 << 20, host=1 << 20, slots=8, step_pairs=1 << 40, max_items=1 << 20)
    ts = [f.submit(1, 1, dev=100_000, host=10) for _ in range(8)]
    f.admit()
    f.plan()
    f.complete_oldest()
    for t in ts:
        lib.sched_finish(f.s, t)
    assert lib.sched_dev_largest(f.s) == 1 << 20
    f.close()


def test_min_items_overrides_a_small_budget(lib):
    """A step of a few long items would leave the device idle: with a minimum,
    the step takes that many items even past the pair budget."""
    f = Fake(lib, slots=2, step_pairs=10, max_items=100)
    lib.sched_set_min_items(f.s, 6)
    t = f.submit(tiles=20, splits=1, pairs=1000)
    f.admit()
    step, items, comp, pairs = f.plan()
    assert len(items) == 6 and pairs == 6000
    f.close()
