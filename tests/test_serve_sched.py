"""Host-side scheduling of the serving layer: which slot takes which jobs.

The server's dispatch decisions (micro-batch composition, the slot an
oversized job goes to, memory admission) are plain host logic; these tests
drive them on CPU tensors without contexts, streams or threads.
"""
from __future__ import annotations

import collections
import threading

import pytest

torch = pytest.importorskip("torch")

from paper_2410_08946_amd import serve  # noqa: E402


def make_server(slots=4, budget=1 << 40, max_batch_jobs=64, max_batch_pixels=1000):
    s = serve.Server.__new__(serve.Server)
    s.budget = budget
    s.max_batch_jobs = max_batch_jobs
    s.max_batch_pixels = max_batch_pixels
    s.in_use = 0
    s.queue = collections.deque()
    s.lock = threading.Condition()
    s.slots = [{"k": k, "work": None} for k in range(slots)]
    return s


def job(jid, shape, conn=8, NL=4, dtype=torch.uint8, footprint=1):
    j = serve.Job(grad=torch.zeros(shape, dtype=dtype), conn=conn, NL=NL, jid=jid)
    j.footprint = footprint
    return j


def ids(batch):
    return [j.jid for j in batch]


def test_batch_groups_compatible_jobs_in_order():
    s = make_server()
    s.queue.extend([job(0, (10, 10)), job(1, (4, 4, 4), conn=6), job(2, (20, 20)), job(3, (10, 10), NL=3),
                    job(4, (5, 5))])
    slot, allow_big = s._pick_slot()
    assert slot["k"] == 1 and not allow_big  # ordinary work prefers the slots other than 0
    batch, foot = s._take_batch(allow_big)
    # 2D and 3D jobs of any connectivity share a micro-batch; NL must match
    assert ids(batch) == [0, 1, 2, 4] and foot == 4
    assert [j.jid for j in s.queue] == [3]  # skipped jobs keep their order
    s.queue.extend([job(5, (4, 4, 4), conn=26, dtype=torch.uint16), job(6, (9, 9), NL=3)])
    batch, _ = s._take_batch(allow_big)
    assert ids(batch) == [3, 6] and [j.jid for j in s.queue] == [5]  # one grey type per micro-batch


def test_pixel_cap_closes_the_batch():
    s = make_server(max_batch_pixels=500)
    s.queue.extend([job(0, (10, 20)), job(1, (10, 20)), job(2, (10, 20)), job(3, (2, 2))])
    batch, _ = s._take_batch(False)
    assert ids(batch) == [0, 1]  # the third would exceed 500 pixels: it and all after wait
    assert [j.jid for j in s.queue] == [2, 3]


def test_oversized_head_runs_on_slot_zero_alone():
    s = make_server(max_batch_pixels=1000)
    s.queue.extend([job(0, (50, 50)), job(1, (10, 10)), job(2, (10, 10))])
    slot, allow_big = s._pick_slot()
    assert slot["k"] == 0 and allow_big
    batch, _ = s._take_batch(allow_big)
    assert ids(batch) == [0]
    assert [j.jid for j in s.queue] == [1, 2]


def test_oversized_head_does_not_block_other_slots():
    s = make_server(max_batch_pixels=1000)
    s.slots[0]["work"] = ("busy", 0)
    s.queue.extend([job(0, (50, 50)), job(1, (10, 10)), job(2, (60, 60)), job(3, (10, 10))])
    slot, allow_big = s._pick_slot()
    assert slot["k"] != 0 and not allow_big
    batch, _ = s._take_batch(allow_big)
    assert ids(batch) == [1, 3]  # the oversized jobs stay queued, in order, for slot 0
    assert [j.jid for j in s.queue] == [0, 2]
    # nothing ordinary is left: the other slots take nothing, slot 0 gets them when free
    assert s._take_batch(False)[0] == []
    s.slots[0]["work"] = None
    slot, allow_big = s._pick_slot()
    assert slot["k"] == 0 and allow_big
    assert ids(s._take_batch(True)[0]) == [0]


def test_only_slot_zero_free_takes_ordinary_work():
    s = make_server(slots=3)
    for k in (1, 2):
        s.slots[k]["work"] = ("busy", 0)
    s.queue.extend([job(0, (10, 10))])
    slot, allow_big = s._pick_slot()
    assert slot["k"] == 0
    assert ids(s._take_batch(allow_big)[0]) == [0]


def test_no_free_slot():
    s = make_server(slots=2)
    for sl in s.slots:
        sl["work"] = ("busy", 0)
    s.queue.append(job(0, (10, 10)))
    assert s._pick_slot() is None


def test_memory_admission():
    s = make_server(budget=100)
    s.in_use = 60
    s.queue.extend([job(0, (10, 10), footprint=30), job(1, (10, 10), footprint=30), job(2, (10, 10), footprint=5)])
    batch, foot = s._take_batch(False)
    assert ids(batch) == [0] and foot == 30  # the second does not fit: the batch closes in order
    s.in_use += foot
    assert s._take_batch(False)[0] == []  # memory busy: nothing until a completion
    assert [j.jid for j in s.queue] == [1, 2]


def test_job_cap():
    s = make_server(max_batch_jobs=3)
    s.queue.extend(job(k, (4, 4)) for k in range(7))
    assert ids(s._take_batch(False)[0]) == [0, 1, 2]
    assert ids(s._take_batch(False)[0]) == [3, 4, 5]
    assert ids(s._take_batch(False)[0]) == [6]
