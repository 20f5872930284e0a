"""CPU checks of the serving admission logic with a fake device budget:
the pool allocator and the footprint admission policy (no GPU)."""
import random

from paper_0912_3912_amd.serve import ALIGN, Admission, Pool


def test_pool_alloc_release_coalesce():
    p = Pool(10 * ALIGN)
    a = p.alloc(1)
    b = p.alloc(ALIGN + 1)
    c = p.alloc(3 * ALIGN)
    assert (a, b, c) == (0, ALIGN, 3 * ALIGN)
    assert p.used == 6 * ALIGN and p.largest_free() == 4 * ALIGN
    assert p.alloc(5 * ALIGN) is None
    p.release(b, ALIGN + 1)
    assert p.alloc(3 * ALIGN) == 6 * ALIGN           # first fit skips the 2-unit hole
    p.release(a, 1)
    p.release(c, 3 * ALIGN)
    assert p.largest_free() == 6 * ALIGN               # holes merged: [0, 6)
    assert p.alloc(6 * ALIGN) == 0
    assert p.peak == 9 * ALIGN


def test_pool_random_never_overlaps():
    rng = random.Random(3)
    p = Pool(1 << 20)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            p.release(off, live.pop(off))
        else:
            n = rng.randint(1, 40000)
            off = p.alloc(n)
            if off is not None:
                need = (n + ALIGN - 1) // ALIGN * ALIGN
                for o, m in live.items():
                    mm = (m + ALIGN - 1) // ALIGN * ALIGN
                    assert off + need <= o or o + mm <= off
                assert off % ALIGN == 0 and off + need <= p.size
                live[off] = n
        assert p.used == sum((m + ALIGN - 1) // ALIGN * ALIGN for m in live.values())
    for off, n in list(live.items()):
        p.release(off, n)
    assert p.free == [(0, p.size)]


def test_admission_skips_ahead_and_respects_slots():
    pool = Pool(100 * ALIGN)
    adm = Admission(pool, slots=2)
    assert adm.add(0, rid=10, footprint=80 * ALIGN)
    assert adm.add(1, rid=11, footprint=60 * ALIGN)
    assert adm.add(2, rid=12, footprint=10 * ALIGN)
    assert not adm.add(3, rid=13, footprint=101 * ALIGN)   # larger than the pool: rejected
    r1 = adm.next()
    assert r1[0] == 10
    r2 = adm.next()
    assert r2[0] == 12                                      # 11 does not fit yet, 12 does
    assert adm.next() is None                               # no slot left
    adm.finish(r1[1], r1[2], 80 * ALIGN)
    r3 = adm.next()
    assert r3[0] == 11 and r3[1] == r1[1]
    assert adm.cancel(11) is False                          # already admitted
    assert adm.add(4, rid=14, footprint=1)
    assert adm.cancel(14) is True and adm.next() is None


def test_admission_budget_is_never_exceeded():
    rng = random.Random(9)
    pool = Pool(1000 * ALIGN)
    adm = Admission(pool, slots=4)
    footprint = {}
    running = []
    order = 0
    for _ in range(2000):
        if rng.random() < 0.6:
            footprint[order] = rng.randint(1, 400) * ALIGN
            adm.add(order, order, footprint[order])
            order += 1
        if running and rng.random() < 0.5:
            rid, slot, off = running.pop(rng.randrange(len(running)))
            adm.finish(slot, off, footprint[rid])
        while True:
            nxt = adm.next()
            if nxt is None:
                break
            running.append(nxt)
        assert pool.used == sum(footprint[r[0]] for r in running) <= pool.size
        assert len(running) <= 4
        assert len({r[1] for r in running}) == len(running)
