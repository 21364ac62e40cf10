"""Host-side batching and admission of the serving loop (no GPU)."""
from dataclasses import dataclass

import pytest

from paper_2511_00735_amd.serve import Planner, Record, summarize


@dataclass
class Req:
    name: str
    n: int
    N: int
    arrival: float = 0.0


def fp(shape, count):
    n, N = shape
    return count * n * n * N      # bytes proportional to elements x order


def test_batches_one_shape_in_arrival_order():
    pl = Planner(fp, budget=10 ** 9, max_batch=3)
    reqs = [Req("a", 8, 8), Req("b", 16, 8), Req("c", 8, 8), Req("d", 8, 8), Req("e", 8, 8)]
    for r in reqs:
        pl.add(r)
    batch, need = pl.take()
    assert [r.name for r in batch] == ["a", "c", "d"]       # oldest fixes the shape; max_batch 3
    assert need == fp((8, 8), 3)
    batch, _ = pl.take()
    assert [r.name for r in batch] == ["b"]
    batch, _ = pl.take()
    assert [r.name for r in batch] == ["e"]
    assert pl.take() is None


def test_admission_by_footprint_shrinks_then_waits():
    one = fp((8, 8), 1)
    pl = Planner(fp, budget=2 * one, max_batch=8)
    for i in range(5):
        pl.add(Req(f"r{i}", 8, 8))
    batch, need = pl.take()
    assert len(batch) == 2 and need == 2 * one            # shrunk to what fits
    assert pl.take() is None                               # nothing left: waits
    pl.release(need)
    batch2, need2 = pl.take()
    assert [r.name for r in batch2] == ["r2", "r3"]
    pl.release(need2)
    batch3, _ = pl.take()
    assert [r.name for r in batch3] == ["r4"]


def test_request_larger_than_budget_is_an_error():
    pl = Planner(fp, budget=fp((8, 8), 1) - 1)
    pl.add(Req("big", 8, 8))
    with pytest.raises(ValueError):
        pl.take()


def test_summary_percentiles():
    recs = []
    for i in range(100):
        r = Record(f"q{i}", 8, 8, arrival=0.01 * i, dof=10)
        r.finish = r.arrival + 0.001 * (i + 1)
        r.status = 0
        r.relres = 1e-9
        r.batch = 1
        recs.append(r)
    s = summarize(recs)
    assert s["completed"] == 100 and s["converged"] == 100
    assert abs(s["latency_p50_ms"] - 50.5) < 1e-6
    assert abs(s["latency_p99_ms"] - 99.01) < 1e-6


def test_batch_budget_caps_a_batch_but_not_a_lone_request():
    one = fp((8, 8), 1)
    pl = Planner(fp, budget=10 * one, max_batch=8, batch_budget=3 * one)
    for i in range(5):
        pl.add(Req(f"r{i}", 8, 8, arrival=float(i)))
    batch, need = pl.take()
    assert [r.name for r in batch] == ["r0", "r1", "r2"] and need == 3 * one
    # a request larger than the per-batch budget still runs alone while it
    # fits the free budget
    big = fp((16, 8), 1)
    assert big > 3 * one
    pl2 = Planner(fp, budget=10 * one, max_batch=8, batch_budget=3 * one)
    pl2.add(Req("big", 16, 8))
    pl2.add(Req("big2", 16, 8))
    batch, need = pl2.take()
    assert [r.name for r in batch] == ["big"] and need == big


def test_arena_layout_is_aligned_disjoint_and_exact():
    """A batch's buffers inside a worker's arena: 256-byte aligned, disjoint,
    the group workspace first at the library's exact footprint (host-side
    sizing through the C ABI; no GPU)."""
    from paper_2511_00735_amd.serve import Server
    from paper_2511_00735_amd import hps
    srv = Server(precision="mixed", workers=2, memory_budget=64 << 30)
    for shape, count in (((8, 8), 1), ((16, 12), 5), ((32, 16), 3)):
        off, total = srv.layout(shape, count)
        ws = hps.group_workspace_bytes(srv.desc(*shape), count)
        n, N = shape
        E, p = n * n, N - 1
        spans = [(0, ws)]
        for r in off["req"]:
            spans += [(r["b"], 8 * E * (N + 1) ** 2)] + [(r[k], 16 * E * 4 * p) for k in ("t", "rhs", "g")]
        spans += [(off[k], 8 * E * (N + 1) ** 2) for k in ("tmpa", "tmpb", "tmpc")]
        spans.sort()
        for (o1, l1), (o2, _) in zip(spans, spans[1:]):
            assert o1 % 256 == 0 and o1 + l1 <= o2
        assert spans[-1][0] + spans[-1][1] <= total == srv.footprint(shape, count)
        assert srv.footprint(shape, count + 1) > total


def test_request_larger_than_an_arena_is_refused():
    from paper_2511_00735_amd.serve import Server
    from paper_2511_00735_amd import workloads
    pr = workloads.c3()
    srv = Server(precision="fp64", workers=4, memory_budget=4 << 30)   # 1 GiB arenas
    with pytest.raises(ValueError):
        srv.run([pr])
