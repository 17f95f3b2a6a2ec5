"""Host-side serving arithmetic (no GPU): the one-at-a-time latencies from
measured service times, and the latency summary.

The one-at-a-time leg is the FIFO queue: request i starts at
max(arrival_i, finish_{i-1}) and runs for its measured service time.  The
expected values are worked out by hand below.
"""

import dataclasses

import numpy as np

from paper_2506_15411_amd.serve import (ServedResult, ServiceTime, fifo_one_at_a_time,
                                        service_times, summarize)


@dataclasses.dataclass
class _Scene:
    shape: tuple


@dataclasses.dataclass
class _Req:
    rid: int
    kind: str
    scene: _Scene
    arrival: float


def test_fifo_recurrence_by_hand():
    # arrivals 0, 1, 1.5, 10; services 2, 1, 3, 0.5
    reqs = [_Req(3, "forward", _Scene((4, 4, 4)), 10.0), _Req(0, "forward", _Scene((4, 4, 4)), 0.0),
            _Req(2, "adjoint", _Scene((4, 4, 4)), 1.5), _Req(1, "forward", _Scene((4, 4, 4)), 1.0)]
    service = {0: ServiceTime(2.0, 0, (5, 0)), 1: ServiceTime(1.0, 0, (3, 0)),
               2: ServiceTime(3.0, 0, (4, 4)), 3: ServiceTime(0.5, 1, (9, 0))}
    out = fifo_one_at_a_time(reqs, service)
    assert [r.rid for r in out] == [0, 1, 2, 3]          # served in arrival order
    # 0: [0, 2]; 1: waits for 0, [2, 3]; 2: waits for 1, [3, 6]; 3: idle queue, [10, 10.5]
    assert [(r.admitted, r.finished) for r in out] == [(0.0, 2.0), (2.0, 3.0), (3.0, 6.0),
                                                       (10.0, 10.5)]
    assert [r.latency for r in out] == [2.0, 2.0, 4.5, 0.5]
    assert out[3].status == 1 and out[2].iterations == (4, 4)


def test_service_times_and_summary():
    res = [ServedResult(i, "forward", (2, 3, 4), 0, (10, 0), float(i), float(i) + 0.5,
                        float(i) + 0.5 + 0.1 * (i + 1)) for i in range(7)]
    st = service_times(res)
    assert np.allclose([st[i].seconds for i in range(7)], [0.1 * (i + 1) for i in range(7)])
    s = summarize(res)
    lat = np.array([0.5 + 0.1 * (i + 1) for i in range(7)])
    assert s["requests"] == 7
    assert np.isclose(s["p50_latency_s"], np.percentile(lat, 50))
    assert np.isclose(s["p99_latency_s"], np.percentile(lat, 99))
    wall = res[-1].finished - res[0].arrival
    assert np.isclose(s["wall_s"], wall)
    assert np.isclose(s["throughput_solves_per_s"], 7 / wall)
    assert np.isclose(s["gvoxel_iter_per_s"], 7 * 24 * 10 / wall / 1e9)
    assert s["not_ok"] == 0
