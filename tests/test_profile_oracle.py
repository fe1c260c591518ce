"""Pins of the event-profile oracle (oracle/profile.py).

* Fig. 3 of the paper (Section 6.1) prints one profile summary. Its printed
  inputs (three aggregate times, one overlap, the elapsed time) determine its
  printed outputs (relative times, effective time, device/host split); a
  synthetic event list with exactly those inputs must reproduce the printed
  outputs to within the rounding of the printed inputs.
* With two in-order queues at most two events are in flight at once, so
  "sum of durations minus pairwise overlaps" must equal the measure of the
  union of all event intervals, which a brute-force count over a tiny integer
  time grid gives independently.
"""
import numpy as np
import pytest

from oracle import profile as prof


def fig3_events():
    """Event list whose totals equal Fig. 3's printed inputs.

    INIT_KERNEL: one event of 6.2464e-05 s on the main queue. READ_BUFFER:
    100 reads of 66.521 ms (6.6521 s) on the comms queue. RNG_KERNEL: 99
    kernels (0.81531 s) on the main queue; kernel k starts before read k ends
    and overlaps it, 15.790 ms of overlap in all; read k+1 starts when kernel
    k ends (the paper's pipeline order).
    """
    ev = [prof.Event("INIT_KERNEL", "Main", 0, 62464)]
    read_d = 66_521_000
    rng_d = [8_235_455] * 98 + [815_310_000 - 98 * 8_235_455]
    ov = [159_495] * 98 + [15_790_000 - 98 * 159_495]
    t = 62464
    for k in range(100):
        ev.append(prof.Event("READ_BUFFER", "Comms", t, t + read_d))
        if k < 99:
            s = t + read_d - ov[k]
            ev.append(prof.Event("RNG_KERNEL", "Main", s, s + rng_d[k]))
            t = s + rng_d[k]
    return ev


def test_fig3_summary_reproduced():
    p = prof.analyze(fig3_events(), 9.054619)
    names = [r[0] for r in p.agg]
    assert names == ["READ_BUFFER", "RNG_KERNEL", "INIT_KERNEL"]
    counts = {r[0]: r[1] for r in p.agg}
    assert counts == {"READ_BUFFER": 100, "RNG_KERNEL": 99, "INIT_KERNEL": 1}
    rel = {r[0]: r[3] for r in p.agg}
    ab = {r[0]: r[2] for r in p.agg}
    # Absolute times are the inputs.
    assert ab["READ_BUFFER"] == pytest.approx(6.6521, abs=1e-12)
    assert ab["RNG_KERNEL"] == pytest.approx(0.81531, abs=1e-12)
    assert ab["INIT_KERNEL"] == pytest.approx(6.2464e-05, abs=1e-15)
    # Printed with 4 decimals (+-5e-5 %); the printed inputs are themselves
    # rounded (READ_BUFFER to +-5e-5 s), which moves the shares by at most
    # ~7e-5 %: allow 1.5e-4 %.
    assert rel["READ_BUFFER"] == pytest.approx(89.0810, abs=1.5e-4)
    assert rel["RNG_KERNEL"] == pytest.approx(10.9182, abs=1.5e-4)
    assert rel["INIT_KERNEL"] == pytest.approx(0.0008, abs=5e-5 + 1e-5)
    assert p.total_s == pytest.approx(7.4674, abs=5e-5 + 5.6e-5)
    assert p.overlaps == [("RNG_KERNEL", "READ_BUFFER", pytest.approx(1.5790e-02, abs=1e-12))]
    # Printed eff is 7.451659; the sum of the rounded printed inputs minus the
    # overlap differs from it by their rounding (<= 5.6e-5 s).
    assert p.eff_s == pytest.approx(7.451659, abs=5.6e-5)
    assert p.elapsed_s == 9.054619
    assert p.device_pct == pytest.approx(82.30, abs=0.005 + 1e-3)
    assert p.host_pct == pytest.approx(17.70, abs=0.005 + 1e-3)
    assert p.device_pct + p.host_pct == pytest.approx(100.0)


def _union_measure(events):
    hi = max(e.end_ns for e in events)
    covered = np.zeros(hi + 1, dtype=bool)
    for e in events:
        covered[e.start_ns:e.end_ns] = True
    return int(covered.sum())


@pytest.mark.parametrize("seed", range(40))
def test_two_queues_eff_equals_union(seed):
    rng = np.random.default_rng(seed)
    events = []
    for q in ("A", "B"):
        t = int(rng.integers(0, 5))
        for _ in range(int(rng.integers(1, 12))):
            d = int(rng.integers(0, 9))
            name = str(rng.choice(["K", "R", "I"]))
            events.append(prof.Event(name, q, t, t + d))
            t += d + int(rng.integers(0, 4))
    p = prof.analyze(events, 1.0)
    assert round(p.eff_s * 1e9) == _union_measure(events)
    assert round(p.total_s * 1e9) == sum(e.end_ns - e.start_ns for e in events)
    assert round(sum(o[2] for o in p.overlaps) * 1e9) == round(p.overlap_s * 1e9)


def test_hand_examples():
    ev = [prof.Event("K", "main", 0, 10), prof.Event("R", "comms", 4, 20),
          prof.Event("K", "main", 12, 15)]
    p = prof.analyze(ev, 40e-9)
    assert [(r[0], r[1], round(r[2] * 1e9)) for r in p.agg] == [("R", 1, 16), ("K", 2, 13)]
    assert [(a, b, round(c * 1e9)) for a, b, c in p.overlaps] == [("K", "R", 9)]
    assert round(p.eff_s * 1e9) == 20
    assert p.device_pct == pytest.approx(50.0)
    # Same-queue events never count as overlapping.
    p2 = prof.analyze([prof.Event("K", "q", 0, 10), prof.Event("K", "q", 5, 8)], 1.0)
    assert p2.overlaps == []
    # Same-name events on different queues form a (name, name) row.
    p3 = prof.analyze([prof.Event("K", "a", 0, 10), prof.Event("K", "b", 5, 8)], 1.0)
    assert [(a, b, round(c * 1e9)) for a, b, c in p3.overlaps] == [("K", "K", 3)]
    with pytest.raises(ValueError):
        prof.analyze([prof.Event("K", "a", 5, 4)], 1.0)
