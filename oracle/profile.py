"""Event-profile arithmetic, written out plainly -- TEST INFRASTRUCTURE.

Follows the profiler module of the cf4ocl paper (Section 4.3) and the summary
of Fig. 3 (Section 6.1):

* aggregate times by event name: the sum of (end - start) over the events of
  one name, and its share of the sum over all events;
* event overlaps: for two events on different queues, the length of the
  intersection of their [start, end) intervals, summed per pair of names
  (events of one in-order queue never overlap, Section 4.3);
* "Tot. of all events (eff.)": the sum of all durations minus the sum of all
  overlaps;
* "Time spent in device": eff / total elapsed host time; "in host": the rest.

Readings (the paper does not define them): an overlap row is an unordered
pair of names; it is printed with the name of smaller aggregate time first
(ties: by name), which matches Fig. 3's "RNG_KERNEL | READ_BUFFER" row.
Aggregates are sorted by time, descending, and overlap rows by duration,
descending (the flags passed in Section 6.1); ties by name.

Every pair of events is examined (O(E^2)); this is the definition, not a fast
algorithm.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class Event:
    name: str
    queue: str
    start_ns: int
    end_ns: int


@dataclass
class Profile:
    agg: list = field(default_factory=list)      # (name, count, abs_s, rel_pct)
    overlaps: list = field(default_factory=list)  # (name1, name2, overlap_s)
    total_s: float = 0.0
    overlap_s: float = 0.0
    eff_s: float = 0.0
    elapsed_s: float = 0.0
    device_pct: float = 0.0
    host_pct: float = 0.0


def analyze(events, elapsed_s: float) -> Profile:
    events = [e if isinstance(e, Event) else Event(*e) for e in events]
    for e in events:
        if e.end_ns < e.start_ns:
            raise ValueError("event %r ends before it starts" % (e,))
    total_ns = 0
    per_name = {}
    for e in events:
        d = e.end_ns - e.start_ns
        total_ns += d
        cnt, s = per_name.get(e.name, (0, 0))
        per_name[e.name] = (cnt + 1, s + d)

    pair_ns = {}
    for i in range(len(events)):
        a = events[i]
        for j in range(i + 1, len(events)):
            b = events[j]
            if a.queue == b.queue:
                continue
            ov = min(a.end_ns, b.end_ns) - max(a.start_ns, b.start_ns)
            if ov <= 0:
                continue
            key = frozenset((a.name, b.name)) if a.name != b.name else frozenset((a.name,))
            pair_ns[key] = pair_ns.get(key, 0) + ov
    overlap_ns = sum(pair_ns.values())

    p = Profile()
    p.total_s = total_ns * 1e-9
    p.overlap_s = overlap_ns * 1e-9
    p.eff_s = (total_ns - overlap_ns) * 1e-9
    p.elapsed_s = float(elapsed_s)
    if p.elapsed_s > 0:
        p.device_pct = 100.0 * p.eff_s / p.elapsed_s
        p.host_pct = 100.0 - p.device_pct
    rows = []
    for name, (cnt, s) in per_name.items():
        rel = 100.0 * s / total_ns if total_ns > 0 else 0.0
        rows.append((name, cnt, s * 1e-9, rel))
    rows.sort(key=lambda r: (-r[2], r[0]))
    p.agg = rows
    ovs = []
    for key, ns in pair_ns.items():
        names = sorted(key)
        if len(names) == 1:
            n1 = n2 = names[0]
        else:
            x, y = names
            tx, ty = per_name[x][1], per_name[y][1]
            n1, n2 = (x, y) if (tx, x) <= (ty, y) else (y, x)
        ovs.append((n1, n2, ns * 1e-9))
    ovs.sort(key=lambda r: (-r[2], r[0], r[1]))
    p.overlaps = ovs
    return p
