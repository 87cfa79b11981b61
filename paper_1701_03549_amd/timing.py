"""Load balance of a persistent simulation launch from its per-simulation
clocks (fire_set_sim_timing): when each simulation was taken by a workgroup
and when its result was written, in ticks of the device's 100 MHz clock.

* span: first take to last result;
* slots: the most simulations running at once (the resident workgroups);
* efficiency: simulation-time summed over all simulations / (slots x span),
  1.0 when every slot is busy from the first take to the last result;
* tail: last result minus the last take (after the last simulation has
  started, slots only empty);
* drain: last result minus the last moment every slot was busy (from then
  on at least one slot stays idle).
"""
from __future__ import annotations

import numpy as np

CLOCK_HZ = 100e6


def load_balance(times: np.ndarray, hz: float = CLOCK_HZ) -> dict:
    t = np.asarray(times, dtype=np.int64).reshape(-1, 2)
    t = t[(t[:, 0] > 0) & (t[:, 1] >= t[:, 0])]
    if t.shape[0] == 0:
        raise ValueError("no complete (take, finish) pairs")
    start, end = t[:, 0], t[:, 1]
    t0, t1 = int(start.min()), int(end.max())
    span = max(t1 - t0, 1)
    # running count over the sorted take (+1) and finish (-1) events; at
    # equal times finishes come first (a slot freed and retaken)
    ev_t = np.concatenate([start, end])
    ev_d = np.concatenate([np.ones_like(start), -np.ones_like(end)])
    order = np.lexsort((ev_d, ev_t))
    ev_t, ev_d = ev_t[order], ev_d[order]
    running = np.cumsum(ev_d)
    slots = int(running.max())
    busy = int((end - start).sum())
    # the event after which the running count never again reaches `slots`
    full = np.nonzero(running == slots)[0]
    drain_from = int(ev_t[full[-1] + 1]) if full[-1] + 1 < ev_t.size else t1
    dur = end - start
    return {
        "sims": int(t.shape[0]),
        "span_ms": span / hz * 1e3,
        "slots": slots,
        "efficiency": busy / (slots * span),
        "tail_ms": (t1 - int(start.max())) / hz * 1e3,
        "drain_ms": (t1 - drain_from) / hz * 1e3,
        "longest_sim_ms": float(dur.max()) / hz * 1e3,
        "median_sim_ms": float(np.median(dur)) / hz * 1e3,
    }
