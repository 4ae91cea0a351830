"""The oracle's plane loops run in parallel (OpenMP); each iteration writes
only the entries of its own plane, so the geometry, the redistribution
tables and a full stage are bitwise the same for any thread count.  CPU
only."""
import numpy as np

import oracle
import synth


def test_results_do_not_depend_on_thread_count():
    w = synth.make_workload(1)
    U = synth.state_random(w.grid, 17, amp=2.0)
    Un = synth.state_random(w.grid, 18, amp=2.0)
    keep = oracle.set_threads()
    runs = []
    try:
        for th in (1, 3, 8):
            oracle.set_threads(th)
            o = oracle.Oracle(w.grid, w.h_nodes)
            R = o.redistribute(o.advance(Un, U, 0.3 * w.dt))
            runs.append((o, R))
    finally:
        oracle.set_threads(keep)
    o1, R1 = runs[0]
    for o, R in runs[1:]:
        for inst in range(4):
            assert np.array_equal(o.geo[inst], o1.geo[inst])
            assert np.array_equal(o.w[inst], o1.w[inst])
            assert np.array_equal(o.ctype[inst], o1.ctype[inst])
        for f in oracle.FIELDS:
            assert np.array_equal(R[f], R1[f]), f
