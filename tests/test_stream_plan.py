"""Host logic of the streaming service, without a device.

The chunk arithmetic is pinned by what a stream must satisfy: the outputs of
successive chunks tile [0, inf) with no gap and no overlap, and every output
of chunk k needs only input that has arrived by the end of chunk k and
nothing older than the max_delay samples a beam keeps.  The admission rule is
pinned against a plain model of the rule as the header states it, on random
cases, and on hand-made cases for each of its clauses (order within a beam,
busy beams, memory blocking without overtaking, the in-flight and batch caps).
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


@pytest.mark.parametrize("L,D", [(6104, 5791), (6104, 11593), (100, 0), (1, 7), (64, 64), (50, 49), (7, 300)])
def test_chunk_spans_tile_the_stream(amber, L, D):
    covered = []
    for k in range(0, 4 * (D // L + 2)):
        t0, n = amber.chunk_span(k, L, D)
        assert n >= 0 and t0 >= 0
        if n:
            # inputs t0 .. t0+n-1+D have all arrived by the end of chunk k ...
            assert t0 + n - 1 + D <= (k + 1) * L - 1
            # ... and none is older than the D samples kept from earlier chunks
            assert t0 >= k * L - D
            covered.append((t0, n))
        else:
            assert (k + 1) * L <= D
    # contiguous from 0, no overlap
    pos = 0
    for t0, n in covered:
        assert t0 == pos
        pos += n
    k_last = 4 * (D // L + 2) - 1
    assert pos == (k_last + 1) * L - D


def test_chunk_span_rejects(amber):
    for args in ((-1, 10, 0), (0, 0, 0), (0, 10, -1)):
        with pytest.raises(amber.AmberError):
            amber.chunk_span(*args)


def _model(pending, busy, inflight, in_use, max_inflight, max_batch, budget):
    """The rule as stated: arrival order; a beam that is busy or already seen
    in this pass is passed over; the first other chunk that does not fit the
    budget stops the pass; the in-flight and batch caps stop it too."""
    seen = set(b for b, v in enumerate(busy) if v)
    out = []
    for i, (beam, nbytes) in enumerate(pending):
        if inflight + len(out) >= max_inflight or len(out) >= max_batch:
            return out, -1
        if beam in seen:
            continue
        seen.add(beam)
        if in_use + nbytes > budget:
            return out, i
        in_use += nbytes
        out.append(i)
    return out, -1


def test_admission_rule_matches_model(amber):
    rng = np.random.default_rng(11)
    for _ in range(400):
        n_beams = int(rng.integers(1, 9))
        n_pending = int(rng.integers(0, 25))
        pending = [(int(rng.integers(0, n_beams)), int(rng.integers(0, 60))) for _ in range(n_pending)]
        busy = [bool(rng.random() < 0.3) for _ in range(n_beams)]
        inflight = int(rng.integers(0, 5))
        in_use = int(rng.integers(0, 100))
        max_inflight = int(rng.integers(1, 12))
        max_batch = int(rng.integers(1, 8))
        budget = int(rng.integers(0, 250))
        cfg = amber.server_config(max_inflight=max_inflight, max_batch=max_batch, memory_budget=budget)
        got = amber.admit(pending, busy, inflight, in_use, cfg)
        want = _model(pending, busy, inflight, in_use, max_inflight, max_batch, budget)
        assert got == (want[0], want[1]), (pending, busy, inflight, in_use, max_inflight, max_batch, budget)


def test_admission_clauses(amber):
    big = amber.server_config(max_inflight=100, max_batch=100, memory_budget=1000)
    # one chunk per beam per pass, in arrival order
    assert amber.admit([(0, 1), (0, 1), (1, 1), (1, 1), (2, 1)], [0, 0, 0], 0, 0, big) == ([0, 2, 4], -1)
    # busy beams wait
    assert amber.admit([(0, 1), (1, 1), (2, 1)], [1, 0, 1], 0, 0, big) == ([1], -1)
    # memory: the first chunk that does not fit stops the pass (no overtaking)
    mem = amber.server_config(max_inflight=100, max_batch=100, memory_budget=100)
    assert amber.admit([(0, 40), (1, 70), (2, 10)], [0, 0, 0], 0, 0, mem) == ([0], 1)
    assert amber.admit([(0, 40), (1, 60), (2, 10)], [0, 0, 0], 0, 0, mem) == ([0, 1], 2)
    assert amber.admit([(0, 40)], [0], 0, 61, mem) == ([], 0)
    # caps
    cap = amber.server_config(max_inflight=3, max_batch=2, memory_budget=1000)
    assert amber.admit([(0, 1), (1, 1), (2, 1)], [0, 0, 0], 0, 0, cap) == ([0, 1], -1)
    assert amber.admit([(0, 1), (1, 1), (2, 1)], [0, 0, 0], 2, 0, cap) == ([0], -1)
    assert amber.admit([(0, 1)], [0], 3, 0, cap) == ([], -1)
    # empty queue
    assert amber.admit([], [0, 0], 0, 0, cap) == ([], -1)


def test_admission_rejects_bad_input(amber):
    cfg = amber.server_config(max_inflight=4, max_batch=2, memory_budget=10)
    with pytest.raises(amber.AmberError):
        amber.admit([(2, 1)], [0, 0], 0, 0, cfg)          # beam out of range
    with pytest.raises(amber.AmberError):
        amber.admit([(0, -1)], [0], 0, 0, cfg)            # negative bytes
    with pytest.raises(amber.AmberError):
        amber.admit([(0, 1)], [0], 0, 0, amber.server_config(max_inflight=0))
    with pytest.raises(amber.AmberError):
        amber.admit([(0, 1)], [0], 0, 0, amber.server_config(n_streams=9))


def test_poisson_arrivals_recipe():
    import workloads
    ev = workloads.poisson_arrivals(40, 10.0, 30.0, seed=5)
    t = np.array([e[0] for e in ev])
    assert np.all(np.diff(t) >= 0) and t.min() >= 0 and t.max() < 30.0
    # 12000 expected; Poisson sd ~ 110
    assert abs(len(ev) - 12000) < 600
    for b in (0, 17, 39):
        seqs = [e[2] for e in ev if e[1] == b]
        assert seqs == list(range(len(seqs)))
    assert ev == workloads.poisson_arrivals(40, 10.0, 30.0, seed=5)
