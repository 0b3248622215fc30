"""The streaming service against the oracle on the whole stream.

Each beam's chunks are the consecutive pieces of one seeded input; the
oracle dedisperses that input in one piece, and every chunk's S/N table must
equal the oracle's boxcar/S/N over the chunk's span of outputs (S/N within
1e-5 relative, peaks exactly).  The same chunks run alone on a fresh server
must give bit-identical tables to the ones they gave in the mix, and a memory
budget that admits one chunk at a time must change nothing but the schedule.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5
WIDTHS = (1, 2, 4, 8, 16)
L = 1024
N_CHUNKS = 6

# largest delays about 1065, 714 and 1767 samples: the last is longer than a
# chunk, so its first chunk yields nothing and its second starts mid-chunk
GEOMS = [
    workloads.Geometry(n_chan=128, n_dm=48, dm_first=0.0, dm_step=2.0),
    workloads.Geometry(n_chan=256, n_dm=64, dm_first=0.0, dm_step=1.0),
    workloads.Geometry(n_chan=96, n_dm=40, dm_first=0.0, dm_step=4.0),
]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


@pytest.fixture(scope="module")
def streams():
    """Per beam: (geometry, delays, max_delay, whole input, oracle dd)."""
    out = []
    for b, g in enumerate(GEOMS):
        d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        total = N_CHUNKS * L
        x = workloads.noise(g.n_chan, total, total, seed=700 + b)
        # one pulse per beam, late enough to land inside the outputs
        i = g.n_dm * 2 // 3
        workloads.inject(x, d[i], t0=total - mx - 900, width=4, amp=50)
        dd = oracle.dedisperse(d, x, total, total - mx)
        out.append((g, d, mx, x, dd))
    return out


def _expected(dd, t0, n):
    s, p = [], []
    for w in WIDTHS:
        a, b = oracle.snr(oracle.boxcar(dd[:, t0:t0 + n], w))
        s.append(a)
        p.append(b)
    return np.array(s), np.array(p)


def _add_beams(amber, srv, streams):
    return [srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, L, WIDTHS) for g, *_ in streams]


def _collect(srv, n, timeout=60.0):
    res = {}
    for _ in range(n):
        r = srv.wait(timeout)
        assert r is not None, "a chunk did not complete within %g s" % timeout
        res[(r["beam"], r["seq"])] = r
    return res


def _check_against_oracle(amber, streams, res):
    for b, (g, d, mx, x, dd) in enumerate(streams):
        for k in range(N_CHUNKS):
            r = res[(b, k)]
            t0, n = amber.chunk_span(k, L, mx)
            assert (r["t_first"], r["n_out"]) == (t0, n)
            if n < max(WIDTHS):
                assert r["has_snr"] == 0
                continue
            assert r["has_snr"] == 1
            s, p = _expected(dd, t0, n)
            np.testing.assert_allclose(r["snr"].astype(np.float64), s, rtol=SNR_RTOL, atol=1e-6)
            assert np.array_equal(r["peak"], p), (b, k)


def test_stream_matches_one_shot_and_alone(amber, streams):
    say("serve: %d beams x %d chunks of %d, all submitted at once" % (len(streams), N_CHUNKS, L))
    with amber.Server(max_inflight=8, max_batch=4, n_streams=3) as srv:
        ids = _add_beams(amber, srv, streams)
        assert ids == list(range(len(streams)))
        for k in range(N_CHUNKS):
            for b, (g, d, mx, x, dd) in enumerate(streams):
                srv.submit(b, x[:, k * L:(k + 1) * L], tag=1000 * b + k)
        mix = _collect(srv, N_CHUNKS * len(streams))
        st = srv.stats()
    assert st["completed"] == st["submitted"] == N_CHUNKS * len(streams)
    assert st["inflight"] == 0 and st["queued"] == 0
    assert all(r["tag"] == 1000 * r["beam"] + r["seq"] for r in mix.values())
    assert max(r["batch_size"] for r in mix.values()) > 1     # chunks of different beams shared launches
    assert st["batches"] < st["submitted"]
    _check_against_oracle(amber, streams, mix)

    say("serve: each beam alone, one chunk at a time")
    for b, (g, d, mx, x, dd) in enumerate(streams):
        with amber.Server(max_inflight=1, max_batch=1, n_streams=1) as srv:
            _add_beams(amber, srv, streams)
            for k in range(N_CHUNKS):
                srv.submit(b, np.ascontiguousarray(x[:, k * L:(k + 1) * L]))
                r = srv.wait(60.0)
                assert r is not None and r["batch_size"] == 1 and (r["beam"], r["seq"]) == (b, k)
                m = mix[(b, k)]
                assert (r["t_first"], r["n_out"], r["has_snr"]) == (m["t_first"], m["n_out"], m["has_snr"])
                if r["has_snr"]:
                    assert np.array_equal(r["snr"], m["snr"]) and np.array_equal(r["peak"], m["peak"])


def test_memory_budget_admits_one_chunk_at_a_time(amber, streams):
    say("serve: budget for the resident buffers plus one chunk")
    with amber.Server(max_inflight=16, max_batch=8, n_streams=2) as probe:
        _add_beams(amber, probe, streams)
        resident = probe.stats()["memory_in_use"]
    # chunk blocks: int32 dd [n_dm][round64(L)], the S/N and peak tables and
    # the staged chunk [n_chan][L], each part 256-byte aligned
    def r256(n):
        return (n + 255) // 256 * 256
    blocks = []
    for g, *_ in streams:
        res_off = r256(g.n_dm * ((L + 63) // 64 * 64) * 4)
        stage_off = r256(res_off + len(WIDTHS) * g.n_dm * 8)
        blocks.append(r256(stage_off + g.n_chan * L))
    budget = resident + max(blocks)
    with amber.Server(max_inflight=16, max_batch=8, n_streams=2, memory_budget=budget) as srv:
        _add_beams(amber, srv, streams)
        for k in range(N_CHUNKS):
            for b, (g, d, mx, x, dd) in enumerate(streams):
                srv.submit(b, x[:, k * L:(k + 1) * L], tag=k)
        res = _collect(srv, N_CHUNKS * len(streams))
        st = srv.stats()
    assert st["memory_peak"] <= budget
    assert st["admissions_deferred_for_memory"] > 0
    assert all(r["batch_size"] == 1 for r in res.values())
    _check_against_oracle(amber, streams, res)


def test_server_rejects(amber, streams):
    g = streams[0][0]
    with amber.Server(max_inflight=2, max_batch=2, n_streams=1, memory_budget=1 << 20) as srv:
        with pytest.raises(amber.AmberError):      # 128 ch x (1065 + 1024) x 2 buffers does not fit 1 MiB
            srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, 4096, WIDTHS)
    with amber.Server(max_inflight=2, max_batch=2, n_streams=1) as srv:
        with pytest.raises(amber.AmberError):      # width longer than a chunk
            srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, 8, WIDTHS)
        b = srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, L, WIDTHS)
        with pytest.raises(ValueError):
            srv.submit(b, np.zeros((g.n_chan, L - 1), np.uint8))
        with pytest.raises(amber.AmberError):
            srv.submit(b + 1, np.zeros((g.n_chan, L), np.uint8))
        assert srv.wait(0.05) is None              # nothing submitted: the wait times out


def test_process_exits_cleanly_with_open_handles():
    """A process that leaves a Server (with a chunk done) and a Batch open
    exits with status 0: the binding closes them at exit."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import sys
sys.path.insert(0, %r)
import numpy as np, torch
import paper_1811_04165_amd as amber, workloads
g = workloads.Geometry(n_chan=64, n_dm=16, dm_first=0.0, dm_step=1.0)
srv = amber.Server(max_inflight=4, max_batch=2, n_streams=2)
srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, 1024, (1, 2, 4))
srv.submit(0, np.full((64, 1024), 100, np.uint8), tag=0)
assert srv.wait(30.0) is not None
d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
n_in = 1000 + info.max_delay
bm = dict(delays=torch.from_numpy(d).cuda(), info=info, x=torch.zeros((64, (n_in + 127) // 128 * 128), dtype=torch.uint8, device="cuda"),
          n_in=n_in, n_out=1000, dd=torch.zeros((16, 1000), dtype=torch.int32, device="cuda"),
          snr=torch.zeros((3, 16), dtype=torch.float32, device="cuda"), peak=torch.zeros((3, 16), dtype=torch.int32, device="cuda"))
b = amber.Batch([bm], (1, 2, 4))
b.run()
torch.cuda.synchronize()
print("left open", flush=True)
''' % root
    say("child process exiting with an open Server and Batch")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "left open" in r.stdout
