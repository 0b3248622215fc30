"""Parity at the workloads' full sizes, against the oracle.

* The 1536-channel beam (2048 DM trials x 12208 samples, widths 1..64) in the
  benchmark's launch configuration: every dedispersed value bit for bit and
  the whole S/N and peak tables (1e-5 relative, peaks exact).
* The 40 uneven beams of the batched workload, in one batch with automatic
  tiles (its boxcar / S/N launch takes single-wavefront groups, since the
  batch has more than 4096 rows) and with one tile set shared by every beam,
  eager and replayed from a HIP graph: 16 rows per beam (first, last, the
  pulse's row and 13 seeded random rows) against the oracle.
* The streaming service on the stream workload's two beam shapes (768
  channels / 1024 trials and 1536 channels / 2048 trials) in chunks of 6104
  samples: sampled rows of every chunk's S/N table against the oracle run on
  the whole concatenated input.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _check_snr(got_s, got_p, ref_s, ref_p, what=""):
    np.testing.assert_allclose(got_s.astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6, err_msg=what)
    assert np.array_equal(got_p, ref_p), what


def _oracle_snr_rows(dd, widths):
    s = np.empty((len(widths), dd.shape[0]))
    p = np.empty((len(widths), dd.shape[0]), dtype=np.int32)
    for k, w in enumerate(widths):
        s[k], p[k] = oracle.snr(oracle.boxcar(dd, w))
    return s, p


# --- the 1536-channel beam, every value ---------------------------------------------------

def test_beam_whole_tables(amber, torch):
    wl = workloads.beam()
    g = wl.geom
    do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, do, mx)
    say("beam 1536 ch x 2048 DM x %d samples: device search (default launch configuration)" % wl.n_out)
    s = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths,
                     tiles=amber.default_tiles())
    assert np.array_equal(s.delays_host, do)
    dd, sn, pk = s.run(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    dd, sn, pk = dd.cpu().numpy(), sn.cpu().numpy(), pk.cpu().numpy()
    say("beam: oracle on all 2048 trials")
    ref_dd = oracle.dedisperse(do, x, n_in, wl.n_out)
    assert np.array_equal(dd[:, :wl.n_out], ref_dd)
    ref_s, ref_p = _oracle_snr_rows(ref_dd, wl.widths)
    _check_snr(sn, pk, ref_s, ref_p, "beam S/N table")
    # the five pulses are the strongest candidates at their own DM rows
    for p in wl.pulses:
        k = list(wl.widths).index(p.width)
        assert sn[k, p.dm_index] > 8.0


# --- the 40-beam batch ------------------------------------------------------------------

@pytest.fixture(scope="module")
def batch40(amber, torch):
    wls = workloads.batch_beams(40)
    widths = wls[0].widths
    beams = []
    for k, wl in enumerate(wls):
        g = wl.geom
        d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        assert np.array_equal(d, do)
        x, n_in = workloads.make_input(wl, do, mx)
        rng = np.random.default_rng(7000 + k)
        rows = sorted(set([0, g.n_dm - 1, wl.pulses[0].dm_index] +
                          [int(r) for r in rng.choice(g.n_dm, size=13, replace=False)]))
        ref_dd = oracle.dedisperse(do[rows], x, n_in, wl.n_out)
        ref_s, ref_p = _oracle_snr_rows(ref_dd, widths)
        beams.append(dict(delays=torch.from_numpy(d).cuda(), info=info, x=torch.from_numpy(x).cuda(), n_in=n_in,
                          n_out=wl.n_out, dd=torch.full((g.n_dm, wl.n_out), -1, dtype=torch.int32, device="cuda"),
                          snr=torch.zeros((len(widths), g.n_dm), dtype=torch.float32, device="cuda"),
                          peak=torch.zeros((len(widths), g.n_dm), dtype=torch.int32, device="cuda"),
                          rows=rows, ref=(ref_dd, ref_s, ref_p)))
        if k % 10 == 9:
            say("batch: %d of 40 beams built with their oracle rows" % (k + 1))
    return beams, widths


def _check_batch(beams, what):
    for b, bm in enumerate(beams):
        ref_dd, ref_s, ref_p = bm["ref"]
        rows = bm["rows"]
        assert np.array_equal(bm["dd"][rows].cpu().numpy(), ref_dd), (what, b)
        _check_snr(bm["snr"][:, rows].cpu().numpy(), bm["peak"][:, rows].cpu().numpy(), ref_s, ref_p,
                   "%s beam %d" % (what, b))


def _reset(beams):
    for bm in beams:
        bm["dd"].fill_(-1)
        bm["snr"].zero_()
        bm["peak"].fill_(-1)


@pytest.mark.parametrize("shared", [False, True], ids=["auto-tiles", "one-tile-set"])
def test_batch40_against_oracle(amber, torch, batch40, shared):
    beams, widths = batch40
    tiles = None
    if shared:
        # one configuration valid for every beam: the defaults fitted to the
        # largest DM-to-DM delay step of the batch
        worst = max(beams, key=lambda bm: bm["info"].max_step)["info"]
        t = amber.auto_tiles(worst, 0)
        for bm in beams:
            amber.validate_tiles(t, bm["info"], len(widths))
        tiles = [t] * len(beams)
    _reset(beams)
    say("batch40 %s: eager" % ("one tile set" if shared else "automatic tiles"))
    batch = amber.Batch(beams, widths, tiles=tiles)
    n_dd, n_snr = batch.launches()
    if shared:
        assert (n_dd, n_snr) == (1, 1)
    assert n_snr == 1
    batch.run()
    torch.cuda.synchronize()
    _check_batch(beams, "eager")
    stream = torch.cuda.Stream()
    say("batch40: graph capture and 2 replays")
    with torch.cuda.stream(stream):
        batch.capture(stream)
    for rep in range(2):
        _reset(beams)
        torch.cuda.synchronize()
        batch.launch(stream)
        stream.synchronize()
        _check_batch(beams, "replay %d" % rep)
        _ = torch.ones(1000, device="cuda").sum()   # unrelated eager work between replays
    batch.close()


# --- streaming at the stream workload's shapes ---------------------------------------------

STREAM_WIDTHS = (1, 2, 4, 8, 16, 32, 64)
N_CHUNKS = 4


def test_stream_full_size_chunks(amber):
    L = workloads.STREAM_CHUNK
    geoms = workloads.stream_geometries(2)     # 768 ch / 1024 trials, 1536 ch / 2048 trials
    cases = []
    for b, g in enumerate(geoms):
        d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        total = N_CHUNKS * L
        x = workloads.noise(g.n_chan, total, total, seed=5100 + b)
        workloads.inject(x, d[g.n_dm // 3], t0=total - mx - 3000, width=8, amp=40)
        rng = np.random.default_rng(5200 + b)
        rows = sorted(set([0, g.n_dm // 3, g.n_dm - 1] + [int(r) for r in rng.choice(g.n_dm, 21, replace=False)]))
        say("stream beam %d (%d ch, %d trials, max delay %d): oracle rows" % (b, g.n_chan, g.n_dm, mx))
        dd = oracle.dedisperse(d[rows], x, total, total - mx)
        cases.append((g, mx, x, rows, dd))
    say("stream: 2 beams x %d chunks of %d samples through the service" % (N_CHUNKS, L))
    with amber.Server(max_inflight=8, max_batch=4, n_streams=2) as srv:
        for g, *_ in cases:
            srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, L, STREAM_WIDTHS)
        for k in range(N_CHUNKS):
            for b, (g, mx, x, rows, dd) in enumerate(cases):
                srv.submit(b, x[:, k * L:(k + 1) * L], tag=k)
        res = {}
        for _ in range(N_CHUNKS * len(cases)):
            r = srv.wait(60.0)
            assert r is not None
            res[(r["beam"], r["seq"])] = r
    checked = 0
    for b, (g, mx, x, rows, dd) in enumerate(cases):
        for k in range(N_CHUNKS):
            r = res[(b, k)]
            t0, n = amber.chunk_span(k, L, mx)
            assert (r["t_first"], r["n_out"]) == (t0, n)
            if n < max(STREAM_WIDTHS):
                assert r["has_snr"] == 0
                continue
            ref_s, ref_p = _oracle_snr_rows(dd[:, t0:t0 + n], STREAM_WIDTHS)
            _check_snr(r["snr"][:, rows], r["peak"][:, rows], ref_s, ref_p, "stream beam %d chunk %d" % (b, k))
            checked += 1
    assert checked >= 5     # 768 ch: chunks 0-3 all yield outputs; 1536 ch: chunks 1-3
