"""Seeded random parity cases: shapes, tiles and masks drawn at random, the
HIP path against the CPU oracle element by element.

Each case draws a geometry (1..700 channels in random non-uniform order,
1..70 DM trials from a random first DM and step, 1..3000 output samples, a
random row padding), a dedispersion tile from the whole tile space (any
work-group shape, one or two DMs per wavefront, LDS staging or direct
reads), sometimes a random channel mask, then 1..6 boxcar widths up to
min(n_out, 1024) with random S/N tiles.  Tiles the library refuses
(AMBER_E_CONFIG, checked on the host before any launch) are redrawn.
Dedispersion must match bit for bit; S/N within 1e-5 relative, peaks exactly.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

N_CASES = 40
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


def _draw_dedisp_tiles(amber, rng, info):
    for _ in range(60):
        kw = dict(threads_per_dm=int(rng.choice([64, 128, 256, 512, 1024])),
                  samples_per_thread=int(rng.choice([4, 8, 16, 32])),
                  dms_per_block=int(rng.choice([1, 2, 3, 4, 5, 8, 16])),
                  channel_unroll=int(rng.choice([1, 2, 4, 8, 16, 32])),
                  dms_per_thread=int(rng.choice([1, 2])),
                  direct_reads=int(rng.random() < 0.25))
        t = amber.make_tiles(**kw)
        try:
            amber.validate_tiles(t, info, 1)
        except amber.AmberError:
            continue
        return t, kw
    return None, "auto"


def _draw_widths(rng, n_out):
    cap = min(n_out, 1024)
    pool = sorted({1, 2, 3, 4, 7, 8, 16, 31, 32, 64, 100, 128, 256, 512, 1000, 1024} & set(range(1, cap + 1)))
    k = int(rng.integers(1, min(6, len(pool)) + 1))
    return tuple(sorted(rng.choice(pool, size=k, replace=False).tolist()))


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_case(amber, torch, case):
    rng = np.random.default_rng(7000 + case)
    n_chan = int(rng.integers(1, 701))
    n_dm = int(rng.integers(1, 71))
    n_out = int(rng.integers(1, 3001))
    freqs = rng.uniform(1100.0, 1700.0, size=n_chan)          # any order, non-uniform
    dm_first, dm_step = float(rng.uniform(0.0, 50.0)), float(rng.uniform(0.0, 3.0))
    d, mx = oracle.delay_table(freqs, 81.92e-6, n_dm, dm_first, dm_step)
    dl, info = amber.delay_table(freqs, 81.92e-6, n_dm, dm_first, dm_step)
    assert np.array_equal(dl, d) and info.max_delay == mx
    n_in = n_out + mx
    stride = (n_in + 3) // 4 * 4 + int(rng.choice([0, 4, 60, 124]))
    x = rng.integers(0, 256, size=(n_chan, stride), dtype=np.uint8)
    keep = (rng.random(n_chan) >= 0.2).astype(np.uint8) if rng.random() < 0.3 else None
    tiles, desc = _draw_dedisp_tiles(amber, rng, info)
    say("fuzz", case, "ch", n_chan, "dm", n_dm, "out", n_out, "max_delay", mx, "stride", stride,
        "masked", keep is not None, "tiles", desc)
    ref = oracle.dedisperse_masked(d, x, n_in, n_out, keep) if keep is not None else \
        oracle.dedisperse(d, x, n_in, n_out)
    dev, xd = torch.from_numpy(d).cuda(), torch.from_numpy(x).cuda()
    kd = torch.from_numpy(keep).cuda() if keep is not None else None
    try:
        got = amber.dedisperse(dev, info, xd, n_in, n_out, tiles, keep=kd)
    except amber.AmberError as e:
        # a mask adds a zeroed LDS region the tile check does not count; the
        # library refuses such a tile on the host
        assert e.status == -3 and keep is not None
        say("fuzz", case, "masked tile refused, automatic tiles")
        got = amber.dedisperse(dev, info, xd, n_in, n_out, None, keep=kd)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), ref)

    widths = _draw_widths(rng, n_out)
    ref_s, ref_p = [], []
    for w in widths:
        s, p = oracle.snr(oracle.boxcar(ref, w))
        ref_s.append(s)
        ref_p.append(p)
    ref_s, ref_p = np.array(ref_s), np.array(ref_p)
    for _ in range(30):
        st = amber.make_tiles(snr_threads=int(rng.choice([64, 128, 256, 512, 1024])),
                              boxcar_step=[int(v) for v in rng.choice([1, 2, 4, 8], size=len(widths))])
        say("fuzz", case, "widths", widths, "snr_threads", st.snr_threads,
            "steps", [st.boxcar_step[k] for k in range(len(widths))])
        try:
            s, p = amber.integrate_snr(got, n_out, widths, st)
        except amber.AmberError as e:
            assert e.status == -3       # a refused tile (chunk too short for the widths): redraw
            continue
        torch.cuda.synchronize()
        np.testing.assert_allclose(s.cpu().numpy().astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6)
        assert np.array_equal(p.cpu().numpy(), ref_p)
        break
    else:
        pytest.fail("no valid S/N tile drawn")


N_SUBBAND_CASES = 16


def _draw_step_tiles(rng, step):
    if step == 1:   # uint8 input, 16-bit sums
        return amber_tiles_kw(rng, [64, 128, 256], [4, 8, 16], [1, 2, 3, 4, 8], [1, 2, 4, 8, 16], [1, 2])
    return amber_tiles_kw(rng, [64, 128, 256], [8, 16], [1, 2, 4, 6, 8, 16], [4, 8, 16, 32], [1])


def amber_tiles_kw(rng, tpd, spt, dpb, cu, dpt):
    return dict(threads_per_dm=int(rng.choice(tpd)), samples_per_thread=int(rng.choice(spt)),
                dms_per_block=int(rng.choice(dpb)), channel_unroll=int(rng.choice(cu)),
                dms_per_thread=int(rng.choice(dpt)))


@pytest.mark.parametrize("case", range(N_SUBBAND_CASES))
def test_random_subband_case(amber, torch, case):
    """Two-step subband dedispersion on a random grid (1..32 subbands of
    1..24 channels, 1..12 coarse DMs x 1..12 fine DMs), random step tiles
    (redrawn while the library refuses them), sometimes zapped channels."""
    rng = np.random.default_rng(8000 + case)
    n_sub = int(rng.choice([1, 2, 4, 8, 16, 32]))
    m = int(rng.integers(1, 25))
    n_chan = n_sub * m
    n_coarse, n_fine = int(rng.integers(1, 13)), int(rng.integers(1, 13))
    coarse_step = float(rng.uniform(0.5, 8.0))
    grid = (n_sub, n_coarse, float(rng.uniform(0.0, 30.0)), coarse_step, n_fine, 0.0,
            coarse_step / n_fine * float(rng.uniform(0.5, 1.0)))
    n_out = int(rng.integers(1, 2501))
    freqs = rng.uniform(1100.0, 1700.0, size=n_chan)
    d1, d2, info = amber.subband_delay_tables(freqs, 81.92e-6, *grid)
    o1, o2, _, _ = oracle.subband_delays(freqs, 81.92e-6, *grid)
    n_in = n_out + info.max_delay
    stride = (n_in + 3) // 4 * 4 + int(rng.choice([0, 4, 124]))
    x = rng.integers(0, 256, size=(n_chan, stride), dtype=np.uint8)
    keep = (rng.random(n_chan) >= 0.2).astype(np.uint8) if rng.random() < 0.3 else None
    xz = x.copy()
    if keep is not None:
        xz[keep == 0] = 0
    ref = oracle.subband_dedisperse(o1, o2, xz, n_in, n_out)
    dev1, dev2, xd = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda(), torch.from_numpy(x).cuda()
    kd = torch.from_numpy(keep).cuda() if keep is not None else None
    for attempt in range(40):
        kw1, kw2 = (_draw_step_tiles(rng, 1), _draw_step_tiles(rng, 2)) if attempt < 39 else (None, None)
        t1 = amber.make_tiles(**kw1) if kw1 else None
        t2 = amber.make_tiles(**kw2) if kw2 else None
        say("fuzz subband", case, "grid", grid, "ch", n_chan, "out", n_out, "masked", keep is not None,
            "tiles", kw1, kw2)
        try:
            got = amber.subband_dedisperse(dev1, dev2, info, xd, n_in, n_out, tiles1=t1, tiles2=t2, keep=kd)
        except amber.AmberError as e:
            assert e.status == -3       # refused on the host before any launch: redraw
            continue
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref)
        break
    else:
        pytest.fail("no subband tiles accepted")


N_DECIMATION_CASES = 16


@pytest.mark.parametrize("case", range(N_DECIMATION_CASES))
def test_random_decimation_case(amber, torch, case):
    """Decimation (materialised and fused with S/N) of random series by 1..8
    random factors up to min(n_out, 4096), random S/N tiles."""
    rng = np.random.default_rng(9000 + case)
    n_dm, n_out = int(rng.integers(1, 41)), int(rng.integers(1, 20001))
    dd = rng.integers(0, 391680, size=(n_dm, n_out)).astype(np.int32)
    pool = sorted({1, 2, 3, 5, 10, 16, 20, 33, 40, 64, 80, 160, 320, 640, 1000, 1280, 2048, 3200, 4096} &
                  set(range(1, min(n_out, 4096) + 1)))
    k = int(rng.integers(1, min(8, len(pool)) + 1))
    factors = tuple(sorted(rng.choice(pool, size=k, replace=False).tolist()))
    ddd = torch.from_numpy(dd).cuda()
    say("fuzz decimation", case, "dm", n_dm, "out", n_out, "factors", factors)
    ys = [oracle.downsample(dd, f) for f in factors]
    y = amber.downsample(ddd, n_out, factors).cpu().numpy()
    for j, f in enumerate(factors):
        assert np.array_equal(y[j, :, :n_out // f], ys[j]), f
    ref = [oracle.snr(v) for v in ys]
    ref_s, ref_p = np.array([r[0] for r in ref]), np.array([r[1] for r in ref])
    for _ in range(30):
        st = amber.make_tiles(snr_threads=int(rng.choice([64, 128, 256, 512, 1024])),
                              boxcar_step=[int(v) for v in rng.choice([1, 2, 4, 8], size=len(factors))])
        say("fuzz decimation", case, "snr_threads", st.snr_threads,
            "steps", [st.boxcar_step[j] for j in range(len(factors))])
        try:
            s, p = amber.downsample_snr(ddd, n_out, factors, st)
        except amber.AmberError as e:
            assert e.status == -3
            continue
        torch.cuda.synchronize()
        np.testing.assert_allclose(s.cpu().numpy().astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6)
        assert np.array_equal(p.cpu().numpy(), ref_p)
        break
    else:
        pytest.fail("no valid S/N tile drawn")
