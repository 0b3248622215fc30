"""The allocation-free subband entry point against the one with a work buffer.

amber_subband_dedisperse_noalloc keeps step one's sums in the library's own
device array and runs the coarse DMs in slices that fit it; its dedispersed
trials must equal amber_subband_dedisperse's bit for bit with the same tiles.
Two calls in a row, the second with a smaller input, so that the second runs
over what the first left in the array:

1. the 1536-channel beam, 32 subbands, 128 coarse x 16 fine trials, 12208
   samples: step one's rows of all coarse DMs exceed the array, so the call
   runs in several slices;
2. 256 channels, 16 subbands, 24 coarse x 8 fine trials, 3000 samples, with
   zapped channels: one slice.

A problem whose single coarse DM does not fit the array is refused before any
launch.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


def _case(amber, torch, g, grid, n_out, seed, zap=None):
    f = g.freqs()
    d1, d2, info = amber.subband_delay_tables(f, g.t_samp_s, *grid)
    n_in = n_out + info.max_delay
    x = workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=seed)
    keep = None
    if zap is not None:
        k = np.ones(g.n_chan, dtype=np.uint8)
        k[np.asarray(zap)] = 0
        keep = torch.from_numpy(k).cuda()
    return (torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda(), info, torch.from_numpy(x).cuda(), n_in,
            keep)


def _compare(amber, torch, case, n_out):
    d1, d2, info, x, n_in, keep = case
    ref = amber.subband_dedisperse(d1, d2, info, x, n_in, n_out, keep=keep)
    out = torch.full((info.n_coarse * info.n_fine, n_out), -7, dtype=torch.int32, device="cuda")
    got = amber.subband_dedisperse_noalloc(d1, d2, info, x, n_in, n_out, out=out, keep=keep)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, ref)


def test_noalloc_matches_work_buffer_two_calls(amber, torch):
    cap = amber.subband_static_bytes()
    assert cap == 32 << 20
    beam = workloads.beam().geom
    grid1 = (32, 128, 0.0, 8.0, 16, 0.0, 0.5)
    case1 = _case(amber, torch, beam, grid1, 12208, seed=21)
    info1 = case1[2]
    row_bytes = (12208 + info1.max_delay2 + 63) // 64 * 64 * 2
    assert info1.n_subbands * info1.n_coarse * row_bytes > cap      # needs several slices
    say("noalloc call 1: 1536 ch, 32 subbands, 128 x 16 trials, 12208 samples")
    _compare(amber, torch, case1, 12208)

    small = workloads.small().geom
    grid2 = (16, 24, 0.0, 4.0, 8, 0.0, 0.5)
    case2 = _case(amber, torch, small, grid2, 3000, seed=22, zap=[0, 5, 17, 100, 255])
    say("noalloc call 2: 256 ch, 16 subbands, 24 x 8 trials, 3000 samples, 5 zapped channels")
    _compare(amber, torch, case2, 3000)


def test_noalloc_refuses_rows_beyond_the_array(amber, torch):
    # 256 subbands of one channel: one coarse DM's rows are 256 x >= 65600 x 2 B > 32 MiB
    g = workloads.Geometry(n_chan=256, n_dm=1, dm_first=0.0, dm_step=1.0)
    f = g.freqs()
    d1, d2, info = amber.subband_delay_tables(f, g.t_samp_s, 256, 2, 0.0, 1.0, 2, 0.0, 0.5)
    n_out = 65600
    n_in = n_out + info.max_delay
    x = torch.zeros((256, workloads.padded_stride(n_in)), dtype=torch.uint8, device="cuda")
    out = torch.full((4, n_out), -7, dtype=torch.int32, device="cuda")
    say("noalloc refusal: 256 subbands x 65600 samples")
    with pytest.raises(amber.AmberError) as e:
        amber.subband_dedisperse_noalloc(torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda(), info, x, n_in,
                                         n_out, out=out)
    assert e.value.status == -2 and "work buffer" in str(e.value)
    torch.cuda.synchronize()
    assert int((out != -7).sum()) == 0
