"""Parameter validation of the newer C-ABI options: every bad value is rejected with an error and nothing changes."""
import pytest

from gpu_util import gpu_available
from paper_2603_28848_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bm():
    from paper_2603_28848_amd import boltzmc
    return boltzmc


@pytest.mark.parametrize("bad", [
    dict(width_mode=2), dict(width_mode=wl.WIDTH_REL, sigma_E=1.5), dict(width_adapt=2),
    dict(width_adapt=1, width_lo=0.0), dict(width_adapt=1, width_lo=0.02, width_hi=0.01),
    dict(width_adapt=1, width_factor=1.0), dict(width_adapt=1, width_min=0.0),
    dict(width_adapt=1, width_min=0.3, width_max=0.2), dict(m2_kind=3), dict(vegas_plus=2), dict(beta=2.5),
    dict(n_samples=1 << 32),  # D n_samples >= 2^34: the word stream's block index would pass 32 bits
])
def test_bad_process_parameters_are_rejected(bad):
    bm = _bm()
    ctx = bm.Context()
    sid = ctx.add_species("phi", wl.BOSE, 32, 0.01, 20.0)
    with pytest.raises(bm.BmcError):
        ctx.add_process([sid, sid], [sid, sid], **bad)


def test_bad_width_and_interp_calls_are_rejected():
    bm = _bm()
    w = wl.w22_mb()
    w.processes[0].width_mode = wl.WIDTH_REL
    w.processes[0].sigma_E = 0.01
    ctx = bm.from_workload(w)
    for v in (0.0, -1.0, 1.5, float("nan")):
        with pytest.raises(bm.BmcError):
            ctx.set_width(0, v)
    assert ctx.get_width(0) == 0.01
    with pytest.raises(bm.BmcError):
        ctx.set_width(3, 0.01)
    for mode in (-1, 3):
        with pytest.raises(bm.BmcError):
            ctx.set_interp(0, mode)
    with pytest.raises(bm.BmcError):
        ctx.set_interp(5, wl.INTERP_SPLINE)


def test_sample_count_beyond_the_word_stream_is_rejected():
    """A call whose samples per item would take the word stream's block index past 32 bits (D N >= 2^34) fails with
    an error before anything runs."""
    bm = _bm()
    ctx = bm.from_workload(wl.w22_mb())
    with pytest.raises(bm.BmcError):
        ctx.collision(-1, -1, bm.default_opts(n_samples=1 << 32, n_iter=1))


def test_timing_every_kth_sample_phase():
    """set_timing(every=k) times phases 0, k, 2k, ... of the calls that follow; every < 0 is rejected."""
    bm = _bm()
    ctx = bm.from_workload(wl.w22_mb())
    o = bm.default_opts(seed=1, n_iter=4)
    ctx.collision(-1, -1, o)  # plan and maps
    for every, calls, want in ((1, 1, 4), (3, 1, 2), (3, 2, 3), (5, 2, 2)):
        ctx.set_timing(True, every=every)
        ctx.get_timing(reset=True)
        for _ in range(calls):
            ctx.collision(-1, -1, o)
        ms, n = ctx.get_timing(reset=True)
        assert n == want and ms > 0.0, (every, calls, n, ms)
    ctx.set_timing(False)
    ctx.collision(-1, -1, o)
    assert ctx.get_timing(reset=True)[1] == 0
    with pytest.raises(bm.BmcError):
        ctx.set_timing(True, every=-1)


def test_kernel_timing_splits_the_sample_phase():
    """get_kernel_timing reports the same timed phases as get_timing, split at the event between the screening pass
    and the second pass: screen + second = the phase total (float event times), both positive; reading either
    with reset clears both."""
    bm = _bm()
    ctx = bm.from_workload(wl.w23_be(n_grid=32, N=1 << 14, nitn=3))
    o = bm.default_opts(seed=2, n_iter=3)
    ctx.collision(-1, -1, o)
    ctx.set_timing(True, every=1)
    ctx.get_kernel_timing(reset=True)
    ctx.collision(-1, -1, o)
    ctx.collision(-1, -1, o)
    scr, sec, n = ctx.get_kernel_timing(reset=False)
    ms, n2 = ctx.get_timing(reset=True)
    assert n == n2 == 6 and scr > 0.0 and sec > 0.0
    assert abs((scr + sec) - ms) <= 1e-3 * ms + 1e-3, (scr, sec, ms)
    assert ctx.get_kernel_timing(reset=True) == (0.0, 0.0, 0)
    ctx.set_timing(False)


def test_device_outputs_equal_host_outputs_and_are_checked():
    """C and sigma written into device tensors (MEM_DEVICE) equal the host outputs bitwise; a tensor of the wrong
    dtype, too short or on the host is refused before the call."""
    import numpy as np
    import torch
    bm = _bm()
    w = wl.w22_mb(n_grid=16, N=4096, nitn=2)
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=2, freeze_maps=1)
    C, S = ctx.collision(-1, -1, opts)
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    sig = torch.zeros(16, dtype=torch.float64, device="cuda")
    ctx.collision(-1, -1, opts, out=out, sigma=sig)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), C) and np.array_equal(sig.cpu().numpy(), S)
    for bad in (torch.zeros(16, dtype=torch.float32, device="cuda"), torch.zeros(8, dtype=torch.float64, device="cuda"),
                torch.zeros(16, dtype=torch.float64)):
        with pytest.raises(ValueError):
            ctx.collision(-1, -1, opts, out=bad, sigma=sig)
