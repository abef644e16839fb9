"""The allocation-free entry point (bmc_collision_noalloc) against bmc_collision on the same inputs: two contexts
with the same model and state, one evaluated through each entry point, adaptive maps, two calls in a row (the second
with fewer samples per item); outputs must agree bitwise (the same kernels sum in the same fixed order; only where
the scratch lives differs).  A call beyond the static scratch is refused."""
import numpy as np
import pytest

from gpu_util import gpu_available, say
from paper_2603_28848_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bm():
    from paper_2603_28848_amd import boltzmc
    return boltzmc


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_collision_two_calls(precision):
    bm = _bm()
    w = wl.w23_be(n_grid=128, N=1 << 16, nitn=3)
    ref, na = bm.from_workload(w), bm.from_workload(w)
    for k, N in enumerate((1 << 16, 1 << 13)):  # the second call has a smaller input
        opts = bm.default_opts(seed=3, epoch=k, precision=precision, n_samples=N, n_iter=3)
        say("noalloc call %d precision=%d N=%d" % (k, precision, N))
        C1, S1 = ref.collision(-1, -1, opts)
        C2, S2 = na.collision_noalloc(-1, -1, opts)
        say("noalloc call %d: max |dC| %.3e, max |dsigma| %.3e" % (k, np.max(np.abs(C1 - C2)), np.max(np.abs(S1 - S2))))
        assert np.array_equal(C1, C2) and np.array_equal(S1, S2)
        assert np.any(C1 != 0)


def test_noalloc_full_size_batched_matches_and_plain_is_refused():
    """The 2<->3 benchmark workload (128 nodes, 2^18 samples, sliced to fit the static lists) matches bmc_collision
    bitwise on frozen maps; a per-grid-point launch of the same plan needs more scratch and is refused."""
    bm = _bm()
    w = wl.w23_be(nitn=1)
    ref, na = bm.from_workload(w), bm.from_workload(w)
    opts = bm.default_opts(seed=0, precision=1, freeze_maps=1, n_iter=1)
    C1, S1 = ref.collision(-1, -1, opts)
    C2, S2 = na.collision_noalloc(-1, -1, opts)
    assert np.array_equal(C1, C2) and np.array_equal(S1, S2)
    opts.launch = bm.LAUNCH_PLAIN
    with pytest.raises(bm.BmcError) as e:
        na.collision_noalloc(-1, -1, opts)
    assert e.value.code == bm.ENOMEM
