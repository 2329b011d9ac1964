"""The give-up path of the bank kernels' count wait, forced from the host.

The workgroup that scans the per-workgroup (streaming kernel) or per-tile
(tiled kernel) candidate counts polls each count word at most `spin` times.
With the context's spin set to one poll, a search whose spectrum puts dozens
of strong tones in a range that another workgroup searches long after the
scanner has finished (the first workgroup's range for the streaming kernel,
whose scanner is the last; the tile just before the last for the tiled
kernel, whose last tile scans) loses that count: the search must return
PULSCAN_EHIP with every kernel having run to its end, and the next search
with the default spin must give exactly the candidates of a clean search.
"""

import pytest

import synth
from gpu_helpers import say, to_device

pytestmark = pytest.mark.gpu

N, Z, C = 1 << 23, 200, 1024
DEFAULT_SPIN = 1 << 20


@pytest.fixture(scope="module")
def pk():
    import paper_2406_15186_amd as pk
    pk.lib()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    import torch
    assert torch.cuda.is_available()
    c = pk.Context(0)
    yield c
    c.close()


def heavy_spectrum(oracle_lib, lo, hi, seed):
    # 48 tones of 2..61 bins at 12-20 sigma, first bins in [lo, hi]
    wl = synth.Workload("giveup", N, Z, C, 6.0, seed, 48, None, (1, 60), (12.0, 20.0), (lo, hi))
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=N)
    return x


@pytest.mark.parametrize("kernel,lo,hi", [
    ("stream", 64, 15000),                # the first workgroup's 16 blocks
    ("tiled", 1169 * 7168 + 64, 1170 * 7168 - 300),  # tile 1169 of 1171
])
def test_lost_count_gives_ehip_and_the_next_search_is_clean(ctx, pk, oracle_lib, kernel, lo, hi):
    k = pk.PULSCAN_KERNEL_STREAM if kernel == "stream" else pk.PULSCAN_KERNEL_TILED
    d = to_device(heavy_spectrum(oracle_lib, lo, hi, seed=17 if kernel == "stream" else 19))
    ctx.pulscan_ctx_set_kernel(k)
    try:
        say(f"give-up {kernel}: reference search")
        ref, nref = ctx.pulscan_search_ex(d, Z, C, 6.0)
        assert ctx.pulscan_ctx_last_kernel() == k
        assert nref > 0
        say(f"give-up {kernel}: one poll per count word")
        ctx.pulscan_ctx_set_spin(1)
        with pytest.raises(pk.PulscanError) as e:
            ctx.pulscan_search_ex(d, Z, C, 6.0)
        assert e.value.status == pk.PULSCAN_EHIP
        ctx.pulscan_ctx_set_spin(DEFAULT_SPIN)
        for rep in range(2):
            say(f"give-up {kernel}: clean search {rep}")
            got, ngot = ctx.pulscan_search_ex(d, Z, C, 6.0)
            assert ngot == nref
            assert got.tobytes() == ref.tobytes()
    finally:
        ctx.pulscan_ctx_set_spin(DEFAULT_SPIN)
        ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_AUTO)
