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
The same holds for asynchronous calls, whose count word then carries
PULSCAN_COUNT_LOST.
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

        # asynchronous: the count word carries the failure, and the next
        # asynchronous search (which the host cannot have re-armed for) is
        # clean: the failed launch's emit cleared what its late workgroups
        # left behind
        import torch
        cap = nref + 64
        buf = torch.zeros(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        aopts = pk.make_opts(async_=True, stream=torch.cuda.current_stream())
        say(f"give-up {kernel}: asynchronous, one poll per count word")
        ctx.pulscan_ctx_set_spin(1)
        ctx.pulscan_search_ex(d, Z, C, 6.0, capacity=cap, opts=aopts, out_device=buf,
                              count_device=cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) & 0xFFFFFFFFFFFFFFFF == pk.PULSCAN_COUNT_LOST
        ctx.pulscan_ctx_set_spin(DEFAULT_SPIN)
        say(f"give-up {kernel}: asynchronous clean search")
        buf.zero_()
        ctx.pulscan_search_ex(d, Z, C, 6.0, capacity=cap, opts=aopts, out_device=buf,
                              count_device=cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == nref
        got = buf[:nref * pk.CANDIDATE_DTYPE.itemsize].cpu().numpy().view(pk.CANDIDATE_DTYPE)
        assert got.tobytes() == ref.tobytes()
    finally:
        ctx.pulscan_ctx_set_spin(DEFAULT_SPIN)
        ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_AUTO)
