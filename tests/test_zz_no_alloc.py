"""me_compute_channels_noalloc: the multi-subprocess entry point whose
workspace is the library's fixed device array, for callers that cannot
allocate.  Through the C ABI its results equal those of me_compute_channels
(same kernels, same partition: bit for bit) on two calls in a row, the second
with a smaller batch; oversized batches and processes that need a workspace
of their own are rejected before anything is launched."""
import numpy as np
import pytest

from paper_2312_02898_amd.inputs import config_events

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHAS = np.array([0.100, 0.118, 0.130])


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _batch(cfg, n, nch, seed):
    rng = np.random.default_rng(seed)
    mom = config_events(cfg, n)
    ch = rng.integers(0, nch, size=n).astype(np.int32)
    al = ALPHAS[rng.integers(0, 3, size=n)]
    return mom, ch, al


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("cfg,procs", [("ggtt", ["ggtt", "uutt", "uxutt"]),
                                       ("ggttg", ["ggttg", "uuttg", "uxuttg", "ugttu", "guttu"])])
def test_noalloc_equals_allocating_entry_point(dev, cfg, procs, precision):
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import ChannelMix
    mix = ChannelMix(procs, precision)
    handles = [m.handle for m in mix.members]
    stream = torch.cuda.current_stream().cuda_stream
    for n, seed, use_alphas in ((5000 + 17, 3, True), (777, 4, False)):
        print(f"[noalloc] {cfg} {precision} nevt={n}", flush=True)
        mom, ch, al = _batch(cfg, n, len(procs), seed)
        m = torch.from_numpy(mom).to(dev)
        c = torch.from_numpy(ch).to(dev)
        a = torch.from_numpy(al).to(dev) if use_alphas else None
        ref = torch.empty(n, dtype=torch.float64, device=dev)
        got = torch.full((n,), -1.0, dtype=torch.float64, device=dev)
        args = (m.data_ptr(), c.data_ptr(), a.data_ptr() if a is not None else 0, n)
        B.me_compute_channels(handles, *args, ref.data_ptr(), stream)
        B.me_compute_channels_noalloc(handles, *args, got.data_ptr(), stream)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(r).all() and (r > 0).all()
        assert np.array_equal(r, g)
    mix.close()


def test_noalloc_rejects_what_it_cannot_hold(dev):
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import MatrixElement
    stream = torch.cuda.current_stream().cuda_stream
    me = MatrixElement("ggtt", "fp64")
    # more events than the fixed workspace holds (about 144 bytes per
    # event of 4 legs): rejected before any launch (the buffers are real)
    n = B.NOALLOC_SCRATCH_BYTES // 144 + 4096
    m = torch.zeros((n, 4, 4), dtype=torch.float64, device=dev)
    c = torch.zeros(n, dtype=torch.int32, device=dev)
    out = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(B.MeError) as e:
        B.me_compute_channels_noalloc([me.handle], m.data_ptr(), c.data_ptr(), 0, n, out.data_ptr(), stream)
    assert e.value.status == B.ME_EINVAL
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    # the split form needs its own workspace: not supported here
    big = MatrixElement("ggttggg", "mixed")
    mom = torch.from_numpy(config_events("ggttggg", 64)).to(dev)
    c7 = torch.zeros(64, dtype=torch.int32, device=dev)
    o7 = torch.zeros(64, dtype=torch.float64, device=dev)
    with pytest.raises(B.MeError) as e:
        B.me_compute_channels_noalloc([big.handle], mom.data_ptr(), c7.data_ptr(), 0, 64, o7.data_ptr(), stream)
    assert e.value.status == B.ME_ENOTSUP
    # nevt == 0 is a no-op
    B.me_compute_channels_noalloc([me.handle], m.data_ptr(), c.data_ptr(), 0, 0, out.data_ptr(), stream)
    me.close()
    big.close()
