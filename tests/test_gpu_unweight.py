"""GPU-assisted batch unweighting (paper, Sec. 3): device weights and batch
maximum vs the plain definition, bit for bit (a product and a max involve no
rounding-order freedom)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000, 4096 * 256 + 77, 1 << 21])
def test_max_weight_matches_definition(oracle_lib, n):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02898_amd import binding as B
    print(f"[max_weight] n={n}", flush=True)
    rng = np.random.default_rng(n + 1)
    me = rng.lognormal(0, 3, size=n)
    f = rng.lognormal(0, 2, size=n)
    if n > 10:
        f[3] = -1.0          # negative factor counts as 0
        me[5] = np.nan
    d_me = torch.from_numpy(me).cuda()
    d_f = torch.from_numpy(f).cuda()
    d_w = torch.empty(n, dtype=torch.float64, device="cuda")
    d_max = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    B.me_max_weight(d_me.data_ptr(), d_f.data_ptr(), n, d_w.data_ptr() if n else 0, d_max.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    w_ref, m_ref = oracle_lib.max_weight(me, f)
    assert d_max.item() == m_ref
    if n:
        assert np.array_equal(d_w.cpu().numpy(), w_ref)
    # without the weights output
    d_max2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.me_max_weight(d_me.data_ptr(), d_f.data_ptr(), n, 0, d_max2.data_ptr(), 0)
    torch.cuda.synchronize()
    assert d_max2.item() == m_ref


def test_max_weight_errors():
    from paper_2312_02898_amd import binding as B
    assert B.lib().me_max_weight(None, None, 5, None, None, None) == B.ME_EINVAL
    assert B.lib().me_max_weight(None, None, -1, None, None, None) == B.ME_EINVAL


FUSED = [("ggtt", "fp64", 1000), ("ggttgg", "fp64", 4096 + 37), ("ggttgg", "mixed", 4096 + 37),
         ("ggttgg", "mixed_mfma16", 999), ("uuttgg", "fp64", 777), ("ggttggg", "mixed", (1 << 17) + 300),
         ("ggttggg", "fp64", 513)]


@pytest.mark.parametrize("proc,precision,n", FUSED)
def test_fused_weights_equal_separate(oracle_lib, proc, precision, n):
    """me_compute_weighted: |M|^2 bit for bit that of me_compute, the weights
    and their maximum bit for bit the plain definition on those |M|^2; two
    calls in a row (the maximum is cleared; the second is smaller), a batch
    over more than one chunk of the split form, and nevt = 0."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import MatrixElement
    from paper_2312_02898_amd.inputs import config_events
    print(f"[fused weights] {proc} {precision} n={n}", flush=True)
    me = MatrixElement(proc, precision)
    stream = torch.cuda.current_stream().cuda_stream
    mom = torch.from_numpy(config_events(proc, n)).cuda()
    ref_me = me(mom)
    rng = np.random.default_rng(n)
    for scale in (1.0, 0.25):
        f = rng.lognormal(0, 2, size=n) * scale
        f[7] = -1.0
        d_f = torch.from_numpy(f).cuda()
        d_me = torch.full((n,), -3.0, dtype=torch.float64, device="cuda")
        d_w = torch.full((n,), -3.0, dtype=torch.float64, device="cuda")
        d_max = torch.full((1,), 1e300, dtype=torch.float64, device="cuda")
        B.me_compute_weighted(me.handle, mom.data_ptr(), n, d_f.data_ptr(), d_me.data_ptr(), d_w.data_ptr(),
                              d_max.data_ptr(), stream)
        torch.cuda.synchronize()
        got_me = d_me.cpu().numpy()
        assert np.array_equal(got_me, ref_me.cpu().numpy())
        w_ref, m_ref = oracle_lib.max_weight(got_me, f)
        assert np.array_equal(d_w.cpu().numpy(), w_ref)
        assert d_max.item() == m_ref
        # without the weights output
        d_max2 = torch.full((1,), 1e300, dtype=torch.float64, device="cuda")
        B.me_compute_weighted(me.handle, mom.data_ptr(), n, d_f.data_ptr(), d_me.data_ptr(), 0, d_max2.data_ptr(),
                              stream)
        torch.cuda.synchronize()
        assert d_max2.item() == m_ref
    d_max0 = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    B.me_compute_weighted(me.handle, 0, 0, 0, 0, 0, d_max0.data_ptr(), stream)
    torch.cuda.synchronize()
    assert d_max0.item() == 0.0
    me.close()


def test_fused_weights_errors():
    from paper_2312_02898_amd import binding as B
    L = B.lib()
    assert L.me_compute_weighted(None, None, 5, None, None, None, None, None) == B.ME_EINVAL
