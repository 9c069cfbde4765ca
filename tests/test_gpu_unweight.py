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
