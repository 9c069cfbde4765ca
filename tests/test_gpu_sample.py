"""Device importance-sampled phase space (me_sample) against the oracle's
implementation of the same mapping on the same Philox4x32-10 stream, and the
device pipeline sample -> me_compute -> me_max_weight (weights |M|^2 x phase-
space weight, their batch maximum) without a host copy, against the oracle's
|M|^2 of the same points."""
import numpy as np
import pytest

from fp64_bar import check_fp64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [("ggtt", [173.0, 173.0]), ("ggttg", [173.0, 173.0, 0.0]), ("ggttgg", [173.0, 173.0, 0.0, 0.0]),
         ("ggttggg", [173.0, 173.0, 0.0, 0.0, 0.0])]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,masses", CASES)
@pytest.mark.parametrize("n", [1, 255, 257, 100000])
def test_device_sampler_matches_oracle(oracle_lib, dev, name, masses, n):
    from paper_2312_02898_amd import binding as B
    print(f"[sample] {name} n={n}", flush=True)
    d = torch.empty((n, len(masses) + 2, 4), dtype=torch.float64, device=dev)
    w = torch.empty(n, dtype=torch.float64, device=dev)
    B.me_sample(n, masses, 1500.0, 91, d.data_ptr(), w.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got, gw = d.cpu().numpy(), w.cpu().numpy()
    ref, rw = oracle_lib.sample(n, masses, 1500.0, 91)
    # the same arithmetic up to contraction and the device's transcendental
    # functions: componentwise within a few ulp of sqrt(s), weights relative
    assert np.abs(got - ref).max() <= 1e-12 * 1500.0
    assert np.abs(gw / rw - 1).max() <= 1e-11
    bal = got[:, 0] + got[:, 1] - got[:, 2:].sum(axis=1)
    assert np.abs(bal).max() <= 1e-11 * 1500.0


def test_sample_compute_max_weight_pipeline(oracle_lib, dev):
    """g g > t t~ g g: 2^17 sampled points, their |M|^2 (FP64) and weights
    |M|^2 x W / (2 s) with the batch maximum, all on the device; the oracle's
    |M|^2 of a sample of the points and the exact maximum of the device
    weights (a product and a maximum: no rounding freedom)."""
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import MatrixElement
    n = 1 << 17
    masses = [173.0, 173.0, 0.0, 0.0]
    s = 1500.0 ** 2
    stream = torch.cuda.current_stream().cuda_stream
    d = torch.empty((n, 6, 4), dtype=torch.float64, device=dev)
    w = torch.empty(n, dtype=torch.float64, device=dev)
    B.me_sample(n, masses, 1500.0, 5, d.data_ptr(), w.data_ptr(), stream)
    me = MatrixElement("ggttgg", "fp64")
    m2 = me(d)
    fac = w / (2 * s)
    ww = torch.empty(n, dtype=torch.float64, device=dev)
    mx = torch.empty(1, dtype=torch.float64, device=dev)
    B.me_max_weight(m2.data_ptr(), fac.data_ptr(), n, ww.data_ptr(), mx.data_ptr(), stream)
    torch.cuda.synchronize()
    m2n, facn, wwn = m2.cpu().numpy(), fac.cpu().numpy(), ww.cpu().numpy()
    assert np.array_equal(wwn, np.where(m2n * facn > 0, m2n * facn, 0.0))
    assert float(mx.item()) == wwn.max()
    idx = np.sort(np.random.default_rng(2).choice(n, size=256, replace=False))
    pts = d.cpu().numpy()[idx]
    ref = oracle_lib.me("g g > t t~ g g", pts)
    # the sampler concentrates points near soft and collinear limits, where the
    # FP64 oracle's own rounding grows: every point is judged against long double
    check_fp64(m2n[idx], ref, lambda i: oracle_lib.me("g g > t t~ g g", pts[i], long_double=True), "sampled",
               flag=0.0, median=None)
    me.close()
