"""Serving form on the GPU: requests of several processes and uneven sizes
arrive while others run; every result equals the same request evaluated
alone (bit for bit: events are independent and each lane's arithmetic does
not depend on its neighbours), memory admission holds the budget, and a
request larger than the whole budget is rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NAMES = ["eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg"]


@pytest.fixture(scope="module")
def handles():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import PROCESS_NAMES
    hs = {}
    for nm in NAMES:
        h = B.me_create(PROCESS_NAMES[nm], B.me_default_params(precision=B.ME_MIXED))
        B.me_helicity_filter(h)
        hs[nm] = h
    yield hs
    for h in hs.values():
        B.me_destroy(h)


def _alone(B, h, mom):
    m = torch.from_numpy(mom).to("cuda:0")
    out = torch.empty(mom.shape[0], dtype=torch.float64, device="cuda:0")
    B.me_compute(h, m.data_ptr(), mom.shape[0], out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("budget,slots", [(1 << 30, 8), (6 << 20, 4)])
def test_mix_equals_alone(handles, budget, slots):
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.serving import make_stream, run_stream
    print(f"[serving] budget={budget} slots={slots}", flush=True)
    arr, procs, moms = make_stream(NAMES, 48, rate_hz=2000.0, seed=5, nmin=256, nmax=16384)
    times = []
    lat, status, outs, wall, st = run_stream(handles, arr, procs, moms, budget_bytes=budget, n_slots=slots,
                                             times=times)
    assert (status == 0).all()
    q = np.array([t[0] for t in times])
    sv = np.array([t[1] for t in times])
    assert (q >= 0).all() and (sv > 0).all() and np.allclose(q + sv, lat, rtol=0, atol=1e-9)
    assert st["completed"] == 48 and st["failed"] == 0
    assert st["peak_bytes_in_use"] <= budget and st["bytes_in_use"] == 0
    for name, m, o in zip(procs, moms, outs):
        ref = _alone(B, handles[name], m)
        assert np.array_equal(o, ref), name
    print(f"  p50 {np.median(lat) * 1e3:.2f} ms p99 {np.quantile(lat, 0.99) * 1e3:.2f} ms wall {wall:.3f} s",
          flush=True)


def test_over_budget_and_invalid(handles):
    from paper_2312_02898_amd import binding as B
    srv = B.me_server_create(1 << 20, 2)
    try:
        big = np.zeros((100000, 6, 4))
        out = np.zeros(100000)
        with pytest.raises(B.MeError) as e:
            B.me_server_submit(srv, handles["ggttgg"], big, out)
        assert e.value.status == B.ME_ENOMEM
        with pytest.raises(B.MeError) as e:
            B.me_server_submit(srv, handles["ggttgg"], big[:0], out[:0])
        assert e.value.status == B.ME_EINVAL
        st = B.me_server_stats(srv)
        assert st["rejected"] == 1 and st["submitted"] == 0
    finally:
        B.me_server_destroy(srv)
