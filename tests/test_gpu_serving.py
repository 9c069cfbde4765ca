"""Serving form on the GPU: requests of several processes and uneven sizes
arrive while others run; every result equals the same request evaluated
alone (bit for bit: events are independent and each lane's arithmetic does
not depend on its neighbours), memory admission holds the budget with each
request's workspace counted in its footprint (free device memory does not
move while a g g > t t~ g g g heavy stream runs), and a request larger than
the whole budget is rejected."""
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


@pytest.mark.parametrize("budget,slots", [(1 << 30, 8), (64 << 20, 4)])
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


def test_workspace_inside_the_budget(handles):
    """g g > t t~ g g g requests carry their jamp workspace in their
    footprint: the server's arena (allocated at creation) is all the device
    memory the stream uses, so free memory sampled while it runs never drops
    below its value after creation, and peak arena use stays within the
    budget, with the budget small enough that admission waits for memory."""
    import threading
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.serving import make_stream, run_stream
    budget = 96 << 20
    names = ["ggttggg", "ggttgg", "ggttggg"]
    arr, procs, moms = make_stream(names, 24, rate_hz=5000.0, seed=9, nmin=256, nmax=12000)
    ws = {nm: B.me_workspace_bytes(handles[nm], 12000) for nm in ("ggttgg", "ggttggg")}
    assert ws["ggttgg"] == 0 and ws["ggttggg"] > 0
    print(f"[serving workspace] budget={budget} requests={len(procs)}", flush=True)
    torch.cuda.synchronize()
    base, samples, stop = [], [], threading.Event()

    def created(_srv):
        torch.cuda.synchronize()
        base.append(torch.cuda.mem_get_info()[0])

    def poll():
        while not stop.is_set():
            samples.append(torch.cuda.mem_get_info()[0])
            stop.wait(0.0005)
    th = threading.Thread(target=poll)
    th.start()
    try:
        lat, status, outs, wall, st = run_stream(handles, arr, procs, moms, budget_bytes=budget, n_slots=8,
                                                 on_created=created)
    finally:
        stop.set()
        th.join()
    assert (status == 0).all() and st["completed"] == len(procs)
    assert st["peak_bytes_in_use"] <= budget
    during = samples
    print(f"  free after creation {base[0] / 2**20:.1f} MiB, lowest while serving {min(during) / 2**20:.1f} MiB, "
          f"peak arena {st['peak_bytes_in_use'] / 2**20:.1f} MiB, passes {st['bypassed']}", flush=True)
    assert min(during) >= base[0] - (2 << 20)
    for name, m, o in zip(procs, moms, outs):
        assert np.array_equal(o, _alone(B, handles[name], m)), name


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


def test_large_requests_run_in_pieces(handles):
    """g g > t t~ g g g requests above 2e11 flop (here 40 000 and 16 385
    events) run in pieces of 16 384 events, one piece's kernels queued at a
    time, with small requests arriving meanwhile: every result equals the
    same request evaluated in one call, bit for bit."""
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.inputs import CONFIGS, process_events
    from paper_2312_02898_amd.serving import run_stream
    rng = np.random.default_rng(3)
    procs = ["ggttggg", "ggtt", "ggttgg", "ggttggg", "eemumu", "ggttg", "ggtt", "ggttgg"]
    sizes = [40000, 300, 2000, 16385, 256, 1000, 5000, 700]
    moms = [process_events(CONFIGS[p][0], n, CONFIGS[p][1], 100 + i) for i, (p, n) in enumerate(zip(procs, sizes))]
    arr = np.cumsum(rng.exponential(0.002, size=len(procs))) - 0.002
    print(f"[serving pieces] sizes={sizes}", flush=True)
    lat, status, outs, wall, st = run_stream(handles, np.maximum(arr, 0.0), procs, moms, budget_bytes=1 << 30,
                                             n_slots=8)
    assert (status == 0).all() and st["completed"] == len(procs)
    for name, m, o in zip(procs, moms, outs):
        assert np.array_equal(o, _alone(B, handles[name], m)), name
