"""GPU path vs the CPU oracle, element by element, through the C ABI.

FP64 form: within 1e-12 of the exact |M|^2 on every event.  Events where
the GPU and the FP64 oracle differ by more than 1e-13 are re-evaluated with
the long-double oracle, and the GPU must be within 1e-12 of it on each of
them (fp64_bar.py).  Mixed form: median relative error <= 1e-5 and
maximum <= 1e-3.  Sizes: the oracle checks every event of batches that span
many 256-event blocks plus a ragged tail, and a random sample of events of
the full-size configurations the benchmark runs.
"""
import numpy as np
import pytest

from paper_2312_02898_amd.inputs import CONFIGS, config_events

from fp64_bar import check_fp64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

QQG = ["uuttg", "uxuttg", "ugttu", "guttu", "uxgttux", "guxttux"]
PROCS = ["eemumu", "ggtt", "ggttg", "ggttgg", "uutt", "uxutt"] + QQG
# events checked element-wise against the oracle (all of ee->mumu's batch)
NCHECK = {"eemumu": 16384, "ggtt": 4096 + 37, "ggttg": 2048 + 37, "ggttgg": 1024 + 37, "uutt": 4096 + 37,
          "uxutt": 4096 + 37}
NCHECK.update({p: 2048 + 37 for p in QQG})


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def B():
    from paper_2312_02898_amd import binding
    binding.lib()
    return binding


def _me(B, proc, precision, **kw):
    from paper_2312_02898_amd.engine import MatrixElement
    return MatrixElement(proc, precision=precision, **kw)


def _run(me, mom_np, dev):
    m = torch.from_numpy(mom_np).to(dev)
    out = me(m)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _rel(a, b):
    return np.abs(a / b - 1.0)


def _check_fp64(oracle_lib, name, mom, gpu, ref):
    check_fp64(gpu, ref, lambda idx: oracle_lib.me(name, mom[idx], long_double=True), name)


@pytest.mark.parametrize("proc", PROCS)
def test_fp64_matches_oracle(oracle_lib, B, dev, proc):
    mom = config_events(proc, NCHECK[proc])
    name = CONFIGS[proc][0]
    print(f"[fp64 parity] {proc} nevt={mom.shape[0]}", flush=True)
    me = _me(B, proc, "fp64")
    gpu = _run(me, mom, dev)
    ref = oracle_lib.me(name, mom)
    _check_fp64(oracle_lib, name, mom, gpu, ref)


@pytest.mark.parametrize("proc", PROCS)
def test_fp64_full_size_sampled(oracle_lib, B, dev, proc):
    """Full benchmark batch in the launch configuration the benchmark uses;
    the oracle checks a random sample of its events."""
    mom = config_events(proc)
    name = CONFIGS[proc][0]
    print(f"[fp64 full] {proc} nevt={mom.shape[0]}", flush=True)
    me = _me(B, proc, "fp64")
    gpu = _run(me, mom, dev)
    assert np.isfinite(gpu).all() and (gpu > 0).all()
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(mom.shape[0], size=256, replace=False))
    ref = oracle_lib.me(name, mom[idx])
    _check_fp64(oracle_lib, name, mom[idx], gpu[idx], ref)


@pytest.mark.parametrize("precision", ["mixed", "mixed_valu", "mixed_mfma16", "mixed_mfma32", "mixed_mfma_bf16"])
@pytest.mark.parametrize("proc", PROCS)
def test_mixed_precision_error(oracle_lib, B, dev, proc, precision):
    mom = config_events(proc, NCHECK[proc])
    name = CONFIGS[proc][0]
    print(f"[{precision} parity] {proc} nevt={mom.shape[0]}", flush=True)
    me = _me(B, proc, precision)
    gpu = _run(me, mom, dev)
    ref = oracle_lib.me(name, mom)
    rel = _rel(gpu, ref)
    print(f"  mixed median {np.median(rel):.3e} p99 {np.quantile(rel, 0.99):.3e} max {rel.max():.3e}", flush=True)
    assert np.median(rel) <= 1e-5
    assert rel.max() <= 1e-3


@pytest.mark.parametrize("proc", PROCS)
def test_per_helicity_and_filter(oracle_lib, B, dev, proc):
    """|M_h|^2 of every helicity matches the oracle; the filter keeps every
    helicity that is alive on the configuration's events."""
    mom = config_events(proc, 64)
    name = CONFIGS[proc][0]
    me = _me(B, proc, "fp64")
    m = torch.from_numpy(mom).to(dev)
    gh = me.helicities(m)
    torch.cuda.synchronize()
    gh = gh.cpu().numpy()
    oh = oracle_lib.me_hel(name, mom)
    scale = oh.sum(axis=1, keepdims=True)
    assert (np.abs(gh - oh) / scale).max() <= 1e-12
    live = np.nonzero((oh / scale).max(axis=0) > 1e-20)[0]
    good = set(me.good_helicities())
    assert set(live.tolist()) <= good
    # the filtered sum equals the unfiltered one
    me_all = _me(B, proc, "fp64", filter_helicities=False)
    a = _run(me, mom, dev)
    b = _run(me_all, mom, dev)
    assert _rel(a, b).max() <= 1e-13


@pytest.mark.parametrize("proc", ["ggtt", "ggttgg"])
def test_ragged_sizes_and_determinism(B, dev, proc):
    """nevt in {1, 63, 64, 65, 255, 257}: each result equals the same events
    inside a larger batch bit for bit, and reruns are bitwise identical."""
    mom = config_events(proc, 1000)
    me = _me(B, proc, "fp64")
    full = _run(me, mom, dev)
    again = _run(me, mom, dev)
    assert np.array_equal(full, again)
    for n in (1, 63, 64, 65, 255, 257):
        part = _run(me, np.ascontiguousarray(mom[:n]), dev)
        assert np.array_equal(part, full[:n])
    off = _run(me, np.ascontiguousarray(mom[311:311 + 77]), dev)
    assert np.array_equal(off, full[311:311 + 77])


def test_abi_errors(B, dev):
    import ctypes
    with pytest.raises(B.MeError) as e:
        B.me_create("g g > t t~ t t~")
    assert e.value.status == B.ME_EPROCESS
    h = B.me_create("g g > t t~")
    # nevt == 0 is a no-op, null pointers and negative sizes are rejected
    assert B.lib().me_compute(h, None, 0, None, None) == B.ME_OK
    assert B.lib().me_compute(h, None, 5, None, None) == B.ME_EINVAL
    assert B.lib().me_compute(h, ctypes.c_void_p(16), -1, ctypes.c_void_p(16), None) == B.ME_EINVAL
    assert B.lib().me_compute(None, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None) == B.ME_EINVAL
    info = B.me_info(h)
    assert info["npar"] == 4 and info["ndiagrams"] == 3 and info["ncolor"] == 2 and info["nhel"] == 16
    B.me_helicity_filter(h)
    B.me_helicity_filter(h)   # idempotent
    assert B.me_info(h)["nhel_good"] == 12
    B.me_destroy(h)


# BF16 hi+lo carries 16 significant bits of each jamp (2^-16 = 1.5e-5 at
# most, a few 1e-6 typically); FP16 hi+lo about 22 and FP32 operands 24
@pytest.mark.parametrize("variant,med,mx", [("mixed_mfma16", 1e-6, 1e-5), ("mixed_mfma32", 1e-6, 1e-5),
                                            ("mixed_mfma_bf16", 1e-5, 1e-3)])
@pytest.mark.parametrize("proc", ["ggttg", "ggttgg"])
def test_mfma_colour_sum_matches_valu(B, dev, proc, variant, med, mx):
    """The MFMA colour sums (FP16 or BF16 hi+lo jamps or FP32 operands, FP32
    accumulation) agree with the FP32 vector-ALU colour sum of the same FP32
    jamps, including a batch with a ragged last wave."""
    mom = config_events(proc, 2048 + 29)
    a = _run(_me(B, proc, variant), mom, dev)
    b = _run(_me(B, proc, "mixed_valu"), mom, dev)
    rel = _rel(a, b)
    print(f"  {variant} vs valu median {np.median(rel):.3e} max {rel.max():.3e}", flush=True)
    assert np.median(rel) < med and rel.max() < mx


def test_debug_validation(B, dev, monkeypatch):
    """With ME_DEBUG set at creation, me_compute rejects batches with
    non-finite or unbalanced momenta (and computes valid ones)."""
    monkeypatch.setenv("ME_DEBUG", "1")
    me = _me(B, "ggtt", "fp64")
    mom = config_events("ggtt", 300)
    ok = _run(me, mom, dev)
    assert np.isfinite(ok).all()
    for bad in ("nan", "balance"):
        m = mom.copy()
        if bad == "nan":
            m[17, 2, 1] = np.nan
        else:
            m[250, 3, 0] += 1e-3
        with pytest.raises(B.MeError) as e:
            _run(me, m, dev)
        assert e.value.status == B.ME_EINVAL
    me.close()


def test_batch_beyond_2gib_of_momenta(oracle_lib, B, dev):
    """2^24 + 13 g g > t t~ events (2.1 GB of momenta: byte offsets past
    2^31) generated on the device, both forms; sampled events, the last ones
    among them, against the oracle."""
    n = (1 << 24) + 13
    print(f"[beyond 2 GiB] ggtt nevt={n}", flush=True)
    m = torch.empty((n, 4, 4), dtype=torch.float64, device=dev)
    B.me_rambo(n, [173.0, 173.0], 1500.0, 77, m.data_ptr(), torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.choice(n, size=200, replace=False), np.arange(n - 40, n)]))
    sel = torch.from_numpy(idx).to(dev)
    mom = m[sel].cpu().numpy()
    ref = oracle_lib.me("g g > t t~", mom)
    for precision in ("fp64", "mixed"):
        me = _me(B, "ggtt", precision)
        out = me(m)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).all()) and bool((out > 0).all())
        got = out[sel].cpu().numpy()
        if precision == "fp64":
            _check_fp64(oracle_lib, "g g > t t~", mom, got, ref)
        else:
            rel = _rel(got, ref)
            assert np.median(rel) <= 1e-5 and rel.max() <= 1e-3
        me.close()
        del out
