"""gg -> t tbar ggg (1240 diagrams, 120 colour flows, 128 helicities) on the
split form: amplitude parts writing jamps to a workspace, colour sum on MFMA.

Same bars as the other processes: FP64 within 1e-12 of the exact |M|^2 on
every event (events above 1e-13 against the FP64 oracle re-evaluated with
the long-double oracle, fp64_bar.py), mixed form
median <= 1e-5 and max <= 1e-3.  The oracle takes about 0.2 s per event on
one core, so element-wise checks use a few hundred events; the chunked
launch (events beyond one chunk of 2^14, helicities in several workspace
slices) is checked on sampled events and against the same events in a small
batch.
"""
import numpy as np
import pytest

from paper_2312_02898_amd.inputs import CONFIGS, config_events

from fp64_bar import check_fp64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NAME = CONFIGS["ggttggg"][0]
CHUNK = 1 << 14


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _me(precision, **kw):
    from paper_2312_02898_amd.engine import MatrixElement
    return MatrixElement("ggttggg", precision=precision, **kw)


def _run(me, mom_np, dev):
    out = me(torch.from_numpy(mom_np).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _rel(a, b):
    return np.abs(a / b - 1.0)


def _check_fp64(oracle_lib, mom, gpu, ref):
    check_fp64(gpu, ref, lambda idx: oracle_lib.me(NAME, mom[idx], long_double=True), "ggttggg")


@pytest.fixture(scope="module")
def small(oracle_lib):
    mom = config_events("ggttggg", 256 + 37)
    return mom, oracle_lib.me(NAME, mom)


def test_fp64_matches_oracle(oracle_lib, dev, small):
    mom, ref = small
    print(f"[ggttggg fp64] nevt={mom.shape[0]}", flush=True)
    gpu = _run(_me("fp64"), mom, dev)
    _check_fp64(oracle_lib, mom, gpu, ref)


# every mixed form of the split process sums colours on FP16 hi+lo MFMA
@pytest.mark.parametrize("precision", ["mixed", "mixed_valu", "mixed_mfma_bf16"])
def test_mixed_matches_oracle(dev, small, precision):
    mom, ref = small
    print(f"[ggttggg {precision}] nevt={mom.shape[0]}", flush=True)
    gpu = _run(_me(precision), mom, dev)
    rel = _rel(gpu, ref)
    print(f"  median {np.median(rel):.3e} p99 {np.quantile(rel, 0.99):.3e} max {rel.max():.3e}", flush=True)
    assert np.isfinite(gpu).all()
    assert np.median(rel) <= 1e-5
    assert rel.max() <= 1e-3


def test_per_helicity_and_filter(oracle_lib, dev):
    mom = config_events("ggttggg", 12)
    print("[ggttggg per-helicity]", flush=True)
    me = _me("fp64")
    gh = me.helicities(torch.from_numpy(mom).to(dev))
    torch.cuda.synchronize()
    gh = gh.cpu().numpy()
    oh = oracle_lib.me_hel(NAME, mom)
    scale = oh.sum(axis=1, keepdims=True)
    err = (np.abs(gh - oh) / scale).max()
    print(f"  max |dM_h|/sum {err:.3e}", flush=True)
    assert err <= 1e-12
    live = np.nonzero((oh / scale).max(axis=0) > 1e-20)[0]
    assert set(live.tolist()) <= set(me.good_helicities())
    a = _run(me, mom, dev)
    b = _run(_me("fp64", filter_helicities=False), mom, dev)
    assert _rel(a, b).max() <= 1e-13


def test_ragged_sizes_bitwise(dev):
    """Batches of 1..257 events give the same bits as the same events inside
    a larger (single-chunk) batch, and reruns are bitwise identical."""
    mom = config_events("ggttggg", 600)
    for prec in ("fp64", "mixed"):
        print(f"[ggttggg ragged] {prec}", flush=True)
        me = _me(prec)
        full = _run(me, mom, dev)
        assert np.array_equal(full, _run(me, mom, dev))
        for n in (1, 15, 16, 17, 63, 65, 257):
            assert np.array_equal(_run(me, np.ascontiguousarray(mom[:n]), dev), full[:n])
        assert np.array_equal(_run(me, np.ascontiguousarray(mom[311:311 + 77]), dev), full[311:311 + 77])


def test_chunked_launch_sampled(oracle_lib, dev):
    """More than one chunk of events (and, in FP64, several helicity slices of
    the workspace): sampled events near both chunk edges and elsewhere match
    the oracle, and the same events computed in a small batch agree to
    rounding (only the order of the helicity sum differs)."""
    n = CHUNK + 300
    mom = config_events("ggttggg", n)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(CHUNK - 8, CHUNK + 8), [0, n - 1],
                                    rng.choice(n, size=40, replace=False)]))
    ref = oracle_lib.me(NAME, mom[idx])
    sub = np.ascontiguousarray(mom[idx])
    for prec in ("fp64", "mixed"):
        print(f"[ggttggg chunked] {prec} nevt={n}", flush=True)
        me = _me(prec)
        got = _run(me, mom, dev)
        assert np.isfinite(got).all() and (got > 0).all()
        alone = _run(me, sub, dev)
        if prec == "fp64":
            _check_fp64(oracle_lib, mom[idx], got[idx], ref)
            assert _rel(got[idx], alone).max() <= 1e-14
        else:
            rel = _rel(got[idx], ref)
            print(f"  median {np.median(rel):.3e} max {rel.max():.3e}", flush=True)
            assert np.median(rel) <= 1e-5 and rel.max() <= 1e-3
            assert _rel(got[idx], alone).max() <= 1e-6
