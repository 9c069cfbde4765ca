"""Two-jet channels of p p > t t~ on the GPU, through the C ABI, against the
diagram-by-diagram oracle: q qbar > t tbar g g, q g > t tbar q g and their
crossings, g g > t tbar q qbar, and the four-quark channels with one and two
light flavours (Fermi signs between the fermion pairings of identical quarks).

FP64 within 1e-12 of the exact value on every event (fp64_bar.py), mixed
form median <= 1e-5 and max <= 1e-3; per-helicity values and the helicity
filter; large batches on sampled events; and p p > t t~ + 2 jets as one channel mix with the
g g > t t~ g g channel at per-event alpha_s.
"""
import numpy as np
import pytest

from paper_2312_02898_amd.inputs import CONFIGS, config_events

from fp64_bar import check_fp64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TWO_JET = ["uuttgg", "uxuttgg", "ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux", "uuttuux", "uuttddx",
           "uuttuu", "udttud", "uxuxttuxux"]
NCHECK = 1024 + 37
_REF = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ref(oracle_lib, proc, n):
    key = (proc, n)
    if key not in _REF:
        _REF[key] = oracle_lib.me(CONFIGS[proc][0], config_events(proc, n))
    return _REF[key]


def _run(proc, precision, mom, dev, **kw):
    from paper_2312_02898_amd.engine import MatrixElement
    me = MatrixElement(proc, precision, **kw)
    out = me(torch.from_numpy(mom).to(dev))
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    me.close()
    return r


@pytest.mark.parametrize("proc", TWO_JET)
def test_fp64_matches_oracle(oracle_lib, dev, proc):
    mom = config_events(proc, NCHECK)
    print(f"[two-jet fp64] {proc} nevt={NCHECK}", flush=True)
    gpu = _run(proc, "fp64", mom, dev)
    name = CONFIGS[proc][0]
    check_fp64(gpu, _ref(oracle_lib, proc, NCHECK), lambda idx: oracle_lib.me(name, mom[idx], long_double=True),
               proc)


@pytest.mark.parametrize("precision", ["mixed", "mixed_mfma16", "mixed_mfma_bf16"])
@pytest.mark.parametrize("proc", TWO_JET)
def test_mixed_matches_oracle(oracle_lib, dev, proc, precision):
    mom = config_events(proc, NCHECK)
    print(f"[two-jet {precision}] {proc} nevt={NCHECK}", flush=True)
    gpu = _run(proc, precision, mom, dev)
    rel = np.abs(gpu / _ref(oracle_lib, proc, NCHECK) - 1)
    print(f"  median {np.median(rel):.3e} max {rel.max():.3e}", flush=True)
    assert np.median(rel) <= 1e-5 and rel.max() <= 1e-3


@pytest.mark.parametrize("proc", TWO_JET)
def test_large_batch_sampled(oracle_lib, dev, proc):
    """2^18 events (1024 blocks, the benchmark's launch shape): sampled."""
    mom = config_events(proc, 1 << 18)
    print(f"[two-jet full] {proc} nevt={mom.shape[0]}", flush=True)
    gpu = _run(proc, "fp64", mom, dev)
    assert np.isfinite(gpu).all() and (gpu > 0).all()
    idx = np.sort(np.random.default_rng(7).choice(mom.shape[0], size=128, replace=False))
    name = CONFIGS[proc][0]
    ref = oracle_lib.me(name, mom[idx])
    check_fp64(gpu[idx], ref, lambda i: oracle_lib.me(name, mom[idx][i], long_double=True), proc)


@pytest.mark.parametrize("proc", ["uuttgg", "ugttug", "ggttuux", "uuttuu", "uuttddx"])
def test_per_helicity_and_filter(oracle_lib, dev, proc):
    from paper_2312_02898_amd.engine import MatrixElement
    mom = config_events(proc, 48)
    me = MatrixElement(proc, "fp64")
    gh = me.helicities(torch.from_numpy(mom).to(dev))
    torch.cuda.synchronize()
    gh = gh.cpu().numpy()
    oh = oracle_lib.me_hel(CONFIGS[proc][0], mom)
    scale = oh.sum(axis=1, keepdims=True)
    assert (np.abs(gh - oh) / scale).max() <= 1e-12
    live = np.nonzero((oh / scale).max(axis=0) > 1e-20)[0]
    assert set(live.tolist()) <= set(me.good_helicities())
    me.close()


def test_ragged_and_deterministic(dev):
    mom = config_events("uuttgg", 700)
    full = _run("uuttgg", "fp64", mom, dev)
    assert np.array_equal(full, _run("uuttgg", "fp64", mom, dev))
    for n in (1, 63, 65, 257):
        assert np.array_equal(_run("uuttgg", "fp64", np.ascontiguousarray(mom[:n]), dev), full[:n])


ALPHAS = np.array([0.100, 0.118, 0.130])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_jet_channel_mix(oracle_lib, dev, precision):
    """p p > t t~ + 2 jets: g g > t t~ g g and the twelve quark channels in
    one batch, each event at its own alpha_s (|M|^2 ~ alpha_s^4)."""
    from paper_2312_02898_amd.engine import ChannelMix
    procs = ["ggttgg"] + TWO_JET
    n = 1500 + 11
    rng = np.random.default_rng(31)
    mom = config_events("ggttgg", n)
    ch = rng.integers(0, len(procs), size=n).astype(np.int32)
    al = ALPHAS[rng.integers(0, 3, size=n)]
    print(f"[two-jet mix] {precision} nevt={n}", flush=True)
    mix = ChannelMix(procs, precision)
    got = mix(torch.from_numpy(mom).to(dev), torch.from_numpy(ch).to(dev), torch.from_numpy(al).to(dev))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    mix.close()

    def oracle_of(idx_all, long_double=False):
        out = np.empty(idx_all.size)
        for c, p in enumerate(procs):
            for a in ALPHAS:
                sel = np.nonzero((ch[idx_all] == c) & (al[idx_all] == a))[0]
                if sel.size:
                    out[sel] = oracle_lib.me(CONFIGS[p][0], mom[idx_all[sel]],
                                             oracle_lib.default_params(alpha_s=float(a)), long_double=long_double)
        return out
    ref = oracle_of(np.arange(n))
    if precision == "fp64":
        check_fp64(got, ref, lambda idx: oracle_of(idx, long_double=True), "2-jet mix")
    else:
        rel = np.abs(got / ref - 1)
        print(f"  median {np.median(rel):.3e} max {rel.max():.3e}", flush=True)
        assert np.median(rel) <= 1e-5 and rel.max() <= 1e-3
