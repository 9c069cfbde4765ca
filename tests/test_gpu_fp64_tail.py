"""FP64 on the ill-conditioned tail of the benchmark samples.

Flat phase space without cuts puts some events close to collinear limits:
a final gluon nearly parallel to a beam or to another final gluon, or the
outgoing light quark of a q g channel nearly parallel to its beam.  There a
propagator invariant is 1e-5..1e-7 of the beam energy squared and diagrams
cancel strongly, and an FP64 evaluation that forms such an invariant as
E^2 - |p|^2 loses up to 1e-9.  These tests run large prefixes of the
benchmark samples, flag every event on which the GPU and the FP64 oracle
differ by more than 1e-13, and require the GPU to be within 1e-12 of the
long-double oracle on each flagged event (fp64_bar.py).
"""
import numpy as np
import pytest

from paper_2312_02898_amd.inputs import CONFIGS, config_events

from fp64_bar import check_fp64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# process -> prefix of its benchmark sample
TAIL = {"ggttgg": 65536, "ggttg": 65536, "ugttu": 8192, "guttu": 8192, "uxgttux": 8192, "guxttux": 8192,
        "uuttg": 8192, "uxuttg": 8192}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("proc", list(TAIL))
def test_fp64_tail_against_long_double(oracle_lib, dev, proc):
    from paper_2312_02898_amd.engine import MatrixElement
    mom = config_events(proc, TAIL[proc])
    name = CONFIGS[proc][0]
    print(f"[fp64 tail] {proc} nevt={mom.shape[0]}", flush=True)
    me = MatrixElement(proc, "fp64")
    gpu = me(torch.from_numpy(mom).to(dev))
    torch.cuda.synchronize()
    gpu = gpu.cpu().numpy()
    me.close()
    ref = oracle_lib.me(name, mom)
    check_fp64(gpu, ref, lambda idx: oracle_lib.me(name, mom[idx], long_double=True), proc)
