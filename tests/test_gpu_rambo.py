"""Device-side phase-space generation vs the oracle's RAMBO on the same
Philox4x32-10 stream, and the device pipeline RAMBO -> me_compute without a
host copy vs the oracle's |M|^2 of the same events."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [("eemumu", [0.0, 0.0], 500.0), ("ggtt", [173.0, 173.0], 1500.0),
         ("ggttg", [173.0, 173.0, 0.0], 1500.0), ("ggttgg", [173.0, 173.0, 0.0, 0.0], 1500.0),
         ("ggttggg", [173.0, 173.0, 0.0, 0.0, 0.0], 1500.0)]


@pytest.mark.parametrize("name,masses,sqs", CASES)
@pytest.mark.parametrize("n", [1, 255, 257, 100000])
def test_device_rambo_matches_oracle(oracle_lib, name, masses, sqs, n):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02898_amd import binding as B
    print(f"[rambo] {name} n={n}", flush=True)
    d = torch.empty((n, len(masses) + 2, 4), dtype=torch.float64, device="cuda")
    B.me_rambo(n, masses, sqs, 77, d.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    ref = oracle_lib.rambo(n, masses, sqs, 77)
    rel = np.abs(got - ref).max(axis=(1, 2)) / sqs
    # RAMBO boosts the massless system of mass M and energy Q0 to rest: the
    # rounding of both sides is amplified by about gamma^2, gamma = Q0 / M,
    # which is large when the random directions nearly coincide.  gamma
    # comes from the shared Philox uniforms.
    u = oracle_lib.uniforms(n, len(masses), 77)
    c = 2.0 * u[..., 0] - 1.0
    phi = 2.0 * np.pi * u[..., 1]
    q0 = -np.log((1.0 - u[..., 2]) * (1.0 - u[..., 3]))
    st = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    nh = np.stack([st * np.cos(phi), st * np.sin(phi), c], axis=-1)
    m2 = np.zeros(n)
    for i in range(len(masses)):
        for j in range(i + 1, len(masses)):
            m2 += q0[:, i] * q0[:, j] * ((nh[:, i] - nh[:, j]) ** 2).sum(axis=1)
    gamma = q0.sum(axis=1) / np.sqrt(m2)
    tol = np.maximum(1e-12, 64 * np.finfo(np.float64).eps * gamma ** 2)
    worst = int(np.argmax(rel / tol))
    print(f"[rambo] worst rel {rel[worst]:.2e} at gamma {gamma[worst]:.1f} (tol {tol[worst]:.2e})")
    assert np.median(rel) <= 1e-15
    assert (rel <= tol).all()
    bal = got[:, 0] + got[:, 1] - got[:, 2:].sum(axis=1)
    assert np.abs(bal).max() <= 1e-11 * sqs


def test_device_pipeline_no_host_copy(oracle_lib):
    """me_rambo -> me_compute on device for gg -> ttbar gg, checked against
    the oracle on the same (device-generated) events."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02898_amd import binding as B
    from paper_2312_02898_amd.engine import MatrixElement
    n = 2048 + 13
    d = torch.empty((n, 6, 4), dtype=torch.float64, device="cuda")
    B.me_rambo(n, [173.0, 173.0, 0.0, 0.0], 1500.0, 4, d.data_ptr(), torch.cuda.current_stream().cuda_stream)
    me = MatrixElement("ggttgg", precision="fp64")
    out = me(d)
    torch.cuda.synchronize()
    mom = d.cpu().numpy()
    ref = oracle_lib.me("g g > t t~ g g", mom)
    rel = np.abs(out.cpu().numpy() / ref - 1)
    assert np.median(rel) <= 1e-14 and (rel > 1e-12).sum() <= max(1, n // 1000)


def test_rambo_errors():
    from paper_2312_02898_amd import binding as B
    import ctypes
    m = (ctypes.c_double * 2)(100.0, 100.0)
    assert B.lib().me_rambo(10, 2, m, 150.0, 1, ctypes.c_void_p(16), None) == B.ME_EINVAL   # below threshold
    assert B.lib().me_rambo(10, 1, m, 500.0, 1, ctypes.c_void_p(16), None) == B.ME_EINVAL   # nfinal < 2
    assert B.lib().me_rambo(-1, 2, m, 500.0, 1, ctypes.c_void_p(16), None) == B.ME_EINVAL
    assert B.lib().me_rambo(0, 2, m, 500.0, 1, None, None) == B.ME_OK
