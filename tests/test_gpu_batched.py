"""Batched launches: one launch over many shots.

A shot in a batch must give bit-for-bit what a single call with the same RNG
counter word gives, and agree with the oracle to the single-shot tolerances."""
import numpy as np
import pytest

from paper_2308_09348_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    ctx = qs.Context(0)
    yield ctx
    ctx.close()


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _mixed_shots():
    base = workloads.scaled(workloads.focused_3d(), n_steps=256)
    shots = []
    for k, (n, a0, w0, xo, dl, g0) in enumerate([(1, 20.0, 3.0, 0.0, 0.0, 2000.0),
                                                  (300, 50.0, 2.0, 1.0, -5.0, 1500.0),
                                                  (5037, 80.0, 4.0, -2.0, 12.0, 3000.0),
                                                  (4096, 5.0, 6.0, 0.5, 0.0, 1000.0),
                                                  (8193, 35.0, 0.0, 0.0, 3.0, 2500.0)]):
        shots.append(dict(base, n_samples=n, a0=a0, w0_um=w0, x_off_um=xo, delay_fs=dl,
                          gamma0=g0, sigma_gamma=0.05 * g0, e_hi=1.5 * g0, shot=base["shot"]))
    return shots


@pytest.mark.parametrize("precision,chi64", [("fp32", 0.0), ("fp32", 0.1), ("fp64", 0.0)])
def test_batch_equals_single_shots(gpu, precision, chi64):
    shots = [dict(p, precision=precision, chi_fp64=chi64) for p in _mixed_shots()]
    batch = [_np(o) for o in gpu.forward_batched(shots)]
    for k, p in enumerate(shots):
        single = _np(gpu.forward(dict(p, shot=p["shot"] + k)))
        for key in ("energy_hist", "angle_hist", "a0eff_hist", "moments", "status"):
            assert np.array_equal(batch[k][key], single[key]), (k, key)


def test_batch_parity_with_oracle(gpu, oracle):
    shots = workloads.batched_shots(n_shots=6)
    shots = [dict(p, n_samples=min(p["n_samples"], 3000), n_steps=256) for p in shots]
    out = [_np(o) for o in gpu.forward_batched(shots)]
    base = shots[0]["shot"]
    for k, p in enumerate(shots):
        o = oracle.forward(dict(p, shot=base + k))
        g = out[k]
        assert g["moments"][0] == p["n_samples"]
        for m in (1, 2, 4, 7, 9, 10):
            assert abs(g["moments"][m] - o["moments"][m]) <= 1e-5 * abs(o["moments"][m]), (k, m)
        tol = 1e-4 * o["energy_hist"] + 1e-7 * o["energy_hist"].sum()
        assert np.all(np.abs(g["energy_hist"] - o["energy_hist"]) <= tol), k
        assert g["energy_hist"].sum() == p["n_samples"]


def test_batch_rejects_mixed_wavelength(gpu):
    from paper_2308_09348_amd import QScatterError
    shots = _mixed_shots()[:2]
    shots[1] = dict(shots[1], lambda_um=1.0)
    with pytest.raises(QScatterError) as ei:
        gpu.forward_batched(shots)
    assert ei.value.status == 5


def test_batch_repeat_is_deterministic(gpu):
    shots = workloads.batched_shots(n_shots=64)
    shots = [dict(p, n_samples=min(p["n_samples"], 20000)) for p in shots]
    a = [_np(o) for o in gpu.forward_batched(shots)]
    b = [_np(o) for o in gpu.forward_batched(shots)]
    for x, y in zip(a, b):
        for key in x:
            assert np.array_equal(x[key], y[key])
