"""The derivative tape: a forward pass that records, per sample, mu_f, sig2_f
and their derivatives along the eight parameters, and the adjoint read from
it.

  - the adjoint from the tape is bit-for-bit the adjoint that integrates the
    trajectories again (same per-sample arithmetic, same reduction order);
  - the tape's per-sample derivatives match the oracle's forward-mode
    derivatives of the same sample (FP64: 1e-8 relative; FP32: 1e-4, with a
    floor of 1e-9 (FP64) / 1e-6 (FP32) of mu_f per unit of the parameter's
    scale for derivatives that are nearly zero);
  - the tape forward's histograms and moments pass the forward parity bar
    against the oracle (they are not bit-identical to qs_forward's: the FP32
    step arithmetic differs);
  - a batched tape holds each shot's single-call tape at the shot's offset.
"""
import numpy as np
import pytest

from paper_2308_09348_amd import workloads

pytestmark = pytest.mark.gpu

NAMES = ["a0", "w0_um", "x_off_um", "y_off_um", "delay_fs", "gamma0", "sigma_gamma", "div_mrad"]
SCALE = {"a0": 1.0, "w0_um": 3.0, "x_off_um": 3.0, "y_off_um": 3.0, "delay_fs": 30.0,
         "gamma0": 1.0, "sigma_gamma": 1.0, "div_mrad": 1.0}


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    ctx = qs.Context(0)
    yield ctx
    ctx.close()


def _case(n_samples=600, n_steps=256, **kw):
    p = workloads.scaled(workloads.differentiation(), n_samples=n_samples, n_steps=n_steps)
    p.update(kw)
    return p


def _weights(n, seed=5):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.tensor(rng.normal(size=n + 2), dtype=torch.float64, device="cuda")


CONFIGS = [dict(rr_model="quantum", amp_mode="local", deposit="gauss"),
           dict(rr_model="quantum", amp_mode="a0eff", deposit="cic"),
           dict(rr_model="classical", amp_mode="local", deposit="gauss")]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_tape_adjoint_equals_recompute(gpu, precision, cfg):
    p = _case(precision=precision, **CONFIGS[cfg])
    tape = gpu.new_tape(p["n_samples"])
    gpu.forward(p, tape=tape)
    w = _weights(p["n_e"])
    a = gpu.backward(p, w, tape=tape).cpu().numpy()
    b = gpu.backward(p, w).cpu().numpy()
    assert np.array_equal(a, b), (a, b)


def _check_sample_derivs(oracle, p, tape, idx, rtol, floor):
    t = tape.cpu().numpy()
    worst = 0.0
    for i in idx:
        m, s2 = oracle.sample_grad(p, int(i))
        assert abs(t[0, i] - m[0]) <= rtol * abs(m[0]), (i, t[0, i], m[0])
        assert abs(t[1, i] - s2[0]) <= rtol * abs(s2[0]) + floor * m[0] ** 2, (i, t[1, i], s2[0])
        for k, name in enumerate(NAMES):
            fl = floor * abs(m[0]) / SCALE[name]
            dm = abs(t[2 + k, i] - m[1 + k])
            ds = abs(t[10 + k, i] - s2[1 + k])
            worst = max(worst, dm / (abs(m[1 + k]) + fl), ds / (abs(s2[1 + k]) + fl * abs(m[0])))
            assert dm <= rtol * abs(m[1 + k]) + fl, (i, name, t[2 + k, i], m[1 + k])
            assert ds <= rtol * abs(s2[1 + k]) + fl * abs(m[0]), (i, name, t[10 + k, i], s2[1 + k])
    return worst


@pytest.mark.parametrize("precision,rtol,floor", [("fp64", 1e-8, 1e-9), ("fp32", 1e-4, 1e-6)])
@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_tape_matches_oracle_sample_derivatives(gpu, oracle, precision, rtol, floor, cfg):
    p = _case(n_samples=300, precision=precision, **CONFIGS[cfg])
    tape = gpu.new_tape(p["n_samples"])
    gpu.forward(p, tape=tape)
    worst = _check_sample_derivs(oracle, p, tape, range(0, 300, 23), rtol, floor)
    print(precision, CONFIGS[cfg], "worst relative", worst)


def test_tape_forward_parity_with_oracle(gpu, oracle):
    p = _case(n_samples=3000, n_steps=512, deposit="cic")
    g = gpu.forward(p, tape=gpu.new_tape(p["n_samples"]))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = oracle.forward(p)
    assert g["moments"][0] == p["n_samples"]
    for m in (1, 2, 4, 6, 7, 9, 10):
        assert abs(g["moments"][m] - o["moments"][m]) <= 1e-5 * abs(o["moments"][m]), m
    assert abs(g["moments"][8] - o["moments"][8]) <= 1e-5 * o["moments"][8]
    for key in ("energy_hist", "angle_hist"):
        tol = 1e-4 * o[key] + 1e-7 * o[key].sum()
        assert np.all(np.abs(g[key] - o[key]) <= tol), key
    assert np.array_equal(g["a0eff_hist"], o["a0eff_hist"])


def test_full_size_sampled(gpu, oracle):
    """The differentiation workload at its full size (2^20 samples x 1024
    steps, FP32, the launch the benchmark times): sampled tape entries
    against the oracle's per-sample derivatives, and the gradient's
    consistency between tape and recompute."""
    p = workloads.differentiation()
    n = p["n_samples"]
    tape = gpu.new_tape(n)
    out = gpu.forward(p, tape=tape)
    assert out["energy_hist"].sum().item() == n
    idx = np.linspace(0, n - 1, 12).astype(np.int64)
    worst = _check_sample_derivs(oracle, p, tape, idx, 1e-4, 1e-6)
    print("full size worst relative", worst)
    w = _weights(p["n_e"])
    a = gpu.backward(p, w, tape=tape).cpu().numpy()
    b = gpu.backward(p, w).cpu().numpy()
    assert np.array_equal(a, b)


def test_batched_tape_equals_single(gpu):
    import torch
    base = _case(n_samples=300)
    shots = [dict(base, n_samples=n, a0=a0, gamma0=g0, sigma_gamma=0.05 * g0, e_hi=1.5 * g0)
             for n, a0, g0 in [(1, 20.0, 2000.0), (700, 50.0, 1500.0), (2500, 80.0, 3000.0)]]
    total = sum(s["n_samples"] for s in shots)
    tape = gpu.new_tape(total)
    outs = gpu.forward_batched(shots, tape=tape)
    ws = [_weights(s["n_e"], seed=k) for k, s in enumerate(shots)]
    grads = gpu.backward_batched(shots, ws, tape=tape)
    off = 0
    for k, s in enumerate(shots):
        q = dict(s, shot=s["shot"] + k)
        t1 = gpu.new_tape(s["n_samples"])
        o1 = gpu.forward(q, tape=t1)
        assert torch.equal(tape[:, off:off + s["n_samples"]], t1), k
        for key in ("energy_hist", "angle_hist", "a0eff_hist", "moments"):
            assert torch.equal(outs[k][key], o1[key]), (k, key)
        assert torch.equal(grads[k], gpu.backward(q, ws[k], tape=t1)), k
        off += s["n_samples"]


def test_tape_rejects_bad_tensor(gpu):
    import torch
    p = _case(n_samples=100)
    with pytest.raises(ValueError):
        gpu.forward(p, tape=torch.empty((18, 99), dtype=torch.float64, device="cuda"))
