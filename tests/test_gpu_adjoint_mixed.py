"""Derivatives in mixed precision: FP32 with FP64 steps wherever some lane of
a wavefront has chi above the threshold at a step start (the forward pass's
rule), for the quantum model.  In those steps the state, the amplitudes and
the step's linearisation are FP64; the tangents stay FP32.

  - at quantum-batch physics (gamma0 = 2e4, a0 = 120, W0 = 2 um: chi up to
    several, so FP64 segments start and end inside the pulse) the adjoint,
    recomputed or from the tape, matches the oracle's gradient to the FP32
    bar (1e-5 of the scale s_m of the summed terms), and the tape's sampled
    entries match the oracle's per-sample derivatives (FP32 bars);
  - a threshold below every chi runs every step in FP64: the tape's mu_f and
    sig2_f are then the FP64 tape's up to the FP32 pair that holds the state
    on return (1e-13 relative), the derivatives within the FP32 tangents'
    precision;
  - the tape forward's histograms and moments pass the forward parity bar
    against the oracle;
  - a batch of shots gives each shot's single-call tape and gradient, bit for
    bit.
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


def _case(n_samples=300, n_steps=512, amp_mode="local", **kw):
    shot = workloads.quantum_batch(n_shots=4)[1]
    p = dict(shot, a0=120.0, n_samples=n_samples, n_steps=n_steps, amp_mode=amp_mode)
    p.update(kw)
    return p


def _weights(n, seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=n + 2)


def _t(x):
    import torch
    return torch.tensor(x, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("amp", ["local", "a0eff"])
def test_mixed_adjoint_matches_oracle(gpu, oracle, amp):
    p = _case(amp_mode=amp)
    w = _weights(p["n_e"])
    _, jac = oracle.grad(p)
    og, scale = w @ jac, np.abs(w) @ np.abs(jac)
    out = gpu.forward(p)
    assert out["moments"][8].item() > 1.0  # FP64 steps were taken
    tape = gpu.new_tape(p["n_samples"])
    gpu.forward(p, tape=tape)
    a = gpu.backward(p, _t(w)).cpu().numpy()
    b = gpu.backward(p, _t(w), tape=tape).cpu().numpy()
    assert np.array_equal(a, b)
    err = np.abs(a - og) / np.maximum(scale, 1e-300)
    print(amp, "mixed max err / scale", err.max(), dict(zip(NAMES, err)))
    assert np.all(np.abs(a - og) <= 1e-5 * scale + 1e-300), dict(zip(NAMES, err))


def test_mixed_tape_matches_oracle_sample_derivatives(gpu, oracle):
    p = _case()
    tape = gpu.new_tape(p["n_samples"])
    gpu.forward(p, tape=tape)
    t = tape.cpu().numpy()
    rtol, floor = 1e-4, 1e-6
    for i in range(0, p["n_samples"], 29):
        m, s2 = oracle.sample_grad(p, i)
        assert abs(t[0, i] - m[0]) <= 3e-6 * abs(m[0]), (i, t[0, i], m[0])
        assert abs(t[1, i] - s2[0]) <= 3e-5 * abs(s2[0]) + floor * m[0] ** 2, (i, t[1, i], s2[0])
        for k, name in enumerate(NAMES):
            fl = floor * abs(m[0]) / SCALE[name]
            assert abs(t[2 + k, i] - m[1 + k]) <= rtol * abs(m[1 + k]) + fl, (i, name)
            assert abs(t[10 + k, i] - s2[1 + k]) <= rtol * abs(s2[1 + k]) + fl * abs(m[0]), \
                (i, name)


@pytest.mark.parametrize("amp", ["local", "a0eff"])
def test_mixed_promotion_everywhere_is_the_fp64_trajectory(gpu, amp):
    p = _case(n_samples=1500, n_steps=384, amp_mode=amp)
    n = p["n_samples"]
    tm = gpu.new_tape(n)
    gpu.forward(dict(p, chi_fp64=1e-30), tape=tm)
    td = gpu.new_tape(n)
    gpu.forward(dict(p, precision="fp64"), tape=td)
    m, d = tm.cpu().numpy(), td.cpu().numpy()
    assert np.allclose(m[0], d[0], rtol=1e-13, atol=0)
    assert np.allclose(m[1], d[1], rtol=1e-12, atol=1e-12 * d[1].max())
    # FP32 tangents: the bars of the tape's per-sample check (floor 1e-6 of
    # mu_f per unit of the parameter's scale, times mu_f for the variance)
    mu = np.abs(d[0])
    for k, name in enumerate(NAMES):
        fl = 1e-6 * mu / SCALE[name]
        assert np.all(np.abs(m[2 + k] - d[2 + k]) <= 1e-4 * np.abs(d[2 + k]) + fl), name
        assert np.all(np.abs(m[10 + k] - d[10 + k]) <= 1e-4 * np.abs(d[10 + k]) + fl * mu), name


def test_mixed_tape_forward_parity_with_oracle(gpu, oracle):
    p = _case(n_samples=2000, deposit="cic")
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


def test_mixed_batch_equals_single_shots(gpu):
    import torch
    shots = workloads.quantum_batch(n_shots=3)
    shots = [dict(s, n_samples=n, n_steps=256, shot=0) for s, n in zip(shots, (900, 1, 333))]
    total = sum(s["n_samples"] for s in shots)
    tape = gpu.new_tape(total)
    gpu.forward_batched(shots, tape=tape)
    ws = [_t(_weights(s["n_e"], seed=k)) for k, s in enumerate(shots)]
    grads = gpu.backward_batched(shots, ws, tape=tape)
    again = gpu.backward_batched(shots, ws)
    off = 0
    for k, s in enumerate(shots):
        q = dict(s, shot=k)
        t1 = gpu.new_tape(s["n_samples"])
        gpu.forward(q, tape=t1)
        assert torch.equal(tape[:, off:off + s["n_samples"]], t1), k
        assert torch.equal(grads[k], gpu.backward(q, ws[k], tape=t1)), k
        assert torch.equal(again[k], grads[k]), k
        off += s["n_samples"]
