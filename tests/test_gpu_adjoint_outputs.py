"""GPU adjoint of the angle histogram and the moments (through the C ABI)
against the oracle's forward-mode derivatives, which are pinned to central
differences of the oracle's forward pass.

For L = w.H + u.T + v.M with seeded upstream weights, the oracle's Jacobians
give dL/dp = w J_H + u J_T + v J_M; errors are measured against the scale
s_m = |w| |J_H| + |u| |J_T| + |v| |J_M| of the summed terms, with the bars of
the energy-histogram adjoint (FP64 1e-9 s_m, FP32 1e-5 s_m).  The moment
weights are nonzero on every field, including the weight, the largest chi and
the FP64-shadow fields, whose derivatives are zero (the oracle has no shadow
fields; its Jacobian covers the first sixteen).
"""
import numpy as np
import pytest

from paper_2308_09348_amd import _lib, workloads

pytestmark = pytest.mark.gpu

NAMES = ["a0", "w0_um", "x_off_um", "y_off_um", "delay_fs", "gamma0", "sigma_gamma", "div_mrad"]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    ctx = qs.Context(0)
    yield ctx
    ctx.close()


CASES = {
    "quantum-local-gauss": dict(rr_model="quantum", amp_mode="local", deposit="gauss"),
    "quantum-a0eff-cic": dict(rr_model="quantum", amp_mode="a0eff", deposit="cic"),
    "classical-local-gauss": dict(rr_model="classical", amp_mode="local", deposit="gauss"),
}


def _case(name, n_samples=400, n_steps=256, **kw):
    p = workloads.scaled(workloads.differentiation(), n_samples=n_samples, n_steps=n_steps)
    p.update(CASES[name])
    p.update(kw)
    return p


def _weights(p, seed, energy=True, angle=True, moments=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.normal(size=p["n_e"] + 2) if energy else None
    u = rng.normal(size=p["n_th"] + 2) if angle else None
    # one weight per moment, the FP64-shadow fields included (their derivative
    # is zero on the device; the oracle has no shadow fields)
    v = rng.normal(size=_lib.M_N) / np.array([1, 1e3, 1e2] + [1] * (_lib.M_N - 3)) \
        if moments else None
    return w, u, v


def _oracle(oracle, p, w, u, v):
    g = np.zeros(8)
    s = np.zeros(8)
    if w is not None:
        _, je = oracle.grad(p)
        g += w @ je
        s += np.abs(w) @ np.abs(je)
    if u is not None or v is not None:
        _, jt, _, jm = oracle.grad_outputs(p)
        if u is not None:
            g += u @ jt
            s += np.abs(u) @ np.abs(jt)
        if v is not None:
            g += v[:jm.shape[0]] @ jm
            s += np.abs(v[:jm.shape[0]]) @ np.abs(jm)
    return g, s


def _gpu(ctx, p, w, u, v, tape=False):
    import torch
    t = lambda x: None if x is None else torch.tensor(x, dtype=torch.float64, device="cuda")
    kw = {}
    if tape:
        kw["tape"] = ctx.new_tape(p["n_samples"])
        out = ctx.forward(p, tape=kw["tape"])
    else:
        out = ctx.forward(p)
    g = ctx.backward(p, t(w), d_angle=t(u), d_moments=t(v), moments=out["moments"], **kw)
    return g.cpu().numpy()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
@pytest.mark.parametrize("name", list(CASES))
def test_angle_and_moment_adjoint_matches_oracle(gpu, oracle, name, precision, tol):
    p = _case(name, precision=precision)
    w, u, v = _weights(p, 5)
    og, scale = _oracle(oracle, p, w, u, v)
    for tape in (False, True):
        go = _gpu(gpu, p, w, u, v, tape=tape)
        err = np.abs(go - og) / np.maximum(scale, 1e-300)
        print(name, precision, "tape" if tape else "recompute", err.max())
        assert np.all(np.abs(go - og) <= tol * scale + 1e-300), (tape, dict(zip(NAMES, err)))


@pytest.mark.parametrize("which", ["angle", "moments"])
def test_single_upstream_kinds(gpu, oracle, which):
    p = _case("quantum-local-gauss", precision="fp64", n_samples=300)
    w, u, v = _weights(p, 9, energy=False, angle=which == "angle", moments=which == "moments")
    og, scale = _oracle(oracle, p, w, u, v)
    go = _gpu(gpu, p, w, u, v)
    assert np.all(scale[[0, 7]] > 0)
    assert np.all(np.abs(go - og) <= 1e-9 * scale + 1e-300), (go, og)


def test_autograd_spectra_matches_backward(gpu):
    import torch
    import paper_2308_09348_amd as qs
    p = _case("quantum-local-gauss", precision="fp64", n_samples=500)
    w, u, v = _weights(p, 3)
    theta = torch.tensor([p[k] for k in NAMES], dtype=torch.float64, requires_grad=True)
    H, T, M = qs.spectra(theta, p, context=gpu)
    W, U, V = (torch.tensor(x, dtype=torch.float64, device="cuda") for x in (w, u, v))
    loss = (H * W).sum() + (T * U).sum() + (M * V).sum()
    loss.backward()
    ref = _gpu(gpu, p, w, u, v, tape=True)
    assert np.allclose(theta.grad.numpy(), ref, rtol=1e-13, atol=0)


def test_batched_equals_single(gpu):
    import torch
    base = _case("quantum-local-gauss", precision="fp32", n_samples=700)
    shots = [dict(base, n_samples=n, a0=a, shot=0) for n, a in ((700, 20.0), (1, 35.0),
                                                                (300, 50.0))]
    ups = [_weights(s, 20 + k) for k, s in enumerate(shots)]
    t = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    outs = gpu.forward_batched(shots)
    grads = gpu.backward_batched(shots, [t(w) for w, _, _ in ups], d_angle=[t(u) for _, u, _ in ups],
                                 d_moments=[t(v) for _, _, v in ups],
                                 moments=[o["moments"] for o in outs])
    for k, s in enumerate(shots):
        q = dict(s, shot=k)
        m = gpu.forward(q)["moments"]
        w, u, v = ups[k]
        single = gpu.backward(q, t(w), d_angle=t(u), d_moments=t(v), moments=m)
        assert np.array_equal(grads[k].cpu().numpy(), single.cpu().numpy()), k


def test_backward_argument_checks(gpu):
    import torch
    import paper_2308_09348_amd as qs
    p = _case("quantum-local-gauss", n_samples=64, n_steps=32)
    with pytest.raises(ValueError):
        gpu.backward(p)  # no upstream weights
    with pytest.raises(ValueError):
        gpu.backward(p, d_moments=torch.zeros(_lib.M_N, dtype=torch.float64, device="cuda"))
    assert qs.QScatterError is not None
