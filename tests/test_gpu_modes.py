"""Hermite- and Laguerre-Gauss laser modes on the GPU path against the
oracle (the same tolerances as the Gaussian-focus parity tests): forward
passes with the amplitude at the collision point and along the path, the
photon spectrum, the plane-wave reconstruction; the derivative entry points
refuse higher modes.
"""
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


def _check_bins(gh, oh, rel=1e-4, floor=1e-7):
    tol = rel * np.abs(oh) + floor * oh.sum()
    bad = np.abs(gh - oh) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:10], gh[bad][:5], oh[bad][:5])


MODES = [("hg", 1, 2), ("hg", 3, 0), ("lg", 1, 1), ("lg", 0, -3)]


def _case(kind, m, n, **kw):
    p = workloads.scaled(workloads.focused_3d(), n_samples=3037, n_steps=256, mode=kind,
                         mode_m=m, mode_n=n)
    p.update(kw)
    return p


@pytest.mark.parametrize("kind,m,n", MODES)
@pytest.mark.parametrize("amp,precision", [("local", "fp32"), ("local", "fp64"),
                                           ("a0eff", "fp32")])
def test_mode_forward_parity(gpu, oracle, kind, m, n, amp, precision):
    p = _case(kind, m, n, amp_mode=amp, precision=precision, deposit="cic")
    nsamp = p["n_samples"]
    print("case", kind, m, n, amp, precision, flush=True)
    g = _np(gpu.forward(p, sample_stride=7, n_sample_records=nsamp // 7 + 1))
    o = oracle.forward(p)
    ref = oracle.samples(p, range(0, nsamp, 7))
    tol = 2e-9 if precision == "fp64" else 3e-6
    assert np.allclose(g["samples"][:, 5], ref[:, oracle.S_AEFF], rtol=1e-12, atol=1e-12)
    assert np.allclose(g["samples"][:, 0], ref[:, oracle.S_MU], rtol=tol, atol=0)
    for key in ("energy_hist", "angle_hist"):
        _check_bins(g[key], o[key])
    for k in (1, 2, 4, 7, 9, 10):
        assert abs(g["moments"][k] - o["moments"][k]) <= 1e-5 * abs(o["moments"][k]), k


def test_mode_photon_parity(gpu, oracle):
    p = _case("lg", 1, 1, n_samples=200, precision="fp64", n_ph=64, ph_lo=0.0, ph_hi=2400.0)
    g = _np(gpu.photons(p, angles=True))
    oh, oe = oracle.photons(p, p["n_ph"], p["ph_lo"], p["ph_hi"])
    assert np.all(np.abs(g["energy"] - oe) <= 1e-10 * np.abs(oe))
    # the spectrum bar, per bin
    assert np.all(np.abs(g["photon_hist"] - oh) <= 1e-4 * np.abs(oh) + 1e-7 * oh.sum())
    oa = oracle.photon_angles(p)
    assert np.all(np.abs(g["angles"] - oa) <= 2e-6 * np.abs(oa))


def test_mode_reconstruction_parity(gpu, oracle):
    p = _case("hg", 1, 2, amp_mode="a0eff", deposit="gauss", precision="fp64")
    nsamp = p["n_samples"]
    g = _np(gpu.forward_factorised(p, 21, 17, nodes=True, sample_stride=1,
                                   n_sample_records=nsamp))
    o = oracle.factorised(p, 21, 17)
    orec = oracle.factorised_samples(p, 21, 17, range(nsamp))
    assert np.allclose(g["samples"][:, 0], orec[:, oracle.S_MU], rtol=2e-9, atol=0)
    assert np.all(np.abs(g["node_weights"] - o["node_weights"]) <= 1e-9 * nsamp)
    _check_bins(g["energy_hist"], o["energy_hist"])


def test_derivatives_refuse_higher_modes(gpu):
    import torch
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib
    p = _case("hg", 1, 0, n_samples=100)
    w = torch.zeros(p["n_e"] + 2, dtype=torch.float64, device="cuda")
    with pytest.raises(qs.QScatterError) as e:
        gpu.backward(p, w)
    assert e.value.status == _lib.QS_EUNSUPPORTED
    with pytest.raises(qs.QScatterError) as e:
        gpu.forward(p, tape=gpu.new_tape(p["n_samples"]))
    assert e.value.status == _lib.QS_EUNSUPPORTED
    # the Gaussian mode still differentiates
    gpu.backward(dict(p, mode="gauss"), w)


def test_invalid_mode_indices(gpu):
    import paper_2308_09348_amd as qs
    for kw in (dict(mode="hg", mode_m=9), dict(mode="hg", mode_n=-1), dict(mode="lg", mode_n=9),
               dict(mode="lg", mode_m=-1)):
        with pytest.raises(qs.QScatterError):
            gpu.forward(_case("gauss", 0, 0, n_samples=10, **kw))
