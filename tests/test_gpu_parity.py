"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded samples.

Tolerances (from the FP32 arithmetic of the phase loop):
  moments:  relative 1e-5 (absolute 1e-5 of the spread for means near zero)
  bins:     |G_k - O_k| <= 1e-4 O_k + 1e-7 sum(O) for smooth deposits;
  NGP bins: |G_k - O_k| <= the number of samples whose oracle value lies within
            a relative 1e-5 (FP32) or 1e-12 (FP64) of an edge of bin k, since a
            floating-point comparison decides the bin.
"""
import math

import numpy as np
import pytest

from paper_2308_09348_amd import workloads

pytestmark = pytest.mark.gpu

MOMENT_KEYS = [1, 2, 3, 4, 5, 6, 7, 9, 10]  # mean/std g, theta x/y, a_eff, rad frac, sigma_f


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    ctx = qs.Context(0)
    yield ctx
    ctx.close()


def test_loaded_library_matches_the_sources(gpu):
    from paper_2308_09348_amd import _lib
    assert len(_lib.check_build()) == 64


def _run(ctx, params, **kw):
    out = ctx.forward(params, **kw)
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check_moments(g, o, params, rtol=1e-5):
    gm, om = g["moments"], o["moments"]
    assert gm[0] == om[0] == params["n_samples"]
    for k in MOMENT_KEYS:
        scale = abs(om[k])
        if k in (3, 5):  # mean angles: near zero, compare against the rms
            scale = max(scale, om[k + 1])
        assert abs(gm[k] - om[k]) <= rtol * scale + 1e-300, (k, gm[k], om[k])
    # max chi: FP32 chi at the step starts
    assert abs(gm[8] - om[8]) <= 1e-5 * om[8] + 1e-30


def _check_bins(gh, oh, rel=1e-4, floor=1e-7):
    tol = rel * np.abs(oh) + floor * oh.sum()
    bad = np.abs(gh - oh) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:10], gh[bad][:5], oh[bad][:5])


def _edge_allowance(values, lo, hi, n, rel):
    """Per-bin count of samples whose value is within rel*|v| of a bin edge
    (such a sample may land on either side in the other precision)."""
    w = (hi - lo) / n
    allow = np.zeros(n + 2)
    for v in values:
        x = (v - lo) / w
        k = int(round(x))
        if abs(lo + k * w - v) <= rel * max(abs(v), w):
            # edge k separates bin k-1 (or underflow) and bin k (or overflow)
            below = n if k <= 0 else min(k - 1, n + 1)
            above = n + 1 if k >= n else max(k, 0)
            if k < 0:
                below = above = n
            allow[below] += 1
            allow[above] += 1
    return allow


def _check_ngp(gh, oh, values, lo, hi, n, rel):
    allow = _edge_allowance(values, lo, hi, n, rel)
    diff = np.abs(gh - oh)
    assert np.all(diff <= allow + 1e-9), (np.nonzero(diff > allow + 1e-9)[0][:10])
    assert abs(gh.sum() - oh.sum()) < 1e-6


# ---- radiation tables ------------------------------------------------------

def test_radiation_tables_against_definition(gpu, oracle):
    import torch
    rng = np.random.default_rng(3)
    chi = np.concatenate([np.exp(rng.uniform(np.log(1e-8), np.log(200.0), 3000)),
                          [0.0, 1e-7, 2.0 ** -20, 0.1, 1.0, 2.0, 100.0]])
    ref = np.stack([oracle.radiation(c) if c > 0 else np.array([1.0, 0, 0, 1.0]) for c in chi])
    for prec, tol in (("fp32", (1e-6, 2e-6, 2e-6, 3e-6)), ("fp64", (1e-9, 1e-9, 1e-9, 1e-8))):
        got = gpu.radiation_eval(torch.tensor(chi), prec).cpu().numpy()
        for f in range(4):
            # chi g' and chi^2 g'' enter the drift next to 2 g: scale them by g
            scale = np.abs(ref[:, f]) if f in (0, 3) else np.maximum(np.abs(ref[:, f]),
                                                                     np.abs(ref[:, 0]))
            err = np.abs(got[:, f] - ref[:, f]) / scale
            assert err.max() <= tol[f], (prec, f, chi[np.argmax(err)], err.max())


# ---- the plane-wave 1D configuration ----------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plane_wave_1d_full(gpu, oracle, precision):
    p = dict(workloads.plane_wave_1d(), precision=precision)
    g = _run(gpu, p, sample_stride=1, n_sample_records=p["n_samples"])
    o = oracle.forward(p)
    _check_moments(g, o, p, rtol=1e-12 if precision == "fp64" else 1e-5)
    ov = oracle.samples(p, range(p["n_samples"]))[:, oracle.S_MU]
    rel = 1e-12 if precision == "fp64" else 1e-5
    _check_ngp(g["energy_hist"], o["energy_hist"], ov, p["e_lo"], p["e_hi"], p["n_e"], rel)
    gv = g["samples"][:, 0]
    assert np.max(np.abs(gv - ov) / ov) <= (1e-13 if precision == "fp64" else 2e-6)


# ---- the focused configuration at parity-test sizes --------------------------

FOCUSED_CASES = [
    # (rr, amp, deposit, precision, chi_fp64)
    ("quantum", "local", "cic", "fp32", 0.0),
    ("quantum", "local", "cic", "fp32", 0.1),
    ("quantum", "local", "cic", "fp64", 0.0),
    ("quantum", "a0eff", "gauss", "fp32", 0.0),
    ("quantum", "local", "point", "fp32", 0.0),
    ("classical", "local", "gauss", "fp32", 0.0),
    ("classical", "a0eff", "cic", "fp64", 0.0),
]


@pytest.mark.parametrize("rr,amp,dep,prec,chi64", FOCUSED_CASES)
def test_focused_parity(gpu, oracle, rr, amp, dep, prec, chi64):
    # 5000 + 37 samples: several phase blocks and a ragged tail
    p = workloads.scaled(workloads.focused_3d(), n_samples=5037, n_steps=512, rr_model=rr,
                         amp_mode=amp, deposit=dep, precision=prec, chi_fp64=chi64)
    g = _run(gpu, p, sample_stride=97, n_sample_records=52)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    smooth = rr == "quantum" or dep != "point"
    if smooth:
        _check_bins(g["energy_hist"], o["energy_hist"])
    if rr == "quantum" or dep != "point":
        _check_bins(g["angle_hist"], o["angle_hist"])
    # a0,eff histogram: NGP on the FP64 spatial factor on both sides
    idx = range(p["n_samples"])
    S0 = oracle.samples(p, idx)[:, oracle.S_AEFF] / p["a0"]
    allow = np.zeros(p["n_a"])
    for s in S0:
        x = s * p["n_a"]
        k = int(round(x))
        if abs(x - k) < 1e-9 and 0 < k < p["n_a"]:
            allow[k - 1] += 1
            allow[k] += 1
    assert np.all(np.abs(g["a0eff_hist"] - o["a0eff_hist"]) <= allow)
    # per-sample records
    recs = g["samples"]
    ref = oracle.samples(p, range(0, p["n_samples"], 97))
    # FP64: the two sides interpolate independent radiation tables (~1e-10)
    tol = 2e-9 if prec == "fp64" else 3e-6
    assert np.allclose(recs[:, 0], ref[:, oracle.S_MU], rtol=tol, atol=0)
    s2tol = 2e-8 if prec == "fp64" else 3e-5
    assert np.allclose(recs[:, 1], ref[:, oracle.S_SIG2], rtol=s2tol,
                       atol=s2tol * max(ref[:, oracle.S_SIG2].max(), 1.0))
    assert np.allclose(recs[:, 5], ref[:, oracle.S_AEFF], rtol=1e-13, atol=0)
    assert np.allclose(recs[:, 7], ref[:, oracle.S_GAMMA0], rtol=1e-15, atol=0)


@pytest.mark.parametrize("amp", ["local", "a0eff"])
def test_promotion_everywhere_is_the_fp64_pass(gpu, amp):
    """A threshold below every chi promotes every step of every wavefront: the
    mixed-precision pass then integrates in FP64 from start to end (one FP64
    segment) and differs from the FP64 pass only by the FP32 pair that holds
    the state on return (2^-48 relative)."""
    p = workloads.scaled(workloads.focused_3d(), n_samples=3037, n_steps=384,
                         amp_mode=amp, deposit="gauss")
    n = p["n_samples"]
    g = _run(gpu, dict(p, precision="fp32", chi_fp64=1e-30), sample_stride=1,
             n_sample_records=n)
    d = _run(gpu, dict(p, precision="fp64"), sample_stride=1, n_sample_records=n)
    assert np.allclose(g["samples"][:, 0], d["samples"][:, 0], rtol=1e-13, atol=0)
    assert np.allclose(g["samples"][:, 1], d["samples"][:, 1], rtol=1e-12,
                       atol=1e-12 * d["samples"][:, 1].max())
    _check_bins(g["energy_hist"], d["energy_hist"], rel=1e-9, floor=1e-12)


def test_promotion_at_high_chi(gpu, oracle):
    """Quantum-batch physics (gamma0 = 2e4, a0 = 120, W0 = 2 um: chi up to
    several): FP64 steps where chi > 0.1, FP32 elsewhere, against the oracle;
    segments of FP64 steps start and end inside the pulse."""
    shot = workloads.quantum_batch(n_shots=4)[1]
    p = dict(shot, a0=120.0, n_samples=2037, n_steps=1024)
    g = _run(gpu, p, sample_stride=13, n_sample_records=p["n_samples"] // 13 + 1)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    _check_bins(g["energy_hist"], o["energy_hist"])
    ref = oracle.samples(p, range(0, p["n_samples"], 13))
    assert np.allclose(g["samples"][:, 0], ref[:, oracle.S_MU], rtol=3e-6, atol=0)
    assert np.allclose(g["samples"][:, 1], ref[:, oracle.S_SIG2], rtol=3e-5,
                       atol=3e-5 * ref[:, oracle.S_SIG2].max())
    assert g["moments"][8] > 1.0  # the promoted steps were taken


def test_fp64_step_share(gpu):
    """The moment QS_M_FP64_STEPS: 1 for the FP64 pass, 0 for FP32 without the
    threshold, 1 when the threshold lies below every chi (each wavefront takes
    every step in FP64), strictly between at quantum-batch physics, -1 for the
    derivative-tape pass (not counted)."""
    from paper_2308_09348_amd import _lib
    p = workloads.scaled(workloads.focused_3d(), n_samples=3037, n_steps=256)
    m = lambda q: _run(gpu, q)["moments"][_lib.M_FP64_STEPS]
    assert m(dict(p, precision="fp64")) == 1.0
    assert m(dict(p, precision="fp32", chi_fp64=0.0)) == 0.0
    assert m(dict(p, precision="fp32", chi_fp64=1e-30)) == 1.0
    shot = workloads.quantum_batch(n_shots=4)[1]
    q = dict(shot, a0=120.0, n_samples=2037, n_steps=512)
    share = m(q)
    assert 0.0 < share < 1.0, share
    tape = gpu.new_tape(q["n_samples"])
    out = gpu.forward(q, tape=tape)
    assert out["moments"][_lib.M_FP64_STEPS].item() == -1.0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_wide_box_gaussian_laws(gpu, oracle, prec):
    """Quantum-batch physics with the CIC deposit: samples that keep about 1 %
    of their energy have angle laws hundreds of bins wide (width a0,eff
    sigma_f / mu_f^2), deposited with the box-average series of the law's CDF;
    every bin of both spectra within the parity bar."""
    shot = workloads.quantum_batch(n_shots=4)[1]
    p = dict(shot, a0=120.0, n_samples=2000, n_steps=512, deposit="cic", precision=prec)
    g = _run(gpu, p)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    _check_bins(g["energy_hist"], o["energy_hist"])
    _check_bins(g["angle_hist"], o["angle_hist"])
    assert o["angle_hist"][:-2].min() > 0.5  # the tails are populated


@pytest.mark.parametrize("ksig", [4.5, 9.0, 11.0, 20.0])
def test_gauss_runs_on_both_sides_of_the_rule_bound(gpu, oracle, ksig):
    """GAUSS deposits with kernels of ksig bins: every law is at least ksig
    bins wide, so its edges are at most 1/ksig of its width apart and its
    edges are walked in runs, by Boole's rule on quarter edges where some law
    of the wavefront has them more than a tenth of its width apart (ksig 4.5
    and 9) and by Simpson's on half edges where none has (ksig 11 and 20):
    every bin of both spectra within the parity bar on either side."""
    p = workloads.scaled(workloads.focused_3d(), n_samples=3000, n_steps=256,
                         deposit="gauss", kernel_sigma_bins=ksig)
    g = _run(gpu, p)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    _check_bins(g["energy_hist"], o["energy_hist"])
    _check_bins(g["angle_hist"], o["angle_hist"])


def test_fine_histograms_keep_the_single_edge_array(gpu, oracle):
    """4096 energy and 4096 angle bins: the deposit's LDS words exceed what the
    split upper-tail arrays may take, so the runs add their upper tails as
    2^32 - 2^32 F into the one edge array; every bin within the bar."""
    p = workloads.scaled(workloads.focused_3d(), n_samples=2000, n_steps=128,
                         n_e=4096, n_th=4096, n_a=64)
    g = _run(gpu, p)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    _check_bins(g["energy_hist"], o["energy_hist"])
    _check_bins(g["angle_hist"], o["angle_hist"])


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257])
def test_small_and_ragged_sizes(gpu, oracle, n):
    p = workloads.scaled(workloads.focused_3d(), n_samples=n, n_steps=64)
    g = _run(gpu, p)
    o = oracle.forward(p)
    _check_moments(g, o, p)
    for k in ("energy_hist", "angle_hist", "a0eff_hist"):
        assert abs(g[k].sum() - n) < 1e-9


def test_single_step_and_sin2(gpu, oracle):
    # one RK4 step across the whole window is only sane for a weak field
    p = workloads.scaled(workloads.focused_3d(), n_samples=300, n_steps=1, a0=0.5)
    _check_moments(_run(gpu, p), oracle.forward(p), p)
    q = workloads.scaled(workloads.focused_3d(), n_samples=300, n_steps=256, envelope="sin2",
                         tau_fs=20.0)
    _check_moments(_run(gpu, q), oracle.forward(q), q)


def test_no_field_is_exact(gpu, oracle):
    p = workloads.scaled(workloads.focused_3d(), n_samples=2000, n_steps=64, a0=0.0)
    g = _run(gpu, p, sample_stride=1, n_sample_records=2000)
    assert np.array_equal(g["samples"][:, 0], g["samples"][:, 7])
    assert np.all(g["samples"][:, 1] == 0.0)
    ref = oracle.samples(p, range(0, 2000, 50))
    # Box-Muller and the affine maps round differently on the two sides (an ulp)
    assert np.allclose(g["samples"][::50, 0], ref[:, oracle.S_MU], rtol=1e-15, atol=0)


def test_deterministic_repeat(gpu):
    p = workloads.scaled(workloads.focused_3d(), n_samples=20000, n_steps=128)
    a = _run(gpu, p)
    b = _run(gpu, p)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_invalid_arguments_enqueue_nothing(gpu):
    import torch
    from paper_2308_09348_amd import QScatterError
    p = workloads.scaled(workloads.focused_3d(), n_samples=100, n_steps=16)
    out = gpu.forward(p)
    sentinel = {k: v.clone() for k, v in out.items()}
    for bad in (dict(a0=-1.0), dict(gamma0=0.5), dict(n_steps=0), dict(n_samples=0),
                dict(e_hi=-1.0), dict(tau_fs=float("nan")), dict(n_e=0), dict(deposit=7)):
        q = dict(p, **bad)
        with pytest.raises(QScatterError) as ei:
            gpu.forward(q, out=out)
        assert ei.value.status == 1
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], sentinel[k]), (bad, k)


# ---- full size of the focused configuration, sampled -------------------------

def test_focused_full_size_sampled(gpu, oracle):
    p = workloads.focused_3d()
    n = p["n_samples"]
    stride = n // 64 + 1
    g = _run(gpu, p, sample_stride=stride, n_sample_records=64)
    # every sample adds exactly one unit to each histogram
    for k in ("energy_hist", "angle_hist", "a0eff_hist"):
        assert g[k].sum() == float(n), k
    assert g["status"][0] == 0
    ref = oracle.samples(p, range(0, n, stride))
    assert np.allclose(g["samples"][:, 0], ref[:, oracle.S_MU], rtol=3e-6, atol=0)
    assert np.allclose(g["samples"][:, 1], ref[:, oracle.S_SIG2], rtol=3e-5,
                       atol=3e-5 * ref[:, oracle.S_SIG2].max())
    # moments against the oracle on a bounded prefix, through a separate GPU run
    q = dict(p, n_samples=1 << 14)
    _check_moments(_run(gpu, q), oracle.forward(q), q)
    m = g["moments"]
    assert 0 < m[1] < p["gamma0"] and m[2] > 0 and math.isfinite(m[4])
