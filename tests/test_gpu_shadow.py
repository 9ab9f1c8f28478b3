"""FP64 shadow of an FP32 pass (QS_VALIDATE_FP64): every shadow_stride-th
sample is integrated again in FP64 and the differences are reported in the
moments QS_M_SHADOW_N .. QS_M_ERR_MEAN_G.  Checked against the FP64 pass's
own per-sample records (the shadow runs the same FP64 integration of the same
samples), and the rest of the output must be the FP32 pass's bits.
"""
import numpy as np
import pytest

from paper_2308_09348_amd import _lib, workloads

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


def _run(ctx, p):
    n = p["n_samples"]
    return _np(ctx.forward(p, sample_stride=1, n_sample_records=n))


@pytest.mark.parametrize("chi64,stride", [(0.0, 7), (0.1, 1), (0.1, 64)])
def test_shadow_matches_the_fp64_pass(gpu, chi64, stride):
    p = workloads.scaled(workloads.focused_3d(), n_samples=5037, n_steps=256, deposit="cic",
                         chi_fp64=chi64)
    plain = _run(gpu, p)
    g = _run(gpu, dict(p, validate_fp64=True, shadow_stride=stride))
    d = _run(gpu, dict(p, precision="fp64"))
    # everything but the shadow fields is the FP32 pass
    for k in ("energy_hist", "angle_hist", "a0eff_hist", "samples"):
        assert np.array_equal(g[k], plain[k]), k
    assert np.array_equal(g["moments"][:11], plain["moments"][:11])
    assert not plain["moments"][11:_lib.M_FP64_STEPS].any()
    # the shadow's FP64 launch counts no FP32-loop steps: the share is the pass's
    assert g["moments"][_lib.M_FP64_STEPS] == plain["moments"][_lib.M_FP64_STEPS]
    m = g["moments"]
    idx = np.arange(0, p["n_samples"], stride)
    mu32, mu64 = g["samples"][idx, 0], d["samples"][idx, 0]
    s32 = np.sqrt(np.maximum(g["samples"][idx, 1], 0.0))
    s64 = np.sqrt(np.maximum(d["samples"][idx, 1], 0.0))
    diff = mu32 - mu64
    assert m[_lib.M_SHADOW_N] == len(idx)
    assert m[_lib.M_ERR_MU_MAX] == np.max(np.abs(diff) / mu64)
    assert m[_lib.M_ERR_SIG_MAX] == np.max(np.abs(s32 - s64) / mu64)
    assert abs(m[_lib.M_ERR_MU_MEAN] - np.mean(diff / mu64)) <= 1e-12 * np.max(np.abs(diff / mu64))
    assert abs(m[_lib.M_ERR_MEAN_G] - np.mean(diff)) <= 1e-12 * np.max(np.abs(diff))
    # the FP32 pass is within its tolerance of the FP64 one, and not identical
    assert 0 < m[_lib.M_ERR_MU_MAX] < 3e-6
    assert m[_lib.M_ERR_SIG_MAX] < 3e-6


def test_no_shadow_for_fp64_passes(gpu):
    p = workloads.scaled(workloads.focused_3d(), n_samples=1000, n_steps=64, precision="fp64",
                         validate_fp64=True, shadow_stride=3)
    g = _run(gpu, p)
    assert not g["moments"][11:_lib.M_FP64_STEPS].any()
    assert g["moments"][_lib.M_FP64_STEPS] == 1.0


def test_shadow_in_a_batch_equals_single_shots(gpu):
    base = workloads.scaled(workloads.focused_3d(), n_samples=3000, n_steps=128,
                            validate_fp64=True, shadow_stride=5)
    shots = [dict(base, n_samples=n, a0=a, shot=0) for n, a in ((3000, 30.0), (1, 50.0),
                                                                 (777, 80.0))]
    batch = [_np(o) for o in gpu.forward_batched(shots)]
    for k, s in enumerate(shots):
        single = _np(gpu.forward(dict(s, shot=k)))
        for key in single:
            assert np.array_equal(batch[k][key], single[key]), (k, key)
    assert batch[1]["moments"][_lib.M_SHADOW_N] == 1


@pytest.mark.parametrize("deposit", ["cic", "gauss", "point"])
def test_shadow_spectrum_errors(gpu, oracle, deposit):
    """The histogram-level shadow fields: D_k = sum over the shadowed samples
    of the law deposited from the FP32 state minus that from the FP64 state
    (the FP64 pass's records give the latter), through the oracle's deposit;
    L1 and largest bin per shadowed sample, energy and angle.  Bars: the
    device quantises each edge's CDF difference to 2^-40 (at most 2^-40 per
    bin and shadowed sample), and the oracle's law stops at 6 standard
    deviations (the device's difference runs to 9: 2e-9 of a law's mass,
    times the relative shift of the two laws)."""
    stride = 7
    p = workloads.scaled(workloads.focused_3d(), n_samples=5037, n_steps=256, deposit=deposit)
    n = p["n_samples"]
    g = _run(gpu, dict(p, validate_fp64=True, shadow_stride=stride))
    d = _run(gpu, dict(p, precision="fp64"))
    idx = np.arange(0, n, stride)
    r32, r64 = g["samples"][idx], d["samples"][idx]
    De = np.zeros(p["n_e"] + 2)
    Dt = np.zeros(p["n_th"] + 2)
    for a, b in zip(r32, r64):
        De += oracle.deposit(a[0], np.sqrt(max(a[1], 0.0)), deposit, p["kernel_sigma_bins"],
                             p["e_lo"], p["e_hi"], p["n_e"])
        De -= oracle.deposit(b[0], np.sqrt(max(b[1], 0.0)), deposit, p["kernel_sigma_bins"],
                             p["e_lo"], p["e_hi"], p["n_e"])
        Dt += oracle.deposit(a[2], a[4], deposit, p["kernel_sigma_bins"], p["th_lo_mrad"],
                             p["th_hi_mrad"], p["n_th"])
        Dt -= oracle.deposit(b[2], b[4], deposit, p["kernel_sigma_bins"], p["th_lo_mrad"],
                             p["th_hi_mrad"], p["n_th"])
    ns = len(idx)
    m = g["moments"]
    want = [np.abs(De).sum() / ns, np.abs(De).max() / ns, np.abs(Dt).sum() / ns,
            np.abs(Dt).max() / ns]
    got = [m[_lib.M_ERR_E_L1], m[_lib.M_ERR_E_MAX], m[_lib.M_ERR_T_L1], m[_lib.M_ERR_T_MAX]]
    print(deposit, "want", want, "got", got)
    # the FP32 pass differs from the FP64 one, and the fields say by how much
    assert want[0] > 0 and got[0] > 0
    # quantisation: at most 2^-40 a bin and shadowed sample (L1: times the bins)
    for w_, g_, nb in zip(want, got, (p["n_e"] + 2, 1, p["n_th"] + 2, 1)):
        assert abs(g_ - w_) <= 1e-6 * w_ + nb * 2.0 ** -40, (deposit, want, got)
    # an FP32 pass without the shadow leaves them zero
    assert not _run(gpu, p)["moments"][11:_lib.M_FP64_STEPS].any()
