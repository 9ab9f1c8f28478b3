"""qs_forward_noalloc (the forward pass for callers that cannot allocate)
against qs_forward, through the C ABI: two calls in a row on one context, the
second with a smaller input and other bins, then the largest input the static
scratch holds.  The two entry points share every kernel, so the outputs must
agree bit for bit (stronger than the parity bar of the pass itself).
"""
import numpy as np
import pytest

from paper_2308_09348_amd import workloads

pytestmark = pytest.mark.gpu

KEYS = ("energy_hist", "angle_hist", "a0eff_hist", "moments", "status", "samples")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    ctx = qs.Context(0)
    yield ctx
    ctx.close()


def _both(ctx, params, records=8):
    stride = max(params["n_samples"] // records, 1)
    print(f"noalloc: {params['n_samples']} samples x {params['n_steps']} steps, "
          f"bins {params['n_e']}/{params['n_th']}/{params['n_a']}", flush=True)
    ref = ctx.forward(params, sample_stride=stride, n_sample_records=records)
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    got = ctx.forward(params, sample_stride=stride, n_sample_records=records, noalloc=True)
    got = {k: v.cpu().numpy() for k, v in got.items()}
    return ref, got


def _same(ref, got):
    for k in KEYS:
        assert np.array_equal(ref[k], got[k]), (k, ref[k][:4], got[k][:4])


def test_noalloc_equals_forward_twice_smaller_second(gpu):
    big = workloads.scaled(workloads.focused_3d(), n_samples=3 * 4096 + 77, n_steps=256)
    ref, got = _both(gpu, big)
    _same(ref, got)
    assert got["energy_hist"].sum() == big["n_samples"]
    small = workloads.scaled(workloads.focused_3d(), n_samples=1000 + 3, n_steps=128)
    small.update(n_e=100, n_th=64, n_a=32, deposit="gauss", kernel_sigma_bins=1.0, seed=11)
    ref2, got2 = _both(gpu, small)
    _same(ref2, got2)
    assert got2["energy_hist"].sum() == small["n_samples"]


def test_noalloc_at_its_largest_input(gpu):
    from paper_2308_09348_amd import _lib
    p = workloads.scaled(workloads.focused_3d(), n_samples=_lib.NOALLOC_MAX_SAMPLES, n_steps=64)
    p.update(n_e=4096, n_th=4096, n_a=4096)
    ref, got = _both(gpu, p)
    _same(ref, got)


def test_noalloc_rejects_what_its_scratch_cannot_hold(gpu):
    import torch
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib
    p = workloads.scaled(workloads.focused_3d(), n_samples=_lib.NOALLOC_MAX_SAMPLES + 1,
                         n_steps=16)
    with pytest.raises(qs.QScatterError) as e:
        gpu.forward(p, noalloc=True)
    assert e.value.status == _lib.QS_EINVAL
    p = workloads.scaled(workloads.focused_3d(), n_samples=4096, n_steps=16)
    p["validate_fp64"] = True
    with pytest.raises(qs.QScatterError) as e:
        gpu.forward(p, noalloc=True)
    assert e.value.status == _lib.QS_EUNSUPPORTED
    torch.cuda.synchronize()
    # the context still works after the rejections
    p = workloads.scaled(workloads.focused_3d(), n_samples=500, n_steps=32)
    ref, got = _both(gpu, p)
    _same(ref, got)
