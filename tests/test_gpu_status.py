"""Device-side status paths, driven by valid extreme inputs (host validation
accepts them; every table lookup clamps its index, so nothing leaves its
buffer):

- QS_ERANGE: chi = 2 gamma |a| / a_S beyond the tabulated radiation functions
  (chi >= 256; Sec. 4 eq. dpdtRR).  gamma0 = 1e6 and a0 = 500 enter at
  chi ~ 3000, and the quantum drift (g ~ chi^(-4/3)) cannot cool them below
  256 on the rising edge.  Forward (FP32, mixed, FP64), adjoint and photon
  passes all report it; the classical model has no table and reports nothing.
- QS_ENONFINITE: a0 = 1e30 is a finite double whose square overflows FP32 and
  drives the FP64 state past the largest double within a step, so the final
  energy is not finite; the deposit skips such samples.

Each status is read back through qs_sync_status (the C ABI) and raised by the
binding; the next valid call on the same context reports QS_OK.
"""
import ctypes

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


def _small(**kw):
    p = workloads.scaled(workloads.focused_3d(), n_samples=300, n_steps=128)
    p.update(kw)
    return p


def _hot(**kw):
    # chi ~ 3000 at entry, beyond the tables' 256
    return _small(gamma0=1e6, sigma_gamma=1e4, a0=500.0, e_hi=1.5e6, **kw)


def _status(ctx, status_tensor):
    import torch
    from paper_2308_09348_amd import _lib
    return _lib.lib().qs_sync_status(ctx.handle, ctypes.c_void_p(status_tensor.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec,chi64", [("fp32", 0.0), ("fp32", 0.1), ("fp64", 0.0)])
def test_chi_beyond_the_table_is_reported(gpu, prec, chi64):
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib
    p = _hot(precision=prec, chi_fp64=chi64)
    print(f"status: range, forward {prec} chi_fp64={chi64}", flush=True)
    out = gpu.forward(p, check=False)
    assert _status(gpu, out["status"]) == _lib.QS_ERANGE
    with pytest.raises(qs.QScatterError) as e:
        gpu.forward(p)
    assert e.value.status == _lib.QS_ERANGE
    # the deposit still conserves the weight of the clamped samples
    assert float(out["energy_hist"].sum().item()) == p["n_samples"]
    # a valid call on the same context reports ok again
    ok = gpu.forward(_small(precision=prec, chi_fp64=chi64), check=False)
    assert _status(gpu, ok["status"]) == _lib.QS_OK


def test_classical_model_has_no_range(gpu):
    from paper_2308_09348_amd import _lib
    print("status: classical at the same chi", flush=True)
    out = gpu.forward(_hot(rr_model="classical"), check=False)
    assert _status(gpu, out["status"]) == _lib.QS_OK


def test_range_in_adjoint_and_photon_passes(gpu):
    import torch
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib
    p = _hot(deposit="gauss")
    print("status: range, adjoint and photons", flush=True)
    w = torch.ones(p["n_e"] + 2, dtype=torch.float64, device="cuda")
    with pytest.raises(qs.QScatterError) as e:
        gpu.backward(p, w)
    assert e.value.status == _lib.QS_ERANGE
    with pytest.raises(qs.QScatterError) as e:
        gpu.photons(dict(p, n_ph=64, ph_hi=1e6))
    assert e.value.status == _lib.QS_ERANGE


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_non_finite_state_is_reported(gpu, prec):
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib
    p = _small(a0=1e30, rr_model="classical", precision=prec)
    print(f"status: non-finite, forward {prec}", flush=True)
    out = gpu.forward(p, check=False)
    assert _status(gpu, out["status"]) == _lib.QS_ENONFINITE
    with pytest.raises(qs.QScatterError) as e:
        gpu.forward(p)
    assert e.value.status == _lib.QS_ENONFINITE
    # samples whose state is not finite deposit nothing
    assert float(out["energy_hist"].sum().item()) < p["n_samples"]
    ok = gpu.forward(_small(precision=prec), check=False)
    assert _status(gpu, ok["status"]) == _lib.QS_OK
