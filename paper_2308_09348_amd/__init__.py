"""MI355X (gfx950) beam-phase-space integrator of QScatter (arXiv 2308.09348).

``forward(params)`` predicts the asymptotic electron energy / angle / a0,eff
distributions and moments after a relativistic electron beam meets a focused,
possibly misaligned laser pulse head-on; ``energy_histogram(theta, params)``
is the same energy histogram as a differentiable function of the eight shot
parameters ``PARAM_NAMES`` (adjoint on the device).  All computation runs in
the HIP kernels of ``libqscatter.so``; PyTorch only provides device memory and
the stream.
"""
import ctypes
import os

from . import _lib

__all__ = ["Context", "forward", "energy_histogram", "spectra", "radiation_eval",
           "QScatterError", "PARAM_NAMES"]

QScatterError = _lib.QScatterError
PARAM_NAMES = _lib.PARAM_NAMES


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required (torch.cuda.is_available() is False)")
    return torch


class Context:
    """Owns a qs_ctx (radiation tables and device scratch) on one device."""

    def __init__(self, device=0):
        self._ptr = ctypes.c_void_p()
        self.device = int(device)
        st = _lib.lib().qs_create(ctypes.byref(self._ptr), self.device)
        if st != _lib.QS_OK:
            raise QScatterError(st, "qs_create")

    @property
    def handle(self):
        return self._ptr

    def close(self):
        if self._ptr:
            _lib.lib().qs_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return _lib.lib().qs_last_error(self._ptr).decode()

    def new_tape(self, n_samples):
        """A device tensor for a derivative tape of n_samples samples:
        [TAPE_FIELDS, n_samples] float64 (fields T_MU, T_SIG2, T_DMU + p,
        T_DSIG2 + p)."""
        torch = _torch()
        return torch.empty((_lib.TAPE_FIELDS, int(n_samples)), dtype=torch.float64,
                           device=torch.device("cuda", self.device))

    def forward(self, params, sample_stride=0, n_sample_records=0, stream=None, out=None,
                check=True, tape=None, noalloc=False):
        """Enqueue one forward pass; returns a dict of device tensors.

        ``out`` may hold preallocated tensors (same keys as the result) to
        avoid allocation.  With ``check`` the stream is synchronised and the
        device status word raised as an error.  With ``tape`` (from new_tape)
        the pass also records the per-sample parameter derivatives there.
        With ``noalloc`` the pass runs through qs_forward_noalloc (the
        library allocates nothing; at most NOALLOC_MAX_SAMPLES samples)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        la, be, nu, bi = _lib.structs(params)
        if out is None:
            out = {
                "energy_hist": torch.empty(params["n_e"] + 2, dtype=torch.float64, device=dev),
                "angle_hist": torch.empty(params["n_th"] + 2, dtype=torch.float64, device=dev),
                "a0eff_hist": torch.empty(params["n_a"], dtype=torch.float64, device=dev),
                "moments": torch.empty(_lib.M_N, dtype=torch.float64, device=dev),
                "status": torch.empty(1, dtype=torch.int32, device=dev),
            }
            if n_sample_records > 0:
                out["samples"] = torch.empty((n_sample_records, _lib.S_N), dtype=torch.float64,
                                             device=dev)
        o = _lib.Outputs(
            energy_hist=out["energy_hist"].data_ptr(), angle_hist=out["angle_hist"].data_ptr(),
            a0eff_hist=out["a0eff_hist"].data_ptr(), moments=out["moments"].data_ptr(),
            status=out["status"].data_ptr(),
            samples=out["samples"].data_ptr() if "samples" in out else None,
            sample_stride=max(int(sample_stride), 1), n_sample_records=int(n_sample_records))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        if tape is not None:
            _check_tape(tape, params["n_samples"])
            st = _lib.lib().qs_forward_tape(self._ptr, ctypes.byref(la), ctypes.byref(be),
                                            ctypes.byref(nu), ctypes.byref(bi), ctypes.byref(o),
                                            ctypes.c_void_p(tape.data_ptr()),
                                            ctypes.c_void_p(stream.cuda_stream))
        else:
            fn = _lib.lib().qs_forward_noalloc if noalloc else _lib.lib().qs_forward
            st = fn(self._ptr, ctypes.byref(la), ctypes.byref(be), ctypes.byref(nu),
                    ctypes.byref(bi), ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            st = _lib.lib().qs_sync_status(self._ptr, ctypes.c_void_p(out["status"].data_ptr()),
                                           ctypes.c_void_p(stream.cuda_stream))
            if st != _lib.QS_OK:
                raise QScatterError(st, "device status")
        return out

    def prepare_batch(self, shots):
        """Marshal a list of per-shot parameter dictionaries once (ctypes
        arrays and output tensors); run it with run_batch().  The numerics
        (steps, seed, models, deposit, precision) come from shots[0]; shot k
        uses RNG counter word shots[0]["shot"] + k."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = len(shots)
        if n == 0:
            raise ValueError("empty batch")
        b = _Batch()
        _, _, b.nu, _ = _lib.structs(shots[0])
        b.n = n
        b.lasers = (_lib.Laser * n)()
        b.beams = (_lib.Beam * n)()
        b.bins = (_lib.Bins * n)()
        b.outs = (_lib.Outputs * n)()
        b.ns = (ctypes.c_int64 * n)()
        b.out = []
        for k, p in enumerate(shots):
            la, be, _, bi = _lib.structs(p)
            b.lasers[k], b.beams[k], b.bins[k] = la, be, bi
            b.ns[k] = int(p["n_samples"])
            o = {"energy_hist": torch.empty(p["n_e"] + 2, dtype=torch.float64, device=dev),
                 "angle_hist": torch.empty(p["n_th"] + 2, dtype=torch.float64, device=dev),
                 "a0eff_hist": torch.empty(p["n_a"], dtype=torch.float64, device=dev),
                 "moments": torch.empty(_lib.M_N, dtype=torch.float64, device=dev),
                 "status": torch.empty(1, dtype=torch.int32, device=dev)}
            b.out.append(o)
            b.outs[k] = _lib.Outputs(
                energy_hist=o["energy_hist"].data_ptr(), angle_hist=o["angle_hist"].data_ptr(),
                a0eff_hist=o["a0eff_hist"].data_ptr(), moments=o["moments"].data_ptr(),
                status=o["status"].data_ptr(), samples=None, sample_stride=1,
                n_sample_records=0)
        return b

    def run_batch(self, batch, stream=None, check=True, tape=None):
        """Enqueue one launch over a prepared batch; returns its outputs.  With
        ``tape`` ([TAPE_FIELDS, total samples]) the launch records the
        per-sample parameter derivatives of every shot."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        if tape is not None:
            _check_tape(tape, sum(batch.ns))
            st = _lib.lib().qs_forward_tape_batched(
                self._ptr, batch.n, batch.lasers, batch.beams, batch.ns, ctypes.byref(batch.nu),
                batch.bins, batch.outs, ctypes.c_void_p(tape.data_ptr()),
                ctypes.c_void_p(stream.cuda_stream))
        else:
            st = _lib.lib().qs_forward_batched(self._ptr, batch.n, batch.lasers, batch.beams,
                                               batch.ns, ctypes.byref(batch.nu), batch.bins,
                                               batch.outs, ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            torch.cuda.synchronize(dev)
            bad = int(torch.stack([o["status"] for o in batch.out]).max().item())
            if bad != _lib.QS_OK:
                raise QScatterError(bad, "device status of a shot")
        return batch.out

    def forward_batched(self, shots, stream=None, check=True, tape=None):
        """One launch over a list of per-shot parameter dictionaries; returns a
        list of per-shot result dictionaries (device tensors)."""
        return self.run_batch(self.prepare_batch(shots), stream=stream, check=check, tape=tape)

    def forward_factorised(self, params, n_anodes=61, n_gnodes=None, nodes=False, stream=None,
                           check=True, sample_stride=0, n_sample_records=0):
        """The A0EFF forward pass by plane-wave reconstruction on an n_anodes x
        n_gnodes node grid (n_gnodes defaults to 64, or 1 without an energy
        spread); returns a dict of device tensors, with "node_states"
        [nodes, NODE_FIELDS] and "node_weights" [nodes] when ``nodes``, and
        "samples" [n_sample_records, S_N] (every sample_stride-th sample)."""
        torch = _torch()
        b = self.prepare_factorised([params], n_anodes, n_gnodes, nodes)
        if n_sample_records > 0:
            o = b.out[0]
            o["samples"] = torch.empty((n_sample_records, _lib.S_N), dtype=torch.float64,
                                       device=torch.device("cuda", self.device))
            b.outs[0].samples = o["samples"].data_ptr()
            b.outs[0].sample_stride = max(int(sample_stride), 1)
            b.outs[0].n_sample_records = int(n_sample_records)
        return self.run_factorised(b, stream=stream, check=check, single=True)[0]

    def forward_factorised_batched(self, shots, n_anodes=61, n_gnodes=None, nodes=False,
                                   stream=None, check=True, single=False):
        """forward_factorised over a list of shots in one launch (numerics from
        shots[0], shot k with RNG counter word shots[0]["shot"] + k); with
        ``single`` the one-shot entry point is called instead."""
        batch = self.prepare_factorised(shots, n_anodes, n_gnodes, nodes)
        return self.run_factorised(batch, stream=stream, check=check, single=single)

    def prepare_factorised(self, shots, n_anodes=61, n_gnodes=None, nodes=False):
        """Marshal a reconstruction launch once (see prepare_batch); run it
        with run_factorised()."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        b = self.prepare_batch(shots)
        b.grids = (_lib.NodeGrid * b.n)()
        for k, p in enumerate(shots):
            ng = n_gnodes if n_gnodes is not None else (64 if p["sigma_gamma"] > 0 else 1)
            b.grids[k] = _lib.NodeGrid(n_a=int(n_anodes), n_g=int(ng))
            if nodes:
                o = b.out[k]
                o["node_states"] = torch.empty((n_anodes * ng, _lib.NODE_FIELDS),
                                               dtype=torch.float64, device=dev)
                o["node_weights"] = torch.empty(n_anodes * ng, dtype=torch.float64, device=dev)
                b.grids[k].node_states = o["node_states"].data_ptr()
                b.grids[k].node_weights = o["node_weights"].data_ptr()
        return b

    def run_factorised(self, b, stream=None, check=True, single=False):
        """Enqueue one reconstruction launch over a prepared batch."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        if single:
            if b.n != 1:
                raise ValueError("single needs one shot")
            st = _lib.lib().qs_forward_factorised(
                self._ptr, ctypes.byref(b.lasers[0]), ctypes.byref(b.beams[0]),
                ctypes.byref(b.nu), ctypes.byref(b.bins[0]), ctypes.byref(b.grids[0]),
                ctypes.byref(b.outs[0]), ctypes.c_void_p(stream.cuda_stream))
        else:
            st = _lib.lib().qs_forward_factorised_batched(
                self._ptr, b.n, b.lasers, b.beams, b.ns, ctypes.byref(b.nu), b.bins, b.grids,
                b.outs, ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            torch.cuda.synchronize(dev)
            bad = int(torch.stack([o["status"] for o in b.out]).max().item())
            if bad != _lib.QS_OK:
                raise QScatterError(bad, "device status of a shot")
        return b.out

    def _upstream(self, params, stream, d_energy, d_angle, d_moments, moments, keep):
        """Device float64 copies of the upstream weights (None stays None)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        sizes = (params["n_e"] + 2, params["n_th"] + 2, _lib.M_N, _lib.M_N)
        names = ("d_energy", "d_angle", "d_moments", "moments")
        out = []
        for t, n, name in zip((d_energy, d_angle, d_moments, moments), sizes, names):
            if t is None:
                out.append(None)
                continue
            d = t.to(device=dev, dtype=torch.float64).contiguous()
            if d.numel() != n:
                raise ValueError(f"{name} needs {n} entries")
            if d.data_ptr() != t.data_ptr():
                d.record_stream(stream)
            keep.append(d)
            out.append(d)
        if out[2] is not None and out[3] is None:
            raise ValueError("d_moments needs the forward moments")
        if all(o is None for o in out[:3]):
            raise ValueError("no upstream weights")
        return out

    def backward(self, params, d_energy=None, stream=None, check=True, tape=None, d_angle=None,
                 d_moments=None, moments=None, errors=False):
        """Derivatives of L = d_energy . H + d_angle . T + d_moments . M (H, T, M:
        the energy histogram, angle histogram and moments of forward(params);
        each weight vector optional, ``moments`` = M is needed with d_moments)
        with respect to PARAM_NAMES; returns a float64 device tensor of 8.  With
        ``tape`` (recorded by forward(params, tape=...)) the energy-state
        derivatives are read from it instead of integrating the trajectories
        again.  With ``errors`` returns (gradient, report): the FP64-shadow
        report [GE_N] (zeros unless params["validate_fp64"] on an FP32 pass)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        la, be, nu, bi = _lib.structs(params)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        keep = []
        de, dt, dm, mo = self._upstream(params, stream, d_energy, d_angle, d_moments, moments,
                                        keep)
        ptr = lambda t: None if t is None else t.data_ptr()
        grad = torch.empty(len(PARAM_NAMES), dtype=torch.float64, device=dev)
        status = torch.empty(1, dtype=torch.int32, device=dev)
        err = torch.empty(_lib.GE_N, dtype=torch.float64, device=dev) if errors else None
        g = _lib.GradOutputs(d_energy_hist=ptr(de), grad=grad.data_ptr(),
                             status=status.data_ptr(), d_angle_hist=ptr(dt), d_moments=ptr(dm),
                             moments=ptr(mo), errors=ptr(err))
        if tape is not None:
            _check_tape(tape, params["n_samples"])
            st = _lib.lib().qs_backward_tape(self._ptr, ctypes.byref(la), ctypes.byref(be),
                                             ctypes.byref(nu), ctypes.byref(bi), ctypes.byref(g),
                                             ctypes.c_void_p(tape.data_ptr()),
                                             ctypes.c_void_p(stream.cuda_stream))
        else:
            st = _lib.lib().qs_backward(self._ptr, ctypes.byref(la), ctypes.byref(be),
                                        ctypes.byref(nu), ctypes.byref(bi), ctypes.byref(g),
                                        ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            st = _lib.lib().qs_sync_status(self._ptr, ctypes.c_void_p(status.data_ptr()),
                                           ctypes.c_void_p(stream.cuda_stream))
            if st != _lib.QS_OK:
                raise QScatterError(st, "device status")
        return (grad, err) if errors else grad

    def backward_batched(self, shots, d_energy=None, stream=None, check=True, tape=None,
                         d_angle=None, d_moments=None, moments=None, errors=False):
        """Adjoint of forward_batched(shots): d_energy, d_angle, d_moments and
        moments are lists of per-shot tensors (or None) as in backward();
        returns a list of gradient tensors (with ``errors``: and a list of
        FP64-shadow reports, as in backward()).  ``tape``: as recorded by
        forward_batched(shots, tape=...)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = len(shots)
        lists = [x if x is not None else [None] * n for x in (d_energy, d_angle, d_moments,
                                                               moments)]
        if n == 0 or any(len(x) != n for x in lists):
            raise ValueError("one upstream weight vector per shot")
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _, _, nu, _ = _lib.structs(shots[0])
        lasers, beams, bins = (_lib.Laser * n)(), (_lib.Beam * n)(), (_lib.Bins * n)()
        outs, ns = (_lib.GradOutputs * n)(), (ctypes.c_int64 * n)()
        keep, grads = [], []
        status = torch.empty(n, dtype=torch.int32, device=dev)
        errs = [torch.empty(_lib.GE_N, dtype=torch.float64, device=dev) if errors else None
                for _ in range(n)]
        ptr = lambda t: None if t is None else t.data_ptr()
        for k, p in enumerate(shots):
            la, be, _, bi = _lib.structs(p)
            lasers[k], beams[k], bins[k] = la, be, bi
            ns[k] = int(p["n_samples"])
            de, dt, dm, mo = self._upstream(p, stream, *(x[k] for x in lists), keep)
            grads.append(torch.empty(len(PARAM_NAMES), dtype=torch.float64, device=dev))
            outs[k] = _lib.GradOutputs(d_energy_hist=ptr(de), grad=grads[k].data_ptr(),
                                       status=status[k:].data_ptr(), d_angle_hist=ptr(dt),
                                       d_moments=ptr(dm), moments=ptr(mo), errors=ptr(errs[k]))
        if tape is not None:
            _check_tape(tape, sum(ns))
            st = _lib.lib().qs_backward_tape_batched(self._ptr, n, lasers, beams, ns,
                                                     ctypes.byref(nu), bins, outs,
                                                     ctypes.c_void_p(tape.data_ptr()),
                                                     ctypes.c_void_p(stream.cuda_stream))
        else:
            st = _lib.lib().qs_backward_batched(self._ptr, n, lasers, beams, ns,
                                                ctypes.byref(nu), bins, outs,
                                                ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            torch.cuda.synchronize(dev)
            bad = int(status.max().item())
            if bad != _lib.QS_OK:
                raise QScatterError(bad, "device status of a shot")
        return (grads, errs) if errors else grads

    def photons(self, params, stream=None, check=True, angles=False):
        """Photon spectrum of one shot (Sec. 4): returns {"photon_hist": [n_ph + 2]
        expected photon number per bin, "energy": [emitted photon energy,
        electron energy loss], "status"}; bins from photon_bins(params).  With
        ``angles`` also "angles" [6]: photon number and its rms theta_x,
        theta_y (mrad), photon energy and its rms theta_x, theta_y (Sec. 5.1).
        With params["validate_fp64"] also "errors" [PE_N]: the FP64-shadow
        report (zeros for an FP64 pass)."""
        return self.photons_batched([params], stream=stream, check=check, single=True,
                                    angles=angles)[0]

    def photons_batched(self, shots, stream=None, check=True, single=False, angles=False):
        """Photon spectra of many shots in one launch (shot k uses RNG counter
        word shots[0]["shot"] + k)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = len(shots)
        if n == 0:
            raise ValueError("empty batch")
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _, _, nu, _ = _lib.structs(shots[0])
        report = bool(shots[0].get("validate_fp64", False))
        lasers, beams = (_lib.Laser * n)(), (_lib.Beam * n)()
        pbins, pouts, ns = (_lib.PhotonBins * n)(), (_lib.PhotonOutputs * n)(), (ctypes.c_int64 * n)()
        outs = []
        for k, p in enumerate(shots):
            la, be, _, _ = _lib.structs(p)
            lasers[k], beams[k] = la, be
            pbins[k] = _lib.photon_bins(p)
            ns[k] = int(p["n_samples"])
            o = {"photon_hist": torch.empty(pbins[k].n_ph + 2, dtype=torch.float64, device=dev),
                 "energy": torch.empty(2, dtype=torch.float64, device=dev),
                 "status": torch.empty(1, dtype=torch.int32, device=dev)}
            if angles:
                o["angles"] = torch.empty(6, dtype=torch.float64, device=dev)
            if report:
                o["errors"] = torch.empty(_lib.PE_N, dtype=torch.float64, device=dev)
            outs.append(o)
            pouts[k] = _lib.PhotonOutputs(photon_hist=o["photon_hist"].data_ptr(),
                                          energy=o["energy"].data_ptr(),
                                          status=o["status"].data_ptr(),
                                          angles=o["angles"].data_ptr() if angles else None,
                                          errors=o["errors"].data_ptr() if report else None)
        if single:
            st = _lib.lib().qs_photons(self._ptr, ctypes.byref(lasers[0]), ctypes.byref(beams[0]),
                                       ctypes.byref(nu), ctypes.byref(pbins[0]),
                                       ctypes.byref(pouts[0]), ctypes.c_void_p(stream.cuda_stream))
        else:
            st = _lib.lib().qs_photons_batched(self._ptr, n, lasers, beams, ns, ctypes.byref(nu),
                                               pbins, pouts, ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        if check:
            torch.cuda.synchronize(dev)
            bad = int(torch.stack([o["status"] for o in outs]).max().item())
            if bad != _lib.QS_OK:
                raise QScatterError(bad, "device status of a shot")
        return outs

    def photon_cdf(self, chi, xi):
        """The device's LCFA number CDF Phi(xi; chi) (1-D float64 tensors)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        chi = chi.to(device=dev, dtype=torch.float64).contiguous()
        xi = xi.to(device=dev, dtype=torch.float64).contiguous()
        out = torch.empty_like(chi)
        stream = torch.cuda.current_stream(dev)
        st = _lib.lib().qs_photon_cdf(self._ptr, chi.numel(), ctypes.c_void_p(chi.data_ptr()),
                                      ctypes.c_void_p(xi.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        torch.cuda.synchronize(dev)
        return out

    def tune(self, shots, cache_path=None, stream=None):
        """Time the launch choices for the launch class of `shots` (one
        parameter dictionary, a list of them, or a prepared batch; qs_tune)
        and keep the fastest for later launches of that class on this
        context; with cache_path, read the choice from / append it to that
        text file.  Returns the choice as a dict."""
        torch = _torch()
        if isinstance(shots, dict):
            shots = [shots]
        b = shots if isinstance(shots, _Batch) else self.prepare_batch(shots)
        stream = stream or torch.cuda.current_stream(torch.device("cuda", self.device))
        t = _lib.Tuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        st = _lib.lib().qs_tune(self._ptr, b.n, b.lasers, b.beams, b.ns, ctypes.byref(b.nu),
                                b.bins, path, ctypes.byref(t),
                                ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        return {"dep_tile": t.dep_tile, "phase_cap": t.phase_cap, "dep_cap": t.dep_cap,
                "from_cache": bool(t.from_cache), "phase_ms": t.phase_ms,
                "deposit_ms": t.deposit_ms}

    def set_graphs(self, on=True):
        """Capture forward launches into HIP graphs and replay them for
        launches with identical kernel arguments (qs_set_graphs)."""
        st = _lib.lib().qs_set_graphs(self._ptr, 1 if on else 0)
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())

    def set_profiling(self, on=True):
        st = _lib.lib().qs_set_profiling(self._ptr, 1 if on else 0)
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())

    def last_timings(self):
        """Kernel durations [ms] of the last profiled forward: envelope, clear,
        phase, deposit, finalize."""
        ms = (ctypes.c_double * 5)()
        st = _lib.lib().qs_last_timings(self._ptr, ms)
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        return dict(zip(["envelope", "clear", "phase", "deposit", "finalize"], list(ms)))

    def timings_sum(self):
        """(calls, sums) of the kernel durations [ms] that last_timings reports,
        over the last min(n, 64) of the n profiled forwards since profiling was
        switched on; read once after many back-to-back calls."""
        ms = (ctypes.c_double * 5)()
        n = ctypes.c_int32(0)
        st = _lib.lib().qs_timings_sum(self._ptr, ctypes.byref(n), ms)
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        return n.value, dict(zip(["envelope", "clear", "phase", "deposit", "finalize"], list(ms)))

    def radiation_eval(self, chi, precision="fp32"):
        """{g, chi g', chi^2 g'', h} of the device tables at chi (1-D float64 tensor)."""
        torch = _torch()
        chi = chi.to(device=torch.device("cuda", self.device), dtype=torch.float64).contiguous()
        out = torch.empty((chi.numel(), 4), dtype=torch.float64, device=chi.device)
        stream = torch.cuda.current_stream(chi.device)
        st = _lib.lib().qs_radiation_eval(self._ptr, _lib.PRECISION[precision], chi.numel(),
                                          ctypes.c_void_p(chi.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        torch.cuda.synchronize(chi.device)
        return out

    def radiation_derivs(self, chi, precision="fp32"):
        """The adjoint's device tables at chi (1-D float64 tensor): columns g,
        chi g', chi^2 g'', h, chi^3 d3g/dchi3, chi h'."""
        torch = _torch()
        chi = chi.to(device=torch.device("cuda", self.device), dtype=torch.float64).contiguous()
        out = torch.empty((chi.numel(), 6), dtype=torch.float64, device=chi.device)
        stream = torch.cuda.current_stream(chi.device)
        st = _lib.lib().qs_radiation_derivs(self._ptr, _lib.PRECISION[precision], chi.numel(),
                                            ctypes.c_void_p(chi.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.QS_OK:
            raise QScatterError(st, self.last_error())
        torch.cuda.synchronize(chi.device)
        return out


class _Batch:
    """Marshalled arguments and output tensors of a batched launch."""


def _check_tape(tape, n_samples):
    import torch
    if (tape.dtype != torch.float64 or not tape.is_cuda or not tape.is_contiguous()
            or tape.numel() != _lib.TAPE_FIELDS * int(n_samples)):
        raise ValueError("tape must be a contiguous float64 device tensor of "
                         "TAPE_FIELDS x n_samples")


_default = {}


def _ctx(device=0):
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def forward(params, device=0, **kw):
    """One forward pass on ``device`` with a cached context."""
    return _ctx(device).forward(params, **kw)


def radiation_eval(chi, precision="fp32", device=0):
    return _ctx(device).radiation_eval(chi, precision)


def _with_theta(params, theta):
    p = dict(params)
    for name, v in zip(PARAM_NAMES, theta.detach().to("cpu", dtype=_torch().float64).tolist()):
        p[name] = v
    return p


def _energy_hist_fn():
    torch = _torch()

    class EnergyHistogram(torch.autograd.Function):
        """H(theta): the energy histogram (n_e + 2 raw weights) of one shot as a
        function of theta = the PARAM_NAMES values.  The forward records the
        derivative tape; the backward contracts it with dL/dH on the device."""

        @staticmethod
        def forward(fctx, theta, qctx, params):
            p = _with_theta(params, theta)
            tape = qctx.new_tape(p["n_samples"])
            fctx.qctx, fctx.p, fctx.tape = qctx, p, tape
            fctx.theta_meta = (theta.dtype, theta.device)
            return qctx.forward(p, tape=tape)["energy_hist"]

        @staticmethod
        def backward(fctx, grad_h):
            g = fctx.qctx.backward(fctx.p, grad_h, tape=fctx.tape)
            dtype, device = fctx.theta_meta
            return g.to(device=device, dtype=dtype), None, None

    return EnergyHistogram


_fn_cache = []


def energy_histogram(theta, params, context=None, device=0):
    """Differentiable energy histogram: theta (8 values, PARAM_NAMES order)
    overrides those entries of ``params``."""
    if not _fn_cache:
        _fn_cache.append(_energy_hist_fn())
    return _fn_cache[0].apply(theta, context or _ctx(device), params)


def _spectra_fn():
    torch = _torch()

    class Spectra(torch.autograd.Function):
        """(H, T, M)(theta): the energy histogram, the angle histogram and the
        moments of one shot as functions of theta = the PARAM_NAMES values.
        The forward records the derivative tape; the backward contracts it
        with dL/dH, dL/dT and dL/dM on the device (the weight, the largest chi
        and the FP64-shadow moments have no derivative)."""

        @staticmethod
        def forward(fctx, theta, qctx, params):
            p = _with_theta(params, theta)
            tape = qctx.new_tape(p["n_samples"])
            out = qctx.forward(p, tape=tape)
            fctx.qctx, fctx.p, fctx.tape, fctx.moments = qctx, p, tape, out["moments"]
            fctx.theta_meta = (theta.dtype, theta.device)
            return out["energy_hist"], out["angle_hist"], out["moments"]

        @staticmethod
        def backward(fctx, grad_h, grad_t, grad_m):
            g = fctx.qctx.backward(fctx.p, grad_h, tape=fctx.tape, d_angle=grad_t,
                                   d_moments=grad_m, moments=fctx.moments)
            dtype, device = fctx.theta_meta
            return g.to(device=device, dtype=dtype), None, None

    return Spectra


_spectra_cache = []


def spectra(theta, params, context=None, device=0):
    """Differentiable (energy histogram, angle histogram, moments): theta (8
    values, PARAM_NAMES order) overrides those entries of ``params``."""
    if not _spectra_cache:
        _spectra_cache.append(_spectra_fn())
    return _spectra_cache[0].apply(theta, context or _ctx(device), params)
