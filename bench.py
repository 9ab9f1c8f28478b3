"""Throughput of the beam-phase-space integration on one MI355X.

One step = one full forward pass (sample generation, phase integration,
deposit, reductions, normalisation) of the focused single-shot workload:
a0 = 50, W0 = 3 um, 30 fs, beam 3 um x 5 um, gamma0 = 2000 +- 5 %, 1 mrad,
2^22 samples x 1024 phase steps, quantum-corrected moments, local amplitude.

Prints one JSON line.  The roofline block describes the phase-integration
kernel (the dominant one): algorithmic FLOPs per launch over its average
duration, timed with HIP events on the stream it runs on.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sample·phase-steps/s (fwd, fwd+adjoint), batched spectra/s; % FP32 VALU peak"
UNIT = "sample·phase-steps/s"
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
# launch choices found by the tuner on this machine type, one line per class
DEFAULT_TUNE_CACHE = os.path.join(ROOT, "paper_2308_09348_amd", "tune_cache.txt")

# Algorithmic floating-point operations per sample-step of the phase loop:
# the oracle's own operation tally (oracle/flop_table.py writes the table; it
# is read here as data).
FLOP_TABLE = os.path.join(ROOT, "oracle", "flop_table.json")


def alg_flops(rr, amp):
    with open(FLOP_TABLE) as f:
        return float(json.load(f)["modes"][f"{rr}/{amp}"]["per_sample_step"])


PROFILE = os.path.join(ROOT, "profiles", "phase_kernel_focused_2p22.md")
# the forward kernels and the device helpers they use
KERNEL_SRC = [os.path.join(ROOT, "paper_2308_09348_amd", "csrc", f)
              for f in ("qs_kernels.hip", "qs_device.h")]


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def profile_values():
    """The machine-readable block of the committed phase-kernel profile
    (rocprofv3 average duration, HBM traffic, hardware-counted FP32 FLOPs per
    sample-step), or {} when the kernel source changed since it was taken."""
    try:
        kv = {}
        for line in open(PROFILE):
            parts = line.split()
            if len(parts) == 2:
                kv[parts[0]] = parts[1]
        if kv.get("kernel_source_sha256") != kernel_source_sha256():
            return {}
        return {k: float(v) for k, v in kv.items() if k != "kernel_source_sha256"}
    except (OSError, ValueError):
        return {}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--chi-fp64", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2,
                    help="timed launches of the 4096-shot batch (0 skips that leg)")
    ap.add_argument("--adjoint-steps", type=int, default=3,
                    help="timed forward+adjoint steps on the differentiation workload (0: skip)")
    ap.add_argument("--quantum-batch-steps", type=int, default=1,
                    help="timed steps of the quantum batch with gradients and photon spectra "
                         "(0: skip)")
    ap.add_argument("--mixed-steps", type=int, default=5,
                    help="timed passes of the focused workload with FP64 steps where chi > 0.1 "
                         "(0: skip)")
    ap.add_argument("--factorised-steps", type=int, default=10,
                    help="steps of the plane-wave reconstruction leg (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=4.0,
                    help="target wall time of one run of the CPU-oracle sample (median of 3)")
    ap.add_argument("--cpu-other-seconds", type=float, default=3.0,
                    help="target wall time of one run of each other workload's CPU-oracle "
                         "sample (median of 3; 0 skips them)")
    ap.add_argument("--tune-cache", default=os.environ.get("QS_TUNE_CACHE", DEFAULT_TUNE_CACHE),
                    help="launch-tuning cache file of the batched leg (read, else timed and "
                         "appended)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this size (the "
                         "reference kernel for scaling HBM byte counters)")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _median_time(fn, reps=3):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def _oracle():
    from oracle import build as obuild, qso
    if not os.path.exists(qso.LIB_PATH):
        obuild.build()
    return qso


def _prefix(run, n_max, target_s, start):
    """Grow a sample prefix until one run of it takes about target_s."""
    n = start
    while True:
        t0 = time.perf_counter()
        run(n)
        dt = time.perf_counter() - t0
        if dt > 0.25 * target_s or n >= n_max:
            break
        n = min(n * 4, n_max)
    return int(max(1, min(n_max, n * target_s / max(dt, 1e-3))))


def cpu_baseline(params, target_s):
    """The FP64 oracle on a bounded prefix of the focused workload, all host
    threads; sample-steps per second, median of 3 runs."""
    qso = _oracle()
    threads = min(os.cpu_count() or 1, 64)
    qso.forward(dict(params, n_samples=threads), 0, threads, threads)  # builds the g/h table
    run = lambda n: qso.forward(dict(params, n_samples=n), 0, n, threads)
    n = _prefix(run, params["n_samples"], target_s, 4 * threads)
    dt = _median_time(lambda: run(n))
    return {"value": n * params["n_steps"] / dt, "unit": UNIT, "cores": threads,
            "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"first {n} of {params['n_samples']} samples x {params['n_steps']} steps "
                      f"(median of 3 runs, {dt:.2f} s each, FP64, {threads} threads)"}


def cpu_baselines(workloads, target_s):
    """The oracle on bounded samples of the other workloads (median of 3 runs
    each, all host threads): the 1D plane wave in full, the 4096-shot batch
    (its first 64 shots, a prefix of each), the differentiation workload
    (forward and the dual-number gradient of the energy histogram) and the
    quantum batch (its first 16 shots: forward, gradient and photon spectrum
    with angular moments, a prefix of each); sample-steps per second of the
    work done, and the time the whole workload would take at that rate."""
    qso = _oracle()
    threads = min(os.cpu_count() or 1, 64)
    out = {"cores": threads, "cpu": cpu_model(), "nproc": os.cpu_count(), "kind": "oracle"}
    p1 = workloads.plane_wave_1d()
    dt = _median_time(lambda: qso.forward(p1, 0, p1["n_samples"], threads))
    out["plane_wave_1d"] = {"value": p1["n_samples"] * p1["n_steps"] / dt, "unit": UNIT,
                            "sample": f"all {p1['n_samples']} samples x {p1['n_steps']} steps",
                            "s": dt}
    shots = workloads.batched_shots()[:64]
    total_b = sum(s["n_samples"] for s in workloads.batched_shots())
    qso.forward(dict(shots[0], n_samples=threads), 0, threads, threads)

    def run_b(n):
        for s in shots:
            m = min(n, s["n_samples"])
            qso.forward(dict(s, n_samples=m), 0, m, threads)
    n = _prefix(run_b, 1 << 18, target_s, threads)
    dt = _median_time(lambda: run_b(n))
    work = sum(min(n, s["n_samples"]) for s in shots) * shots[0]["n_steps"]
    rate = work / dt
    out["batched"] = {"value": rate, "unit": UNIT,
                      "sample": f"first 64 of 4096 shots, first {n} samples of each x "
                                f"{shots[0]['n_steps']} steps",
                      "extrapolated_batch_s": total_b * shots[0]["n_steps"] / rate,
                      "extrapolated_spectra_per_s": 4096 / (total_b * shots[0]["n_steps"] / rate)}
    pd = workloads.differentiation_eval()

    def run_d(n):
        q = dict(pd, n_samples=n)
        qso.forward(q, 0, n, threads)
        qso.grad(q, 0, n, threads)
    n = _prefix(run_d, pd["n_samples"], target_s, threads)
    dt = _median_time(lambda: run_d(n))
    out["differentiation"] = {
        "value": n * pd["n_steps"] / dt, "unit": "sample·phase-steps/s (fwd+adjoint)",
        "sample": f"first {n} of {pd['n_samples']} samples x {pd['n_steps']} steps: forward "
                  "and the dual-number gradient",
        "extrapolated_step_s": pd["n_samples"] * pd["n_steps"] / (n * pd["n_steps"] / dt)}
    qshots = workloads.quantum_batch()[:16]
    qtotal = sum(s["n_samples"] for s in workloads.quantum_batch())

    def run_q(n):
        for s in qshots:
            q = dict(s, n_samples=n)
            qso.forward(q, 0, n, threads)
            qso.grad(q, 0, n, threads)
            qso.photons(q, q["n_ph"], q["ph_lo"], q["ph_hi"], 0, n, threads)
            qso.photon_angles(q, 0, n, threads)
    n = _prefix(run_q, 1 << 18, target_s, threads)
    dt = _median_time(lambda: run_q(n))
    rate = 16 * n * qshots[0]["n_steps"] / dt
    out["quantum_batch"] = {
        "value": rate, "unit": "sample·phase-steps/s (spectra, gradients, photons)",
        "sample": f"first 16 of 256 shots, first {n} samples of each x {qshots[0]['n_steps']} "
                  "steps: forward, dual-number gradient, photon spectrum and angular moments",
        "extrapolated_step_s": qtotal * qshots[0]["n_steps"] / rate}
    return out


def adjoint_leg(ctx, qs, workloads, torch, steps):
    """Forward + adjoint on the differentiation workload: a Neyman chi^2 loss
    against a Poisson target drawn from the histogram at the reference
    parameters, evaluated at perturbed parameters.  One step = forward pass
    recording the derivative tape, loss, upstream weights, adjoint from the
    tape (all on the device).  The parts are also timed alone, with the
    adjoint that integrates the trajectories again instead of reading a tape."""
    ref = workloads.differentiation()
    p = workloads.differentiation_eval()
    n, N = p["n_samples"], p["n_steps"]
    n_tot = 1e6
    h_ref = ctx.forward(ref)["energy_hist"].cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(4))
    target = torch.tensor(rng.poisson(n_tot * h_ref / n).astype(np.float64), device="cuda")
    denom = torch.clamp(target, min=1.0)
    tape = ctx.new_tape(n)
    out = ctx.forward(p, tape=tape)

    def step():
        h = ctx.forward(p, out=out, tape=tape, check=False)["energy_hist"]
        r = n_tot * h / n - target
        loss = (r * r / denom).sum()
        w = 2.0 * r / denom * (n_tot / n)
        g = ctx.backward(p, w, tape=tape, check=False)
        return loss, g, w

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    res = {}
    fwd = lambda: ctx.forward(p, out=out, check=False)
    # the step and the plain forward pass timed in alternating rounds, so that
    # both see the same clock state of the device (kernel durations drift by
    # several percent over a few seconds of load)
    fn_step = lambda: res.update(zip(("loss", "g", "w"), step()))
    dts, fwds = [], []
    for r in range(5):  # the first round warms the device up and is not kept
        dt_r, fwd_r = timed(fn_step), timed(fwd)
        if r > 0:
            dts.append(dt_r)
            fwds.append(fwd_r)
    dt, t_fwd = float(np.mean(dts)), float(np.mean(fwds))
    if int(out["status"].item()) != 0:
        raise RuntimeError("device status in the adjoint leg")
    w = res["w"]
    t_tape = timed(lambda: ctx.forward(p, out=out, tape=tape, check=False))
    t_contract = timed(lambda: ctx.backward(p, w, tape=tape, check=False))
    t_recompute = timed(lambda: ctx.backward(p, w, check=False))
    g = res["g"].cpu().numpy()
    if not np.all(np.isfinite(g)):
        raise RuntimeError("non-finite gradient in the adjoint leg")
    return {"workload": "differentiation: focused-shot physics, GAUSS deposit (1 bin), 2^20 "
                        "samples x 1024 steps, quantum, local amplitude; Neyman chi^2 loss vs a "
                        "Poisson target (1e6 counts) at parameters perturbed by 5%",
            "n_samples": n, "n_steps": N, "steps": steps, "ms_per_step": 1e3 * dt,
            "fwd_ms": 1e3 * t_fwd, "fwd_tape_ms": 1e3 * t_tape,
            "adjoint_from_tape_ms": 1e3 * t_contract,
            "adjoint_recompute_ms": 1e3 * t_recompute,
            "step_over_fwd": dt / t_fwd, "rounds": len(dts),
            "step_over_fwd_by_round": [a / b for a, b in zip(dts, fwds)],
            "sample_steps_per_s": n * N / dt, "loss": float(res["loss"]),
            "grad": dict(zip(qs.PARAM_NAMES, [float(x) for x in g]))}


FP64_VALU_PEAK_TFLOPS = 78.6  # MI355X published FP64 vector peak


def mixed_peak(fp64_share):
    """The VALU ceiling of a pass that takes the given share of its phase
    steps in FP64 (at half the FP32 rate) and the rest in FP32."""
    return 1.0 / (fp64_share / FP64_VALU_PEAK_TFLOPS + (1.0 - fp64_share) / FP32_VALU_PEAK_TFLOPS)


def quantum_batch_leg(ctx, workloads, torch, steps, tune_cache=None):
    """256 shots of 2^18 samples x 2048 steps, quantum (FP64 steps where
    chi > 0.1).  One training step: the forward pass that records the
    derivative tape (it deposits the electron spectra too), per-shot Neyman
    chi^2 losses against Poisson targets and their upstream weights, the
    adjoint from the tape, and the photon spectra with angular moments -- all
    shots in one launch per stage.  The plain forward pass of the batch (the
    spectra alone) is timed beside it for its roofline and its share of FP64
    steps."""
    shots = workloads.quantum_batch()
    total = sum(p["n_samples"] for p in shots)
    N = shots[0]["n_steps"]
    batch = ctx.prepare_batch(shots)
    # launch choices of the forward pass from the tuner cache (tuned once if
    # the class is not there)
    tuning = ctx.tune(batch, cache_path=tune_cache) if tune_cache else None
    tape = ctx.new_tape(total)
    n_tot = 1e6
    ref = ctx.run_batch(batch)
    rng = np.random.Generator(np.random.PCG64(5))
    targets = [torch.tensor(rng.poisson(n_tot * o["energy_hist"].cpu().numpy() / p["n_samples"])
                            .astype(np.float64), device="cuda") for o, p in zip(ref, shots)]
    share = float(np.mean([o["moments"][20].item() for o in ref]))
    parts = {}

    def step():
        t = [time.perf_counter()]
        tout = ctx.run_batch(batch, check=False, tape=tape)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        ws = []
        for o, p, tg in zip(tout, shots, targets):
            r = n_tot * o["energy_hist"] / p["n_samples"] - tg
            ws.append(2.0 * r / torch.clamp(tg, min=1.0) * (n_tot / p["n_samples"]))
        grads = ctx.backward_batched(shots, ws, check=False, tape=tape)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        phot = ctx.photons_batched(shots, check=False, angles=True)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        for k, name in enumerate(("tape_forward", "adjoint", "photons")):
            parts[name] = parts.get(name, 0.0) + t[k + 1] - t[k]
        return tout, grads, phot

    step()  # warm-up
    parts.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        outs, grads, phot = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    bad = int(torch.stack([o["status"] for o in outs] + [o["status"] for o in phot]).max().item())
    if bad != 0:
        raise RuntimeError(f"device status {bad} in the quantum batch leg")
    g = torch.stack(grads).cpu().numpy()
    if not np.all(np.isfinite(g)):
        raise RuntimeError("non-finite gradient in the quantum batch leg")
    # the plain forward pass of the batch: its phase kernel against the
    # mixed FP32/FP64 ceiling
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.run_batch(batch, check=False)
    torch.cuda.synchronize()
    fwd_s = time.perf_counter() - t1
    phase_ms = ctx.last_timings()["phase"]
    ctx.set_profiling(False)
    flops = alg_flops("quantum", "local") * total * N
    peak = mixed_peak(share)
    achieved = flops / (phase_ms * 1e-3) / 1e12
    return {"workload": "256 shots: gamma0 N(2e4, 600^2), a0 U[50,150], W0 2um, no offsets, "
                        "2^18 samples x 2048 steps, quantum with FP64 steps where chi > 0.1, "
                        "local amplitude; one training step: electron spectra with the derivative "
                        "tape, per-shot gradients of chi^2 losses, 256-bin photon spectra with "
                        "photon angular moments",
            "n_shots": len(shots), "n_samples": total, "n_steps": N, "steps": steps,
            "ms_per_step": 1e3 * dt,
            "ms_parts": {k: 1e3 * v / steps for k, v in parts.items()},
            "sample_steps_per_s": total * N / dt, "spectra_per_s": len(shots) / dt,
            "fp64_step_share": share,
            "forward_ms": 1e3 * fwd_s,
            # the batched forward pass with its adjoint (the tape-recording
            # forward and the adjoint from the tape) over the plain batched forward
            "fwd_adjoint_over_fwd": (parts["tape_forward"] + parts["adjoint"]) / steps / fwd_s,
            "roofline": {"bound": "alu", "kernel": "phase_kernel (FP32 with FP64 steps)",
                         "kernel_avg_ms": phase_ms, "achieved": achieved, "peak": peak,
                         "unit": "TFLOP/s", "frac": achieved / peak,
                         "peak_rule": "time-weighted: FP64 steps at 78.6, FP32 at 157.3 TFLOP/s"},
            "tuning": tuning}


def factorised_leg(ctx, workloads, torch, steps):
    """The focused workload in A0EFF mode (2^22 samples x 1024 steps, quantum,
    FP32): the direct pass against the plane-wave reconstruction on a 61 x 64
    (a0,eff, gamma0) node grid, both timed over whole passes."""
    p = dict(workloads.focused_3d(), amp_mode="a0eff")
    n, N = p["n_samples"], p["n_steps"]
    K, M = 61, 64
    out = ctx.forward(p)
    batch = ctx.prepare_factorised([p], K, M)
    fact = ctx.run_factorised(batch, single=True)[0]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_direct = timed(lambda: ctx.forward(p, out=out, check=False))
    t_fact = timed(lambda: ctx.run_factorised(batch, check=False, single=True))
    ctx.set_profiling(True)
    ctx.run_factorised(batch, check=False, single=True)
    parts = ctx.last_timings()
    ctx.set_profiling(False)
    for o in (out, fact):
        if int(o["status"].item()) != 0:
            raise RuntimeError("device status in the reconstruction leg")
    hd, hf = out["energy_hist"].cpu().numpy(), fact["energy_hist"].cpu().numpy()
    md, mf = out["moments"].cpu().numpy(), fact["moments"].cpu().numpy()
    return {"workload": "focused single shot in A0EFF mode (2^22 samples x 1024 steps, quantum, "
                        "FP32, CIC); plane-wave reconstruction on 61 a0,eff x 64 gamma0 nodes",
            "n_samples": n, "n_steps": N, "nodes": K * M, "steps": steps,
            "direct_ms": 1e3 * t_direct, "factorised_ms": 1e3 * t_fact,
            "speedup": t_direct / t_fact,
            "ms_parts": {"node_runs": parts["phase"], "interpolation": parts["deposit"],
                         "deposit_finalize": parts["finalize"]},
            "equivalent_sample_steps_per_s": n * N / t_fact,
            "l1_vs_direct": float(np.abs(hf - hd).sum() / n),
            "mean_gamma_rel_diff": float(abs(mf[1] - md[1]) / md[1])}


def note(msg):
    """A progress line on stderr as each leg ends (stdout holds the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2308_09348_amd as qs
    from paper_2308_09348_amd import _lib, workloads

    build_id = _lib.check_build()  # the library was built from these sources
    params = dict(workloads.focused_3d(), precision=args.precision, chi_fp64=args.chi_fp64)
    n, N = params["n_samples"], params["n_steps"]
    ctx = qs.Context(0)
    dev = torch.device("cuda", 0)
    # launch choices for this class (read from the cache, else timed there)
    tuning = ctx.tune(params, cache_path=args.tune_cache)
    out = ctx.forward(params)  # allocates the outputs and the context scratch
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        ctx.forward(params, out=out, check=False)
    torch.cuda.synchronize()

    # timed region: K whole forward passes, inputs resident, outputs reused
    # (the kernels' events are kept per call and read after the region)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.forward(params, out=out, stream=stream, check=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_timed, ms_sum = ctx.timings_sum()
    ctx.set_profiling(False)
    st = int(out["status"].item())
    if st != 0:
        raise RuntimeError(f"device status {st}")

    ms_per_step = 1e3 * wall / args.steps
    value = n * N / (wall / args.steps)
    note(f"forward: {ms_per_step:.3f} ms per pass")
    phase_avg_ms = ms_sum["phase"] / n_timed
    flops_step = alg_flops(params["rr_model"], params["amp_mode"])
    flops_launch = flops_step * n * N
    achieved = flops_launch / (phase_avg_ms * 1e-3) / 1e12
    prof = profile_values() if args.precision == "fp32" and args.chi_fp64 <= 0 else {}
    peak = FP32_VALU_PEAK_TFLOPS
    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "focused single shot: a0=50, W0=3um, 30fs, x_off=2um, delay=10fs, "
                               "sigma_r=3um, sigma_z=5um, gamma0=2000+-5%, 1mrad; 2^22 samples x "
                               "1024 steps, quantum moments, local amplitude, CIC deposit",
                   "n_samples": n, "n_steps": N, "rr_model": params["rr_model"],
                   "amp_mode": params["amp_mode"], "precision": args.precision,
                   "chi_fp64": args.chi_fp64, "leg": "fwd"},
        "build_id": build_id,
        "tuning": tuning,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": prof.get("phase_kernel_traffic_bytes"),
                     "kernel": "phase_kernel",
                     "kernel_avg_ms": phase_avg_ms,
                     "alg_flops_per_sample_step": flops_step,
                     "alg_flops_source": "oracle/flop_table.json (the oracle's operation tally)",
                     # the same FLOPs over the committed rocprofv3 average of the kernel
                     "kernel_avg_ms_rocprof": prof.get("phase_kernel_avg_ms"),
                     "frac_rocprof": (flops_launch / (prof["phase_kernel_avg_ms"] * 1e-3) / 1e12
                                      / peak if "phase_kernel_avg_ms" in prof else None),
                     # FP32 operations the hardware counted (rocprofv3 VALU classes, FMA = 2)
                     "hw_flops_per_sample_step": prof.get("hw_flops_per_sample_step"),
                     "frac_hw": (prof["hw_flops_per_sample_step"] * n * N /
                                 (phase_avg_ms * 1e-3) / 1e12 / peak
                                 if "hw_flops_per_sample_step" in prof else None),
                     # the algorithmic FLOPs over the whole pass (every kernel of a step)
                     "frac_whole_pass": flops_launch / (ms_per_step * 1e-3) / 1e12 / peak},
    }
    # the same workload with FP64 steps where chi > 0.1 (the stability rule):
    # its phase kernel against the mixed FP32/FP64 ceiling
    if args.chi_fp64 <= 0 and args.precision == "fp32" and args.mixed_steps > 0:
        pm = dict(params, chi_fp64=0.1)
        om = ctx.forward(pm)
        share = float(om["moments"][20].item())
        ctx.set_profiling(True)
        mixed_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.mixed_steps):
            ctx.forward(pm, out=om, stream=stream, check=False)
            mixed_ms.append(ctx.last_timings()["phase"])
        torch.cuda.synchronize()
        wall_m = (time.perf_counter() - t0) / args.mixed_steps
        ctx.set_profiling(False)
        k_ms = sum(mixed_ms) / len(mixed_ms)
        pk = mixed_peak(share)
        ach = flops_launch / (k_ms * 1e-3) / 1e12
        note(f"forward at chi_fp64 = 0.1: {1e3 * wall_m:.3f} ms per pass")
        line["fwd_chi_fp64_0p1"] = {
            "chi_fp64": 0.1, "fp64_step_share": share, "ms_per_step": 1e3 * wall_m,
            "sample_steps_per_s": n * N / wall_m, "kernel_avg_ms": k_ms,
            "roofline": {"achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
                         "peak_rule": "time-weighted: FP64 steps at 78.6, FP32 at 157.3 TFLOP/s"}}
    # FP64 shadow of the same pass (untimed above): every 64th sample again in
    # FP64, the FP32 pass's per-sample error against it
    pv = dict(params, validate_fp64=True, shadow_stride=64)
    ctx.forward(pv, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv = ctx.forward(pv)
    torch.cuda.synchronize()
    mv = sv["moments"].cpu().numpy()
    line["fp64_shadow"] = {
        "shadow_stride": 64, "samples": int(mv[11]), "ms_per_pass": 1e3 * (time.perf_counter() - t0),
        "err_mu_max": float(mv[12]), "err_mu_mean": float(mv[13]), "err_sig_max": float(mv[14]),
        "err_mean_gamma": float(mv[15]), "err_energy_hist_l1": float(mv[16]),
        "err_energy_hist_max_bin": float(mv[17]), "err_angle_hist_l1": float(mv[18]),
        "err_angle_hist_max_bin": float(mv[19])}
    if args.batched_steps > 0:
        # batched leg: 4096 shots of uneven size in one launch, with the launch
        # choices of the tuner (cached per device and launch class) and the
        # launch replayed from a HIP graph
        shots = workloads.batched_shots()
        batch = ctx.prepare_batch(shots)
        tuning = ctx.tune(batch, cache_path=args.tune_cache)
        ctx.set_graphs(True)
        ctx.run_batch(batch)  # scratch allocation, graph capture and warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            ctx.run_batch(batch, check=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.batched_steps
        bad = int(torch.stack([o["status"] for o in batch.out]).max().item())
        if bad != 0:
            raise RuntimeError(f"device status {bad} in the batched leg")
        n_tot = sum(p["n_samples"] for p in shots)
        note(f"batched: {1e3 * dt:.1f} ms per batch")
        line["batched"] = {
            "workload": "4096 shots, samples log-uniform in [2^12, 2^18], a0 U[5,100], "
                        "W0 U[2,6]um, offsets N(0,2^2)um, delay N(0,15^2)fs, gamma0 "
                        "U[1e3,1e4], sigma_gamma 1-10%; 512 steps, quantum, local amplitude",
            "n_shots": len(shots), "n_samples": n_tot, "n_steps": shots[0]["n_steps"],
            "steps": args.batched_steps, "ms_per_batch": 1e3 * dt,
            "spectra_per_s": len(shots) / dt,
            "sample_steps_per_s": n_tot * shots[0]["n_steps"] / dt,
            "tuning": tuning, "hip_graph": True}
        ctx.set_graphs(False)
    if args.factorised_steps > 0:
        line["factorised"] = factorised_leg(ctx, workloads, torch, args.factorised_steps)
        note("factorised leg done")
    if args.adjoint_steps > 0:
        line["adjoint"] = adjoint_leg(ctx, qs, workloads, torch, args.adjoint_steps)
        note("adjoint leg done")
    if args.quantum_batch_steps > 0:
        line["quantum_batch"] = quantum_batch_leg(ctx, workloads, torch, args.quantum_batch_steps,
                                                  args.tune_cache)
        note(f"quantum batch: {line['quantum_batch']['ms_per_step']:.0f} ms per step")
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = nb
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(params, args.cpu_seconds)
        note("CPU baseline of the forward workload done")
        if args.cpu_other_seconds > 0:
            line["cpu_baselines"] = cpu_baselines(workloads, args.cpu_other_seconds)
            note("CPU baselines of the other workloads done")
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
