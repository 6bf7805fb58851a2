#!/usr/bin/env python
"""Throughput of one minSR iteration on one MI355X.

Workload (the metric's configuration): 1D transverse-field Ising chain,
N = 64, periodic, J = h = 1; 1D GRU pRNN with d_h = 64 (13058 parameters);
N_s = 1024 samples with N + 1 connected configurations each; regularised
minSR step with lambda = 1e-3, eta = 0.05, momentum 0.7.  The timed region is
a training run of K consecutive steps from the seeded initialisation; the
energy of every step is kept on the device.  Reported per form: E/N - E0/N
(closed-form ground energy) averaged over the last 100 steps with its
standard error, and between the two forms the difference of those averages
(the equal-energy condition of the metric).

value: steps/s of the BF16 + FP64 form (BF16 O'/Gram on MFMA with FP32
accumulation, FP64 reductions, solve and update; FP32 recurrence).  The
plain FP32 form is timed the same way and reported beside it.

The timed steps replay a captured hip graph of the step (the Philox
counter lives in device memory and advances on every replay).  Per-kernel
times come from HIP events the library records on the step's stream over
further eager steps of the same run; `roofline` is given for the kernel
with the largest share of the step.  `cpu_baseline` times the FP64 CPU
oracle on one full step of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("minSR steps/sec at fixed ΔE/N; Jacobian GB/s & Gram MFMA util vs peak")
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6         # dense FP64 matrix cores (equal to the FP64 vector peak)

# traffic measured with rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE) per launch,
# scaled by the counter's reading on a plain copy of known size; None until
# taken for the current kernel version
TRAFFIC_BYTES = {
    # k_eloc_mfma_w (FP16 hi/lo split products): 10006.6 KiB fetched x 2.000 +
    # 1371.7 KiB written x 1.000
    "eloc": 10006.6 * 1024 * 2.0 + 1371.7 * 1024,
    # k_chol_prep + k_chol_persist_f64 + k_trsv_back_mt:
    # (78.2 + 9287.3 + 2254.3) KiB fetched x 2.000 + (17.4 + 4692.5 + 8.5) KiB written
    "solve": (78.2 + 9287.3 + 2254.3) * 1024 * 2.0 + (17.4 + 4692.5 + 8.5) * 1024,
    # k_jacobian (gate-tape path, gate adjoints stored per site) + k_jac_wgrad:
    # (42359.0 + 33373.7) KiB fetched x 2.000 + (55328.0 + 50254.2) KiB written x 1.000
    "jacobian": (42359.0 + 33373.7) * 1024 * 2.0 + (55328.0 + 50254.2) * 1024,
    # k_gram_bf16 (split form, four products, eight-wave 128 x 128 tiles, FP64
    # partial tiles): 43333.6 KiB fetched x 2.000 + 32256.0 KiB written x 1.000
    "gram": 43333.6 * 1024 * 2.0 + 32256.0 * 1024}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 form")
    ap.add_argument("--eager", action="store_true", help="time eager steps instead of graph replays")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the short timings of the cluster100, heis10x10 and J1-J2 batch "
                         "systems")
    ap.add_argument("--only-workload", default="", metavar="NAME",
                    help="only time NAME (tfim64, cluster100 or heis10x10: a few BF16 + FP64 steps "
                         "with per-phase events; for profiler runs), print its JSON, exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (for scaling the HBM "
                         "traffic counters of a profiler run), then exit")
    return ap.parse_args()


def work_units(wl):
    """Algorithmic work per launch of the three graded kernels."""
    N, H, Ns = wl.Lx * wl.Ly, wl.H, wl.Ns
    Np = 3 * H * H + 4 * 2 * H + 4 * H + 2      # 1D pRNN, local dimension 2
    seq_sites = Ns * N * (N - 1) // 2           # flip at k re-runs sites k+1..N-1
    return dict(
        Np=Np,
        # GRU gate products (3 H x H) and the two logits per re-evaluated site
        eloc_flop=seq_sites * (6 * H * H + 4 * H),
        # the Jacobian's algorithmic bytes: O written once in FP32 (Ns rows
        # of Np) plus the stored hidden states read once (H per site, FP32)
        jacobian_bytes=Ns * Np * 4 + Ns * N * H * 4,
        # the same with the sampler's gate tape (4 H per site), which this
        # implementation also reads back instead of recomputing the gates
        jacobian_bytes_with_tape=Ns * Np * 4 + Ns * N * 5 * H * 4,
        # useful flops of the symmetric Gram: n (n + 1) Np
        gram_flop=Ns * (Ns + 1) * Np,
        # Cholesky of the n x n system (n^3 / 3) and its two triangular solves
        solve_flop=Ns ** 3 / 3 + 2 * Ns * Ns,
    )


def run_form(pm, wl, form, K, W, dtype="f32", graph=True, kernel_steps=20):
    """W warmup steps, then the timed run of K steps (replays of a captured
    graph of the step, or eager steps), then `kernel_steps` eager steps with
    per-phase HIP events for the kernel breakdown."""
    import numpy as np
    import torch
    ham = pm.hamiltonian("tfim", J=wl.J, h=wl.h, pbc=wl.pbc)
    m = pm.Model(wl.Lx, wl.Ly, wl.dim, wl.H, wl.complex_head, wl.marshall, wl.zero_mag,
                 dtype=dtype, seed=wl.seed, max_Ns=wl.Ns)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    outs = m.step_outputs(wl.Ns)
    # E, Var, the third energy slot and the status word side by side, so one
    # copy per step records them
    rec = torch.zeros(4, dtype=torch.float64, device="cuda")
    outs["energy"] = rec[0:3]
    outs["status"] = rec[3:4].view(torch.int32)[0:1]
    hist = torch.zeros((max(K, 1), 4), dtype=torch.float64, device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")

    def eager():
        m.step(ham, wl.Ns, wl.eta, wl.lam, wl.mu, mom, wl.key, 0, form=form,
               ckpt_every=wl.ckpt_every, outputs=outs, dev_counter=ctr)

    for _ in range(W):
        eager()
    g = None
    if graph:
        g, _ = m.capture_step(ham, wl.Ns, wl.eta, wl.lam, wl.mu, mom, wl.key, ctr, form=form,
                              ckpt_every=wl.ckpt_every, outputs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        if g is not None:
            g.replay()
        else:
            eager()
        hist[i].copy_(rec, non_blocking=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel breakdown: eager steps with events on the step's stream
    m.timing_begin(kernel_steps)
    for _ in range(kernel_steps):
        eager()
    torch.cuda.synchronize()
    phases, nrec = m.timing_read()
    hr = hist.cpu().numpy()
    E = hr[:, :3].copy()
    st = hr[:, 3].copy().view(np.int32)[0::2]   # the status word is the low half of its slot
    m.close()
    return dict(seconds=t1 - t0, phases={k: v / max(nrec, 1) for k, v in phases.items()},
                energy=E, status=st, kernel_steps=nrec)


TARGET_DE = 1e-4      # |Delta E / N| of the metric
WINDOW = 50           # steps averaged for the energy at a step


def convergence_leg(pm, wl, form, K=500):
    """K graph-replayed steps of the workload from the seeded init in one
    form, with every step's energy, status word and shift kept on the
    device.  Reports the first step at which the mean of E/N - E0/N over
    the last WINDOW steps lies within TARGET_DE, the time to that step at
    the leg's measured step time, the failure and shift-floor counts and
    the mean over the last 100 steps with its standard error."""
    import numpy as np
    import torch
    ham = pm.hamiltonian("tfim", J=wl.J, h=wl.h, pbc=wl.pbc)
    m = pm.Model(wl.Lx, wl.Ly, wl.dim, wl.H, wl.complex_head, wl.marshall, wl.zero_mag,
                 dtype="f32", seed=wl.seed, max_Ns=wl.Ns)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    outs = m.step_outputs(wl.Ns)
    g, _ = m.capture_step(ham, wl.Ns, wl.eta, wl.lam, wl.mu, mom, wl.key, ctr, form=form,
                          ckpt_every=wl.ckpt_every, outputs=outs)
    hist = torch.zeros((K, 3), dtype=torch.float64, device="cuda")
    status = torch.zeros(K, dtype=torch.int32, device="cuda")
    lam = torch.zeros(K, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        g.replay()
        hist[i].copy_(outs["energy"], non_blocking=True)
        status[i:i + 1].copy_(outs["status"], non_blocking=True)
        lam[i:i + 1].copy_(outs["lambda_used"], non_blocking=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    tn = float(outs["tnorm"].item())
    m.close()
    del g
    N = wl.Lx * wl.Ly
    dE = hist.cpu().numpy()[:, 0] / N - wl.E0 / N
    st = status.cpu().numpy()
    lam = lam.cpu().numpy()
    win = np.convolve(dE, np.ones(WINDOW) / WINDOW, mode="valid")
    hit = np.nonzero(np.abs(win) <= TARGET_DE)[0]
    steps_to = int(hit[0] + WINDOW) if len(hit) else None
    ms = sec / K * 1e3
    tail = dE[-100:]
    return {"steps": K, "ms_per_step": ms,
            "steps_to_target": steps_to,
            "seconds_to_target": steps_to * ms * 1e-3 if steps_to else None,
            "reached_target": steps_to is not None,
            "dE_per_site_last100": [float(tail.mean()), float(tail.std() / math.sqrt(len(tail)))],
            "failed_steps": int(np.count_nonzero(st & pm.ST_ERRORS)),
            "not_pd_steps": int(np.count_nonzero(st & pm.ST_NOT_PD)),
            "shift_floor_steps": int(np.count_nonzero(st & pm.ST_SHIFT_FLOOR)),
            "lambda_used_min_max": [float(lam.min()), float(lam.max())],
            "trace_norm_T_last": tn}


def time_workload(pm, wl, steps=3):
    """One eager warmup step, then `steps` eager steps of one system in the
    BF16 + FP64 form with per-phase events; ms per step and phases."""
    import torch
    ham = pm.hamiltonian(wl.ham, J=wl.J, h=wl.h, J2=wl.J2, pbc=wl.pbc)
    m = pm.Model(wl.Lx, wl.Ly, wl.dim, wl.H, wl.complex_head, wl.marshall, wl.zero_mag,
                 dtype="f32", seed=wl.seed, max_Ns=wl.Ns, pinv=wl.pinv_cutoff > 0)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    outs = m.step_outputs(wl.Ns)
    bad = 0

    def st(i):
        m.step(ham, wl.Ns, wl.eta, wl.lam, wl.mu, mom, wl.key, i, form=pm.FORM_BF16_FP64,
               pinv_cutoff=wl.pinv_cutoff, ckpt_every=wl.ckpt_every, outputs=outs)

    st(0)
    torch.cuda.synchronize()
    m.timing_begin(steps)
    t0 = time.perf_counter()
    for i in range(steps):
        st(1 + i)
        bad += int(outs["status"].item() & pm.ST_ERRORS != 0)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ph, n = m.timing_read()
    res = {"ms_per_step": dt * 1e3, "steps": steps, "Np": m.Np, "Ns": wl.Ns,
           "N": wl.Lx * wl.Ly, "d_h": wl.H, "failed_steps": bad,
           "phase_ms": {k: v / max(n, 1) for k, v in ph.items()}}
    m.close()
    return res


def time_batch(pm, steps=2):
    """The sixteen J1-J2 instances stepped by one captured graph (each
    instance on its own stream): one warmup replay, then `steps` replays."""
    import torch
    from workloads import j1j2_batch
    insts, models = [], []
    for wl in j1j2_batch():
        m = pm.Model(wl.Lx, wl.Ly, wl.dim, wl.H, wl.complex_head, wl.marshall, wl.zero_mag,
                     dtype="f32", seed=wl.seed, max_Ns=wl.Ns)
        models.append(m)
        insts.append(dict(model=m, ham=pm.hamiltonian(wl.ham, J=wl.J, h=wl.h, J2=wl.J2,
                                                       pbc=wl.pbc),
                          Ns=wl.Ns, eta=wl.eta, lam=wl.lam, mu=wl.mu, key=wl.key,
                          form=pm.FORM_BF16_FP64))
    b = pm.Batch(insts)
    b.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    bad = sum(int(o["status"].item() & pm.ST_ERRORS != 0) for o in b.outputs)
    b.close()
    for m in models:
        m.close()
    return {"ms_per_batch_step": dt * 1e3, "instance_steps_per_s": len(insts) / dt,
            "instances": len(insts), "replays": steps, "failed_instances": bad}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl):
    """One full FP64 oracle step of the workload on the host cores (all the
    threads its numerical library uses), then one more with one thread."""
    import numpy as np
    from oracle import hamiltonian, minsr, model
    spec = model.Spec(Lx=wl.Lx, Ly=wl.Ly, dim=wl.dim, H=wl.H, complex_head=wl.complex_head,
                      marshall=wl.marshall, zero_mag=wl.zero_mag)
    th = model.glorot_init(spec, wl.seed)
    ham = hamiltonian.Ham("tfim", J=wl.J, h=wl.h, pbc=wl.pbc)
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1

    def one():
        t0 = time.perf_counter()
        minsr.step(spec, th, np.zeros_like(th), ham, wl.Ns, wl.eta, wl.lam, wl.mu, wl.key, 0)
        return time.perf_counter() - t0

    dt = one()
    dt1 = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt1 = one()
    return {"value": 1.0 / dt, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "value_1thread": (1.0 / dt1) if dt1 else None,
            "sample": "one full FP64 oracle step of the same workload (Ns=1024, N=64, d_h=64): "
                      "uniforms, sampling, local energies, Jacobian, Gram, Cholesky, update; "
                      "%.1f s with %d threads, %s s with one thread"
                      % (dt, cores, "%.1f" % dt1 if dt1 else "n/a")}


def roofline_entry(name, ms, units):
    if name == "gram":
        ach = units["gram_flop"] / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_BF16_TFLOPS, "traffic": TRAFFIC_BYTES["gram"],
                "ms": ms}
    if name == "jacobian":
        ach = units["jacobian_bytes"] / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": TRAFFIC_BYTES["jacobian"], "ms": ms,
                "bytes": units["jacobian_bytes"],
                "achieved_with_gate_tape": units["jacobian_bytes_with_tape"] / (ms * 1e-3) / 1e9}
    if name == "solve":
        # FP64 factorisation on the FP64 matrix cores; a chain of dependent
        # 64 x 64 blocks, so latency rather than throughput sets its time
        ach = units["solve_flop"] / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_TFLOPS, "traffic": TRAFFIC_BYTES["solve"], "ms": ms}
    # FP32 models evaluate the gate products on v_mfma_f32_32x32x16_f16 as
    # three FP16 hi/lo products; the algorithmic flops are those of one
    # product, priced against the FP16 peak
    ach = units["eloc_flop"] / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP16_TFLOPS, "traffic": TRAFFIC_BYTES["eloc"], "ms": ms}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                          "copies": 3}))
        return
    if args.only_workload:
        r = time_workload(pm, WORKLOADS[args.only_workload], steps=max(1, min(args.steps, 5)))
        print(json.dumps({"workload": args.only_workload, **r}), flush=True)
        return
    wl = WORKLOADS["tfim64"]
    K, W = args.steps, args.warmup
    units = work_units(wl)
    N = wl.Lx * wl.Ly

    res = run_form(pm, wl, pm.FORM_BF16_FP64, K, W, graph=not args.eager)
    print("bf16_fp64: %.3f s for %d steps" % (res["seconds"], K), file=sys.stderr, flush=True)
    ms_step = res["seconds"] / K * 1e3
    value = K / res["seconds"]
    ph = res["phases"]

    def tail_mean(E):
        tail = E[-min(100, len(E)):, 0] / N
        return float(tail.mean()), float(tail.std() / math.sqrt(len(tail)))

    def dE(E):
        mu_, se = tail_mean(E)
        return mu_ - wl.E0 / N, se

    graded = {k: roofline_entry(k, ph[k], units) for k in ("eloc", "jacobian", "gram", "solve")}
    dom = max(("sample", "eloc", "jacobian", "gram", "solve"), key=lambda k: ph[k])
    roof = graded.get(dom) or graded["eloc"]

    forms = {"bf16_fp64": {"steps_per_s": value, "ms_per_step": ms_step,
                           "dE_per_site_last100": dE(res["energy"]),
                           "failed_steps": int(np.count_nonzero(res["status"] & pm.ST_ERRORS)),
                           "shift_floor_steps": int(np.count_nonzero(res["status"]
                                                                    & pm.ST_SHIFT_FLOOR))}}
    if not args.no_fp32:
        r32 = run_form(pm, wl, pm.FORM_FP32_PLAIN, K, W, graph=not args.eager)
        print("fp32_plain: %.3f s for %d steps" % (r32["seconds"], K), file=sys.stderr, flush=True)
        forms["fp32_plain"] = {"steps_per_s": K / r32["seconds"],
                               "ms_per_step": r32["seconds"] / K * 1e3,
                               "dE_per_site_last100": dE(r32["energy"]),
                               "failed_steps": int(np.count_nonzero(r32["status"] & pm.ST_ERRORS)),
                               "phase_ms": r32["phases"]}

    if "fp32_plain" in forms:
        (a, sa), (b, sb) = tail_mean(res["energy"]), tail_mean(r32["energy"])
        forms["dE_per_site_bf16_minus_fp32"] = [a - b, math.hypot(sa, sb)]

    # the equal-energy condition of the metric, whatever --steps is: a
    # training run of 500 steps per form from the seeded initialisation
    conv = {"target_abs_dE_per_site": TARGET_DE, "window_steps": WINDOW}
    for fname, fcode in (("bf16_fp64", pm.FORM_BF16_FP64), ("fp32_plain", pm.FORM_FP32_PLAIN)):
        if fname == "fp32_plain" and args.no_fp32:
            continue
        conv[fname] = convergence_leg(pm, wl, fcode)
        print("convergence %s: %s" % (fname, json.dumps(conv[fname])), file=sys.stderr,
              flush=True)

    others = None
    if not args.no_workloads:
        others = {}
        for name in ("cluster100", "heis10x10"):
            others[name] = time_workload(pm, WORKLOADS[name])
            print("%s: %.1f ms/step" % (name, others[name]["ms_per_step"]), file=sys.stderr,
                  flush=True)
        others["j1j2batch"] = time_batch(pm)
        print("j1j2batch: %.1f ms per batch step" % others["j1j2batch"]["ms_per_batch_step"],
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl)
        print("cpu baseline: %s" % cpu["sample"], file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 hi/lo O' and Gram (fp32 accumulate, fp64 flush); fp32 recurrence "
                 "(local-energy state products as fp16 hi/lo pairs, fp32 accumulate); "
                 "fp64 reductions, solve, update",
        "data": "synthetic",
        "config": {"workload": "tfim64: 1D TFIM N=64 periodic J=h=1, 1D GRU pRNN d_h=64 "
                               "(13058 params), Ns=1024 (N+1 connected configs each), "
                               "BF16+FP64 form, lambda=1e-3, eta=0.05, mu=0.7, "
                               "training run from the seeded init",
                   "Ns": wl.Ns, "N": N, "d_h": wl.H, "Np": units["Np"]},
        "roofline": dict(roof, kernel=dom if dom in graded else "eloc"),
        "rooflines": graded,
        "phase_ms": ph,
        "timing": ("value: %d %s steps; per-kernel ms (roofline, phase_ms): HIP events on the "
                   "step's stream over %d further eager steps of the same run"
                   % (K, "eager" if args.eager else "graph-replayed", res["kernel_steps"])),
        "forms": forms,
        "convergence": conv,
        "E0_per_site": wl.E0 / N,
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
