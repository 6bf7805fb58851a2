"""Autotuner for the library's launch parameters.

For one model and workload it sweeps each tunable (see minsr_set_tunable)
over its candidate values, times the phase the tunable governs with the
library's HIP-event phase timers over a few steps that do not update the
parameters, keeps the fastest value, and records the choice in a JSON cache
keyed by device architecture and shape bucket.  `apply` reads the cache and
sets the recorded values on a model; batches are built from models tuned
this way.

    tunable      phase timed                  candidates
    gram_split   Gram tiles + reduction       0 (heuristic), 1, 2, 4, 8, 16, 32
    eloc_grid    local-energy recurrence      0 (one per item), 256, 512, 1024, 2048
    sample_r     vector sampling recurrence   1, 4 (no effect on the matrix-core sampler)
    jac_parts    Jacobian reverse pass        0 (built-in), 1, 2, 4
"""
import json
import os

import torch

from . import FORM_BF16_FP64

CANDIDATES = {
    "gram_split": (0, 1, 2, 4, 8, 16, 32),
    "eloc_grid": (0, 256, 512, 1024, 2048),
    "sample_r": (1, 4),
    "jac_parts": (0, 1, 2, 4),
}
PHASES = {
    "gram_split": ("gram", "gram_reduce"),
    "eloc_grid": ("eloc",),
    "sample_r": ("sample",),
    "jac_parts": ("jacobian",),
}
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def shape_key(model, Ns, form):
    arch = torch.cuda.get_device_properties(model.device).gcnArchName.split(":")[0]
    d = model.desc
    return "%s/dim%d/H%d/N%d/Ns%d/cplx%d/form%d" % (arch, d.dim, d.hidden, model.N, Ns,
                                                   int(d.complex_head), form)


def _time_phase(model, ham, Ns, form, phases, reps):
    mom = torch.zeros(model.Np, dtype=torch.float64, device=model.device)
    outs = model.step_outputs(Ns)
    kw = dict(form=form, apply_update=False, outputs=outs)
    model.step(ham, Ns, 0.01, 1e-3, 0.0, mom, 1, 0, **kw)       # warm caches and code
    torch.cuda.synchronize()
    model.timing_begin(reps)
    for i in range(reps):
        model.step(ham, Ns, 0.01, 1e-3, 0.0, mom, 1, i, **kw)
    torch.cuda.synchronize()
    ms, n = model.timing_read()
    return sum(ms[p] for p in phases) / max(n, 1)


def tune(model, ham, Ns, form=FORM_BF16_FP64, reps=5, keys=None, cache=DEFAULT_CACHE):
    """Sweep the tunables one at a time (in the order of CANDIDATES), set the
    best value of each on the model, and record the result in the cache.
    Returns {key: (best_value, {value: ms})}."""
    result = {}
    for key in keys or CANDIDATES:
        times = {}
        for v in CANDIDATES[key]:
            model.set_tunable(key, v)
            times[v] = _time_phase(model, ham, Ns, form, PHASES[key], reps)
        best = min(times, key=times.get)
        model.set_tunable(key, best)
        result[key] = (best, times)
    if cache:
        data = load(cache)
        data[shape_key(model, Ns, form)] = {k: v[0] for k, v in result.items()}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return result


def load(cache=DEFAULT_CACHE):
    if not os.path.exists(cache):
        return {}
    with open(cache) as f:
        return json.load(f)


def apply(model, Ns, form=FORM_BF16_FP64, cache=DEFAULT_CACHE):
    """Set the cached launch parameters for this model's shape bucket;
    returns the applied dict (empty if the bucket was never tuned)."""
    entry = load(cache).get(shape_key(model, Ns, form), {})
    for k, v in entry.items():
        model.set_tunable(k, v)
    return entry
