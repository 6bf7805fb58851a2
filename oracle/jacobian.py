"""Per-sample log-derivatives d log Psi(sigma^(s)) / d theta.

Sec. 2.3 defines O_ks = (1/sqrt(N_s)) d log Psi(sigma^(s)) / d theta_k
(Alg. 1, step 5).  With log Psi = 0.5 log P + i phi (Eqs. 2, 6, 8;
App. C.1 writes log Psi = 0.5 sum_i log p_i for a positive ansatz) the real
part comes from the conditionals and the imaginary part from the phases;
the Marshall sign does not depend on theta.

The derivative is taken by a hand-written reverse pass through the GRU of
App. A, site by site in reverse path order, with the forward intermediates
kept in full.  Each parameter gradient is a per-sample sum over sites of
outer products (adjoint x input), accumulated in float64.
"""
import math

import numpy as np

from . import model


def _cell_backward(P, t, dh):
    """Reverse of gru_cell for one site.  Returns (d h_in, grads dict),
    every gradient per sample."""
    u, r, g, ht, hin, xs = t["u"], t["r"], t["g"], t["ht"], t["hin"], t["xs"]
    H = hin.shape[1]
    dht = dh * u
    du = dh * (ht - hin)
    dhin = dh * (1.0 - u)
    da = dht * (1.0 - ht * ht)
    dr = da * g
    dg = da * r
    dpu = du * u * (1.0 - u)
    dpr = dr * r * (1.0 - r)
    xin = np.concatenate([hin, xs], axis=1)
    dhin = dhin + dg @ P["Wh"] + dpu @ P["Wu"][:, :H] + dpr @ P["Wr"][:, :H]
    grads = {
        "Wu": np.einsum("si,sj->sij", dpu, xin), "bu": dpu,
        "Wr": np.einsum("si,sj->sij", dpr, xin), "br": dpr,
        "Wh": np.einsum("si,sj->sij", dg, hin), "bh": dg,
        "Win": np.einsum("si,sj->sij", da, xs), "bin": da,
    }
    return dhin, grads


def _reverse(spec, theta, fwd, seed):
    """One reverse sweep.  seed = "re" for 0.5 log P, "im" for phi."""
    P = model.unpack(spec, theta)
    tape, sig = fwd["tape"], fwd["sigma"]
    Ns, N, H = sig.shape[0], spec.N, spec.H
    grads = {name: np.zeros((Ns,) + shape) for name, shape in model.layout(spec)}
    dh_acc = np.zeros((Ns, N, H))
    nb = model.neighbours_2d(spec) if spec.dim == 2 else None
    rows = np.arange(Ns)
    for k in range(N - 1, -1, -1):
        t = tape[k]
        h = t["h"]
        onehot = np.zeros((Ns, 2))
        onehot[rows, sig[:, k]] = 1.0
        dh = dh_acc[:, k]
        if seed == "re":
            dz = 0.5 * (onehot - t["p"])           # d(0.5 log p'_sigma)/dz
            grads["U"] += np.einsum("si,sj->sij", dz, h)
            grads["c"] += dz
            dh = dh + dz @ P["U"]
        else:
            a = t["a_phi"]
            da_phi = onehot * (math.pi / (1.0 + np.abs(a)) ** 2)
            grads["Uphi"] += np.einsum("si,sj->sij", da_phi, h)
            grads["cphi"] += da_phi
            dh = dh + da_phi @ P["Uphi"]
        dhin, gk = _cell_backward(P, t, dh)
        for name, v in gk.items():
            grads[name] += v
        if spec.dim == 1:
            if k > 0:
                dh_acc[:, k - 1] += dhin
        else:
            kh, kv = nb[k]
            if kh >= 0:
                grads["U1"] += np.einsum("si,sj->sij", dhin, t["hh"])
                dh_acc[:, kh] += dhin @ P["U1"]
            if kv >= 0:
                grads["U2"] += np.einsum("si,sj->sij", dhin, t["hv"])
                dh_acc[:, kv] += dhin @ P["U2"]
    flat = [grads[name].reshape(Ns, -1) for name, _ in model.layout(spec)]
    return np.concatenate(flat, axis=1)


def log_derivatives(spec, theta, sigma):
    """D[s, k] = d log Psi(sigma^(s)) / d theta_k; float64 for pRNN,
    complex128 (Re from 0.5 log P, Im from phi) for cRNN."""
    fwd = model.run(spec, theta, sigma=np.asarray(sigma, dtype=np.int64), keep=True)
    d_re = _reverse(spec, theta, fwd, "re")
    if not spec.complex_head:
        return d_re
    d_im = _reverse(spec, theta, fwd, "im")
    return d_re + 1j * d_im
