"""GRU wave function: parameter layout, initialisation, forward pass, sampling.

Follows Sec. 2 (Eqs. 1-7: Psi = sqrt(P) exp(i phi), chain rule, softmax
conditionals, softsign phases, zero initial hidden state and zero first
input), Sec. 2.1 (zigzag path pi(k) for 2D lattices, zero boundary states)
and App. A (the GRU cell: reset gate multiplying W_h h + b_h, input term
W_in sigma + b_in outside it, h = (1 - u) h_prev + u h_tilde; the 2D cell
with h' = U1 h_horizontal + U2 h_vertical and sigma' = [sigma_h; sigma_v]).
Sec. 3.3 gives the Marshall sign (-1)^{sigma_A}.

Readings where the paper is silent (listed in the design notes as well):
  * spin value sigma = 0 is z = +1 (up), sigma = 1 is z = -1;
  * parameter blocks are flattened in the order given by `layout`, each
    row-major; weights Glorot-uniform a*(2u-1), a = sqrt(6/(fan_in+fan_out)),
    u from Philox domain 1; biases zero;
  * sampling is inverse-CDF: sigma_i = 0 iff u < p_i(0), strict;
  * optional zero-magnetisation masking: once either spin value has been
    used N/2 times, the conditional is renormalised onto the other value;
  * Marshall sublattice A = {(i, j): i + j even}.

All arithmetic is float64 numpy; the site loop is a plain Python loop and the
per-site products are batched matmuls over samples.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import philox


@dataclass(frozen=True)
class Spec:
    """Architecture of one wave function.

    Lx, Ly   lattice extent (1D chains use Ly = 1 and dim = 1)
    dim      1 for the 1D GRU, 2 for the 2D GRU of App. A
    H        hidden width d_h
    complex_head   True for cRNN (softsign phase head), False for pRNN
    marshall       multiply Psi by (-1)^{sigma_A}
    zero_mag       restrict sampling to total S^z = 0
    """
    Lx: int
    Ly: int = 1
    dim: int = 1
    H: int = 16
    complex_head: bool = False
    marshall: bool = False
    zero_mag: bool = False

    @property
    def N(self):
        return self.Lx * self.Ly


def layout(spec):
    """Ordered list of (name, shape, fan_in, fan_out or None for biases)."""
    H = spec.H
    ds = 2 if spec.dim == 1 else 4          # width of the spin input
    blocks = []
    if spec.dim == 2:
        blocks += [("U1", (H, H)), ("U2", (H, H))]
    blocks += [("Wu", (H, H + ds)), ("bu", (H,)),
               ("Wr", (H, H + ds)), ("br", (H,)),
               ("Wh", (H, H)), ("bh", (H,)),
               ("Win", (H, ds)), ("bin", (H,)),
               ("U", (2, H)), ("c", (2,))]
    if spec.complex_head:
        blocks += [("Uphi", (2, H)), ("cphi", (2,))]
    return blocks


def num_params(spec):
    return sum(int(np.prod(s)) for _, s in layout(spec))


def unpack(spec, theta):
    """Split the flat float64 vector into named views (no copies)."""
    out, off = {}, 0
    for name, shape in layout(spec):
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    assert off == theta.shape[0]
    return out


def glorot_init(spec, seed):
    """theta_0: Glorot-uniform weights from Philox domain 1, zero biases."""
    theta = np.zeros(num_params(spec), dtype=np.float64)
    off = 0
    for name, shape in layout(spec):
        n = int(np.prod(shape))
        if len(shape) == 2:
            fan_out, fan_in = shape
            a = math.sqrt(6.0 / (fan_in + fan_out))
            for k in range(off, off + n):
                w = philox.philox4x64((k // 4, 0, 0, 1), (seed, 0))[k % 4]
                u = philox.word_to_uniform(w)
                theta[k] = a * (2.0 * u - 1.0)
        off += n
    return theta


# ---------------------------------------------------------------------------
# lattice path (Sec. 2.1, zigzag path pi(k))
# ---------------------------------------------------------------------------

def path_coords(spec):
    """(i_k, j_k) for k = 0..N-1.  1D: (k, 0)."""
    Nx = spec.Lx
    out = []
    for k in range(spec.N):
        j = k // Nx
        i = k % Nx if j % 2 == 0 else (Nx - 1) - (k % Nx)
        out.append((i, j))
    return out


def path_index(spec, i, j):
    Nx = spec.Lx
    return j * Nx + (i if j % 2 == 0 else Nx - 1 - i)


def neighbours_2d(spec):
    """For each path position k: (k_horizontal, k_vertical), -1 if outside.

    Horizontal neighbour is (i - (-1)^j, j), vertical is (i, j - 1)."""
    res = []
    for (i, j) in path_coords(spec):
        ih = i - (1 if j % 2 == 0 else -1)
        kh = path_index(spec, ih, j) if 0 <= ih < spec.Lx else -1
        kv = path_index(spec, i, j - 1) if j >= 1 else -1
        res.append((kh, kv))
    return res


def marshall_mask(spec):
    """Boolean per path position: True if the site is on sublattice A."""
    return np.array([(i + j) % 2 == 0 for (i, j) in path_coords(spec)])


# ---------------------------------------------------------------------------
# GRU forward
# ---------------------------------------------------------------------------

def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _onehot(col):
    """Spin column (Ns,) -> one-hot (Ns, 2)."""
    out = np.zeros((col.shape[0], 2))
    out[np.arange(col.shape[0]), col] = 1.0
    return out


def gru_cell(P, hprev, xs):
    """One GRU update (App. A).  hprev (Ns,H) is h_{i-1} (1D) or h' (2D);
    xs is the spin input sigma_{i-1} (1D) or sigma' (2D)."""
    xin = np.concatenate([hprev, xs], axis=1)
    u = _sigmoid(xin @ P["Wu"].T + P["bu"])
    r = _sigmoid(xin @ P["Wr"].T + P["br"])
    g = hprev @ P["Wh"].T + P["bh"]
    ht = np.tanh(r * g + xs @ P["Win"].T + P["bin"])
    h = (1.0 - u) * hprev + u * ht
    return h, dict(u=u, r=r, g=g, ht=ht)


def conditional(spec, P, h, nup, ndn):
    """Softmax conditional of Eq. 5 with optional S^z = 0 masking.

    Returns logits z (Ns,2), masked probabilities p (Ns,2) and log p (Ns,2)
    (log p = -inf on a masked value)."""
    z = h @ P["U"].T + P["c"]
    m = np.max(z, axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(z[:, 0] - m[:, 0]) + np.exp(z[:, 1] - m[:, 0]))
    logp = z - lse[:, None]
    p = np.exp(logp)
    if spec.zero_mag:
        half = spec.N // 2
        no_up = nup >= half          # value 0 exhausted -> must draw 1
        no_dn = ndn >= half          # value 1 exhausted -> must draw 0
        p = p.copy()
        logp = logp.copy()
        p[no_up] = [0.0, 1.0]
        logp[no_up] = [-np.inf, 0.0]
        p[no_dn] = [1.0, 0.0]
        logp[no_dn] = [0.0, -np.inf]
    return z, p, logp


def _phase_terms(P, h):
    a = h @ P["Uphi"].T + P["cphi"]
    return a, math.pi * a / (1.0 + np.abs(a))


def run(spec, theta, sigma=None, uniforms=None, keep=False):
    """Walk the lattice path once.

    Exactly one of `sigma` (evaluate given configurations, int (Ns,N)) and
    `uniforms` (sample, float64 (Ns,N)) is given.  Returns a dict with
    sigma, log_p (sum of log conditionals), phase (sum of conditional
    phases, 0 for pRNN) and, with keep=True, every intermediate needed by
    the reverse pass."""
    P = unpack(spec, theta)
    N, H = spec.N, spec.H
    sampling = sigma is None
    Ns = uniforms.shape[0] if sampling else sigma.shape[0]
    sig = np.zeros((Ns, N), dtype=np.int64) if sampling else np.asarray(sigma, dtype=np.int64)
    hs = np.zeros((Ns, N, H))
    logp_tot = np.zeros(Ns)
    phase_tot = np.zeros(Ns)
    nup = np.zeros(Ns, dtype=np.int64)
    ndn = np.zeros(Ns, dtype=np.int64)
    nb = neighbours_2d(spec) if spec.dim == 2 else None
    tape = []
    zeros_h = np.zeros((Ns, H))
    zeros_s = np.zeros((Ns, 2))
    for k in range(N):
        if spec.dim == 1:
            hprev = hs[:, k - 1] if k > 0 else zeros_h
            xs = _onehot(sig[:, k - 1]) if k > 0 else zeros_s
            hh = hv = None
            hcell_in = hprev
        else:
            kh, kv = nb[k]
            hh = hs[:, kh] if kh >= 0 else zeros_h
            hv = hs[:, kv] if kv >= 0 else zeros_h
            sh = _onehot(sig[:, kh]) if kh >= 0 else zeros_s
            sv = _onehot(sig[:, kv]) if kv >= 0 else zeros_s
            xs = np.concatenate([sh, sv], axis=1)
            hcell_in = hh @ P["U1"].T + hv @ P["U2"].T
        h, st = gru_cell(P, hcell_in, xs)
        hs[:, k] = h
        z, p, logp = conditional(spec, P, h, nup, ndn)
        if sampling:
            sig[:, k] = np.where(uniforms[:, k] < p[:, 0], 0, 1)
        s_k = sig[:, k]
        lp = logp[np.arange(Ns), s_k]
        logp_tot += lp
        if spec.complex_head:
            a_phi, ph = _phase_terms(P, h)
            phase_tot += ph[np.arange(Ns), s_k]
        else:
            a_phi = None
        nup += (s_k == 0)
        ndn += (s_k == 1)
        if keep:
            tape.append(dict(hin=hcell_in, xs=xs, hh=hh, hv=hv, h=h, p=p,
                             a_phi=a_phi, **st))
    out = dict(sigma=sig, log_p=logp_tot, phase=phase_tot, hs=hs)
    if keep:
        out["tape"] = tape
    return out


def marshall_phase(spec, sigma):
    """pi * sigma_A (Sec. 3.3) or zeros."""
    if not spec.marshall:
        return np.zeros(sigma.shape[0])
    A = marshall_mask(spec)
    return math.pi * np.sum(np.asarray(sigma)[:, A], axis=1)


def log_psi(spec, theta, sigma):
    """Complex log Psi = 0.5 log P + i (phi + pi sigma_A)   (Eqs. 2, 6, 8)."""
    r = run(spec, theta, sigma=sigma)
    return 0.5 * r["log_p"] + 1j * (r["phase"] + marshall_phase(spec, r["sigma"]))


def sample(spec, theta, uniforms):
    """Autoregressive exact sampling (Sec. 2, Eq. 3; Alg. 1 step 3).

    Returns (sigma (Ns,N) int, log Psi (Ns,) complex)."""
    r = run(spec, theta, uniforms=uniforms)
    lp = 0.5 * r["log_p"] + 1j * (r["phase"] + marshall_phase(spec, r["sigma"]))
    return r["sigma"], lp
