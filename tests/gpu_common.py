"""Helpers shared by the GPU parity tests: build a GPU model and an oracle
spec of the same architecture, move parameters between them."""
import numpy as np
import pytest
import torch

from oracle import model as omodel

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def make_pair(Lx, Ly=1, dim=1, H=16, cplx=False, marshall=False, zero_mag=False, dtype="f64",
              seed=2001, max_Ns=256):
    import paper_2608_18065_amd as pm
    spec = omodel.Spec(Lx=Lx, Ly=Ly, dim=dim, H=H, complex_head=cplx, marshall=marshall,
                       zero_mag=zero_mag)
    m = pm.Model(Lx, Ly, dim, H, cplx, marshall, zero_mag, dtype=dtype, seed=seed, max_Ns=max_Ns)
    assert m.Np == omodel.num_params(spec)
    return spec, m


def scaled_theta(spec, seed, scale):
    """Glorot init with weights scaled up (conditionals far from uniform)
    and non-zero biases."""
    th = omodel.glorot_init(spec, seed) * scale
    rng = np.random.default_rng(seed)
    off = 0
    for name, shape in omodel.layout(spec):
        n = int(np.prod(shape))
        if len(shape) == 1:
            th[off:off + n] = rng.uniform(-0.5, 0.5, n)
        off += n
    return th


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(a, b):
    """Largest entrywise difference relative to the largest entry of the
    reference: max|a - b| / max|b| (the floor only avoids 0 / 0)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))
