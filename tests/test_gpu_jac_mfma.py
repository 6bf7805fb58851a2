"""GPU parity of the matrix-core Jacobian of FP32 chains with d_h = 128 (a
sample-batched reverse pass over checkpoint segments, then the rows
assembled from the gate adjoints) against the FP64 oracle: real and complex
heads, checkpoint strides that divide N and that leave a ragged last
segment, sample counts that leave a ragged last workgroup, the longest chain
the path takes (N = 128), the zero-magnetisation mask, weights beyond the
FP16 range, and the per-sample kernel on the same inputs."""
import numpy as np
import pytest
import torch

from oracle import jacobian as ojac
from oracle import model as omodel
from oracle import philox
from tests.gpu_common import gpu, make_pair, need_gpu, rel_err, scaled_theta, to_dev

pytestmark = gpu

# FP32 recurrence with 22-bit split operands, then a sum over N sites per
# entry: the entrywise error relative to the largest entry stays below this
TOL = 1e-4


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _ref(spec, th, sig):
    D = ojac.log_derivatives(spec, th, sig)
    Ns = sig.shape[0]
    return (np.concatenate([D.real, D.imag], axis=0) if spec.complex_head else D) / np.sqrt(Ns)


def _case(arch, seed, Ns, C, scale=1.0):
    spec, m = make_pair(**arch, dtype="f32", max_Ns=max(Ns, 16))
    th = scaled_theta(spec, seed, scale)
    m.set_params(to_dev(th))
    sig, _ = omodel.sample(spec, th, philox.uniforms(seed, 3, Ns, spec.N))
    O, _ = m.jacobian(to_dev(sig.astype(np.uint8)), ckpt_every=C)
    return spec, m, th, sig, O.cpu().numpy()


@pytest.mark.parametrize("arch,C,Ns", [
    (dict(Lx=23, H=128, cplx=True), 1, 13),
    (dict(Lx=23, H=128, cplx=True), 5, 8),
    (dict(Lx=23, H=128, cplx=True), 10, 21),
    (dict(Lx=23, H=128, cplx=True), 16, 9),
    (dict(Lx=37, H=128), 1, 19),
    (dict(Lx=37, H=128), 4, 16),
    (dict(Lx=37, H=128), 11, 33),
    (dict(Lx=30, H=128, zero_mag=True), 7, 17),
], ids=lambda v: "_".join("%s%s" % kv for kv in v.items()) if isinstance(v, dict) else str(v))
def test_h128_matrix_core_jacobian_matches_oracle(arch, C, Ns):
    spec, m, th, sig, O = _case(arch, 31 + C + Ns, Ns, C)
    err = rel_err(O, _ref(spec, th, sig))
    print("%s C=%d Ns=%d: rel err %.2e" % (arch, C, Ns, err))
    assert err < TOL


def test_h128_matrix_core_jacobian_longest_chain():
    # N = 128: four full K-steps of 32 sites in the row assembly
    spec, m, th, sig, O = _case(dict(Lx=128, H=128, cplx=True), 41, 9, 10)
    err = rel_err(O, _ref(spec, th, sig))
    print("N=128: rel err %.2e" % err)
    assert err < TOL


def test_h128_longer_chain_takes_per_sample_kernel():
    # N = 129 is beyond the row assembly's chain length: the per-sample
    # kernel forms the rows (same oracle bound)
    spec, m, th, sig, O = _case(dict(Lx=129, H=128, cplx=True), 43, 5, 10)
    assert rel_err(O, _ref(spec, th, sig)) < TOL


def test_h128_matrix_core_matches_per_sample_kernel():
    # the same inputs through both kernels (an explicit thread split selects
    # the per-sample one)
    spec, m, th, sig, O = _case(dict(Lx=40, H=128, cplx=True), 47, 24, 10)
    m.set_tunable("jac_parts", 2)
    O2, _ = m.jacobian(to_dev(sig.astype(np.uint8)), ckpt_every=10)
    err = rel_err(O, O2.cpu().numpy())
    print("matrix cores vs per-sample kernel: %.2e" % err)
    assert err < 2e-5


def test_h128_matrix_core_jacobian_large_weights():
    # weight columns beyond FP16's range are split scaled by a power of two
    arch = dict(Lx=21, H=128, cplx=True)
    spec, m = make_pair(**arch, dtype="f32")
    th = scaled_theta(spec, 53, 1.0)
    off = 0
    for name, shape in omodel.layout(spec):
        n = int(np.prod(shape))
        if name in ("Wu", "Wr", "Wh"):
            blk = th[off:off + n].reshape(shape)
            blk[3, 5] = 1.0e5
            blk[7, 1] = -4.0e4
        off += n
    m.set_params(to_dev(th))
    Ns = 11
    sig, _ = omodel.sample(spec, th, philox.uniforms(53, 3, Ns, spec.N))
    O, _ = m.jacobian(to_dev(sig.astype(np.uint8)), ckpt_every=10)
    O = O.cpu().numpy()
    assert np.all(np.isfinite(O))
    err = rel_err(O, _ref(spec, th, sig))
    print("large weights: rel err %.2e" % err)
    assert err < TOL


def test_h128_matrix_core_jacobian_strides_agree():
    # stride 1 reads every stored state; stride 10 recomputes nine of every
    # ten on the matrix cores: the rows agree to the split-operand accuracy
    spec, m, th, sig, O10 = _case(dict(Lx=30, H=128, cplx=True), 59, 16, 10)
    O1, _ = m.jacobian(to_dev(sig.astype(np.uint8)), ckpt_every=1)
    err = rel_err(O10, O1.cpu().numpy())
    print("stride 10 vs 1: %.2e" % err)
    assert err < 2e-5
