"""The allocation-free Cholesky entry point, called through the C ABI,
against the model-workspace solve (minsr_solve) on the same inputs: two
calls in a row, the second with a smaller n, plus the oracle's solve."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import minsr as ominsr
from tests import inputs
from tests.gpu_common import gpu, need_gpu, to_dev

pytestmark = gpu


def _free_device_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def test_noalloc_solve_matches_workspace_solve():
    need_gpu()
    import paper_2608_18065_amd as pm
    lib = pm.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lam = 1e-3
    model = pm.Model(16, hidden=16, dtype="f64", seed=1, max_Ns=1024)
    cases = []
    for n, seed in ((1024, 11), (333, 12)):     # the second call is smaller
        rng = np.random.default_rng(seed)
        T, _ = inputs.psd_matrix(inputs.spectrum_loguniform(n, 1e3, rng), seed=200 + seed)
        b = inputs.rhs(n, seed=seed)
        cases.append((n, T, b, to_dev(T), to_dev(b), torch.empty(n, dtype=torch.float64,
                                                                  device="cuda"),
                      torch.zeros(1, dtype=torch.int32, device="cuda")))
    # set-up call: resolves the device array's address, enqueues nothing
    assert lib.minsr_solve_noalloc(0, None, lam, None, None, None, stream) == 0
    for i, (n, T, b, Td, bd, x, st) in enumerate(cases):
        print("noalloc solve n=%d" % n, flush=True)
        torch.cuda.synchronize()
        free0 = _free_device_bytes()
        rc = lib.minsr_solve_noalloc(n, ctypes.c_void_p(Td.data_ptr()), lam,
                                     ctypes.c_void_p(bd.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(st.data_ptr()), stream)
        assert rc == 0, lib.minsr_last_error()
        torch.cuda.synchronize()
        if i > 0:   # after a first call (runtime set-up of the kernels' launches)
            assert _free_device_bytes() == free0   # the call allocated nothing
        assert int(st.item()) == 0
        xr, sr = model.solve(Td, bd, lam=lam)
        torch.cuda.synchronize()
        assert int(sr.item()) == 0
        # the same kernels in the same order: bit for bit
        assert torch.equal(x, xr)
        ref = ominsr.solve(T, b, lam)
        xn = x.cpu().numpy()
        assert np.linalg.norm(xn - ref) / np.linalg.norm(ref) < 1e-10


def test_noalloc_rejects_sizes_beyond_its_array():
    need_gpu()
    import paper_2608_18065_amd as pm
    lib = pm.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.minsr_solve_noalloc(1025, None, 1e-3, None, None, None, stream)
    assert rc == -2
    assert b"1024" in lib.minsr_last_error()
    assert lib.minsr_solve_noalloc(10, None, 0.0, None, None, None, stream) == -1
