"""The allocation-free MLP gradient (sph_mlp_grad_noalloc) through the C ABI
against the allocating entry point (sph_mlp_grad) and the numpy oracle: two
calls in a row, the second on fewer samples, so the second reuses the
library's device array after a larger call."""

import ctypes as C

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _features(n, seed):
    rng = np.random.default_rng(seed)
    F = np.stack([rng.normal(0, 5e-3, n), rng.normal(0, 2e-3, n), rng.normal(1.1, 0.15, n),
                  np.abs(rng.normal(0, 2e-3, n)), rng.normal(1.0, 0.3, n)], axis=1)
    return F.astype(np.float32)


def test_noalloc_gradient_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_11156_amd import sph
    R = _features(4096, 99)
    p = M.init(seed=3, in_shift=R.mean(0), in_scale=1.0 / R.std(0), out_scale=1e-3).astype(np.float32)
    net = sph.MLP(p)
    P = torch.from_numpy(p).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    for call, n in enumerate((20000, 777)):
        print(f"[noalloc] call {call} n={n}", flush=True)
        F = _features(n, 10 + call)
        t = (1e-3 * np.tanh(F[:, 0] * 100 + F[:, 3] * 300)).astype(np.float32)
        Fd, td = torch.from_numpy(F).cuda(), torch.from_numpy(t).cuda()
        loss_ref, g_ref = net.grad(Fd, td)
        grad = torch.full((sph.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        rc = sph.sph_mlp_grad_noalloc(C.c_void_p(P.data_ptr()), C.c_void_p(Fd.data_ptr()), C.c_void_p(td.data_ptr()),
                                      n, C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()),
                                      C.c_void_p(stream))
        assert rc == sph.SPH_OK
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        # the same kernels with the same fixed-order reductions: identical bits
        np.testing.assert_array_equal(g, g_ref)
        assert float(loss.item()) / n == loss_ref
        # and within the oracle's bf16 tolerance, as the allocating call is tested
        lo, go = M.loss_and_grads(p, F, t)
        tol = 2.0 ** -6 * M.grad_scale(p, F, t) + 1e-12
        assert (np.abs(g - go) / tol).max() <= 1.0
    net.close()


def test_noalloc_gradient_rejects_bad_sizes():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_11156_amd import sph
    buf = torch.zeros(8, dtype=torch.float32, device="cuda")
    ptr = C.c_void_p(buf.data_ptr())
    for n in (0, -1, (1 << 24) + 1):
        assert sph.sph_mlp_grad_noalloc(ptr, ptr, ptr, n, ptr, ptr, None) == sph.SPH_ERR_INVALID
    assert sph.sph_mlp_grad_noalloc(None, ptr, ptr, 4, ptr, ptr, None) == sph.SPH_ERR_INVALID
