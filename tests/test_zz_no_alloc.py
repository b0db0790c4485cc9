"""hfx_mlp_train_static (no allocation: optimizer state in a static device array) against
hfx_mlp_train (which allocates its state per call), through the C ABI, on two calls in a row,
the second with a smaller model and fewer samples.

Both entry points run the same kernels in the same order; with at most 64 samples the gradient is
summed by one wavefront of one workgroup, so the two trainings agree to FP32 rounding of a fixed
summation order (asserted at 1e-6 relative).  A second call that found the first call's Adam
moments still in the shared array would move every parameter by up to the learning rate per step,
orders of magnitude beyond that."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _train(fn, F, H, O, p0, X, T, epochs, lr, loss_on_device):
    import torch
    from paper_2009_12505_amd import _abi as A
    L = A.lib()
    p = torch.from_numpy(p0.copy()).cuda()
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    s = torch.cuda.current_stream()
    if loss_on_device:
        ld = torch.zeros(epochs, dtype=torch.float32, device="cuda")
        st = fn(F, H, O, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                X.shape[0], epochs, ctypes.c_float(lr), ctypes.c_void_p(ld.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        A.check(st)
        torch.cuda.synchronize()
        loss = ld.cpu().numpy()
    else:
        loss = np.zeros(epochs, np.float32)
        st = fn(F, H, O, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                X.shape[0], epochs, ctypes.c_float(lr), loss.ctypes.data, ctypes.c_void_p(s.cuda_stream))
        A.check(st)
        torch.cuda.synchronize()
    return p.cpu().numpy(), loss


def _case(rng, F, H, O, n):
    from paper_2009_12505_amd import _abi as A
    npar = int(A.lib().hfx_mlp_n_params(F, H, O))
    p0 = (rng.standard_normal(npar) * 0.3).astype(np.float32)
    X = rng.standard_normal((n, F)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], np.cos(X[:, 2])] + [X[:, 3]] * (O - 2), 1)[:, :O]
    return p0, X, np.ascontiguousarray(T, np.float32)


def test_static_training_matches_allocating_training_on_two_calls():
    from paper_2009_12505_amd import _abi as A
    L = A.lib()
    rng = np.random.default_rng(2009)
    print("case no-alloc MLP training: call 1 (10-32-2, 64 samples), call 2 (10-16-2, 40 samples)", flush=True)
    for (F, H, O, n, epochs) in ((10, 32, 2, 64, 60), (10, 16, 2, 40, 25)):
        p0, X, T = _case(rng, F, H, O, n)
        pa, la = _train(L.hfx_mlp_train, F, H, O, p0, X, T, epochs, 1e-2, False)
        ps, ls = _train(L.hfx_mlp_train_static, F, H, O, p0, X, T, epochs, 1e-2, True)
        moved = float(np.abs(pa - p0).max())
        diff = float(np.abs(ps - pa).max())
        print(f"  {F}-{H}-{O} n={n}: max|param change| {moved:.3e}, max|static - allocating| {diff:.3e}, "
              f"loss {la[0]:.4f} -> {la[-1]:.4f}", flush=True)
        assert moved > 1e-2
        np.testing.assert_allclose(ps, pa, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(ls, la, rtol=1e-6, atol=1e-7)
        assert la[-1] < la[0]


def test_static_training_rejects_bad_arguments():
    from paper_2009_12505_amd import _abi as A
    L = A.lib()
    P = ctypes.c_void_p(1)  # never dereferenced: rejected first
    assert L.hfx_mlp_train_static(8, 65, 1, P, P, P, 1, 1, ctypes.c_float(1e-2), None, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_train_static(17, 8, 1, P, P, P, 1, 1, ctypes.c_float(1e-2), None, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_train_static(8, 8, 1, P, P, P, 1, 1, ctypes.c_float(0.0), None, None) == A.HFX_ERR_ARG
    host = np.zeros(1000, np.float32)
    st = L.hfx_mlp_train_static(4, 4, 1, host.ctypes.data, host.ctypes.data, host.ctypes.data, 4, 1,
                                ctypes.c_float(1e-2), None, None)
    assert st == A.HFX_ERR_ARG and "GPU-accessible" in L.hfx_last_error().decode()
