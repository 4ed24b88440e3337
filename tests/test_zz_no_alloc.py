"""mpmc_mlp_backward_noalloc through the C ABI against mpmc_mlp_backward:
bit-identical gradients on two calls in a row, the second on fewer samples
(the library's shared gradient rows keep the first call's contents)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fns():
    import paper_1211_1646_amd as pkg
    lib = pkg.load()
    vp = C.c_void_p
    bwd = lib.mpmc_mlp_backward
    bwd.restype = C.c_int32
    bwd.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp]
    na = lib.mpmc_mlp_backward_noalloc
    na.restype = C.c_int32
    na.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp]
    fwd = lib.mpmc_mlp_forward
    fwd.restype = C.c_int32
    fwd.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
    wb = lib.mpmc_mlp_work_bytes
    wb.restype = C.c_int32
    wb.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    return lib, fwd, bwd, na, wb


def test_noalloc_backward_matches_backward_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib, fwd, bwd, na, wb = _fns()
    rng = np.random.Generator(np.random.PCG64(7))
    W = torch.from_numpy(rng.uniform(-0.5, 0.5, 1217).astype(np.float32)).cuda()
    st = torch.cuda.current_stream().cuda_stream
    for n in (50000, 777):   # the second call is smaller: stale rows must not leak in
        print("noalloc backward, n=%d" % n, flush=True)
        X = torch.from_numpy(rng.uniform(-2, 2, (n, 3)).astype(np.float32)).cuda()
        dY = torch.from_numpy(rng.uniform(-1, 1, n).astype(np.float32)).cuda()
        Y = torch.empty(n, dtype=torch.float32, device="cuda")
        cache = torch.empty(64 * n, dtype=torch.float32, device="cuda")
        assert fwd(W.data_ptr(), X.data_ptr(), n, Y.data_ptr(), cache.data_ptr(), st) == 0
        nbytes = C.c_size_t()
        assert wb(n, C.byref(nbytes)) == 0
        work = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        dW_ref = torch.full((1217,), float("nan"), device="cuda")
        dX_ref = torch.full((n, 3), float("nan"), device="cuda")
        assert bwd(W.data_ptr(), X.data_ptr(), cache.data_ptr(), dY.data_ptr(), n,
                   dW_ref.data_ptr(), dX_ref.data_ptr(), work.data_ptr(), st) == 0
        dW = torch.full((1217,), float("nan"), device="cuda")
        dX = torch.full((n, 3), float("nan"), device="cuda")
        assert na(W.data_ptr(), X.data_ptr(), cache.data_ptr(), dY.data_ptr(), n,
                  dW.data_ptr(), dX.data_ptr(), st) == 0
        torch.cuda.synchronize()
        a, b = dW.cpu().numpy(), dW_ref.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "dW differs, n=%d" % n
        assert np.array_equal(dX.cpu().numpy().view(np.uint32), dX_ref.cpu().numpy().view(np.uint32))


def test_noalloc_backward_rejects_too_many_samples():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    lib, fwd, bwd, na, wb = _fns()
    W = torch.zeros(1217, device="cuda")
    d = torch.zeros(4, device="cuda")
    n = 65537   # one past the limit: refused on the host before any launch
    st = torch.cuda.current_stream().cuda_stream
    assert na(W.data_ptr(), d.data_ptr(), d.data_ptr(), d.data_ptr(), n, W.data_ptr(), None,
              st) == -1
    lib.mpmc_last_error.restype = C.c_char_p
    assert b"MPMC_MLP_NOALLOC_MAX_SAMPLES" in lib.mpmc_last_error()
