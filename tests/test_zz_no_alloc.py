"""The start network's forward pass without allocation
(sbmds_mlp_forward_noalloc) against the allocating entry point
(sbmds_mlp_forward), through the C ABI (needs a gfx950 GPU)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward(gpu):
    import torch
    from paper_1705_10887_amd import lib, mlp
    fn = lib().sbmds_mlp_forward_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    rng = np.random.default_rng(3)
    stream = torch.cuda.current_stream().cuda_stream
    with mlp.Net(k=3, seed=11, stream=stream) as net:
        net.set_norm(rng.standard_normal(19).astype(np.float32) * 0.1, (0.5 + rng.random(19)).astype(np.float32))
        # first call spans three passes through the work buffer (8,192 rows
        # each, the last one partial); the second is smaller than one pass
        for rows in (20000, 777):
            F = (rng.standard_normal((rows, 19)) * 0.8 + 0.1).astype(np.float32)
            ref = net.forward(F)  # the allocating entry point
            Fd = torch.from_numpy(F).cuda()
            Yd = torch.full((rows, 3), float("nan"), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            rc = fn(net._h, Fd.data_ptr(), rows, Yd.data_ptr())
            torch.cuda.synchronize()
            print(f"rows {rows}: rc {rc}", flush=True)
            assert rc == 0
            np.testing.assert_array_equal(Yd.cpu().numpy(), ref)
        # sizes beyond the maximum are rejected before any launch
        assert fn(net._h, Fd.data_ptr(), 4_000_001, Yd.data_ptr()) == -1
        assert fn(net._h, Fd.data_ptr(), 0, Yd.data_ptr()) == -1
