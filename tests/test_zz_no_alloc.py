"""The allocation-free top-M selection (spasm_select_topm_static, scratch in a static
device array) against the workspace entry point spasm_select_topm_large, through the C
ABI: equal outputs on two calls in a row, the second with a smaller input (the scratch
keeps the first call's contents), across the one-workgroup and radix-select paths."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    return spasm, L


def _static(spasm, L, key, M):
    N = key.shape[0]
    idx = torch.empty(M, dtype=torch.int32, device="cuda")
    rc = L.spasm_select_topm_static(N, ctypes.c_void_p(key.data_ptr()), M, ctypes.c_void_p(idx.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.spasm_last_error().decode()
    return idx


def test_static_topm_equals_workspace_topm(lib):
    spasm, L = lib
    rng = np.random.default_rng(4242)
    for shapes in ([(1 << 20, 8192), (40000, 100)], [(300000, 4096), (16385, 7)], [(16384, 2048), (5000, 17)],
                   [(70000, 513), (20000, 8192)]):
        for N, M in shapes:  # two calls in a row, the second smaller
            key = np.round(rng.uniform(0, 1, N), 4).astype(np.float32)  # many ties
            key[rng.uniform(size=N) < 0.05] = 0.0
            tk = torch.tensor(key, device="cuda")
            got = _static(spasm, L, tk, M)
            ref = spasm.select_topm_large(tk, M)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (N, M)
            assert np.array_equal(got.cpu().numpy(), np.argsort(key.astype(np.float64), kind="stable")[:M])


def test_static_topm_rejects_sizes_beyond_its_scratch(lib):
    spasm, L = lib
    dummy = ctypes.c_void_p(256)
    assert L.spasm_select_topm_static((1 << 20) + 1, dummy, 8, dummy, None) == -4
    assert L.spasm_select_topm_static(20000, dummy, 8193, dummy, None) == -4
    assert L.spasm_select_topm_static(100, dummy, 101, dummy, None) == -1
    assert L.spasm_select_topm_static_bytes() >= L.spasm_select_topm_workspace(1 << 20, 8192)
