"""semd_decompose_ex_noalloc, the entry point for callers that cannot
allocate (its workspace is the library's static device array), against
semd_decompose_ex, both called through the raw C ABI: two calls in a row
into the same array, the second with a smaller input, bit-identical to the
allocating entry point and within the parity tolerance of the oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_2106_15319_amd as semd
import workloads
from parity import TOL

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _run(name, X, dims, p, out, n):
    L = semd.lib()
    d = (C.c_int64 * len(dims))(*dims)
    s = torch.cuda.current_stream().cuda_stream
    args = [X.data_ptr(), d, len(dims), C.byref(p), out.data_ptr(), n.data_ptr()]
    if name == "semd_decompose_ex":
        args += [None, 0]
    rc = getattr(L, name)(*args, s)
    assert rc == semd.SEMD_OK, (name, rc, L.semd_last_error().decode())


@pytest.mark.parametrize("order", ["stream_then_onchip", "onchip_then_stream_smaller"])
def test_noalloc_matches_decompose_ex(order):
    K, S = 6, 10
    # (M, N, D, path): the second call of each pair is the smaller input
    cases = {"stream_then_onchip": [(30000, 3, 0, semd.SEMD_PATH_AUTO),
                                    (1000, 3, 50, semd.SEMD_PATH_AUTO)],
             "onchip_then_stream_smaller": [(5000, 3, 20, semd.SEMD_PATH_AUTO),
                                            (2100, 2, 7, semd.SEMD_PATH_STREAM)]}[order]
    for k, (M, N, D, path) in enumerate(cases):
        Xh = workloads.series(workloads.rng_for(31, 10 * k + M), N, M)
        print(f"case {order}[{k}]: M={M} N={N} D={D} path={path}", flush=True)
        X = torch.from_numpy(Xh).to(DEV)
        p = semd._params(D, K, S, path=path)
        a = torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV)
        na = torch.empty(1, dtype=torch.int32, device=DEV)
        b = torch.full((K + 1, M * N), float("nan"), dtype=torch.float64, device=DEV)
        nb = torch.full((1,), -99, dtype=torch.int32, device=DEV)
        _run("semd_decompose_ex", X, [M, N], p, a, na)
        _run("semd_decompose_ex_noalloc", X, [M, N], p, b, nb)
        torch.cuda.synchronize()
        ah, bh = a.cpu().numpy(), b.cpu().numpy()
        assert ah.tobytes() == bh.tobytes(), float(np.nanmax(np.abs(ah - bh)))
        assert int(na.cpu()[0]) == int(nb.cpu()[0])
        ref, nr = oracle.decompose(Xh, M, N, D, K, S)
        err = float(np.abs(bh - ref).max())
        assert int(nb.cpu()[0]) == nr
        assert err <= TOL * float(np.abs(Xh).max()), err


def test_noalloc_rejects_signals_beyond_the_scratch():
    L = semd.lib()
    cap = semd.semd_noalloc_scratch_bytes()
    assert cap == 64 << 20
    dims = (C.c_int64 * 2)(1_400_000, 1)
    p = semd._params(0, 6, 10)
    assert L.semd_workspace_bytes(dims, 2, C.byref(p)) > cap
    X = torch.zeros(8, dtype=torch.float64, device=DEV)  # never read: refused first
    rc = L.semd_decompose_ex_noalloc(X.data_ptr(), dims, 2, C.byref(p), X.data_ptr(), None,
                                     torch.cuda.current_stream().cuda_stream)
    assert rc == semd.SEMD_EINVAL
    assert "scratch" in L.semd_last_error().decode()
