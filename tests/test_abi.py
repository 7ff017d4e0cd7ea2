"""The C ABI library loads, exports every declared entry point, and rejects
invalid arguments on the host before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_2106_15319_amd as semd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semd.h")

BOGUS = C.c_void_p(0x1000)  # never dereferenced: validation fails first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(semd_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    L = semd.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(semd.exported_names()) == names


def test_abi_version_and_limits():
    assert semd.semd_abi_version() == 3
    assert semd.semd_resident_max_length() >= 16384


@pytest.mark.parametrize("M,N,D,want", [(4, 2, 2, 10), (1000, 3, 0, 3000), (1000, 3, 50, 3100),
                                        (112, 92, 20, 12124), (5, 1, 5, 5), (5, 2, 6, -1),
                                        (0, 3, 0, -1), (3, 0, 0, -1), (3, 3, -1, -1)])
def test_serial_length(M, N, D, want):
    assert semd.semd_serial_length(M, N, D) == want


def _p(**kw):
    p = semd.semd_params(kw.get("D", 0), kw.get("K", 6), kw.get("S", 10), kw.get("b", 0),
                         kw.get("NR", 1), kw.get("path", 0), 0, kw.get("stop", 0),
                         kw.get("res", 0), kw.get("sd", 0.0))
    return p


@pytest.mark.parametrize("kw,dims,code", [
    (dict(K=0), [100, 3], semd.SEMD_EINVAL),
    (dict(S=0), [100, 3], semd.SEMD_EINVAL),
    (dict(b=1), [100, 3], semd.SEMD_EINVAL),
    (dict(D=101), [100, 3], semd.SEMD_EINVAL),
    (dict(D=-1), [100, 3], semd.SEMD_EINVAL),
    (dict(path=7), [100, 3], semd.SEMD_EINVAL),
    (dict(path=-1), [100, 3], semd.SEMD_EINVAL),
    (dict(stop=2), [100, 3], semd.SEMD_EINVAL),
    (dict(stop=semd.SEMD_STOP_SD, sd=0.0), [100, 3], semd.SEMD_EINVAL),
    (dict(stop=semd.SEMD_STOP_SD, sd=-0.2), [100, 3], semd.SEMD_EINVAL),
    (dict(stop=semd.SEMD_STOP_SD, sd=float("inf")), [100, 3], semd.SEMD_EINVAL),
    (dict(stop=semd.SEMD_STOP_SD, sd=float("nan")), [100, 3], semd.SEMD_EINVAL),
    (dict(res=1), [100, 3], semd.SEMD_EINVAL),
    (dict(), [0, 3], semd.SEMD_EINVAL),
    (dict(), [100, -2], semd.SEMD_EINVAL),
])
def test_decompose_ex_rejects_invalid_arguments(kw, dims, code):
    L = semd.lib()
    p = _p(**kw)
    d = (C.c_int64 * len(dims))(*dims)
    rc = L.semd_decompose_ex(BOGUS, d, len(dims), C.byref(p), BOGUS, None, None, 0, None)
    assert rc == code
    assert L.semd_last_error().decode()


def test_length_limits():
    L = semd.lib()
    d = (C.c_int64 * 2)(20000, 3)  # 60000 serialized samples: streaming only
    p = _p(path=semd.SEMD_PATH_ONCHIP)
    assert L.semd_decompose_ex(BOGUS, d, 2, C.byref(p), BOGUS, None, None, 0, None) == \
        semd.SEMD_EUNSUPPORTED
    big = (C.c_int64 * 2)(1 << 20, 1 << 9)  # 2^29 samples: beyond any path
    assert L.semd_decompose_ex(BOGUS, big, 2, C.byref(_p()), BOGUS, None, None, 0, None) == \
        semd.SEMD_EUNSUPPORTED


def test_null_pointers_rejected():
    L = semd.lib()
    p = _p()
    d = (C.c_int64 * 2)(100, 3)
    assert L.semd_decompose_ex(None, d, 2, C.byref(p), BOGUS, None, None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_decompose_ex(BOGUS, d, 2, C.byref(p), None, None, None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_decompose_ex(BOGUS, None, 2, C.byref(p), BOGUS, None, None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_decompose_ex(BOGUS, d, 0, C.byref(p), BOGUS, None, None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_decompose_ex(BOGUS, d, 2, None, BOGUS, None, None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_serialize(None, d, 2, 0, BOGUS, None) == semd.SEMD_EINVAL
    assert L.semd_extrema(BOGUS, 2, BOGUS, BOGUS, BOGUS, None) == semd.SEMD_EINVAL
    assert L.semd_noise(1, 2, 3, 10, None, None) == semd.SEMD_EINVAL


def test_batch_validation():
    L = semd.lib()
    p = _p()
    items = (semd.semd_item * 2)()
    for it in items:
        it.signal = 0x1000
        it.imfs_out = 0x2000
        it.dims[0], it.dims[1] = 100, 3
        it.ndim = 2
    items[1].ndim = 5
    assert L.semd_decompose_batch(items, 2, C.byref(p), None) == semd.SEMD_EINVAL
    assert "item 1" in L.semd_last_error().decode()
    items[1].ndim = 2
    items[1].reserved = 3
    assert L.semd_decompose_batch(items, 2, C.byref(p), None) == semd.SEMD_EINVAL
    items[1].reserved = 0
    items[0].noise_sigma = -1.0
    pe = _p(NR=4)
    assert L.semd_eemd_batch(items, 2, C.byref(pe), None) == semd.SEMD_EINVAL
    pe = _p(NR=0)
    assert L.semd_eemd_batch(items, 2, C.byref(pe), None) == semd.SEMD_EINVAL
    assert L.semd_ceemdan_batch(items, 2, C.byref(_p(NR=4)), None) == semd.SEMD_EINVAL
    assert "eps" in L.semd_last_error().decode()
    items[0].noise_sigma = float("nan")
    assert L.semd_ceemdan_batch(items, 2, C.byref(_p(NR=4)), None) == semd.SEMD_EINVAL
    items[0].noise_sigma = 0.2
    assert L.semd_ceemdan_batch(items, 2, C.byref(_p(NR=0)), None) == semd.SEMD_EINVAL
    assert L.semd_ceemdan_batch(items, 2, C.byref(_p(NR=2, K=0)), None) == semd.SEMD_EINVAL
    assert L.semd_decompose_batch(items, -1, C.byref(p), None) == semd.SEMD_EINVAL
    assert L.semd_decompose_batch(None, 2, C.byref(p), None) == semd.SEMD_EINVAL


def test_engine_validation_without_device():
    L = semd.lib()
    p = _p()
    it = semd.semd_item()
    it.signal = 0x1000
    it.imfs_out = 0x2000
    it.dims[0], it.dims[1] = 1000, 3
    it.ndim = 2
    b = C.c_size_t()
    assert L.semd_engine_footprint(C.byref(it), C.byref(p), C.byref(b)) == semd.SEMD_OK
    assert b.value >= 3000 * 16  # candidate and residue at least
    it.ndim = 0
    assert L.semd_engine_footprint(C.byref(it), C.byref(p), C.byref(b)) == semd.SEMD_EINVAL
    t = C.c_int64()
    assert L.semd_engine_admit(None, C.byref(it), C.byref(p), C.byref(t)) == semd.SEMD_EINVAL
    assert L.semd_engine_step(None, None) == semd.SEMD_EINVAL
    assert L.semd_engine_step_n(None, 1, None) == semd.SEMD_EINVAL
    assert L.semd_engine_step_n(None, 0, None) == semd.SEMD_EINVAL
    h = C.c_void_p()
    assert L.semd_engine_create(1 << 30, 0, C.byref(h)) == semd.SEMD_EINVAL
    assert L.semd_engine_create(10, 4, C.byref(h)) == semd.SEMD_EINVAL


def test_tuning_validation_without_device():
    L = semd.lib()
    assert L.semd_autotune(2, 64, None) == semd.SEMD_EINVAL
    assert L.semd_autotune(1 << 20, 64, None) == semd.SEMD_EINVAL
    assert L.semd_autotune(4096, 0, None) == semd.SEMD_EINVAL
    assert L.semd_tune_get(None, 0, None) == semd.SEMD_EINVAL
    assert L.semd_tune_set(None) == semd.SEMD_EINVAL
    assert L.semd_tune_reset() == semd.SEMD_OK


def test_slices_validation():
    L = semd.lib()
    d = (C.c_int64 * 2)(100, 3)
    assert L.semd_decompose_slices(BOGUS, d, 2, C.byref(_p(D=5)), BOGUS, None, None) == \
        semd.SEMD_EINVAL  # slices are not serialized
    assert L.semd_decompose_slices(None, d, 2, C.byref(_p()), BOGUS, None, None) == \
        semd.SEMD_EINVAL
    big = (C.c_int64 * 2)(20000, 2)
    assert L.semd_decompose_slices(BOGUS, big, 2, C.byref(_p(path=semd.SEMD_PATH_ONCHIP)),
                                   BOGUS, None, None) == semd.SEMD_EUNSUPPORTED


def test_workspace_bytes_and_undersized_workspace():
    """semd_workspace_bytes sizes semd_decompose_ex's workspace; a workspace
    below that size, or not 256-byte aligned, is rejected before anything is
    enqueued (the pointers are never dereferenced)."""
    L = semd.lib()
    for dims, path in [((1000, 3), semd.SEMD_PATH_AUTO), ((1000, 3), semd.SEMD_PATH_STREAM),
                       ((20000, 3), semd.SEMD_PATH_AUTO), ((16384, 1), semd.SEMD_PATH_ONCHIP)]:
        d = (C.c_int64 * 2)(*dims)
        p = _p(path=path)
        need = L.semd_workspace_bytes(d, 2, C.byref(p))
        Ls = dims[0] * dims[1]
        assert need >= 16 * Ls  # residue and candidate at least
        assert need % 256 == 0
        ws = C.c_void_p(0x100000)
        assert L.semd_decompose_ex(BOGUS, d, 2, C.byref(p), BOGUS, None, ws, need - 1,
                                   None) == semd.SEMD_EINVAL
        assert "workspace" in L.semd_last_error().decode()
        assert L.semd_decompose_ex(BOGUS, d, 2, C.byref(p), BOGUS, None, C.c_void_p(0x100008),
                                   need, None) == semd.SEMD_EINVAL
        assert "aligned" in L.semd_last_error().decode()
    # the streaming layout is larger than the on-chip one for the same signal
    d = (C.c_int64 * 2)(1000, 3)
    assert L.semd_workspace_bytes(d, 2, C.byref(_p(path=semd.SEMD_PATH_STREAM))) > \
        L.semd_workspace_bytes(d, 2, C.byref(_p(path=semd.SEMD_PATH_ONCHIP)))
    # invalid arguments: 0 and a message
    assert L.semd_workspace_bytes(d, 2, C.byref(_p(K=0))) == 0
    assert L.semd_last_error().decode()
    assert L.semd_workspace_bytes(d, 0, C.byref(_p())) == 0
    assert L.semd_workspace_bytes(None, 2, C.byref(_p())) == 0
    assert L.semd_workspace_bytes(d, 2, None) == 0
    big = (C.c_int64 * 2)(20000, 3)
    assert L.semd_workspace_bytes(big, 2, C.byref(_p(path=semd.SEMD_PATH_ONCHIP))) == 0


def test_binding_checks_buffer_sizes_before_any_call():
    """The binding compares every buffer with what the dims and K ask for
    (the C ABI cannot see sizes); a mismatch raises before the library is
    called.  CPU tensors of the right sizes are then refused for not being
    on the device."""
    import torch
    f64 = dict(dtype=torch.float64)
    x = torch.zeros(15, **f64)
    with pytest.raises(ValueError, match="dims ask for"):
        semd.semd_decompose_ex(torch.zeros(14, **f64), [5, 3], 0, 2, 3)
    with pytest.raises(ValueError, match="at least"):
        semd.semd_decompose_ex(x, [5, 3], 0, 2, 3, imfs_out=torch.zeros(44, **f64))
    with pytest.raises(TypeError):
        semd.semd_decompose_ex(x, [5, 3], 0, 2, 3, imfs_out=torch.zeros(45, **f64),
                               n_imfs_out=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="at least"):
        semd.semd_decompose_ex(x, [5, 3], 0, 2, 3, imfs_out=torch.zeros(45, **f64),
                               n_imfs_out=torch.zeros(0, dtype=torch.int32))
    with pytest.raises(TypeError, match="HIP device"):
        semd.semd_decompose_ex(x, [5, 3], 0, 2, 3, imfs_out=torch.zeros(45, **f64),
                               n_imfs_out=torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError):
        semd.semd_decompose_ex(x, [5, 0], 0, 2, 3)
    with pytest.raises(ValueError):
        semd.semd_decompose_ex(x, [5, 3], 0, 0, 3)
    with pytest.raises(ValueError, match="at least"):
        semd.semd_decompose_slices(x, [5, 3], 2, 3, imfs_out=torch.zeros(45, **f64),
                                   n_imfs_out=torch.zeros(2, dtype=torch.int32))
    # batches: every item's buffers, counts and stats
    xs = [torch.zeros(15, **f64), torch.zeros(8, **f64)]
    outs = [torch.zeros(45, **f64), torch.zeros(24, **f64)]
    with pytest.raises(ValueError, match="signals\\[1\\]"):
        semd.semd_decompose_batch(xs, [[5, 3], [9, 1]], outs, None, 0, 2, 3)
    with pytest.raises(ValueError, match="imfs_out\\[1\\]"):
        semd.semd_decompose_batch(xs, [[5, 3], [8, 1]], [outs[0], torch.zeros(23, **f64)],
                                  None, 0, 2, 3)
    with pytest.raises(ValueError, match="counts"):
        semd.semd_decompose_batch(xs, [[5, 3], [8, 1]], outs, torch.zeros(1, dtype=torch.int32),
                                  0, 2, 3)
    with pytest.raises(ValueError, match="stats"):
        semd.semd_decompose_batch(xs, [[5, 3], [8, 1]], outs, None, 0, 2, 3,
                                  stats=torch.zeros(5, dtype=torch.int64))
    with pytest.raises(ValueError):
        semd.semd_eemd_batch(xs, [[5, 3]], outs, None, 0, 2, 3, 4, 0, [0.1, 0.1])
    with pytest.raises(ValueError, match="noise sigmas"):
        semd.semd_eemd_batch(xs, [[5, 3], [8, 1]], outs, None, 0, 2, 3, 4, 0, [0.1])
    with pytest.raises(ValueError, match="outside"):
        semd.semd_serialize(x, [5, 3], 6)
    with pytest.raises(ValueError, match="dims ask for"):
        semd.semd_deserialize(torch.zeros(16, **f64), [5, 3], 0)
    with pytest.raises(ValueError, match="at least"):
        semd.semd_noise(1, 2, 3, 10, w=torch.zeros(9, **f64))
