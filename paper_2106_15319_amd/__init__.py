"""Python binding of libsemd (Serial-EMD on MI355X).

Thin ctypes marshalling over the C ABI declared in ``include/semd.h``: every
function below has the name of the C entry point it calls, takes torch tensors
that live on the current HIP device, passes their device pointers and the
current torch stream, and raises ``SemdError`` on a non-zero status.  All the
arithmetic runs in the library's HIP kernels; there is no fallback.

Layout: a set of N signals of length M is an M x N column-major matrix, i.e.
a 1D float64 tensor whose element (m, i) sits at m + M*i (Sec. 3.2 of the
paper).  A (C, L) row-major batch of channels is exactly that with M = L,
N = C; an (H, W) row-major image is passed as ``img.t().contiguous()`` with
M = H, N = W, so that its columns are the signals.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libsemd.so")

SEMD_OK = 0
SEMD_EINVAL = 1
SEMD_ENOMEM = 2
SEMD_EDEVICE = 3
SEMD_EBUSY = 4
SEMD_ENONFINITE = 5
SEMD_EUNSUPPORTED = 6
SEMD_BOUNDARY_MIRROR = 0
SEMD_PATH_AUTO = 0
SEMD_PATH_ONCHIP = 1
SEMD_PATH_STREAM = 2
SEMD_STOP_FIXED = 0
SEMD_STOP_SD = 1
SEMD_ENGINE_MAX_STEPS = 64  # steps per semd_engine_step_n call


class SemdError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed with status {code}: {msg}")
        self.code = code


class semd_params(C.Structure):
    _fields_ = [("transition_len", C.c_int32), ("max_imfs", C.c_int32),
                ("sift_iters", C.c_int32), ("boundary_rule", C.c_int32),
                ("ensemble", C.c_int32), ("path", C.c_int32), ("seed", C.c_uint64),
                ("stop_rule", C.c_int32), ("reserved", C.c_int32), ("sd_threshold", C.c_double)]


class semd_item(C.Structure):
    _fields_ = [("signal", C.c_void_p), ("imfs_out", C.c_void_p), ("n_imfs_out", C.c_void_p),
                ("stats_out", C.c_void_p), ("dims", C.c_int64 * 4), ("ndim", C.c_int32), ("reserved", C.c_int32),
                ("noise_sigma", C.c_double), ("item_id", C.c_uint64)]


_EXPORTS = {
    # name: (restype, argtypes)
    "semd_abi_version": (C.c_int, []),
    "semd_last_error": (C.c_char_p, []),
    "semd_serial_length": (C.c_int64, [C.c_int64, C.c_int64, C.c_int64]),
    "semd_resident_max_length": (C.c_int64, []),
    "semd_autotune": (C.c_int, [C.c_int64, C.c_int, C.c_void_p]),
    "semd_tune_get": (C.c_int, [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "semd_tune_set": (C.c_int, [C.c_char_p]),
    "semd_tune_reset": (C.c_int, []),
    "semd_decompose": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int, C.c_int, C.c_int,
                                 C.c_int, C.c_void_p, C.c_void_p]),
    "semd_workspace_bytes": (C.c_size_t, [C.POINTER(C.c_int64), C.c_int,
                                          C.POINTER(semd_params)]),
    "semd_decompose_ex": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int,
                                    C.POINTER(semd_params), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_size_t, C.c_void_p]),
    "semd_decompose_ex_noalloc": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int,
                                            C.POINTER(semd_params), C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "semd_noalloc_scratch_bytes": (C.c_size_t, []),
    "semd_decompose_trace": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int,
                                       C.POINTER(semd_params), C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_int64, C.c_void_p]),
    "semd_decompose_batch": (C.c_int, [C.POINTER(semd_item), C.c_int, C.POINTER(semd_params),
                                       C.c_void_p]),
    "semd_decompose_slices": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int,
                                        C.POINTER(semd_params), C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    "semd_eemd_batch": (C.c_int, [C.POINTER(semd_item), C.c_int, C.POINTER(semd_params),
                                  C.c_void_p]),
    "semd_ceemdan_batch": (C.c_int, [C.POINTER(semd_item), C.c_int, C.POINTER(semd_params),
                                     C.c_void_p]),
    "semd_serialize": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int, C.c_int,
                                 C.c_void_p, C.c_void_p]),
    "semd_deserialize": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int, C.c_int,
                                   C.c_void_p, C.c_void_p]),
    "semd_extrema": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "semd_noise": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64, C.c_void_p,
                             C.c_void_p]),
    "semd_release_cached_memory": (C.c_int, []),
    "semd_profile_enable": (C.c_int, [C.c_int]),
    "semd_profile_reset": (C.c_int, []),
    "semd_profile_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "semd_engine_create": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    "semd_engine_footprint": (C.c_int, [C.POINTER(semd_item), C.POINTER(semd_params),
                                        C.POINTER(C.c_size_t)]),
    "semd_engine_admit": (C.c_int, [C.c_void_p, C.POINTER(semd_item), C.POINTER(semd_params),
                                    C.POINTER(C.c_int64)]),
    "semd_engine_step": (C.c_int, [C.c_void_p, C.c_void_p]),
    "semd_engine_step_n": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "semd_engine_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int,
                                   C.POINTER(C.c_int)]),
    "semd_engine_resident": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "semd_engine_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libsemd.so (built in-tree by ``paper_2106_15319_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsemd.so is not built ({LIB_PATH}); run "
                              "`python -m paper_2106_15319_amd.build` first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names() -> list[str]:
    return list(_EXPORTS)


def _check(rc: int, what: str):
    if rc != SEMD_OK:
        raise SemdError(rc, what, lib().semd_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _chk(t: torch.Tensor, name: str, dtype: torch.dtype, numel: int | None = None,
         exact: bool = False) -> torch.Tensor:
    """What the C ABI cannot see: `t` is a contiguous tensor of `dtype`
    holding at least (exact: exactly) `numel` elements."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor on the HIP device")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None:
        if exact and t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, the dims ask for {numel}")
        if t.numel() < numel:
            raise ValueError(f"{name} has {t.numel()} elements, at least {numel} are needed")
    return t


def _ptr(t: torch.Tensor, name: str) -> int:
    """Device pointer of `t`, which must live on the current HIP device."""
    if not t.is_cuda:
        raise TypeError(f"{name} must be a tensor on the HIP device")
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}, not on the current device "
                         f"cuda:{torch.cuda.current_device()}")
    return t.data_ptr()


def _dev(t: torch.Tensor, name: str, dtype: torch.dtype, numel: int | None = None,
         exact: bool = False) -> int:
    return _ptr(_chk(t, name, dtype, numel, exact), name)


def _dev_f64(t: torch.Tensor, name: str, numel: int | None = None, exact: bool = False) -> int:
    return _dev(t, name, torch.float64, numel, exact)


def _dims(dims: Sequence[int]):
    dims = [int(d) for d in dims]
    if not 1 <= len(dims) <= 4:
        raise ValueError("dims must have 1..4 entries")
    if any(d < 1 for d in dims):
        raise ValueError(f"every dim must be >= 1, got {dims}")
    arr = (C.c_int64 * len(dims))(*dims)
    return arr, len(dims)


def _mn(dims: Sequence[int]) -> tuple[int, int]:
    """(M, N) of column-major dims: M = dims[0], N = product of the rest."""
    M = int(dims[0])
    N = 1
    for v in dims[1:]:
        N *= int(v)
    return M, N


def _check_shape_params(K: int, S: int) -> None:
    if int(K) < 1 or int(S) < 1:
        raise ValueError(f"max_imfs and sift_iters must be >= 1, got {K}, {S}")


def _params(D: int, K: int, S: int, NR: int = 1, seed: int = 0,
            boundary_rule: int = SEMD_BOUNDARY_MIRROR, path: int = SEMD_PATH_AUTO,
            sd: float = 0.0) -> semd_params:
    """sd > 0 selects the SD stopping rule with that threshold; 0 the fixed
    sift count."""
    rule = SEMD_STOP_SD if sd > 0 else SEMD_STOP_FIXED
    return semd_params(int(D), int(K), int(S), int(boundary_rule), int(NR), int(path),
                       int(seed) & (2**64 - 1), rule, 0, float(sd))


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def semd_abi_version() -> int:
    return int(lib().semd_abi_version())


def semd_serial_length(M: int, N: int, D: int) -> int:
    return int(lib().semd_serial_length(M, N, D))


def semd_resident_max_length() -> int:
    return int(lib().semd_resident_max_length())


def semd_autotune(max_length: int = 16384, batch: int = 512, stream=None) -> None:
    """Time the on-chip launch shapes per length bucket and keep the fastest."""
    _check(lib().semd_autotune(int(max_length), int(batch), _stream(stream)), "semd_autotune")


def semd_tune_get() -> str:
    """The launch-shape table in its text form."""
    need = C.c_size_t()
    lib().semd_tune_get(None, 0, C.byref(need))
    buf = C.create_string_buffer(int(need.value))
    _check(lib().semd_tune_get(buf, need.value, C.byref(need)), "semd_tune_get")
    return buf.value.decode()


def semd_tune_set(text: str) -> None:
    _check(lib().semd_tune_set(text.encode()), "semd_tune_set")


def semd_tune_reset() -> None:
    _check(lib().semd_tune_reset(), "semd_tune_reset")


def autotune(max_length: int = 16384, batch: int = 512, cache: str | None = None,
             stream=None) -> str:
    """Load the launch-shape table from `cache` when it was made for this
    library and GPU; otherwise tune now (about a second) and write it there.
    Returns the table's text."""
    if cache and os.path.exists(cache):
        text = open(cache).read()
        if lib().semd_tune_set(text.encode()) == SEMD_OK:
            return text
    semd_autotune(max_length, batch, stream)
    text = semd_tune_get()
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            fh.write(text)
    return text


def semd_decompose(signal: torch.Tensor, dims: Sequence[int], max_imfs: int, sift_iters: int,
                   boundary_rule: int = SEMD_BOUNDARY_MIRROR, imfs_out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """Serial-EMD with D = round(0.2 M); returns imfs_out ((K+1) x M*N)."""
    d, nd = _dims(dims)
    _check_shape_params(max_imfs, sift_iters)
    M, N = _mn(dims)
    if imfs_out is None:
        imfs_out = torch.empty((max_imfs + 1, M * N), dtype=torch.float64, device=signal.device)
    _check(lib().semd_decompose(_dev_f64(signal, "signal", M * N, exact=True), d, nd, max_imfs,
                                sift_iters, boundary_rule,
                                _dev_f64(imfs_out, "imfs_out", (max_imfs + 1) * M * N),
                                _stream(stream)),
           "semd_decompose")
    return imfs_out


def semd_workspace_bytes(dims: Sequence[int], D: int, max_imfs: int, sift_iters: int,
                         path: int = SEMD_PATH_AUTO, sd: float = 0.0) -> int:
    """Device bytes of the workspace semd_decompose_ex needs for these dims
    and parameters."""
    d, nd = _dims(dims)
    p = _params(D, max_imfs, sift_iters, path=path, sd=sd)
    n = int(lib().semd_workspace_bytes(d, nd, C.byref(p)))
    if n == 0:
        raise SemdError(SEMD_EINVAL, "semd_workspace_bytes", lib().semd_last_error().decode())
    return n


def _single_args(signal, dims, max_imfs, sift_iters, imfs_out, n_imfs_out):
    """Validated (dims array, ndim, signal, imfs_out, n_imfs_out pointers,
    imfs_out, n_imfs_out) of a one-signal call, allocating missing outputs."""
    d, nd = _dims(dims)
    _check_shape_params(max_imfs, sift_iters)
    M, N = _mn(dims)
    dev = signal.device if isinstance(signal, torch.Tensor) else None
    if imfs_out is None:
        imfs_out = torch.empty((max_imfs + 1, M * N), dtype=torch.float64, device=dev)
    if n_imfs_out is None:
        n_imfs_out = torch.empty(1, dtype=torch.int32, device=dev)
    bufs = ((_chk(signal, "signal", torch.float64, M * N, exact=True), "signal"),
            (_chk(imfs_out, "imfs_out", torch.float64, (max_imfs + 1) * M * N), "imfs_out"),
            (_chk(n_imfs_out, "n_imfs_out", torch.int32, 1), "n_imfs_out"))
    ptrs = tuple(_ptr(t, name) for t, name in bufs)
    return d, nd, ptrs, imfs_out, n_imfs_out


def semd_decompose_ex(signal: torch.Tensor, dims: Sequence[int], D: int, max_imfs: int,
                      sift_iters: int, imfs_out: torch.Tensor | None = None,
                      n_imfs_out: torch.Tensor | None = None, stream=None,
                      path: int = SEMD_PATH_AUTO, sd: float = 0.0,
                      workspace: torch.Tensor | None = None):
    """Plain path: one signal per launch.  Returns (imfs_out, n_imfs_out).
    sd > 0: SD stopping rule with that threshold.  workspace: a device
    tensor of at least semd_workspace_bytes(...) bytes (256-byte aligned),
    or None for a library-allocated one."""
    d, nd, (ps, po, pn), imfs_out, n_imfs_out = _single_args(signal, dims, max_imfs, sift_iters,
                                                             imfs_out, n_imfs_out)
    p = _params(D, max_imfs, sift_iters, path=path, sd=sd)
    ws, wsb = None, 0
    if workspace is not None:
        if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or \
                not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous tensor on the HIP device")
        ws = _dev(workspace, "workspace", workspace.dtype)
        wsb = workspace.numel() * workspace.element_size()
    _check(lib().semd_decompose_ex(ps, d, nd, C.byref(p), po, pn, ws, wsb, _stream(stream)),
           "semd_decompose_ex")
    return imfs_out, n_imfs_out


def semd_decompose_ex_noalloc(signal: torch.Tensor, dims: Sequence[int], D: int, max_imfs: int,
                              sift_iters: int, imfs_out: torch.Tensor, n_imfs_out: torch.Tensor,
                              stream=None, path: int = SEMD_PATH_AUTO, sd: float = 0.0):
    """semd_decompose_ex working in the library's static scratch array: no
    allocation by the library (the caller passes the outputs).  Returns
    (imfs_out, n_imfs_out)."""
    d, nd, (ps, po, pn), imfs_out, n_imfs_out = _single_args(signal, dims, max_imfs, sift_iters,
                                                             imfs_out, n_imfs_out)
    p = _params(D, max_imfs, sift_iters, path=path, sd=sd)
    _check(lib().semd_decompose_ex_noalloc(ps, d, nd, C.byref(p), po, pn, _stream(stream)),
           "semd_decompose_ex_noalloc")
    return imfs_out, n_imfs_out


def semd_decompose_trace(signal: torch.Tensor, dims: Sequence[int], D: int, max_imfs: int,
                         sift_iters: int, trace_cap: int | None = None, stream=None,
                         path: int = SEMD_PATH_AUTO, sd: float = 0.0):
    """semd_decompose_ex recording every extremum detection.  Returns
    (imfs_out, n_imfs_out, trace) with trace the int32 device buffer
    (trace[0] entries used, trace[1] complete flag, then the records)."""
    d, nd, (ps, po, pn), imfs_out, n_imfs_out = _single_args(signal, dims, max_imfs, sift_iters,
                                                             None, None)
    M, N = _mn(dims)
    L = semd_serial_length(M, N, int(D))
    if trace_cap is None:
        trace_cap = min(max_imfs * sift_iters * (L + 8) + 64, 2**31 - 1)
    trace = torch.zeros(int(trace_cap), dtype=torch.int32, device=signal.device)
    p = _params(D, max_imfs, sift_iters, path=path, sd=sd)
    _check(lib().semd_decompose_trace(ps, d, nd, C.byref(p), po, pn, trace.data_ptr(),
                                      int(trace_cap), _stream(stream)), "semd_decompose_trace")
    return imfs_out, n_imfs_out, trace


def semd_noalloc_scratch_bytes() -> int:
    return int(lib().semd_noalloc_scratch_bytes())


def semd_decompose_slices(signal: torch.Tensor, dims: Sequence[int], max_imfs: int,
                          sift_iters: int, imfs_out: torch.Tensor | None = None,
                          n_imfs_out: torch.Tensor | None = None, stream=None,
                          path: int = SEMD_PATH_AUTO, sd: float = 0.0):
    """Standard (slice-wise) EMD: every column decomposed on its own.
    Returns (imfs_out (K+1, M*N), n_imfs_out (N,))."""
    d, nd = _dims(dims)
    _check_shape_params(max_imfs, sift_iters)
    M, N = _mn(dims)
    dev = signal.device
    if imfs_out is None:
        imfs_out = torch.empty((max_imfs + 1, M * N), dtype=torch.float64, device=dev)
    if n_imfs_out is None:
        n_imfs_out = torch.empty(N, dtype=torch.int32, device=dev)
    p = _params(0, max_imfs, sift_iters, path=path, sd=sd)
    _chk(signal, "signal", torch.float64, M * N, exact=True)
    _chk(imfs_out, "imfs_out", torch.float64, (max_imfs + 1) * M * N)
    _chk(n_imfs_out, "n_imfs_out", torch.int32, N)
    _check(lib().semd_decompose_slices(_ptr(signal, "signal"), d, nd, C.byref(p),
                                       _ptr(imfs_out, "imfs_out"), _ptr(n_imfs_out, "n_imfs_out"),
                                       _stream(stream)),
           "semd_decompose_slices")
    return imfs_out, n_imfs_out


def _items(signals, dims_list, outs, counts, K, sigmas=None, item_ids=None, stats=None):
    """The semd_item array of a batch, every buffer checked against its dims:
    signal i holds M*N doubles, its output (K+1)*M*N, its count view one
    int32 and its stats view 3 int64."""
    n = len(signals)
    if len(dims_list) != n or len(outs) != n:
        raise ValueError(f"{n} signals, {len(dims_list)} dims and {len(outs)} outputs")
    for name, seq in (("counts", counts), ("noise sigmas", sigmas), ("item ids", item_ids),
                      ("stats", stats)):
        if seq is not None and len(seq) != n:
            raise ValueError(f"{n} signals but {len(seq)} {name}")
    for i in range(n):
        _dims(dims_list[i])
        M, N = _mn(dims_list[i])
        _chk(signals[i], f"signals[{i}]", torch.float64, M * N, exact=True)
        _chk(outs[i], f"imfs_out[{i}]", torch.float64, (K + 1) * M * N)
        if counts is not None:
            _chk(counts[i], f"counts[{i}]", torch.int32, 1)
        if stats is not None:
            _chk(stats[i], f"stats[{i}]", torch.int64, 3)
    arr = (semd_item * max(n, 1))()
    for i in range(n):
        it = arr[i]
        dims = [int(v) for v in dims_list[i]]
        it.signal = _ptr(signals[i], f"signals[{i}]")
        it.imfs_out = _ptr(outs[i], f"imfs_out[{i}]")
        it.n_imfs_out = _ptr(counts[i], f"counts[{i}]") if counts is not None else None
        it.stats_out = _ptr(stats[i], f"stats[{i}]") if stats is not None else None
        for k, v in enumerate(dims):
            it.dims[k] = v
        it.ndim = len(dims)
        it.reserved = 0
        it.noise_sigma = float(sigmas[i]) if sigmas is not None else 0.0
        it.item_id = int(item_ids[i]) if item_ids is not None else i
    return arr, n


def _count_views(counts, n):
    """One-entry views of an int32 count tensor of at least n entries."""
    if counts is None:
        return None
    _chk(counts, "counts", torch.int32, n)
    return [counts[i:i + 1] for i in range(n)]


def _stats_views(stats, n):
    if stats is None:
        return None
    _chk(stats, "stats", torch.int64, 3 * n)
    if stats.dim() != 2 or stats.shape[1] != 3:
        raise ValueError(f"stats must have shape (n, 3), got {tuple(stats.shape)}")
    return [stats[i] for i in range(n)]


def semd_decompose_batch(signals: Sequence[torch.Tensor], dims_list: Sequence[Sequence[int]],
                         outs: Sequence[torch.Tensor], counts: torch.Tensor | None, D: int,
                         max_imfs: int, sift_iters: int, stats: torch.Tensor | None = None,
                         stream=None, path: int = SEMD_PATH_AUTO, sd: float = 0.0) -> None:
    """Batched path: every signal in one launch.  counts: int32 tensor of
    len(signals) entries (or None); stats: int64 tensor (len(signals), 3) of
    (sifts, knots, sample-sifts) per signal (or None)."""
    _check_shape_params(max_imfs, sift_iters)
    cviews = _count_views(counts, len(signals))
    sviews = _stats_views(stats, len(signals))
    arr, n = _items(signals, dims_list, outs, cviews, max_imfs, stats=sviews)
    p = _params(D, max_imfs, sift_iters, path=path, sd=sd)
    _check(lib().semd_decompose_batch(arr, n, C.byref(p), _stream(stream)),
           "semd_decompose_batch")


def semd_eemd_batch(signals: Sequence[torch.Tensor], dims_list: Sequence[Sequence[int]],
                    outs: Sequence[torch.Tensor], counts: torch.Tensor | None, D: int,
                    max_imfs: int, sift_iters: int, ensemble: int, seed: int,
                    noise_sigmas: Sequence[float], item_ids: Sequence[int] | None = None,
                    stream=None, path: int = SEMD_PATH_AUTO, sd: float = 0.0) -> None:
    """Serial-EEMD of every signal (NR = ensemble realizations each)."""
    _check_shape_params(max_imfs, sift_iters)
    cviews = _count_views(counts, len(signals))
    arr, n = _items(signals, dims_list, outs, cviews, max_imfs, noise_sigmas, item_ids)
    p = _params(D, max_imfs, sift_iters, ensemble, seed, path=path, sd=sd)
    _check(lib().semd_eemd_batch(arr, n, C.byref(p), _stream(stream)), "semd_eemd_batch")


def semd_ceemdan_batch(signals: Sequence[torch.Tensor], dims_list: Sequence[Sequence[int]],
                       outs: Sequence[torch.Tensor], counts: torch.Tensor | None, D: int,
                       max_imfs: int, sift_iters: int, ensemble: int, seed: int,
                       eps: Sequence[float], item_ids: Sequence[int] | None = None,
                       stream=None, path: int = SEMD_PATH_AUTO, sd: float = 0.0) -> None:
    """Serial-CEEMDAN of every signal (NR = ensemble noise realizations, eps
    the relative noise amplitude of each item)."""
    _check_shape_params(max_imfs, sift_iters)
    cviews = _count_views(counts, len(signals))
    arr, n = _items(signals, dims_list, outs, cviews, max_imfs, eps, item_ids)
    p = _params(D, max_imfs, sift_iters, ensemble, seed, path=path, sd=sd)
    _check(lib().semd_ceemdan_batch(arr, n, C.byref(p), _stream(stream)), "semd_ceemdan_batch")


def _serial_len(dims: Sequence[int], D: int) -> int:
    M, N = _mn(dims)
    L = semd_serial_length(M, N, int(D))
    if L < 0:
        raise ValueError(f"transition length {D} is outside [0, {M}]")
    return L


def semd_serialize(X: torch.Tensor, dims: Sequence[int], D: int, x: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    d, nd = _dims(dims)
    M, N = _mn(dims)
    L = _serial_len(dims, D)
    if x is None:
        x = torch.empty(L, dtype=torch.float64, device=X.device)
    _chk(X, "X", torch.float64, M * N, exact=True)
    _chk(x, "x", torch.float64, L)
    _check(lib().semd_serialize(_ptr(X, "X"), d, nd, int(D), _ptr(x, "x"), _stream(stream)),
           "semd_serialize")
    return x


def semd_deserialize(y: torch.Tensor, dims: Sequence[int], D: int,
                     out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    d, nd = _dims(dims)
    M, N = _mn(dims)
    L = _serial_len(dims, D)
    if out is None:
        out = torch.empty(M * N, dtype=torch.float64, device=y.device)
    _chk(y, "y", torch.float64, L, exact=True)
    _chk(out, "out", torch.float64, M * N)
    _check(lib().semd_deserialize(_ptr(y, "y"), d, nd, int(D), _ptr(out, "out"),
                                  _stream(stream)),
           "semd_deserialize")
    return out


def semd_extrema(h: torch.Tensor, stream=None):
    """(maxima indices, minima indices) of a 1D device signal, as int32 tensors."""
    L = h.numel()
    ph = _dev_f64(h, "h")
    imax = torch.empty(L // 2 + 1, dtype=torch.int32, device=h.device)
    imin = torch.empty(L // 2 + 1, dtype=torch.int32, device=h.device)
    counts = torch.empty(2, dtype=torch.int32, device=h.device)
    _check(lib().semd_extrema(ph, L, imax.data_ptr(), imin.data_ptr(),
                              counts.data_ptr(), _stream(stream)), "semd_extrema")
    c = counts.cpu()
    return imax[: int(c[0])], imin[: int(c[1])]


def semd_noise(seed: int, item: int, m: int, L: int, w: torch.Tensor | None = None,
               device="cuda", stream=None) -> torch.Tensor:
    if w is None:
        w = torch.empty(L, dtype=torch.float64, device=device)
    _check(lib().semd_noise(int(seed) & (2**64 - 1), int(item), int(m), int(L),
                            _dev_f64(w, "w", int(L)), _stream(stream)), "semd_noise")
    return w


def semd_release_cached_memory() -> None:
    """Return the library pools' cached device memory to the device."""
    _check(lib().semd_release_cached_memory(), "semd_release_cached_memory")


def semd_profile_enable(on: bool = True) -> None:
    _check(lib().semd_profile_enable(1 if on else 0), "semd_profile_enable")


def semd_profile_reset() -> None:
    _check(lib().semd_profile_reset(), "semd_profile_reset")


def semd_profile_read(kernel: str) -> tuple[int, float]:
    """(launches, summed milliseconds) of one kernel since the last reset."""
    n, ms = C.c_int64(), C.c_double()
    _check(lib().semd_profile_read(kernel.encode(), C.byref(n), C.byref(ms)),
           "semd_profile_read")
    return int(n.value), float(ms.value)


# ---------------------------------------------------------------------------
# conveniences
# ---------------------------------------------------------------------------

def decompose(X: torch.Tensor, M: int, N: int, D: int, K: int, S: int, stream=None,
              path: int = SEMD_PATH_AUTO, sd: float = 0.0):
    """Serial-EMD of one column-major M x N signal set (plain path)."""
    return semd_decompose_ex(X, [M, N], D, K, S, stream=stream, path=path, sd=sd)


def decompose_batch(Xs: Sequence[torch.Tensor], shapes: Sequence[tuple[int, int]], D: int, K: int,
                    S: int, stream=None, path: int = SEMD_PATH_AUTO, sd: float = 0.0):
    """Serial-EMD of many signal sets in one launch; returns (outs, counts)."""
    dev = Xs[0].device
    outs = [torch.empty((K + 1, M * N), dtype=torch.float64, device=dev) for (M, N) in shapes]
    counts = torch.empty(len(Xs), dtype=torch.int32, device=dev)
    semd_decompose_batch(Xs, [list(s) for s in shapes], outs, counts, D, K, S, stream=stream,
                         path=path, sd=sd)
    return outs, counts


class PreparedBatch:
    """A semd_item array built once and handed to semd_decompose_batch (or
    semd_eemd_batch) on every call, for loops that decompose the same buffers
    repeatedly without rebuilding the descriptors."""

    def __init__(self, signals, dims_list, outs, counts=None, D=0, max_imfs=8, sift_iters=10,
                 stats=None, ensemble=1, seed=0, noise_sigmas=None, item_ids=None,
                 path=SEMD_PATH_AUTO, sd=0.0):
        _check_shape_params(max_imfs, sift_iters)
        cviews = _count_views(counts, len(signals))
        sviews = _stats_views(stats, len(signals))
        self._keep = (list(signals), list(outs), counts, stats)
        self.items, self.n = _items(signals, dims_list, outs, cviews, max_imfs, noise_sigmas,
                                    item_ids, sviews)
        self.params = _params(D, max_imfs, sift_iters, ensemble, seed, path=path, sd=sd)
        self.eemd = ensemble > 1 or noise_sigmas is not None

    def run(self, stream=None) -> None:
        fn = lib().semd_eemd_batch if self.eemd else lib().semd_decompose_batch
        _check(fn(self.items, self.n, C.byref(self.params), _stream(stream)),
               "semd_eemd_batch" if self.eemd else "semd_decompose_batch")


# ---------------------------------------------------------------------------
# serving engine (continuous batching)
# ---------------------------------------------------------------------------

class Engine:
    """Continuous-batching engine (semd_engine_*): requests are admitted
    between steps while their device footprint fits the budget; every step
    advances all resident requests by one sift."""

    def __init__(self, hbm_budget_bytes: int, max_requests: int):
        h = C.c_void_p()
        _check(lib().semd_engine_create(int(hbm_budget_bytes), int(max_requests), C.byref(h)),
               "semd_engine_create")
        self._h = h
        self._keep: dict[int, tuple] = {}

    @staticmethod
    def footprint(dims: Sequence[int], D: int, K: int, S: int,
                  path: int = SEMD_PATH_AUTO) -> int:
        it = semd_item()
        it.signal = 1
        it.imfs_out = 1
        for k, v in enumerate(dims):
            it.dims[k] = int(v)
        it.ndim = len(dims)
        p = _params(D, K, S, path=path)
        b = C.c_size_t()
        _check(lib().semd_engine_footprint(C.byref(it), C.byref(p), C.byref(b)),
               "semd_engine_footprint")
        return int(b.value)

    def admit(self, signal: torch.Tensor, dims: Sequence[int], out: torch.Tensor,
              n_imfs: torch.Tensor | None, D: int, K: int, S: int,
              sd: float = 0.0, path: int = SEMD_PATH_AUTO) -> int | None:
        """Ticket of the admitted request, or None when it does not fit now."""
        _check_shape_params(K, S)
        arr, _ = _items([signal], [dims], [out],
                        [n_imfs] if n_imfs is not None else None, K)
        p = _params(D, K, S, sd=sd, path=path)
        t = C.c_int64()
        rc = lib().semd_engine_admit(self._h, arr, C.byref(p), C.byref(t))
        if rc == SEMD_EBUSY:
            return None  # fits the budget once resident requests finish
        _check(rc, "semd_engine_admit")
        self._keep[t.value] = (signal, out, n_imfs)
        return int(t.value)

    def step(self, stream=None) -> None:
        _check(lib().semd_engine_step(self._h, _stream(stream)), "semd_engine_step")

    def step_n(self, n_steps: int, stream=None) -> None:
        """n_steps steps in one call; completions are gathered after the last."""
        _check(lib().semd_engine_step_n(self._h, int(n_steps), _stream(stream)),
               "semd_engine_step_n")

    def poll(self, cap: int = 4096) -> list[int]:
        buf = (C.c_int64 * cap)()
        n = C.c_int()
        _check(lib().semd_engine_poll(self._h, buf, cap, C.byref(n)), "semd_engine_poll")
        done = [int(buf[i]) for i in range(n.value)]
        for t in done:
            self._keep.pop(t, None)
        return done

    def resident(self) -> int:
        n = C.c_int()
        _check(lib().semd_engine_resident(self._h, C.byref(n)), "semd_engine_resident")
        return int(n.value)

    def close(self) -> None:
        if self._h:
            _check(lib().semd_engine_destroy(self._h), "semd_engine_destroy")
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
