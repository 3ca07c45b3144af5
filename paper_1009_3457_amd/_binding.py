"""ctypes binding of libfmm2d.so: the C ABI of include/fmm2d.h and
include/fgt2d.h on torch tensors.

Every function here only marshals arguments (device pointers of contiguous
tensors, sizes, the current HIP stream) and allocates outputs with torch; all
arithmetic runs in the library's HIP kernels.  A missing or unloadable library
raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm2d.so")

F32, BF16X3, F16X3, F32_PASCAL, F64_HANKEL = 0, 1, 2, 3, 4
PRECISIONS = {"f32": F32, "bf16x3": BF16X3, "f16x3": F16X3, "f32_pascal": F32_PASCAL, "f64_hankel": F64_HANKEL}

_lock = threading.Lock()
_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t

# name -> (restype, argtypes); mirrors include/fmm2d.h
_SIGNATURES = {
    "fmm2d_abi_version": (_int, []),
    "fmm2d_last_error": (ctypes.c_char_p, []),
    "fmm2d_num_boxes": (_i64, [_int]),
    "fmm2d_level_offset": (_i64, [_int]),
    "fmm2d_translation_count": (_i64, [_int, _int]),
    "fmm2d_build_tree_workspace": (_sz, [_i64, _int]),
    "fmm2d_build_tree": (_int, [_vp, _i64, _int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "fmm2d_build_tree_noalloc": (_int, [_vp, _i64, _int, _vp, _vp, _vp, _vp]),
    "fmm2d_gather": (_int, [_vp, _vp, _i64, _int, _vp, _vp]),
    "fmm2d_scatter": (_int, [_vp, _vp, _i64, _int, _vp, _vp]),
    "fmm2d_p2m": (_int, [_vp, _vp, _vp, _int, _int, _vp, _vp]),
    "fmm2d_m2m": (_int, [_vp, _int, _int, _vp]),
    "fmm2d_m2l_operators_bytes": (_sz, [_int, _int]),
    "fmm2d_m2l_operators": (_int, [_int, _int, _vp, _sz, _vp]),
    "fmm2d_m2l": (_int, [_vp, _vp, _vp, _int, _int, _int, _int, _int, _vp, _sz, _vp]),
    "fmm2d_m2l_backward": (_int, [_vp, _vp, _vp, _int, _int, _int, _int, _int, _vp, _sz, _vp]),
    "fmm2d_l2l": (_int, [_vp, _vp, _vp, _vp, _int, _int, _vp]),
    "fmm2d_l2p": (_int, [_vp, _vp, _i64, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "fmm2d_p2p": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _int, _vp, _vp, _vp]),
    "fmm2d_l2p_backward": (_int, [_vp, _vp, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "fmm2d_l2l_backward": (_int, [_vp, _vp, _vp, _vp, _int, _int, _vp]),
    "fmm2d_m2m_backward": (_int, [_vp, _int, _int, _vp]),
    "fmm2d_p2m_backward": (_int, [_vp, _vp, _vp, _i64, _int, _int, _vp, _vp, _vp, _vp]),
    "fmm2d_p2p_backward": (_int, [_vp, _vp, _vp, _i64, _vp, _vp, _int, _vp, _vp, _vp, _vp, _vp]),
    # include/fgt2d.h
    "fgt2d_hermite_coeffs": (_int, [_vp, _vp, _vp, _int, _int, ctypes.c_float, _vp, _vp]),
    "fgt2d_hermite_eval": (_int, [_vp, _i64, _int, _int, ctypes.c_float, _int, _vp, _vp, _vp]),
}


def load():
    """Load libfmm2d.so (raises OSError if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise OSError(f"{LIB_PATH} is missing: run paper_1009_3457_amd.build.build() first")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
        return _lib


class FMMError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        msg = load().fmm2d_last_error().decode()
        raise FMMError(f"libfmm2d status {rc}: {msg}")


def _p(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return _vp(t.data_ptr())


def _stream(device=None):
    return _vp(torch.cuda.current_stream(device).cuda_stream)


def _dev(*ts):
    """The one GPU device all given tensors (None skipped) live on."""
    ts = [t for t in ts if t is not None]
    dev = ts[0].device
    if dev.type != "cuda":
        raise ValueError("tensors must be on a GPU device")
    for t in ts[1:]:
        if t.device != dev:
            raise ValueError(f"tensors on different devices: {dev} and {t.device}")
    return dev


def _arg(t, name, dtype, shape, optional=False):
    """Checks one tensor argument against the layout the C ABI reads (dtype,
    exact shape, contiguity) before any pointer is passed: a wrong dtype would
    be reinterpreted and a short buffer read or written past its end."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    dts = dtype if isinstance(dtype, tuple) else (dtype,)
    if t.dtype not in dts:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dts)}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _depth_ok(depth: int, lo: int = 2) -> int:
    """The tree entry points take depth 2..12, the fast Gauss transform 0..12."""
    if not lo <= int(depth) <= 12:
        raise ValueError(f"depth {depth} outside {lo}..12")
    return int(depth)


def _nleaf1(depth: int) -> int:
    return (1 << (2 * depth)) + 1


def _points(t, name):
    """[n, 2] float32 points; returns n."""
    _arg(t, name, torch.float32, None)
    if t.dim() != 2 or t.shape[1] != 2:
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected (n, 2)")
    return t.shape[0]


# ------------------------------------------------------------ queries ---

def num_boxes(depth: int) -> int:
    return int(load().fmm2d_num_boxes(depth))


def level_offset(level: int) -> int:
    return int(load().fmm2d_level_offset(level))


def translation_count(lmin: int, lmax: int) -> int:
    return int(load().fmm2d_translation_count(lmin, lmax))


# ---------------------------------------------------------------- tree ---

def build_tree(xy: torch.Tensor, depth: int, check: bool = True):
    """Stable leaf sort: returns (perm [n] int32, leaf_start [4^depth+1] int32).

    The library writes a device-side domain flag instead of waiting for the
    device.  With check=True it is read here (one wait on the stream) and a
    point outside [0,1]^2 or NaN raises FMMError; with check=False the flag
    (uint32 [1], nonzero for such a point) is returned as a third value for
    the caller to read when it chooses."""
    n = _points(xy, "xy")
    depth = _depth_ok(depth)
    dev = _dev(xy)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    ls = torch.empty(_nleaf1(depth), dtype=torch.int32, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    wsb = int(load().fmm2d_build_tree_workspace(n, depth))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    _check(load().fmm2d_build_tree(_p(xy), n, depth, _p(perm), _p(ls), _p(flag), _p(ws), wsb, _stream(dev)))
    if not check:
        return perm, ls, flag
    check_domain(flag)
    return perm, ls


NOALLOC_MAX_POINTS = 1 << 22


def build_tree_noalloc(xy: torch.Tensor, depth: int, perm=None, leaf_start=None, flag=None):
    """build_tree through fmm2d_build_tree_noalloc: the sort's workspace is the
    library's own device array, so the call itself allocates nothing (pass
    perm [n] int32, leaf_start [4^depth+1] int32 and flag [1] int32 to keep
    this wrapper from allocating them).  n <= NOALLOC_MAX_POINTS.  Returns
    (perm, leaf_start, flag); the flag is not read here."""
    n = _points(xy, "xy")
    depth = _depth_ok(depth)
    _arg(perm, "perm", torch.int32, (n,), optional=True)
    _arg(leaf_start, "leaf_start", torch.int32, (_nleaf1(depth),), optional=True)
    _arg(flag, "flag", torch.int32, (1,), optional=True)
    dev = _dev(xy, perm, leaf_start, flag)
    perm = torch.empty(n, dtype=torch.int32, device=dev) if perm is None else perm
    leaf_start = torch.empty(_nleaf1(depth), dtype=torch.int32, device=dev) if leaf_start is None else leaf_start
    flag = torch.empty(1, dtype=torch.int32, device=dev) if flag is None else flag
    _check(load().fmm2d_build_tree_noalloc(_p(xy), n, depth, _p(perm), _p(leaf_start), _p(flag), _stream(dev)))
    return perm, leaf_start, flag


def check_domain(*flags):
    """Raises FMMError when any domain flag from build_tree(check=False) is
    set (this waits for the stream that wrote it)."""
    for f in flags:
        if int(f.item()) != 0:
            raise FMMError("libfmm2d: a point lies outside [0,1]^2 or is NaN")


def _rows(src: torch.Tensor, perm: torch.Tensor):
    _arg(perm, "perm", torch.int32, None)
    if perm.dim() != 1:
        raise ValueError(f"perm: shape {tuple(perm.shape)}, expected (n,)")
    _arg(src, "src", (torch.float32, torch.complex64), None)
    if src.dim() < 1 or src.shape[0] != perm.shape[0]:
        raise ValueError(f"src has {src.shape[0] if src.dim() else 0} rows, perm {perm.shape[0]}")
    per_row = src.numel() // max(src.shape[0], 1)
    return perm.shape[0], per_row * (2 if src.is_complex() else 1)


def gather(src: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """dst[i] = src[perm[i]] for float32 / complex64 rows."""
    n, width = _rows(src, perm)
    dev = _dev(src, perm)
    dst = torch.empty_like(src)
    _check(load().fmm2d_gather(_p(src), _p(perm), n, width, _p(dst), _stream(dev)))
    return dst


def scatter(src: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """dst[perm[i]] = src[i] for float32 / complex64 rows."""
    n, width = _rows(src, perm)
    dev = _dev(src, perm)
    dst = torch.empty_like(src)
    _check(load().fmm2d_scatter(_p(src), _p(perm), n, width, _p(dst), _stream(dev)))
    return dst


def _sources(xy_sorted, q_sorted, leaf_start, depth):
    """Checks the sorted sources of a tree; returns their count."""
    n = _points(xy_sorted, "xy_sorted")
    _arg(q_sorted, "q_sorted", torch.float32, (n,))
    _arg(leaf_start, "leaf_start", torch.int32, (_nleaf1(depth),))
    return n


def _expansion(t, name, depth, p, dtype=torch.complex64, optional=False):
    return _arg(t, name, dtype, (num_boxes(depth), p), optional)


def _per_box(t, name, depth, dtype=torch.complex64, optional=True):
    return _arg(t, name, dtype, (num_boxes(depth),), optional)


# -------------------------------------------------------- upward sweep ---

def p2m(xy_sorted, q_sorted, leaf_start, depth: int, p: int, M=None):
    depth = _depth_ok(depth)
    _sources(xy_sorted, q_sorted, leaf_start, depth)
    _expansion(M, "M", depth, p, optional=True)
    dev = _dev(xy_sorted, q_sorted, leaf_start, M)
    if M is None:
        M = torch.zeros(num_boxes(depth), p, dtype=torch.complex64, device=dev)
    _check(load().fmm2d_p2m(_p(xy_sorted), _p(q_sorted), _p(leaf_start), depth, p, _p(M), _stream(dev)))
    return M


def m2m(M, depth: int, p: int):
    depth = _depth_ok(depth)
    _expansion(M, "M", depth, p)
    _check(load().fmm2d_m2m(_p(M), depth, p, _stream(_dev(M))))
    return M


# ------------------------------------------------------ downward sweep ---

_ops_cache = {}


def m2l_operators(p: int, precision: int, device) -> torch.Tensor:
    """The operator bank for (p, precision) on `device` (generated once)."""
    device = torch.device(device)
    key = (device.index, p, precision)
    ops = _ops_cache.get(key)
    if ops is None:
        nbytes = int(load().fmm2d_m2l_operators_bytes(p, precision))
        if nbytes == 0:
            raise FMMError(f"no operator bank for p={p}, precision={precision}")
        ops = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _check(load().fmm2d_m2l_operators(p, precision, _p(ops), nbytes, _stream(device)))
        _ops_cache[key] = ops
    return ops


def _ops_arg(ops, p, precision):
    _arg(ops, "ops", torch.uint8, None)
    need = int(load().fmm2d_m2l_operators_bytes(p, precision))
    if ops.dim() != 1 or ops.numel() < need:
        raise ValueError(f"ops: {ops.numel()} bytes, the bank for p={p}, precision={precision} needs {need}")
    return ops


def m2l(M, depth: int, p: int, lmin: int = 2, lmax: int | None = None, precision: int = F32,
        L=None, b=None, with_b: bool = True, ops=None):
    """M2L + reduction on levels lmin..lmax; returns (L, b) (b None if not with_b)."""
    depth = _depth_ok(depth)
    lmax = depth if lmax is None else lmax
    _expansion(M, "M", depth, p)
    _expansion(L, "L", depth, p, optional=True)
    _per_box(b, "b", depth)
    if ops is not None:
        _ops_arg(ops, p, precision)
    dev = _dev(M, L, b, ops)
    nb = num_boxes(depth)
    if L is None:
        L = torch.zeros(nb, p, dtype=torch.complex64, device=dev)
    if b is None and with_b:
        b = torch.zeros(nb, dtype=torch.complex64, device=dev)
    ops = m2l_operators(p, precision, dev) if ops is None else ops
    _check(load().fmm2d_m2l(_p(M), _p(L), _p(b), depth, p, lmin, lmax, precision, _p(ops), ops.numel(),
                            _stream(dev)))
    return L, b


def m2l_backward(gL, gb, depth: int, p: int, lmin: int = 2, lmax: int | None = None,
                 precision: int = F32, gM=None, ops=None):
    """Plain transpose of m2l; returns gM (levels lmin..lmax written)."""
    depth = _depth_ok(depth)
    lmax = depth if lmax is None else lmax
    _expansion(gL, "gL", depth, p)
    _per_box(gb, "gb", depth)
    _expansion(gM, "gM", depth, p, optional=True)
    if ops is not None:
        _ops_arg(ops, p, precision)
    dev = _dev(gL, gb, gM, ops)
    if gM is None:
        gM = torch.zeros(num_boxes(depth), p, dtype=torch.complex64, device=dev)
    ops = m2l_operators(p, precision, dev) if ops is None else ops
    _check(load().fmm2d_m2l_backward(_p(gL), _p(gb), _p(gM), depth, p, lmin, lmax, precision, _p(ops),
                                     ops.numel(), _stream(dev)))
    return gM


def l2l(Lm2l, bm2l, depth: int, p: int):
    depth = _depth_ok(depth)
    _expansion(Lm2l, "Lm2l", depth, p)
    _per_box(bm2l, "bm2l", depth)
    dev = _dev(Lm2l, bm2l)
    nb = num_boxes(depth)
    L = torch.empty(nb, p, dtype=torch.complex128, device=dev)
    b = None if bm2l is None else torch.empty(nb, dtype=torch.complex128, device=dev)
    _check(load().fmm2d_l2l(_p(Lm2l), _p(bm2l), _p(L), _p(b), depth, p, _stream(dev)))
    return L, b


def _targets_out(phi, field, nt):
    _arg(phi, "phi", torch.complex64, (nt,), optional=True)
    _arg(field, "field", torch.complex64, (nt,), optional=True)


def l2p(txy_sorted, tleaf_start, L, b, depth: int, p: int, phi=None, field=None):
    depth = _depth_ok(depth)
    nt = _points(txy_sorted, "txy_sorted")
    _arg(tleaf_start, "tleaf_start", torch.int32, (_nleaf1(depth),))
    _expansion(L, "L", depth, p, dtype=torch.complex128)
    _per_box(b, "b", depth, dtype=torch.complex128)
    _targets_out(phi, field, nt)
    dev = _dev(txy_sorted, tleaf_start, L, b, phi, field)
    if phi is None:
        phi = torch.zeros(nt, dtype=torch.complex64, device=dev)
    if field is None:
        field = torch.zeros(nt, dtype=torch.complex64, device=dev)
    _check(load().fmm2d_l2p(_p(txy_sorted), _p(tleaf_start), nt, _p(L), _p(b), depth, p, _p(phi),
                            _p(field), _stream(dev)))
    return phi, field


def p2p(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, depth: int, phi=None, field=None):
    depth = _depth_ok(depth)
    _sources(xy_sorted, q_sorted, leaf_start, depth)
    nt = _points(txy_sorted, "txy_sorted")
    _arg(tleaf_start, "tleaf_start", torch.int32, (_nleaf1(depth),))
    _targets_out(phi, field, nt)
    dev = _dev(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, phi, field)
    if phi is None:
        phi = torch.zeros(nt, dtype=torch.complex64, device=dev)
    if field is None:
        field = torch.zeros(nt, dtype=torch.complex64, device=dev)
    _check(load().fmm2d_p2p(_p(xy_sorted), _p(q_sorted), _p(leaf_start), _p(txy_sorted),
                            _p(tleaf_start), nt, depth, _p(phi), _p(field), _stream(dev)))
    return phi, field


# ---------------------------------------------------------- transposes ---

def l2p_backward(txy_sorted, tleaf_start, cphi, cfield, depth: int, p: int):
    depth = _depth_ok(depth)
    nt = _points(txy_sorted, "txy_sorted")
    _arg(tleaf_start, "tleaf_start", torch.int32, (_nleaf1(depth),))
    _arg(cphi, "cphi", torch.complex64, (nt,), optional=True)
    _arg(cfield, "cfield", torch.complex64, (nt,), optional=True)
    dev = _dev(txy_sorted, tleaf_start, cphi, cfield)
    nb = num_boxes(depth)
    gL = torch.zeros(nb, p, dtype=torch.complex128, device=dev)
    gb = torch.zeros(nb, dtype=torch.complex128, device=dev)
    _check(load().fmm2d_l2p_backward(_p(txy_sorted), _p(tleaf_start), _p(cphi), _p(cfield), depth, p,
                                     _p(gL), _p(gb), _stream(dev)))
    return gL, gb


def l2l_backward(gL, gb, depth: int, p: int):
    depth = _depth_ok(depth)
    _expansion(gL, "gL", depth, p, dtype=torch.complex128)
    _per_box(gb, "gb", depth, dtype=torch.complex128)
    dev = _dev(gL, gb)
    nb = num_boxes(depth)
    gLm = torch.zeros(nb, p, dtype=torch.complex64, device=dev)
    gbm = None if gb is None else torch.zeros(nb, dtype=torch.complex64, device=dev)
    _check(load().fmm2d_l2l_backward(_p(gL), _p(gb), _p(gLm), _p(gbm), depth, p, _stream(dev)))
    return gLm, gbm


def m2m_backward(gM, depth: int, p: int):
    depth = _depth_ok(depth)
    _expansion(gM, "gM", depth, p)
    _check(load().fmm2d_m2m_backward(_p(gM), depth, p, _stream(_dev(gM))))
    return gM


def p2m_backward(xy_sorted, q_sorted, leaf_start, depth: int, p: int, gM):
    depth = _depth_ok(depth)
    n = _sources(xy_sorted, q_sorted, leaf_start, depth)
    _expansion(gM, "gM", depth, p)
    dev = _dev(xy_sorted, q_sorted, leaf_start, gM)
    gq = torch.empty(n, dtype=torch.float32, device=dev)
    G = torch.empty(n, dtype=torch.complex64, device=dev)
    _check(load().fmm2d_p2m_backward(_p(xy_sorted), _p(q_sorted), _p(leaf_start), n, depth, p, _p(gM),
                                     _p(gq), _p(G), _stream(dev)))
    return gq, G


def p2p_backward(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, depth: int, cphi, cfield,
                 gq, G):
    depth = _depth_ok(depth)
    n = _sources(xy_sorted, q_sorted, leaf_start, depth)
    nt = _points(txy_sorted, "txy_sorted")
    _arg(tleaf_start, "tleaf_start", torch.int32, (_nleaf1(depth),))
    _arg(cphi, "cphi", torch.complex64, (nt,), optional=True)
    _arg(cfield, "cfield", torch.complex64, (nt,), optional=True)
    _arg(gq, "gq", torch.float32, (n,))
    _arg(G, "G", torch.complex64, (n,))
    dev = _dev(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, cphi, cfield, gq, G)
    _check(load().fmm2d_p2p_backward(_p(xy_sorted), _p(q_sorted), _p(leaf_start), n, _p(txy_sorted),
                                     _p(tleaf_start), depth, _p(cphi), _p(cfield), _p(gq), _p(G),
                                     _stream(dev)))
    return gq, G


# ------------------------------------------- fast Gauss transform (FGT) ---

def fgt_hermite_coeffs(xy_sorted, q_sorted, leaf_start, depth: int, p: int, sigma: float):
    """Hermite coefficients of every box: float32 [4^depth, p, p] ([box, a, b])."""
    depth = _depth_ok(depth, lo=0)
    _sources(xy_sorted, q_sorted, leaf_start, depth)
    dev = _dev(xy_sorted, q_sorted, leaf_start)
    A = torch.empty(1 << (2 * depth), p, p, dtype=torch.float32, device=dev)
    _check(load().fgt2d_hermite_coeffs(_p(xy_sorted), _p(q_sorted), _p(leaf_start), depth, p, float(sigma),
                                       _p(A), _stream(dev)))
    return A


def fgt_hermite_eval(txy, depth: int, p: int, sigma: float, K: int, A, G=None):
    """Hermite-series evaluation at the targets txy [nt, 2]: float32 [nt]."""
    depth = _depth_ok(depth, lo=0)
    nt = _points(txy, "txy")
    _arg(A, "A", torch.float32, (1 << (2 * depth), p, p))
    _arg(G, "G", torch.float32, (nt,), optional=True)
    dev = _dev(txy, A, G)
    if G is None:
        G = torch.empty(nt, dtype=torch.float32, device=dev)
    _check(load().fgt2d_hermite_eval(_p(txy), nt, depth, p, float(sigma), int(K), _p(A), _p(G),
                                     _stream(dev)))
    return G
