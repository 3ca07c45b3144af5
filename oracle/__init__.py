"""FP64 CPU oracle for the 2D FMM of arXiv:1009.3457 (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does; the two
share no code.  Each function below is a thin ctypes wrapper around the plain C
in ``fmm2d_oracle.c`` (see the citations there), plus the exact power-of-two
change of basis between the paper's unscaled expansions and the scaled ones the
GPU library stores.  The fast Gauss transform's Hermite evaluation (Sec. 4.2)
is in ``fgt2d_oracle.c``, wrapped by ``oracle.fgt``.

Conventions (all arrays numpy):
  * points ``xy`` float64 ``[n, 2]`` (the FP32 inputs promoted exactly);
  * expansions complex128 ``[nbox_total, p]``, levels at offset (4^l-1)/3,
    Morton order inside a level;
  * the log-potential constant ``b`` complex128 ``[nbox_total]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fmm2d_oracle.c"), os.path.join(_HERE, "fgt2d_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int


def _stale() -> bool:
    if not os.path.exists(_LIB_PATH):
        return True
    built = os.path.getmtime(_LIB_PATH)
    return any(os.path.getmtime(src) > built for src in _SRCS)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math) into liboracle.so."""
    if not force and not _stale():
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", "-shared", "-fPIC", *_SRCS, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if _stale():
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ora_num_boxes.restype = _i64
        lib.ora_num_boxes.argtypes = [_int]
        lib.ora_level_offset.restype = _i64
        lib.ora_level_offset.argtypes = [_int]
        lib.ora_morton.restype = _i64
        lib.ora_morton.argtypes = [_i64, _i64, _int]
        lib.ora_build_tree.restype = _int
        lib.ora_build_tree.argtypes = [_dp, _i64, _int, _i32p, _i32p]
        lib.ora_p2m.argtypes = [_dp, _dp, _i32p, _int, _int, _dp]
        lib.ora_m2m.argtypes = [_dp, _int, _int]
        lib.ora_interaction_list.restype = _int
        lib.ora_interaction_list.argtypes = [_int, _i64, _i64, _i64p]
        lib.ora_m2l_operator.argtypes = [ctypes.c_double, ctypes.c_double, _int, _dp]
        lib.ora_log_row.argtypes = [ctypes.c_double, ctypes.c_double, _int, _dp]
        lib.ora_m2l.argtypes = [_dp, _dp, _dp, _int, _int, _int, _int]
        lib.ora_m2l_boxes.argtypes = [_dp, _int, _int, _i64p, _i64, _dp, _dp]
        lib.ora_m2l_transpose.argtypes = [_dp, _dp, _dp, _int, _int, _int, _int]
        lib.ora_m2l_transpose_boxes.argtypes = [_dp, _dp, _int, _int, _i64p, _i64, _dp]
        lib.ora_set_num_threads.argtypes = [_int]
        lib.ora_l2l.argtypes = [_dp, _dp, _dp, _dp, _int, _int]
        lib.ora_l2l_transpose.argtypes = [_dp, _dp, _int, _int]
        lib.ora_m2m_transpose.argtypes = [_dp, _int, _int]
        lib.ora_l2p.argtypes = [_dp, _i32p, _dp, _dp, _int, _int, _dp, _dp]
        lib.ora_l2p_transpose.argtypes = [_dp, _i32p, _dp, _dp, _int, _int, _dp, _dp]
        lib.ora_p2p.argtypes = [_dp, _dp, _i32p, _dp, _i32p, _int, _dp, _dp]
        lib.ora_p2p_transpose.argtypes = [_dp, _dp, _i32p, _dp, _i32p, _int, _dp, _dp,
                                          _dp, _dp]
        lib.ora_p2m_transpose.argtypes = [_dp, _dp, _i32p, _int, _int, _dp, _dp, _dp]
        lib.ora_direct.argtypes = [_dp, _dp, _i64, _dp, _i64, _dp, _dp]
        lib.ora_direct_grad.argtypes = [_dp, _dp, _i64, _dp, _i64, _dp, _dp, _dp]
        lib.ora_hermite_functions.argtypes = [ctypes.c_double, _int, _dp]
        lib.ora_fgt_direct.argtypes = [_dp, _dp, _i64, _dp, _i64, ctypes.c_double, _dp]
        lib.ora_fgt_direct_boxes.argtypes = [_dp, _dp, _i32p, _int, _dp, _i64, ctypes.c_double,
                                             _int, _dp]
        lib.ora_fgt_hermite_coeffs.argtypes = [_dp, _dp, _i32p, _int, _int, ctypes.c_double, _dp]
        lib.ora_fgt_hermite_eval.argtypes = [_dp, _i64, _int, _int, ctypes.c_double, _int, _dp,
                                             _dp]
        lib.ora_num_threads.restype = _int
        lib.ora_num_threads.argtypes = []
        lib.ora_init()
        _lib = lib
        return lib


def _d(a):
    """Pointer to a C-contiguous float64 / complex128 array (or NULL)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"] and a.dtype in (np.float64, np.complex128), a.dtype
    return a.ctypes.data_as(_dp)


def _i32(a):
    assert a.flags["C_CONTIGUOUS"] and a.dtype == np.int32
    return a.ctypes.data_as(_i32p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


# ------------------------------------------------------------------ tree ---

def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Sets the OpenMP threads of the oracle's parallel loops."""
    _load().ora_set_num_threads(int(n))


def num_boxes(depth: int) -> int:
    return int(_load().ora_num_boxes(depth))


def level_offset(level: int) -> int:
    return int(_load().ora_level_offset(level))


def morton(ix: int, iy: int, level: int) -> int:
    return int(_load().ora_morton(ix, iy, level))


def build_tree(xy, depth: int):
    """Initialization stage: returns (perm, leaf_start) (int32)."""
    xy = _f64(xy)
    n = xy.shape[0]
    perm = np.empty(n, np.int32)
    leaf_start = np.empty((1 << (2 * depth)) + 1, np.int32)
    rc = _load().ora_build_tree(_d(xy), n, depth, _i32(perm), _i32(leaf_start))
    if rc != 0:
        raise ValueError("point outside [0,1]^2")
    return perm, leaf_start


def interaction_list(level: int, ix: int, iy: int):
    out = np.zeros(32, np.int64)
    cnt = _load().ora_interaction_list(level, ix, iy, out.ctypes.data_as(_i64p))
    return out[:cnt].copy()


# ------------------------------------------------------------- operators ---

def m2l_operator(d: complex, p: int) -> np.ndarray:
    """Eq. (eq:M2Lmat) for d = target centre - source centre: [p, p], A[n, k]."""
    A = np.zeros((p, p), np.complex128)
    _load().ora_m2l_operator(float(np.real(d)), float(np.imag(d)), p, _d(A))
    return A


def log_row(d: complex, p: int) -> np.ndarray:
    r = np.zeros(p, np.complex128)
    _load().ora_log_row(float(np.real(d)), float(np.imag(d)), p, _d(r))
    return r


# ---------------------------------------------------------------- stages ---

def p2m(xy_sorted, q_sorted, leaf_start, depth: int, p: int) -> np.ndarray:
    M = np.zeros((num_boxes(depth), p), np.complex128)
    _load().ora_p2m(_d(_f64(xy_sorted)), _d(_f64(q_sorted)), _i32(leaf_start), depth, p,
                    _d(M))
    return M


def m2m(M, depth: int, p: int) -> np.ndarray:
    M = _c128(M).copy()
    _load().ora_m2m(_d(M), depth, p)
    return M


def m2l(M, depth: int, p: int, lmin: int = 2, lmax: int | None = None, with_b=True):
    """M2L on levels lmin..lmax; returns (L, b) with other levels zero."""
    lmax = depth if lmax is None else lmax
    M = _c128(M)
    L = np.zeros((num_boxes(depth), p), np.complex128)
    b = np.zeros(num_boxes(depth), np.complex128) if with_b else None
    _load().ora_m2l(_d(M), _d(L), _d(b), depth, p, lmin, lmax)
    return L, b


def m2l_boxes(M_level, level: int, p: int, boxes):
    """M2L for selected target boxes (Morton indices) of one level."""
    M_level = _c128(M_level)
    boxes = np.ascontiguousarray(boxes, dtype=np.int64)
    L = np.zeros((boxes.size, p), np.complex128)
    b = np.zeros(boxes.size, np.complex128)
    _load().ora_m2l_boxes(_d(M_level), level, p, boxes.ctypes.data_as(_i64p), boxes.size,
                          _d(L), _d(b))
    return L, b


def m2l_transpose(gL, gb, depth: int, p: int, lmin: int = 2, lmax: int | None = None):
    lmax = depth if lmax is None else lmax
    gM = np.zeros((num_boxes(depth), p), np.complex128)
    _load().ora_m2l_transpose(_d(_c128(gL)), _d(None if gb is None else _c128(gb)), _d(gM),
                              depth, p, lmin, lmax)
    return gM


def m2l_transpose_boxes(gL_level, gb_level, level: int, p: int, boxes):
    """The transpose of m2l for selected source boxes (Morton indices) of one
    level, gathered over each source's own interaction list; returns gM
    [len(boxes), p]."""
    boxes = np.ascontiguousarray(boxes, dtype=np.int64)
    gM = np.zeros((boxes.size, p), np.complex128)
    _load().ora_m2l_transpose_boxes(_d(_c128(gL_level)), _d(None if gb_level is None else _c128(gb_level)),
                                    level, p, boxes.ctypes.data_as(_i64p), boxes.size, _d(gM))
    return gM


def l2l(Lm2l, bm2l, depth: int, p: int):
    L = np.zeros((num_boxes(depth), p), np.complex128)
    b = None if bm2l is None else np.zeros(num_boxes(depth), np.complex128)
    _load().ora_l2l(_d(_c128(Lm2l)), _d(None if bm2l is None else _c128(bm2l)), _d(L), _d(b),
                    depth, p)
    return L, b


def l2l_transpose(gL, gb, depth: int, p: int):
    gL = _c128(gL).copy()
    gb = None if gb is None else _c128(gb).copy()
    _load().ora_l2l_transpose(_d(gL), _d(gb), depth, p)
    return gL, gb


def m2m_transpose(gM, depth: int, p: int):
    gM = _c128(gM).copy()
    _load().ora_m2m_transpose(_d(gM), depth, p)
    return gM


def l2p(txy_sorted, tleaf_start, L, b, depth: int, p: int):
    nt = txy_sorted.shape[0]
    phi = np.zeros(nt, np.complex128)
    f = np.zeros(nt, np.complex128)
    _load().ora_l2p(_d(_f64(txy_sorted)), _i32(tleaf_start), _d(_c128(L)),
                    _d(None if b is None else _c128(b)), depth, p, _d(phi), _d(f))
    return phi, f


def l2p_transpose(txy_sorted, tleaf_start, cphi, cf, depth: int, p: int):
    gL = np.zeros((num_boxes(depth), p), np.complex128)
    gb = np.zeros(num_boxes(depth), np.complex128)
    _load().ora_l2p_transpose(_d(_f64(txy_sorted)), _i32(tleaf_start),
                              _d(None if cphi is None else _c128(cphi)),
                              _d(None if cf is None else _c128(cf)), depth, p, _d(gL), _d(gb))
    return gL, gb


def p2p(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, depth: int):
    nt = txy_sorted.shape[0]
    phi = np.zeros(nt, np.complex128)
    f = np.zeros(nt, np.complex128)
    _load().ora_p2p(_d(_f64(xy_sorted)), _d(_f64(q_sorted)), _i32(leaf_start),
                    _d(_f64(txy_sorted)), _i32(tleaf_start), depth, _d(phi), _d(f))
    return phi, f


def p2p_transpose(xy_sorted, q_sorted, leaf_start, txy_sorted, tleaf_start, depth, cphi, cf):
    n = xy_sorted.shape[0]
    gq = np.zeros(n, np.float64)
    G = np.zeros(n, np.complex128)
    _load().ora_p2p_transpose(_d(_f64(xy_sorted)), _d(_f64(q_sorted)), _i32(leaf_start),
                              _d(_f64(txy_sorted)), _i32(tleaf_start), depth,
                              _d(None if cphi is None else _c128(cphi)),
                              _d(None if cf is None else _c128(cf)), _d(gq), _d(G))
    return gq, G


def p2m_transpose(xy_sorted, q_sorted, leaf_start, depth: int, p: int, gM):
    n = xy_sorted.shape[0]
    gq = np.zeros(n, np.float64)
    G = np.zeros(n, np.complex128)
    _load().ora_p2m_transpose(_d(_f64(xy_sorted)), _d(_f64(q_sorted)), _i32(leaf_start),
                              depth, p, _d(_c128(gM)), _d(gq), _d(G))
    return gq, G


def direct(xy, q, txy):
    """Eq. (eq:n_body) by direct summation: returns (phi, f) complex128."""
    xy, q, txy = _f64(xy), _f64(q), _f64(txy)
    phi = np.zeros(txy.shape[0], np.complex128)
    f = np.zeros(txy.shape[0], np.complex128)
    _load().ora_direct(_d(xy), _d(q), xy.shape[0], _d(txy), txy.shape[0], _d(phi), _d(f))
    return phi, f


def direct_grad(xy, q, txy, cphi):
    """Exact source gradient of a loss through the direct sum; returns (gq, gxy)."""
    xy, q, txy = _f64(xy), _f64(q), _f64(txy)
    gq = np.zeros(xy.shape[0], np.float64)
    G = np.zeros(xy.shape[0], np.complex128)
    _load().ora_direct_grad(_d(xy), _d(q), xy.shape[0], _d(txy), txy.shape[0],
                            _d(_c128(cphi)), _d(gq), _d(G))
    return gq, np.stack([G.real, -G.imag], axis=1)


# ------------------------------------------------------- change of basis ---
# The GPU library stores M~_k = M_k / h^k and L~_n = L_n h^(n+1), h = 2^-l.
# Both factors are powers of two, so these conversions are exact in FP64.

def _level_of_box(depth: int) -> np.ndarray:
    lev = np.empty(num_boxes(depth), np.int64)
    for l in range(depth + 1):
        lev[level_offset(l):level_offset(l + 1)] = l
    return lev


def scale_multipoles(M, depth: int) -> np.ndarray:
    p = M.shape[1]
    lev = _level_of_box(depth)[:, None].astype(np.float64)
    k = np.arange(p)[None, :].astype(np.float64)
    return M * np.exp2(lev * k)  # M / h^k, h = 2^-l


def unscale_multipoles(Ms, depth: int) -> np.ndarray:
    p = Ms.shape[1]
    lev = _level_of_box(depth)[:, None].astype(np.float64)
    k = np.arange(p)[None, :].astype(np.float64)
    return Ms * np.exp2(-lev * k)


def scale_locals(L, depth: int) -> np.ndarray:
    p = L.shape[1]
    lev = _level_of_box(depth)[:, None].astype(np.float64)
    n = np.arange(p)[None, :].astype(np.float64)
    return L * np.exp2(-lev * (n + 1))  # L h^(n+1)


def unscale_locals(Ls, depth: int) -> np.ndarray:
    p = Ls.shape[1]
    lev = _level_of_box(depth)[:, None].astype(np.float64)
    n = np.arange(p)[None, :].astype(np.float64)
    return Ls * np.exp2(lev * (n + 1))


# ------------------------------------------------------------- pipeline ---

def fmm(xy, q, txy, depth: int, p: int, return_parts: bool = False):
    """The five stages of Sec. 2.1 in FP64; returns (phi, f) at the targets in
    their original order (and the intermediate arrays if return_parts)."""
    xy, q, txy = _f64(xy), _f64(q), _f64(txy)
    perm, ls = build_tree(xy, depth)
    tperm, tls = build_tree(txy, depth)
    xs, qs, ts = xy[perm], q[perm], txy[tperm]
    M = m2m(p2m(xs, qs, ls, depth, p), depth, p)
    Lm, bm = m2l(M, depth, p)
    L, b = l2l(Lm, bm, depth, p)
    phi_s, f_s = l2p(ts, tls, L, b, depth, p)
    pn, fn = p2p(xs, qs, ls, ts, tls, depth)
    phi = np.empty_like(phi_s)
    f = np.empty_like(f_s)
    phi[tperm] = phi_s + pn
    f[tperm] = f_s + fn
    if return_parts:
        parts = dict(perm=perm, leaf_start=ls, tperm=tperm, tleaf_start=tls, M=M, Lm2l=Lm,
                     bm2l=bm, L=L, b=b)
        return phi, f, parts
    return phi, f


def fmm_grad(xy, q, txy, depth: int, p: int, cphi, cf=None):
    """Gradient of a real loss through the FP64 FMM at a frozen tree.

    ``cphi`` = conj(dl/dRe phi + i dl/dIm phi) at the targets (original order),
    ``cf`` likewise for f (optional).  Returns (dl/dq [n], dl/dxy [n, 2]).
    Chain of plain transposes: L2P^T, L2L^T, M2L^T, M2M^T, P2M^T, plus P2P^T.
    """
    xy, q, txy = _f64(xy), _f64(q), _f64(txy)
    perm, ls = build_tree(xy, depth)
    tperm, tls = build_tree(txy, depth)
    xs, qs, ts = xy[perm], q[perm], txy[tperm]
    cp = None if cphi is None else _c128(cphi)[tperm]
    cfs = None if cf is None else _c128(cf)[tperm]
    gL, gb = l2p_transpose(ts, tls, cp, cfs, depth, p)
    gL, gb = l2l_transpose(gL, gb, depth, p)
    gM = m2l_transpose(gL, gb, depth, p)
    gM = m2m_transpose(gM, depth, p)
    gq_far, G_far = p2m_transpose(xs, qs, ls, depth, p, gM)
    gq_near, G_near = p2p_transpose(xs, qs, ls, ts, tls, depth, cp, cfs)
    gq_s = gq_far + gq_near
    G_s = G_far + G_near
    gq = np.empty_like(gq_s)
    G = np.empty_like(G_s)
    gq[perm] = gq_s
    G[perm] = G_s
    return gq, np.stack([G.real, -G.imag], axis=1)
