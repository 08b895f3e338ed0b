"""ctypes wrapper of the FP64 CPU oracle (oracle/gsc_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the benchmark's CPU-baseline
leg are the only callers. The product path never imports this module, and this module imports
nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsc_oracle.c")
_SRC_RLGR = os.path.join(_HERE, "rlgr_oracle.c")
_SRC_RANS = os.path.join(_HERE, "rans_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_CMD = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", _LIB, _SRC,
           _SRC_RLGR, _SRC_RANS, "-lm"]


def build_oracle() -> str:
    """Compile the oracle's shared library with gcc (always rebuilds)."""
    subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC_RLGR), os.path.getmtime(_SRC_RANS)):
            build_oracle()
        L = ctypes.CDLL(_LIB)
        i64, i32, u32, u64, dbl, vp = (ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p)
        L.orc_morton_encode.restype = u64
        L.orc_morton_encode.argtypes = [u32, u32, u32, i32]
        L.orc_morton_encode_n.restype = None
        L.orc_morton_encode_n.argtypes = [vp, i64, i32, vp]
        L.orc_morton_decode.restype = None
        L.orc_morton_decode.argtypes = [u64, i32, vp]
        L.orc_voxelize.restype = i32
        L.orc_voxelize.argtypes = [vp, i64, i32, i32, vp, vp, vp]
        L.orc_sort_merge.restype = i64
        L.orc_sort_merge.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp]
        L.orc_octree_levels.restype = i64
        L.orc_octree_levels.argtypes = [vp, i64, i32, vp, i64, vp, vp]
        L.orc_octree_encode.restype = i64
        L.orc_octree_encode.argtypes = [vp, i64, i32, vp, vp, i64]
        L.orc_octree_decode.restype = i64
        L.orc_octree_decode.argtypes = [vp, i64, vp, i32, vp, i64]
        L.orc_voxel_centres.restype = None
        L.orc_voxel_centres.argtypes = [vp, i64, i32, vp, dbl, vp, vp]
        L.orc_raht_prelude.restype = i64
        L.orc_raht_prelude.argtypes = [vp, i64, i32, vp, vp, vp, vp, i64]
        L.orc_raht_prelude_cap.restype = i64
        L.orc_raht_prelude_cap.argtypes = [i64, i32]
        L.orc_raht_forward.restype = i32
        L.orc_raht_forward.argtypes = [vp, i64, i32, vp, i32]
        L.orc_raht_inverse.restype = i32
        L.orc_raht_inverse.argtypes = [vp, i64, i32, vp, i32]
        L.orc_quantize1.restype = i32
        L.orc_quantize1.argtypes = [dbl, dbl, dbl]
        L.orc_quantize.restype = None
        L.orc_quantize.argtypes = [vp, i64, i32, vp, dbl, vp]
        L.orc_dequantize.restype = None
        L.orc_dequantize.argtypes = [vp, i64, i32, vp, vp]
        L.orc_encode_frame.restype = i32
        L.orc_encode_frame.argtypes = [vp, vp, i64, i32, i32, vp, dbl, i32, vp, vp, vp, vp, vp,
                                       i64, vp, vp, vp, vp]
        L.orc_decode_frame.restype = i64
        L.orc_decode_frame.argtypes = [vp, i64, vp, i32, i32, vp, vp, vp, dbl, i64, vp, vp, vp,
                                       vp]
        L.orc_ste_grad.restype = i32
        L.orc_ste_grad.argtypes = [vp, vp, i64, i32, i32, vp, dbl, dbl, i32, vp, vp, vp, vp, vp,
                                   vp, vp, vp, vp, vp]
        L.orc_rlgr_blocks.restype = i64
        L.orc_rlgr_blocks.argtypes = [i64, i32, i32]
        L.orc_rlgr_encode.restype = i64
        L.orc_rlgr_encode.argtypes = [vp, i64, i32, i32, vp, vp, i64]
        L.orc_rlgr_decode.restype = i32
        L.orc_rlgr_decode.argtypes = [vp, vp, i64, i32, i32, vp]
        L.orc_rans_table.restype = i32
        L.orc_rans_table.argtypes = [vp, i64, vp]
        L.orc_rans_chunks.restype = i64
        L.orc_rans_chunks.argtypes = [i64, i32]
        L.orc_rans_encode.restype = i64
        L.orc_rans_encode.argtypes = [vp, i64, i32, vp, vp, vp, i64]
        L.orc_rans_decode.restype = i32
        L.orc_rans_decode.argtypes = [vp, vp, i64, i32, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# --------------------------------------------------------------------------------------------
def morton_encode(x, y, z, J):
    return int(lib().orc_morton_encode(int(x), int(y), int(z), int(J)))


def morton_decode(code, J):
    out = np.zeros(3, dtype=np.uint32)
    lib().orc_morton_decode(int(code), int(J), _p(out))
    return tuple(int(v) for v in out)


def morton_encode_array(vox, J):
    vox = _c(vox, np.uint32).reshape(-1, 3)
    out = np.zeros(vox.shape[0], dtype=np.uint64)
    lib().orc_morton_encode_n(_p(vox), vox.shape[0], int(J), _p(out))
    return out


def sort_order(pos, J, bbox=None):
    """The stable sorted order of the Gaussians by Morton code and each one's voxel:
    (perm int64[n], voxel_of int64[n]) (voxelize, Morton, then sort_merge)."""
    vox, _, _ = voxelize(pos, J, bbox)
    keys = morton_encode_array(vox, J)
    _, _, perm, vof = sort_merge(keys)
    return perm, vof


def voxelize(pos, J, bbox=None):
    """Returns (vox n x 3 uint32, bbox_min float64[3], cell float)."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    vox = np.zeros((n, 3), dtype=np.uint32)
    bmin = np.zeros(3, dtype=np.float64)
    cell = np.zeros(1, dtype=np.float64)
    mode = 0
    if bbox is not None:
        mode = 1
        bmin[:] = bbox[0]
        cell[0] = bbox[1]
    _check(lib().orc_voxelize(_p(pos), n, J, mode, _p(bmin), _p(cell), _p(vox)), "voxelize")
    return vox, bmin, float(cell[0])


def sort_merge(keys, attr=None, C=0):
    """Returns (leaf codes, merged attributes Nv x C float64 or None, perm, voxel_of)."""
    keys = _c(keys, np.uint64)
    n = keys.shape[0]
    leaf = np.zeros(max(n, 1), dtype=np.uint64)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    vof = np.zeros(max(n, 1), dtype=np.int64)
    va = None
    if attr is not None:
        attr = _c(attr, np.float32).reshape(n, -1)
        C = attr.shape[1]
        va = np.zeros((max(n, 1), C), dtype=np.float64)
    nv = _check(lib().orc_sort_merge(_p(keys), _p(attr), n, C, _p(leaf), _p(va), _p(perm),
                                     _p(vof)), "sort_merge")
    return leaf[:nv], (None if va is None else va[:nv]), perm[:n], vof[:n]


def octree_levels(leaf, J):
    leaf = _c(leaf, np.uint64)
    nv = leaf.shape[0]
    cap = nv * (J + 1) + 1
    nodes = np.zeros(cap, dtype=np.uint64)
    off = np.zeros(J + 1, dtype=np.int64)
    sizes = np.zeros(J + 1, dtype=np.int64)
    _check(lib().orc_octree_levels(_p(leaf), nv, J, _p(nodes), cap, _p(off), _p(sizes)),
           "octree_levels")
    return [nodes[off[d]:off[d] + sizes[d]].copy() for d in range(J + 1)]


def octree_encode(leaf, J):
    """Returns (occupancy bytes uint8, level sizes int64[J+1])."""
    leaf = _c(leaf, np.uint64)
    nv = leaf.shape[0]
    cap = max(nv * J, 1)
    occ = np.zeros(cap, dtype=np.uint8)
    sizes = np.zeros(J + 1, dtype=np.int64)
    nb = _check(lib().orc_octree_encode(_p(leaf), nv, J, _p(sizes), _p(occ), cap),
                "octree_encode")
    return occ[:nb].copy(), sizes


def octree_decode(occ, level_sizes, J, cap=None):
    """Returns the leaf codes, or raises on a corrupt stream."""
    occ = _c(occ, np.uint8)
    sizes = _c(level_sizes, np.int64)
    if cap is None:
        cap = int(sizes[J])
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    nv = lib().orc_octree_decode(_p(occ), occ.shape[0], _p(sizes), J, _p(out), cap)
    if nv == -4:
        raise ValueError("corrupt occupancy stream")
    _check(nv, "octree_decode")
    return out[:nv].copy()


def voxel_centres(leaf, J, bbox_min, cell):
    leaf = _c(leaf, np.uint64)
    nv = leaf.shape[0]
    vox = np.zeros((nv, 3), dtype=np.uint32)
    pos = np.zeros((nv, 3), dtype=np.float64)
    bmin = _c(bbox_min, np.float64)
    lib().orc_voxel_centres(_p(leaf), nv, J, _p(bmin), float(cell), _p(vox), _p(pos))
    return vox, pos


def raht_prelude(M, J):
    """Alg. 4 lists: returns [(I_l, W_l, F_l) for l = 1..3J]."""
    M = _c(M, np.uint64)
    nv = M.shape[0]
    cap = max(int(lib().orc_raht_prelude_cap(nv, J)), 1)
    I = np.zeros(cap, dtype=np.int64)
    W = np.zeros(cap, dtype=np.int64)
    F = np.zeros(cap, dtype=np.uint8)
    off = np.zeros(3 * J + 1, dtype=np.int64)
    _check(lib().orc_raht_prelude(_p(M), nv, J, _p(I), _p(W), _p(F), _p(off), cap), "prelude")
    return [(I[off[l]:off[l + 1]].copy(), W[off[l]:off[l + 1]].copy(),
             F[off[l]:off[l + 1]].astype(bool)) for l in range(3 * J)]


def raht_forward(M, J, A):
    M = _c(M, np.uint64)
    Y = np.array(A, dtype=np.float64, order="C", copy=True)
    nv = M.shape[0]
    C = 1 if Y.ndim == 1 else Y.shape[1]
    _check(lib().orc_raht_forward(_p(M), nv, J, _p(Y), C), "raht_forward")
    return Y


def raht_inverse(M, J, Y):
    M = _c(M, np.uint64)
    A = np.array(Y, dtype=np.float64, order="C", copy=True)
    nv = M.shape[0]
    C = 1 if A.ndim == 1 else A.shape[1]
    _check(lib().orc_raht_inverse(_p(M), nv, J, _p(A), C), "raht_inverse")
    return A


def quantize1(y, step, tau=0.5):
    return int(lib().orc_quantize1(float(y), float(step), float(tau)))


def quantize(Y, step, tau=0.5):
    Y = _c(Y, np.float64)
    nv, C = Y.shape
    step = _c(step, np.float32)
    Q = np.zeros((nv, C), dtype=np.int32)
    lib().orc_quantize(_p(Y), nv, C, _p(step), float(tau), _p(Q))
    return Q


def dequantize(Q, step):
    Q = _c(Q, np.int32)
    nv, C = Q.shape
    step = _c(step, np.float32)
    Y = np.zeros((nv, C), dtype=np.float64)
    lib().orc_dequantize(_p(Q), nv, C, _p(step), _p(Y))
    return Y


def encode_frame(pos, attr, J, step, tau=0.5, bbox=None, want_y=False):
    """Whole-frame encode. Returns a dict with nv, leaf, level_sizes, occ, Q, vattr, (Y),
    bbox_min, cell."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    attr = _c(attr, np.float32)
    n = pos.shape[0]
    C = attr.shape[1]
    step = _c(step, np.float32)
    leaf = np.zeros(max(n, 1), dtype=np.uint64)
    sizes = np.zeros(J + 1, dtype=np.int64)
    occ_cap = max(n * J, 1)
    occ = np.zeros(occ_cap, dtype=np.uint8)
    Q = np.zeros((max(n, 1), C), dtype=np.int32)
    Y = np.zeros((max(n, 1), C), dtype=np.float64) if want_y else None
    va = np.zeros((max(n, 1), C), dtype=np.float64)
    bmin = np.zeros(3, dtype=np.float64)
    cell = np.zeros(1, dtype=np.float64)
    mode = 0
    if bbox is not None:
        mode = 1
        bmin[:] = bbox[0]
        cell[0] = bbox[1]
    res = np.zeros(2, dtype=np.int64)
    _check(lib().orc_encode_frame(_p(pos), _p(attr), n, J, C, _p(step), float(tau), mode,
                                  _p(bmin), _p(cell), _p(leaf), _p(sizes), _p(occ), occ_cap,
                                  _p(Q), _p(Y), _p(va), _p(res)), "encode_frame")
    nv, nb = int(res[0]), int(res[1])
    out = dict(nv=nv, leaf=leaf[:nv], level_sizes=sizes, occ=occ[:nb], Q=Q[:nv], vattr=va[:nv],
               bbox_min=bmin, cell=float(cell[0]))
    if want_y:
        out["Y"] = Y[:nv]
    return out


def decode_frame(occ, level_sizes, J, Q, step, bbox_min, cell):
    """Whole-frame decode. Returns dict(leaf, vox, pos (FP64 centres), attr (FP64))."""
    occ = _c(occ, np.uint8)
    sizes = _c(level_sizes, np.int64)
    Q = _c(Q, np.int32)
    C = Q.shape[1]
    step = _c(step, np.float32)
    nv = int(sizes[J])
    cap = max(nv, 1)
    leaf = np.zeros(cap, dtype=np.uint64)
    vox = np.zeros((cap, 3), dtype=np.uint32)
    pos = np.zeros((cap, 3), dtype=np.float64)
    attr = np.zeros((cap, C), dtype=np.float64)
    r = lib().orc_decode_frame(_p(occ), occ.shape[0], _p(sizes), J, C, _p(Q), _p(step),
                               _p(_c(bbox_min, np.float64)), float(cell), cap, _p(leaf), _p(vox),
                               _p(pos), _p(attr))
    if r == -4:
        raise ValueError("corrupt occupancy stream")
    _check(r, "decode_frame")
    return dict(leaf=leaf[:r], vox=vox[:r], pos=pos[:r], attr=attr[:r])


def ste_grad(pos, attr, J, step, tau=0.5, lam=0.01, bbox=None):
    """Straight-through coding loss and its gradient (R8). Returns a dict with nv, leaf,
    voxel_of, aref, yhat, ahat (Nv x C, FP64), grad (n x C, FP64), loss, dist, rate."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    attr = _c(attr, np.float32)
    n, C = attr.shape
    step = _c(step, np.float32)
    m = max(n, 1)
    leaf = np.zeros(m, dtype=np.uint64)
    vof = np.zeros(m, dtype=np.int64)
    aref = np.zeros((m, C), dtype=np.float64)
    yhat = np.zeros((m, C), dtype=np.float64)
    ahat = np.zeros((m, C), dtype=np.float64)
    grad = np.zeros((m, C), dtype=np.float64)
    loss = np.zeros(3, dtype=np.float64)
    res = np.zeros(1, dtype=np.int64)
    bmin = np.zeros(3, dtype=np.float64)
    cell = np.zeros(1, dtype=np.float64)
    mode = 0
    if bbox is not None:
        mode = 1
        bmin[:] = bbox[0]
        cell[0] = bbox[1]
    _check(lib().orc_ste_grad(_p(pos), _p(attr), n, J, C, _p(step), float(tau), float(lam), mode,
                              _p(bmin), _p(cell), _p(leaf), _p(vof), _p(aref), _p(yhat),
                              _p(ahat), _p(grad), _p(loss), _p(res)), "ste_grad")
    nv = int(res[0])
    return dict(nv=nv, leaf=leaf[:nv], voxel_of=vof[:n], aref=aref[:nv], yhat=yhat[:nv],
                ahat=ahat[:nv], grad=grad[:n], loss=float(loss[0]), dist=float(loss[1]),
                rate=float(loss[2]), bbox_min=bmin, cell=float(cell[0]))


# ------------------------------------------------------------------------- entropy coder
def rlgr_blocks(nv, C, B):
    return int(_check(lib().orc_rlgr_blocks(int(nv), int(C), int(B)), "rlgr_blocks"))


def rlgr_encode(Q, B):
    """Block-parallel RLGR of Q [nv][C] int32 (Sec. 3.4) with blocks of B values per channel.
    Returns (off int64[NB + 1] block word offsets, words uint32[off[-1]])."""
    Q = _c(Q, np.int32)
    nv, C = Q.shape
    NB = rlgr_blocks(nv, C, B)
    off = np.zeros(NB + 1, dtype=np.int64)
    total = _check(lib().orc_rlgr_encode(_p(Q), nv, C, int(B), _p(off), None, 0), "rlgr size")
    words = np.zeros(max(total, 1), dtype=np.uint32)
    _check(lib().orc_rlgr_encode(_p(Q), nv, C, int(B), _p(off), _p(words), total), "rlgr_encode")
    return off, words[:total]


def rlgr_decode(off, words, nv, C, B):
    """Inverse of rlgr_encode; raises ValueError on a block that does not decode exactly."""
    off = _c(off, np.int64)
    words = _c(words, np.uint32)
    if words.size == 0:
        words = np.zeros(1, dtype=np.uint32)
    Q = np.zeros((max(int(nv), 1), int(C)), dtype=np.int32)
    rc = lib().orc_rlgr_decode(_p(off), _p(words), int(nv), int(C), int(B), _p(Q))
    if rc == -3:
        raise ValueError("corrupt entropy-coded block")
    _check(rc, "rlgr_decode")
    return Q[:int(nv)]


# ------------------------------------------------------------------ occupancy-byte rANS coder
def rans_table(data):
    """A1: the frequency table (uint16[256], summing to 4096) of a byte string."""
    d = _c(np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data, np.uint8)
    f = np.zeros(256, dtype=np.uint16)
    _check(lib().orc_rans_table(_p(d), d.size, _p(f)), "rans_table")
    return f


def rans_encode(data, K, freq=None):
    """A2: (freq, chunk offsets int64[nc + 1], coded bytes uint8) of a byte string in chunks of
    K bytes; the table is the stream's own (A1) unless given."""
    d = _c(np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data, np.uint8)
    f = rans_table(d) if freq is None else _c(freq, np.uint16)
    nc = int(_check(lib().orc_rans_chunks(d.size, int(K)), "rans_chunks"))
    off = np.zeros(nc + 1, dtype=np.int64)
    total = _check(lib().orc_rans_encode(_p(d), d.size, int(K), _p(f), _p(off), None, 0), "rans size")
    out = np.zeros(max(total, 1), dtype=np.uint8)
    _check(lib().orc_rans_encode(_p(d), d.size, int(K), _p(f), _p(off), _p(out), total), "rans_encode")
    return f, off, out[:total]


def rans_decode(freq, off, coded, n, K):
    """A3: the n bytes the chunks decode to; raises ValueError on a chunk that does not decode
    exactly."""
    out = np.zeros(max(int(n), 1), dtype=np.uint8)
    cd = _c(coded, np.uint8) if len(coded) else np.zeros(1, dtype=np.uint8)
    rc = lib().orc_rans_decode(_p(_c(off, np.int64)), _p(cd), int(n), int(K), _p(_c(freq, np.uint16)), _p(out))
    if rc == -3:
        raise ValueError("corrupt rANS chunk")
    _check(rc, "rans_decode")
    return out[:int(n)]
