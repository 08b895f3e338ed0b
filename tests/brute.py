"""Pure-Python brute-force references for tiny inputs (<= a few hundred points).

They are written from the *definitions* in the paper, in formulations that differ from the
oracle's, so that a mistake in the oracle (a dropped term, a wrong sign, index or bit order)
shows up as a mismatch:

* octree bytes from voxel *coordinates* by a recursive level-order traversal of cubes
  (Sec. 2.1 "Recursive Octree Encoding"), not from Morton codes and sorted lists;
* RAHT by top-down recursion over the binary tree (Sec. 3.1: each octree level is three binary
  levels, one per axis), plus the equivalent closed form of every coefficient in terms of
  subtree sums;
* exact rational arithmetic (fractions) for voxelization and quantization.
"""
from __future__ import annotations

import math
from fractions import Fraction


# ------------------------------------------------------------------------------------------
# Octree by cubes (Sec. 2.1): the root is the whole 2^J cube; a node's child i covers the
# octant whose x half is bit 0 of i, y half bit 1 and z half bit 2 (the Morton triple is
# z y x with x least significant, Sec. 2.2). Bytes are emitted in level order, children
# visited 0..7.
# ------------------------------------------------------------------------------------------
def octree_bytes_by_cubes(vox, J):
    pts = sorted(set(tuple(int(c) for c in v) for v in vox))
    if not pts:
        return [], [0] * (J + 1)
    level = [((0, 0, 0), pts)]  # (corner, points inside)
    out = []
    sizes = [1]
    for d in range(J):
        half = 1 << (J - d - 1)
        nxt = []
        for corner, inside in level:
            kids = [[] for _ in range(8)]
            for p in inside:
                i = 0
                if p[0] >= corner[0] + half:
                    i |= 1
                if p[1] >= corner[1] + half:
                    i |= 2
                if p[2] >= corner[2] + half:
                    i |= 4
                kids[i].append(p)
            byte = 0
            for i in range(8):
                if kids[i]:
                    byte |= 1 << i
                    c = (corner[0] + half * (i & 1), corner[1] + half * ((i >> 1) & 1),
                         corner[2] + half * ((i >> 2) & 1))
                    nxt.append((c, kids[i]))
            out.append(byte)
        level = nxt
        sizes.append(len(level))
    return out, sizes


def octree_points_from_bytes(occ, J):
    """Inverse of octree_bytes_by_cubes: replay the level-order bytes into voxel corners."""
    level = [(0, 0, 0)]
    k = 0
    for d in range(J):
        half = 1 << (J - d - 1)
        nxt = []
        for corner in level:
            byte = occ[k]
            k += 1
            for i in range(8):
                if byte >> i & 1:
                    nxt.append((corner[0] + half * (i & 1), corner[1] + half * ((i >> 1) & 1),
                                corner[2] + half * ((i >> 2) & 1)))
        level = nxt
    return level


def morton_by_bits(x, y, z, J):
    """Morton code written as a string of bits, most significant triple first (Sec. 2.2)."""
    s = ""
    for b in range(J - 1, -1, -1):
        s += str((z >> b) & 1) + str((y >> b) & 1) + str((x >> b) & 1)
    return int(s, 2) if s else 0


# ------------------------------------------------------------------------------------------
# RAHT by top-down recursion. The binary level l merges the two halves that differ in bit
# l-1 of the Morton code (bit 0 = x at the finest level), so the recursion splits on bit
# 3J-1 first. Weights are leaf counts; the low-pass goes to the parent, the high-pass is
# stored at the first leaf of the right half; a half with no sibling passes through (Sec. 3.1,
# Eq. 1).
# ------------------------------------------------------------------------------------------
def raht_recursive(codes, vals, J):
    """codes: sorted distinct Morton codes; vals: list of float rows. Returns coefficient rows
    (list of lists) in leaf order: index 0 the DC, index i the high-pass stored at leaf i."""
    n = len(codes)
    C = len(vals[0]) if n else 0
    out = [[0.0] * C for _ in range(n)]

    def rec(lo, hi, bit):
        # leaves [lo, hi) share all bits above `bit`; returns (low-pass row, weight)
        if bit < 0:
            assert hi - lo == 1
            return list(vals[lo]), 1
        mid = lo
        while mid < hi and not (codes[mid] >> bit) & 1:
            mid += 1
        if mid == lo:
            return rec(lo, hi, bit - 1)
        if mid == hi:
            return rec(lo, hi, bit - 1)
        l0, w0 = rec(lo, mid, bit - 1)
        l1, w1 = rec(mid, hi, bit - 1)
        s = math.sqrt(w0 + w1)
        a, b = math.sqrt(w0) / s, math.sqrt(w1) / s
        out[mid] = [-b * y0 + a * y1 for y0, y1 in zip(l0, l1)]
        return [a * y0 + b * y1 for y0, y1 in zip(l0, l1)], w0 + w1

    if n:
        dc, _ = rec(0, n, 3 * J - 1)
        out[0] = dc
    return out


def raht_by_subtree_sums(codes, vals, J):
    """Closed form of the same transform: a node's low-pass is (sum of its leaves)/sqrt(w), so
    the high-pass of a merge with left sum S0 (w0 leaves) and right sum S1 (w1 leaves) is
    (w0*S1 - w1*S0) / sqrt(w0*w1*(w0+w1)), and the DC is (sum of all)/sqrt(n)."""
    n = len(codes)
    C = len(vals[0]) if n else 0
    out = [[0.0] * C for _ in range(n)]

    def rec(lo, hi, bit):
        if bit < 0 or hi - lo <= 1:
            return
        mid = lo
        while mid < hi and not (codes[mid] >> bit) & 1:
            mid += 1
        if lo < mid < hi:
            w0, w1 = mid - lo, hi - mid
            for c in range(C):
                s0 = math.fsum(vals[k][c] for k in range(lo, mid))
                s1 = math.fsum(vals[k][c] for k in range(mid, hi))
                out[mid][c] = (w0 * s1 - w1 * s0) / math.sqrt(w0 * w1 * (w0 + w1))
        rec(lo, mid, bit - 1)
        rec(mid, hi, bit - 1)

    if n:
        for c in range(C):
            out[0][c] = math.fsum(v[c] for v in vals) / math.sqrt(n)
        rec(0, n, 3 * J - 1)
    return out


# ------------------------------------------------------------------------------------------
# Exact rational voxelization and quantization.
# ------------------------------------------------------------------------------------------
def voxel_exact(p, lo, cell, J):
    """floor((p - lo)/cell) in exact rational arithmetic, clamped to [0, 2^J - 1]."""
    t = (Fraction(float(p)) - Fraction(float(lo))) / Fraction(float(cell))
    v = math.floor(t)
    return min(max(v, 0), (1 << J) - 1)


def quantize_exact(y, step, tau):
    """sgn(y) * floor(|y|/step + tau) on the exact binary values of y, step and tau."""
    fy = Fraction(float(y))
    if fy == 0:
        return 0
    t = math.floor(abs(fy) / Fraction(float(step)) + Fraction(float(tau)))
    return t if fy > 0 else -t
