"""Pins of the CPU oracle of the block entropy coder (Sec. 3.4: run-length / adaptive
Golomb-Rice coding of independent blocks of quantized coefficients of one channel). The paper
names the method and gives no parameters; readings G1-G5 (oracle/rlgr_oracle.c) fix them. The
pins: hand-worked bit strings of short blocks (tests/golden/rlgr_examples.txt), the closed-form
length of an all-zero block (the run-parameter adaptation), block independence and the block
layout, lossless round trips, and rejection of truncated or inconsistent blocks."""
import os

import numpy as np
import pytest

from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rlgr_examples.txt")


def _examples():
    out = []
    for line in open(GOLDEN):
        if line.startswith("block"):
            vals, words = line[len("block"):].split(":")
            out.append((np.array([int(v) for v in vals.split()], dtype=np.int64),
                        [int(w, 16) for w in words.split()]))
    return out


@pytest.mark.parametrize("vals,words", _examples())
def test_hand_worked_codes(vals, words):
    x = vals.astype(np.int32).reshape(-1, 1)
    off, w = orc.rlgr_encode(x, x.shape[0])
    assert list(off) == [0, len(words)]
    assert [int(v) for v in w] == words
    assert np.array_equal(orc.rlgr_decode(off, w, x.shape[0], 1, x.shape[0]), x)


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_all_zero_block_length(m):
    # In run mode each 0 bit stands for 2^k zeros and raises kp by 4, so k = kp >> 3 takes every
    # value twice: 2m zero bits consume 2 (2 + 4 + ... + 2^m) = 2 (2^(m+1) - 2) zeros and leave
    # k = m + 1, so such a block is 2m bits, then the 1 bit and a count of 0 in m + 1 bits.
    L = 2 * (2 ** (m + 1) - 2)
    off, w = orc.rlgr_encode(np.zeros((L, 1), dtype=np.int32), L)
    bits = 2 * m + 1 + (m + 1)
    assert int(off[-1]) == (bits + 31) // 32
    first = int(w[0]) >> (32 - min(bits, 32))
    # the 2m zero bits, then the terminating 1, then zeros
    assert first == 1 << (min(bits, 32) - 2 * m - 1)


def test_blocks_are_independent_and_laid_out_by_channel():
    # G1: block j * C + c holds rows j*B .. j*B + B - 1 of channel c, coded from a fresh state
    rng = np.random.default_rng(3)
    nv, C, B = 1000, 5, 128
    Q = rng.integers(-6, 7, size=(nv, C)).astype(np.int32)
    Q[rng.random(Q.shape) < 0.5] = 0
    off, w = orc.rlgr_encode(Q, B)
    nb = (nv + B - 1) // B
    assert len(off) == nb * C + 1
    for j in range(nb):
        for c in range(C):
            col = np.ascontiguousarray(Q[j * B:(j + 1) * B, c]).reshape(-1, 1)
            o1, w1 = orc.rlgr_encode(col, B)
            b = j * C + c
            assert np.array_equal(w[off[b]:off[b + 1]], w1)


@pytest.mark.parametrize("B", [1, 3, 64, 512, 4096])
def test_lossless_round_trip(B):
    rng = np.random.default_rng(B)
    nv, C = 3001, 7
    Q = np.round(rng.laplace(0, 3, size=(nv, C))).astype(np.int32)
    Q[rng.random(Q.shape) < 0.3] = 0
    Q[:40, 2] = 0                                    # a long run
    Q[0, 0], Q[1, 0], Q[2, 1] = -2 ** 31, 2 ** 31 - 1, 123456789
    Q[5, :] = rng.integers(-2 ** 20, 2 ** 20, size=C)
    off, w = orc.rlgr_encode(Q, B)
    assert np.array_equal(orc.rlgr_decode(off, w, nv, C, B), Q)


def test_empty_and_single():
    off, w = orc.rlgr_encode(np.zeros((0, 4), dtype=np.int32), 16)
    assert list(off) == [0] and w.size == 0
    x = np.array([[7]], dtype=np.int32)
    off, w = orc.rlgr_encode(x, 512)
    assert np.array_equal(orc.rlgr_decode(off, w, 1, 1, 512), x)


def test_truncated_or_inconsistent_blocks_are_rejected():
    rng = np.random.default_rng(9)
    Q = rng.integers(-50, 50, size=(300, 2)).astype(np.int32)
    off, w = orc.rlgr_encode(Q, 100)
    short = off.copy()
    short[1:] = np.maximum(short[1:], 0)
    short[1] = short[0]  # block 0 given no words
    with pytest.raises(ValueError):
        orc.rlgr_decode(short, w, 300, 2, 100)
    x = Q[:100, :1].copy()
    o1, w1 = orc.rlgr_encode(x, 100)
    with pytest.raises(ValueError):  # the code ends before 120 values
        orc.rlgr_decode(o1, w1, 120, 1, 120)
    with pytest.raises(ValueError):  # 60 values leave whole words of the code unread
        orc.rlgr_decode(o1, w1, 60, 1, 60)
