"""Pins of the CPU oracle of the occupancy-byte rANS coder (an own coder standing in for the
closed ANS library the paper uses for the geometry): hand-worked codes, the table rule, the
closed-form bound of a chunk's length by its information content, chunk independence, the
round trip (also on the oracle's own occupancy bytes) and rejection of damaged chunks."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rans_examples.txt")


def _golden():
    for line in open(GOLDEN):
        if line.startswith("chunk"):
            data, table, code = line[len("chunk"):].split(":", 1)[0], None, None
            parts = line[len("chunk"):].split(" : ")
            data = bytes(int(v) for v in parts[0].split())
            table = dict((int(a), int(b)) for a, b in (t.split(":") for t in parts[1].split()))
            code = bytes(int(v, 16) for v in parts[2].split())
            yield data, table, code


def test_hand_worked_codes():
    cases = list(_golden())
    assert len(cases) == 2
    for data, table, code in cases:
        f, off, out = orc.rans_encode(data, 16)
        assert {s: int(f[s]) for s in np.nonzero(f)[0]} == table
        assert out.tobytes() == code and list(off) == [0, len(code)]
        assert orc.rans_decode(f, off, out, len(data), 16).tobytes() == data


def test_table_rule():
    rng = np.random.default_rng(0)
    for n, alphabet in ((1, 1), (10, 3), (5000, 256), (100_000, 17)):
        d = rng.integers(0, alphabet, size=n).astype(np.uint8)
        d[0] = 255  # a rare byte
        f = orc.rans_table(d)
        c = np.bincount(d, minlength=256)
        P = int((c > 0).sum())
        assert int(f.sum()) == 4096
        assert np.all((f > 0) == (c > 0))
        want = np.where(c > 0, 1 + (c * (4096 - P)) // n, 0)
        most = int(np.argmax(c))  # the first of the most frequent
        want[most] += 4096 - int(want.sum())
        assert np.array_equal(f, want)


def _bits(f, d):
    return sum(math.log2(4096 / int(f[s])) for s in d)


def test_length_bound_by_information_content():
    """bits = 8 (renormalisation bytes) + 32 and the final state lies in [2^23, 2^31), so
    I + 24 - 0.0007 n < bits <= I + 32 with I = sum log2(M / f_s) over the chunk (the floor of
    each state update loses at most 2^-11 / ln 2 bits)."""
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(1, 3000))
        p = rng.dirichlet(np.ones(256) * rng.uniform(0.05, 2.0))
        d = rng.choice(256, size=n, p=p).astype(np.uint8)
        K = int(rng.integers(1, 4097))
        f, off, out = orc.rans_encode(d, K)
        for c in range(len(off) - 1):
            ch = d[c * K:(c + 1) * K]
            I = _bits(f, ch)
            b = 8 * int(off[c + 1] - off[c])
            assert I + 24 - 0.0007 * len(ch) < b <= I + 32 + 1e-9, (trial, c, b, I)
        assert np.array_equal(orc.rans_decode(f, off, out, n, K), d)


def test_chunks_are_independent():
    rng = np.random.default_rng(2)
    d = rng.integers(0, 40, size=10_000).astype(np.uint8)
    f, off, out = orc.rans_encode(d, 1024)
    e = d.copy()
    e[5000] = (e[5000] + 1) % 40  # chunk 4 only, same table
    g, off2, out2 = orc.rans_encode(e, 1024, freq=f)
    for c in range(len(off) - 1):
        a = out[off[c]:off[c + 1]].tobytes()
        b = out2[off2[c]:off2[c + 1]].tobytes()
        assert (a == b) == (c != 4)


def test_round_trip_on_occupancy_bytes():
    pos, _ = synth.make_frame(50_000, seed=3)
    ref = orc.encode_frame(pos, np.zeros((len(pos), 1), np.float32), 10, np.ones(1), 0.5)
    occ = ref["occ"]
    for K in (256, 1024, 4096, len(occ) + 5):
        f, off, out = orc.rans_encode(occ, K)
        assert np.array_equal(orc.rans_decode(f, off, out, len(occ), K), occ)
    # the occupancy bytes are far from uniform: the coder must shrink them
    assert len(out) < 0.8 * len(occ)


def test_empty_and_damaged():
    f, off, out = orc.rans_encode(b"", 64)
    assert len(out) == 0 and list(off) == [0] and int(f.sum()) == 0
    assert orc.rans_decode(f, off, out, 0, 64).size == 0
    rng = np.random.default_rng(4)
    d = rng.integers(0, 8, size=3000).astype(np.uint8)
    f, off, out = orc.rans_encode(d, 512)
    with pytest.raises(ValueError):      # a chunk one byte short
        bad = off.copy()
        bad[1:] -= 1
        orc.rans_decode(f, bad, np.delete(out, off[1] - 1), len(d), 512)
    flipped = out.copy()
    flipped[0] ^= 0x40                   # the first chunk's state
    with pytest.raises(ValueError):
        orc.rans_decode(f, off, flipped, len(d), 512)


def test_first_state_below_the_renormalisation_bound_is_rejected():
    """One byte 0 under the table {0: 4096}: the encoder writes the chunk 00 80 00 00 (its final
    state 2^23). The chunk 00 00 80 00 00 starts in the state 2^15 and would still end in 2^23
    with every byte read (the decoded state stays 2^15, one byte 00 brings it to 2^23); a decoder
    must reject it, since an encoder's first stored state is never below 2^23."""
    f, off, out = orc.rans_encode(b"\x00", 1)
    assert int(f[0]) == 4096 and out.tobytes() == bytes([0x00, 0x80, 0x00, 0x00])
    assert orc.rans_decode(f, off, out, 1, 1).tobytes() == b"\x00"
    crafted = np.array([0x00, 0x00, 0x80, 0x00, 0x00], dtype=np.uint8)
    with pytest.raises(ValueError):
        orc.rans_decode(f, np.array([0, 5], dtype=np.int64), crafted, 1, 1)
