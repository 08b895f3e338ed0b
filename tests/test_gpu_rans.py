"""Parity of the occupancy-byte rANS coder on the GPU with the CPU oracle: the GPU's stream
(header, table, chunk offsets, data) byte for byte equal to the oracle's, the GPU decoder
returning the input exactly (also from the oracle's stream), rejection of damaged streams, and
the codec's own occupancy bytes up to the 1M frame."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import gsc, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _oracle_stream(data, K):
    f, off, coded = orc.rans_encode(data, K)
    nc = len(off) - 1
    h = np.zeros(1, dtype=gsc.RANS_HEADER_DTYPE)
    h["magic"], h["version"], h["n"], h["K"] = gsc.RANS_MAGIC, gsc.VERSION, len(data), K
    h["nchunks"], h["total"] = nc, int(off[-1])
    return (h.tobytes() + f.astype("<u2").tobytes() + off.astype("<u4").tobytes() + coded.tobytes())


def _roundtrip(data, K):
    dev = _dev()
    print(f"case n={len(data)} K={K}", flush=True)
    td = torch.from_numpy(np.ascontiguousarray(data, dtype=np.uint8)).to(dev) if len(data) else \
        torch.empty(0, dtype=torch.uint8, device=dev)
    s = gsc.rans_encode(td, K)
    torch.cuda.synchronize()
    s.check()
    got = s.to_bytes()
    want = _oracle_stream(data, K)
    assert got == want, "stream differs from the oracle's"
    # the GPU decoder on its own stream and on the oracle's
    for blob in (s.buf, torch.from_numpy(np.frombuffer(want, dtype=np.uint8).copy()).to(dev)):
        out, info = gsc.rans_decode(blob, len(data), K, nbytes=len(want))
        torch.cuda.synchronize()
        assert int(info[0].item()) == 0
        assert np.array_equal(out[:len(data)].cpu().numpy(), np.asarray(data, dtype=np.uint8))
    return want


@pytest.mark.parametrize("n,alphabet,K", [(1, 1, 64), (5, 1, 2), (1000, 3, 64), (4097, 256, 4096),
                                          (100_003, 17, 512), (300_000, 200, 1000)])
def test_random_bytes_match_oracle(n, alphabet, K):
    rng = np.random.default_rng(n)
    p = rng.dirichlet(np.ones(alphabet))
    data = rng.choice(alphabet, size=n, p=p).astype(np.uint8)
    _roundtrip(data, K)


@pytest.mark.parametrize("shift", [1, 2, 3, 5])
def test_unaligned_bytes(shift):
    """The raw bytes may start anywhere: the encoder's input and the decoder's output taken as
    views at a byte offset into larger buffers (the stream itself stays aligned)."""
    dev = _dev()
    rng = np.random.default_rng(40 + shift)
    for n, K in ((5, 3), (1000, 7), (20_011, 333), (65_536, 4096)):
        data = rng.choice(7, size=n, p=[0.4, 0.2, 0.15, 0.1, 0.1, 0.04, 0.01]).astype(np.uint8)
        print(f"case shift={shift} n={n} K={K}", flush=True)
        big = torch.zeros(n + 16, dtype=torch.uint8, device=dev)
        big[shift:shift + n] = torch.from_numpy(data).to(dev)
        s = gsc.rans_encode(big[shift:shift + n], K)
        torch.cuda.synchronize()
        s.check()
        assert s.to_bytes() == _oracle_stream(data, K)
        out_big = torch.full((n + 16,), 0xA5, dtype=torch.uint8, device=dev)
        out, info = gsc.rans_decode(s.buf, n, K, out=out_big[shift:shift + n])
        torch.cuda.synchronize()
        assert int(info[0].item()) == 0
        ob = out_big.cpu().numpy()
        assert np.array_equal(ob[shift:shift + n], data)
        assert np.all(ob[:shift] == 0xA5) and np.all(ob[shift + n:] == 0xA5)  # nothing written outside


def test_largest_chunks_and_extreme_tables():
    """Chunks of the largest length (2^20 bytes, the coder's limit) on uniform bytes (every byte
    at frequency 16, about one output byte per input byte), and a table where one byte has
    frequency 1 (12 bits of code each time it occurs) next to one that takes the rest."""
    rng = np.random.default_rng(77)
    _roundtrip(rng.integers(0, 256, size=(1 << 20) + 3).astype(np.uint8), 1 << 20)
    data = np.zeros(200_000, dtype=np.uint8)
    data[rng.choice(data.size, size=7, replace=False)] = 255
    want = _roundtrip(data, 5000)
    f = np.frombuffer(want[32:32 + 512], dtype="<u2")
    assert f[255] == 1 and f[0] == 4095


def test_empty_input():
    _roundtrip(np.zeros(0, dtype=np.uint8), 128)


@pytest.mark.parametrize("n,J,K", [(100_000, 10, 512), (1_000_000, 12, 512), (1_000_000, 12, 4096)])
def test_occupancy_bytes_of_the_codec(n, J, K):
    """The occupancy section of the GPU codec's own stream for the benchmark frames."""
    dev = _dev()
    pos, attr = synth.make_frame(n, seed=2)
    e = gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev),
                         gsc.make_params(J, attr.shape[1], synth.quant_steps(synth.STEPS_GROUPED)))
    torch.cuda.synchronize()
    e.check()
    blob = np.frombuffer(e.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    occ = blob[int(h["occ_offset"]):int(h["occ_offset"]) + int(h["occ_bytes"])]
    want = _roundtrip(occ, K)
    assert len(want) < 0.8 * len(occ)  # the bytes shrink


def test_damaged_streams_are_rejected():
    dev = _dev()
    rng = np.random.default_rng(5)
    data = rng.integers(0, 9, size=20_000).astype(np.uint8)
    K = 1000
    good = np.frombuffer(_oracle_stream(data, K), dtype=np.uint8)
    hsz, nc = 32, -(-len(data) // K)
    d0 = hsz + 512 + 4 * (nc + 1)
    cases = []
    b = good.copy()
    b[0] ^= 1                                    # magic
    cases.append(b)
    b = good.copy()
    b[hsz] = (int(b[hsz]) + 1) % 256             # the table no longer sums to 4096
    cases.append(b)
    b = good.copy()
    b[d0 + 1] ^= 0x20                            # chunk 0's state
    cases.append(b)
    b = good.copy()
    off = b[hsz + 512:d0].view("<u4")
    off[3] += 1                                  # chunk 2 one byte longer, chunk 3 one shorter
    cases.append(b)
    for k, bad in enumerate(cases):
        out, info = gsc.rans_decode(torch.from_numpy(bad.copy()).to(dev), len(data), K)
        torch.cuda.synchronize()
        assert int(info[0].item()) == 5, f"case {k}"   # GSC_ERR_CORRUPT_STREAM
    # a size or chunk length that does not match the header
    for n_, K_ in ((len(data) - 1, K), (len(data), K + 1)):
        out, info = gsc.rans_decode(torch.from_numpy(good.copy()).to(dev), n_, K_)
        torch.cuda.synchronize()
        assert int(info[0].item()) == 5


def test_first_state_below_the_bound_is_rejected():
    """The oracle's pin of the same rule: one byte 0 under the table {0: 4096} stored as the chunk
    00 00 80 00 00 (first state 2^15) instead of the encoder's 00 80 00 00."""
    dev = _dev()
    good = np.frombuffer(_oracle_stream(np.zeros(1, dtype=np.uint8), 1), dtype=np.uint8)
    hsz = 32
    h = np.frombuffer(good[:hsz].tobytes(), dtype=gsc.RANS_HEADER_DTYPE).copy()
    assert good[hsz + 520:].tolist() == [0x00, 0x80, 0x00, 0x00]
    h["total"] = 5
    crafted = np.concatenate([np.frombuffer(h.tobytes(), dtype=np.uint8), good[hsz:hsz + 512],
                              np.array([0, 5], dtype="<u4").view(np.uint8),
                              np.array([0x00, 0x00, 0x80, 0x00, 0x00], dtype=np.uint8)])
    for blob, want in ((good, 0), (crafted, 5)):
        out, info = gsc.rans_decode(torch.from_numpy(blob.copy()).to(dev), 1, 1)
        torch.cuda.synchronize()
        assert int(info[0].item()) == want
