"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: Morton codes, level sizes, occupancy bytes and decoded positions bit-exact; FP32
coefficients within 1e-5 of the per-channel maximum of the FP64 ones; quantized coefficients
equal to the oracle's except at rounding ties (at most 1e-4 of them, off by one, each within the
FP32 error of a decision boundary), and exactly equal to the oracle's quantizer applied to the
GPU's own coefficients; decoded attributes within 1e-5 of the per-channel maximum of the FP64
decode of the same quantized coefficients.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import gsc, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
TIE_FRAC = 1e-4


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_encode(pos, attr, J, steps, tau=0.5, bbox=None):
    dev = _dev()
    n, C = attr.shape
    p = gsc.make_params(J, C, steps, tau, bbox)
    coef = torch.full((max(n, 1), C), np.nan, dtype=torch.float32, device=dev)
    codes = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    enc = gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev), p,
                           coef_f32=coef, leaf_codes=codes)
    torch.cuda.synchronize()
    enc.check()
    blob = np.frombuffer(enc.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    nv = int(h["n_vox"])
    return dict(enc=enc, h=h, nv=nv, blob=blob,
                occ=blob[1024:1024 + int(h["occ_bytes"])],
                Q=blob[int(h["coef_offset"]):int(h["total_bytes"])].view(np.int32).reshape(nv, C),
                Y=coef[:nv].cpu().numpy().astype(np.float64),
                codes=codes[:nv].cpu().numpy().view(np.uint64))


def check_encode(g, ref, J, steps, tau=0.5):
    nv = ref["nv"]
    assert g["nv"] == nv
    assert np.array_equal(g["codes"], ref["leaf"]), "Morton codes differ"
    assert list(g["h"]["level_sizes"][:J + 1]) == list(ref["level_sizes"])
    assert np.array_equal(g["occ"], ref["occ"]), "occupancy bytes differ"
    assert np.array_equal(g["h"]["bbox_min"], ref["bbox_min"]) and g["h"]["cell"] == ref["cell"]
    if nv == 0:
        return
    Y64, Y32 = ref["Y"], g["Y"]
    scale = np.abs(Y64).max(axis=0)
    scale[scale == 0] = 1.0
    rel = np.abs(Y32 - Y64).max(axis=0) / scale
    assert rel.max() <= REL_TOL, f"coefficient error {rel.max():.3g} (channel {rel.argmax()})"
    # the GPU's decision on its own coefficients is the oracle's quantizer, exactly
    assert np.array_equal(g["Q"], orc.quantize(Y32, steps, tau))
    diff = g["Q"] != ref["Q"]
    assert diff.mean() <= TIE_FRAC, f"{diff.sum()} quantized coefficients differ"
    if diff.any():
        assert np.abs(g["Q"] - ref["Q"])[diff].max() == 1
        cols = np.nonzero(diff)[1]
        t = np.abs(Y64[diff]) / steps[cols].astype(np.float64) + tau
        dist = np.abs(t - np.round(t))  # distance of the FP64 decision to its boundary
        bound = np.abs(Y32 - Y64)[diff] / steps[cols] + 1e-12
        assert np.all(dist <= bound)


def check_decode(g, ref, J, steps):
    dev = _dev()
    nv, C = g["nv"], g["Q"].shape[1] if g["nv"] else 0
    dec = gsc.decode_frame(g["enc"].stream, J, g["enc"].C, max(nv, 1), want_vox=True,
                           want_codes=True)
    torch.cuda.synchronize()
    dec.check()
    assert dec.n_vox() == nv
    if nv == 0:
        return
    assert np.array_equal(dec.codes[:nv].cpu().numpy().view(np.uint64), ref["leaf"])
    vox, cen = orc.voxel_centres(ref["leaf"], J, ref["bbox_min"], ref["cell"])
    assert np.array_equal(dec.vox[:nv].cpu().numpy().astype(np.uint32), vox)
    assert np.array_equal(dec.pos[:nv].cpu().numpy(), cen.astype(np.float32)), "positions differ"
    want = orc.decode_frame(ref["occ"], ref["level_sizes"], J, g["Q"], steps, ref["bbox_min"],
                            ref["cell"])["attr"]
    got = dec.attr[:nv].cpu().numpy().astype(np.float64)
    scale = np.abs(want).max(axis=0)
    scale[scale == 0] = 1.0
    rel = np.abs(got - want).max(axis=0) / scale
    assert rel.max() <= REL_TOL, f"decoded attribute error {rel.max():.3g}"


def roundtrip(pos, attr, J, steps, tau=0.5, bbox=None):
    print(f"case n={pos.shape[0]} C={attr.shape[1]} J={J} tau={tau} bbox={bbox is not None}",
          flush=True)
    ref = orc.encode_frame(pos, attr, J, steps, tau, bbox=bbox, want_y=True)
    g = gpu_encode(pos, attr, J, steps, tau, bbox)
    check_encode(g, ref, J, steps, tau)
    check_decode(g, ref, J, steps)
    return g, ref


GROUPED = synth.quant_steps(synth.STEPS_GROUPED)
UNIFORM = synth.quant_steps(synth.STEPS_UNIFORM_64)


@pytest.mark.parametrize("n,J,seed", [
    (100_000, 10, 1),      # the 100K-Gaussian depth-10 workload
    (20_000, 8, 2),
    (5_000, 12, 3),
    (700, 21, 4),          # deepest octree: 63-bit codes, level 63
    (4097, 9, 5),          # one past a sort tile
    (2049, 7, 6),          # one past an occupancy tile
    (513, 11, 7),          # one past a transform tile
    (1, 5, 8),
    (2, 1, 9),
])
def test_frame_roundtrip(n, J, seed):
    pos, attr = synth.make_frame(n, seed=seed)
    roundtrip(pos, attr, J, UNIFORM if J == 10 else GROUPED)


@pytest.mark.parametrize("C", [1, 3, 5, 64])
def test_channel_counts(C):
    pos, _ = synth.make_frame(3000, seed=10 + C)
    rng = np.random.default_rng(C)
    attr = rng.normal(0, 1, size=(3000, C)).astype(np.float32)
    roundtrip(pos, attr, 8, np.full(C, 1 / 32, np.float32))


def test_duplicates_merge():
    pos, attr = synth.make_duplicates_frame(30_000, seed=11, grid=16)
    roundtrip(pos, attr, 6, GROUPED)   # 4096 sites: ~7 Gaussians per voxel
    roundtrip(pos, attr, 3, GROUPED)   # 512 voxels hold everything


def test_degenerate_frames():
    C = 56
    rng = np.random.default_rng(12)
    attr = synth.sample_attributes(rng, 100)
    roundtrip(np.full((100, 3), 0.25, np.float32), attr, 9, GROUPED)   # zero extent
    roundtrip(np.zeros((0, 3), np.float32), np.zeros((0, C), np.float32), 9, GROUPED)
    pos, attr = synth.make_frame(5000, seed=13)
    roundtrip(pos * 2 - 0.5, attr, 9, GROUPED, bbox=(np.zeros(3), 1 / 512))  # clamped points


def test_quantizer_variants():
    pos, attr = synth.make_frame(20_000, seed=14)
    odd = np.linspace(0.011, 0.3, 56).astype(np.float32)   # steps that are not powers of two
    roundtrip(pos, attr, 9, odd, tau=0.5)
    roundtrip(pos, attr, 9, GROUPED, tau=0.25)
    roundtrip(pos, attr, 9, GROUPED, tau=0.0)


@pytest.mark.slow
def test_frame_1M_depth12_full():
    pos, attr = synth.make_frame(1_000_000, seed=2)
    roundtrip(pos, attr, 12, GROUPED)


def test_corrupt_streams_are_rejected():
    dev = _dev()
    pos, attr = synth.make_frame(3000, seed=15)
    g = gpu_encode(pos, attr, 7, GROUPED)
    nv = g["nv"]

    def dec(blob, J=7):
        t = torch.from_numpy(blob.copy()).to(dev)
        d = gsc.decode_frame(t, J, 56, nv)
        torch.cuda.synchronize()
        return int(d.info[0].item())

    assert dec(g["blob"]) == 0
    bad = g["blob"].copy()
    bad[1024 + 5] = 0                       # a node without children
    assert dec(bad) == 5
    bad = g["blob"].copy()
    bad[1024 + 1] = 0xFF if bad[1024 + 1] != 0xFF else 0x01   # child count changes
    assert dec(bad) == 5
    bad = g["blob"].copy()
    bad[:4] = 0                             # magic
    assert dec(bad) == 5
    assert dec(g["blob"], J=8) == 5         # depth mismatch
    assert dec(g["blob"][:2000]) == 5       # truncated


def test_transform_entry_points():
    dev = _dev()
    rng = np.random.default_rng(16)
    for n, J in [(3000, 7), (50_000, 12)]:
        pos, _ = synth.make_frame(n, seed=17)
        vox, _, _ = orc.voxelize(pos, J)
        codes = np.unique(orc.morton_encode_array(vox, J))
        A = rng.normal(-1, 2, size=(codes.size, 6))
        Y = orc.raht_forward(codes, J, A)
        tc = torch.from_numpy(codes.view(np.int64)).to(dev)
        out, info = gsc.raht_forward(tc, torch.from_numpy(A.astype(np.float32)).to(dev), J)
        back, info2 = gsc.raht_adjoint(tc, out, J)
        torch.cuda.synchronize()
        assert int(info[0]) == 0 and int(info2[0]) == 0
        scale = np.abs(Y).max(axis=0)
        assert (np.abs(out.cpu().numpy() - Y).max(axis=0) / scale).max() <= REL_TOL
        assert np.abs(back.cpu().numpy() - A).max() <= 1e-5 * np.abs(A).max()


def test_batch_equals_per_frame():
    dev = _dev()
    frames = [synth.make_frame(n, seed=20 + i) for i, n in enumerate([3000, 17_000, 1, 0, 9000])]
    p = gsc.make_params(9, 56, GROUPED)
    tens = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in frames]
    outs = gsc.encode_batch(tens, p)
    torch.cuda.synchronize()
    singles = []
    for a, b in tens:
        e = gsc.encode_frame(a, b, p)
        torch.cuda.synchronize()
        singles.append(e)
    for e, s in zip(outs, singles):
        e.check()
        assert e.to_bytes() == s.to_bytes()
    decs = gsc.decode_batch(outs, [max(f[0].shape[0], 1) for f in frames])
    torch.cuda.synchronize()
    for d, e in zip(decs, outs):
        d.check()
        nv = e.n_vox()
        ref = gsc.decode_frame(e.stream, 9, 56, max(nv, 1))
        torch.cuda.synchronize()
        assert torch.equal(d.attr[:nv], ref.attr[:nv]) and torch.equal(d.pos[:nv], ref.pos[:nv])


def test_deterministic_bytes():
    dev = _dev()
    pos, attr = synth.make_frame(200_000, seed=30)
    p = gsc.make_params(12, 56, GROUPED)
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    a = gsc.encode_frame(tp, ta, p)
    b = gsc.encode_frame(tp, ta, p)
    torch.cuda.synchronize()
    assert a.to_bytes() == b.to_bytes()
