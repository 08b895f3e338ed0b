"""GPU-versus-oracle checks shared by the GPU parity tests (helpers only, no tests).

Bars: Morton codes, level sizes, occupancy bytes, header fields and decoded positions
bit-exact; FP32 coefficients within 1e-5 of the per-channel maximum of the FP64 ones; quantized
coefficients equal to the oracle's except at rounding ties (at most 1e-4 of them, off by one,
each within the FP32 error of a decision boundary), and equal to the decision rule applied to
the GPU's own coefficients; attributes decoded by the GPU from the oracle's stream within 1e-5
of the per-channel maximum of the oracle's FP64 decode of the same stream.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import gsc
from streamfmt import pack_stream, quantize_rule

torch = pytest.importorskip("torch")

REL_TOL = 1e-5
TIE_FRAC = 1e-4


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_encode(pos, attr, J, steps, tau=0.5, bbox=None, flags=0):
    dev = _dev()
    n, C = attr.shape
    p = gsc.make_params(J, C, steps, tau, bbox, flags=flags)
    coef = torch.full((max(n, 1), C), np.nan, dtype=torch.float32, device=dev)
    codes = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev)
    vof = torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev)
    enc = gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev), p,
                           coef_f32=coef, leaf_codes=codes, perm=perm, voxel_of=vof)
    torch.cuda.synchronize()
    enc.check()
    blob = np.frombuffer(enc.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    nv = int(h["n_vox"])
    return dict(enc=enc, h=h, nv=nv, blob=blob,
                occ=blob[1024:1024 + int(h["occ_bytes"])],
                Q=blob[int(h["coef_offset"]):int(h["total_bytes"])].view(np.int32).reshape(nv, C),
                Y=coef[:nv].cpu().numpy().astype(np.float64),
                codes=codes[:nv].cpu().numpy().view(np.uint64),
                perm=perm[:n].cpu().numpy(), voxel_of=vof[:n].cpu().numpy())


def check_encode(g, ref, J, steps, tau, n_in, flags=0):
    nv = ref["nv"]
    assert g["nv"] == nv
    assert np.array_equal(g["codes"], ref["leaf"]), "Morton codes differ"
    if "perm" in ref:  # the stable sort (Alg. 1 step 1) and the Gaussian -> voxel map
        assert np.array_equal(g["perm"].astype(np.int64), ref["perm"]), "sorted order differs"
        assert np.array_equal(g["voxel_of"].astype(np.int64), ref["voxel_of"]), "voxel map differs"
    assert int(g["h"]["flags"]) == flags
    assert list(g["h"]["level_sizes"][:J + 1]) == list(ref["level_sizes"])
    assert np.array_equal(g["occ"], ref["occ"]), "occupancy bytes differ"
    assert np.array_equal(g["h"]["bbox_min"], ref["bbox_min"]) and g["h"]["cell"] == ref["cell"]
    C = g["Q"].shape[1] if nv else int(g["h"]["C"])
    # every header byte but the coefficients equals the oracle's stream in the documented layout
    packed = pack_stream(ref, J, C, steps, tau, n_in, flags)
    co = int(g["h"]["coef_offset"])
    assert g["blob"].size == packed.size and np.array_equal(g["blob"][:co], packed[:co])
    if nv == 0:
        return
    Y64, Y32 = ref["Y"], g["Y"]
    scale = np.abs(Y64).max(axis=0)
    scale[scale == 0] = 1.0
    rel = np.abs(Y32 - Y64).max(axis=0) / scale
    assert rel.max() <= REL_TOL, f"coefficient error {rel.max():.3g} (channel {rel.argmax()})"
    # the GPU's decision on its own coefficients follows the decision rule exactly
    assert np.array_equal(g["Q"], quantize_rule(Y32, steps, tau))
    diff = g["Q"] != ref["Q"]
    assert diff.mean() <= TIE_FRAC, f"{diff.sum()} quantized coefficients differ"
    if diff.any():
        assert np.abs(g["Q"] - ref["Q"])[diff].max() == 1
        cols = np.nonzero(diff)[1]
        t = np.abs(Y64[diff]) / steps[cols].astype(np.float64) + tau
        dist = np.abs(t - np.round(t))  # distance of the FP64 decision to its boundary
        bound = np.abs(Y32 - Y64)[diff] / steps[cols] + 1e-12
        assert np.all(dist <= bound)


def check_decode(g, ref, J, steps, tau, n_in, flags=0):
    """Decodes the GPU's own stream (geometry) and the oracle's stream (geometry and
    attributes) on the GPU; compares with the oracle's decode of the oracle's stream."""
    dev = _dev()
    nv = g["nv"]
    C = int(g["h"]["C"])
    packed = pack_stream(ref, J, C, steps, tau, n_in, flags)
    decs = []
    for stream in (g["enc"].stream, torch.from_numpy(packed).to(dev)):
        d = gsc.decode_frame(stream, J, C, max(nv, 1), want_vox=True, want_codes=True)
        torch.cuda.synchronize()
        d.check()
        assert d.n_vox() == nv
        decs.append(d)
    if nv == 0:
        return
    vox, cen = orc.voxel_centres(ref["leaf"], J, ref["bbox_min"], ref["cell"])
    for d in decs:
        assert np.array_equal(d.codes[:nv].cpu().numpy().view(np.uint64), ref["leaf"])
        assert np.array_equal(d.vox[:nv].cpu().numpy().astype(np.uint32), vox)
        assert np.array_equal(d.pos[:nv].cpu().numpy(), cen.astype(np.float32)), "positions differ"
    want = orc.decode_frame(ref["occ"], ref["level_sizes"], J, ref["Q"], steps, ref["bbox_min"],
                            ref["cell"])["attr"]
    got = decs[1].attr[:nv].cpu().numpy().astype(np.float64)
    scale = np.abs(want).max(axis=0)
    scale[scale == 0] = 1.0
    rel = np.abs(got - want).max(axis=0) / scale
    assert rel.max() <= REL_TOL, f"decoded attribute error {rel.max():.3g}"


def roundtrip(pos, attr, J, steps, tau=0.5, bbox=None, flags=0, sort_order=True):
    print(f"case n={pos.shape[0]} C={attr.shape[1]} J={J} tau={tau} bbox={bbox is not None} "
          f"flags={flags}", flush=True)
    ref = orc.encode_frame(pos, attr, J, steps, tau, bbox=bbox, want_y=True)
    if sort_order:
        ref["perm"], ref["voxel_of"] = orc.sort_order(pos, J, bbox)
    g = gpu_encode(pos, attr, J, steps, tau, bbox, flags)
    check_encode(g, ref, J, steps, tau, pos.shape[0], flags)
    check_decode(g, ref, J, steps, tau, pos.shape[0], flags)
    return g, ref
