"""Batched coding of a dynamic sequence on the GPU: one launch per stage for the whole batch,
the same launches captured into a HIP graph and replayed, and the sort-tiling autotuner.

A batch must produce, frame by frame, the bytes of the per-frame encoder (whose parity with
the oracle the per-frame tests establish) and the per-frame decoder's output; frames of the
sequence are also checked against the oracle directly. Every sort tiling must give the same
stream. Graph replays are checked against the eager result after each replay, with eager work
and synchronizations in between.
"""
import numpy as np
import pytest

from paper_2606_05650_amd import gsc, synth
from gpucheck import _dev, roundtrip

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GROUPED = synth.quant_steps(synth.STEPS_GROUPED)
J = 12
BBOX = (np.zeros(3), 1.0 / (1 << J))   # one fixed grid for the whole sequence: [0,1]^3


def _params():
    return gsc.make_params(J, 56, GROUPED, bbox=BBOX)


def _to_dev(frames):
    dev = _dev()
    return [(torch.from_numpy(p).to(dev), torch.from_numpy(a).to(dev)) for p, a in frames]


def _check_batch(tens, params):
    outs = gsc.encode_batch(tens, params)
    torch.cuda.synchronize()
    for (tp, ta), e in zip(tens, outs):
        e.check()
        s = gsc.encode_frame(tp, ta, params)
        torch.cuda.synchronize()
        assert e.to_bytes() == s.to_bytes()
    caps = [max(int(t[0].shape[0]), 1) for t in tens]
    decs = gsc.decode_batch(outs, caps)
    torch.cuda.synchronize()
    for d, e in zip(decs, outs):
        d.check()
        nv = e.n_vox()
        ref = gsc.decode_frame(e.stream, J, 56, max(nv, 1))
        torch.cuda.synchronize()
        assert torch.equal(d.attr[:nv], ref.attr[:nv]) and torch.equal(d.pos[:nv], ref.pos[:nv])
    return outs


def test_small_sequence_batch():
    frames = list(synth.make_sequence(6, 2_000, 40_000, seed=5))
    for i in (0, 3):
        roundtrip(*frames[i], J, GROUPED, bbox=BBOX)
    _check_batch(_to_dev(frames), _params())


@pytest.mark.slow
def test_sequence_30_frames():
    """The 30-frame sequence (counts U[200K, 1.5M]) as one batch."""
    frames = list(synth.make_sequence())
    print("sequence", [f[0].shape[0] for f in frames], flush=True)
    sizes = [f[0].shape[0] for f in frames]
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        roundtrip(*frames[i], J, GROUPED, bbox=BBOX)
    tens = _to_dev(frames)
    del frames
    _check_batch(tens, _params())


def test_graph_capture_replays():
    dev = _dev()
    frames = list(synth.make_sequence(6, 2_000, 40_000, seed=6))
    tens = _to_dev(frames)
    p = _params()
    caps = [int(t[0].shape[0]) for t in tens]
    wse = [gsc.Workspace(n, J, 56, dev) for n in caps]
    wsd = [gsc.Workspace(n, J, 56, dev) for n in caps]
    eager = gsc.encode_batch(tens, p, workspaces=wse)
    edec = gsc.decode_batch(eager, caps, workspaces=wsd)
    torch.cuda.synchronize()
    want = [e.to_bytes() for e in eager]
    want_attr = [d.attr.clone() for d in edec]
    # warm up on a side stream, then capture encode + decode of the whole batch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gsc.encode_batch(tens, p, workspaces=wse)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = gsc.encode_batch(tens, p, workspaces=wse)
        decs = gsc.decode_batch(outs, caps, workspaces=wsd)
    other = synth.make_frame(10_000, seed=7)
    to, ao = torch.from_numpy(other[0]).to(dev), torch.from_numpy(other[1]).to(dev)
    for rep in range(3):
        for o in outs:
            o.stream.fill_(0xAB)
        g.replay()
        torch.cuda.synchronize()
        for o, w, d, wa in zip(outs, want, decs, want_attr):
            o.check()
            assert o.to_bytes() == w, f"replay {rep}: stream differs"
            d.check()
            nv = o.n_vox()
            assert torch.equal(d.attr[:nv], wa[:nv]), f"replay {rep}: decoded attributes differ"
        # eager work of the program between replays
        gsc.encode_frame(to, ao, p).check()
        torch.cuda.synchronize()


def test_every_sort_tiling_gives_the_same_stream():
    dev = _dev()
    pos, attr = synth.make_frame(300_000, seed=8)
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    p = _params()
    try:
        blobs = []
        for v in range(gsc.SORT_VARIANTS):
            gsc.tune_set(J, 300_000, v)
            assert gsc.tune_get(J, 300_000) == v
            e = gsc.encode_frame(tp, ta, p)
            torch.cuda.synchronize()
            e.check()
            blobs.append(e.to_bytes())
        assert all(b == blobs[0] for b in blobs)
    finally:
        gsc.tune_set(J, 300_000, -1)
    # one tiling checked against the oracle on a smaller frame of another size class
    try:
        gsc.tune_set(J, 20_000, 1)
        roundtrip(*synth.make_frame(20_000, seed=9), J, GROUPED, bbox=BBOX)
    finally:
        gsc.tune_set(J, 20_000, -1)


def test_autotune_picks_a_variant():
    frames = list(synth.make_sequence(4, 50_000, 120_000, seed=10))
    tens = _to_dev(frames)
    p = _params()
    nmax = max(f[0].shape[0] for f in frames)
    try:
        v, times, outs = gsc.autotune(tens, p, reps=2)
        assert 0 <= v < gsc.SORT_VARIANTS and all(t > 0 for t in times)
        d = gsc.sort_default_variant(nmax)  # kept unless the fastest beats it by the margin
        if min(times) < (1 - gsc.SORT_TUNE_MARGIN) * times[d]:
            assert times[v] == min(times)
        else:
            assert v == d
        assert gsc.tune_get(J, nmax) == v
        torch.cuda.synchronize()
        ref = gsc.encode_batch(tens, p)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert a.check().to_bytes() == b.check().to_bytes()
    finally:
        gsc.tune_set(J, nmax, -1)
