"""The C ABI library loads and exports every symbol include/gsc.h declares; host-side argument
checks and size queries behave as documented. No call here reaches the GPU: every checked call
returns before enqueueing work."""
import ctypes

import numpy as np
import pytest

from paper_2606_05650_amd import gsc


def test_library_exports_every_declared_symbol():
    L = gsc.lib()
    names = gsc.declared_symbols()
    assert {"gsc_encode_frame", "gsc_decode_frame", "gsc_encode_batch", "gsc_workspace_size",
            "gsc_stream_capacity", "gsc_status_string", "gsc_decode_batch", "gsc_raht_forward",
            "gsc_raht_adjoint", "gsc_ste_forward", "gsc_ste_backward",
            "gsc_profile_events", "gsc_encode_frame_noalloc", "gsc_rlgr_encode", "gsc_rlgr_decode",
            "gsc_rlgr_capacity", "gsc_rlgr_workspace_size", "gsc_color_workspace_size",
            "gsc_color_forward", "gsc_color_inverse", "gsc_rans_capacity",
            "gsc_rans_workspace_size", "gsc_rans_encode", "gsc_rans_decode"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    assert gsc.status_string(0) == "ok"
    assert gsc.status_string(5) == "corrupt stream"
    assert gsc.status_string(99) == "unknown status"


def test_size_queries():
    # the stream holds a 1 KiB header, at most min(8^d, n) bytes per level d < J, padding to
    # 256 bytes, and n * C int32 coefficients
    n, J, C = 1000, 5, 56
    occ = sum(min(8 ** d, n) for d in range(J))
    want = ((1024 + occ + 255) // 256) * 256 + n * C * 4
    assert gsc.stream_capacity(n, J, C) == want
    assert gsc.stream_capacity(0, J, C) == 1024
    ws = [gsc.workspace_size(k, 12, 56) for k in (0, 1, 1000, 10 ** 6)]
    assert ws == sorted(ws) and ws[0] > 0
    with pytest.raises(gsc.GscError) as e:
        gsc.workspace_size(10, 22, 56)
    assert e.value.code == 2
    with pytest.raises(gsc.GscError):
        gsc.workspace_size(10, 12, 65)
    with pytest.raises(gsc.GscError):
        gsc.workspace_size(-1, 12, 56)


def _encode_rc(n=10, J=5, C=4, steps=0.1, tau=0.5, ws_bytes=None, cap=None, null_ws=False,
               params=True, **kw):
    L = gsc.lib()
    p = gsc.make_params(J, C, steps, tau, **kw) if params else None
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    ws_need = gsc.workspace_size(max(n, 0), min(J, 21), min(C, 64)) if 1 <= J <= 21 and 1 <= C <= 64 else 0
    return L.gsc_encode_frame(fake, fake, n, ctypes.byref(p) if p else None, fake,
                              cap if cap is not None else 1 << 40, None if null_ws else fake,
                              ws_bytes if ws_bytes is not None else ws_need, fake, None, None,
                              None, None, None)


def test_encode_argument_checks():
    assert _encode_rc(J=0) == 2
    assert _encode_rc(J=22) == 2
    assert _encode_rc(steps=0.0) == 1
    assert _encode_rc(steps=np.inf) == 1
    assert _encode_rc(tau=1.0) == 1
    assert _encode_rc(tau=-0.1) == 1
    assert _encode_rc(n=-1) == 1
    assert _encode_rc(null_ws=True) == 1
    assert _encode_rc(params=False) == 1
    assert _encode_rc(ws_bytes=100) == 3
    assert _encode_rc(cap=100) == 4
    assert _encode_rc(bbox=((0, 0, 0), 0.0)) == 1
    assert _encode_rc(flags=0x2) == 1            # an unknown flag


def test_noalloc_encode_limits():
    # the static-scratch encode rejects, before anything is enqueued, a frame whose workspace
    # exceeds GSC_STATIC_SCRATCH_BYTES, and checks its other arguments like gsc_encode_frame
    L = gsc.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    J, C = 12, 56
    lo, hi = 1, 2_000_000
    while lo < hi:  # the largest frame that fits
        m = (lo + hi + 1) // 2
        lo, hi = (m, hi) if gsc.workspace_size(m, J, C) <= gsc.STATIC_SCRATCH_BYTES else (lo, m - 1)
    assert 400_000 < lo < 600_000
    p = gsc.make_params(J, C, 0.1)
    args = lambda n, pp=p: (fake, fake, n, ctypes.byref(pp), fake, 1 << 40, fake, None, None,
                            None, None, None)
    assert L.gsc_encode_frame_noalloc(*args(lo + 1)) == 8
    assert gsc.status_string(8) == "frame too large for the static scratch"
    assert L.gsc_encode_frame_noalloc(*args(-1)) == 1
    bad = gsc.make_params(J, C, 0.0)
    assert L.gsc_encode_frame_noalloc(*args(10, bad)) == 1
    assert L.gsc_encode_frame_noalloc(fake, fake, 10, None, fake, 1 << 40, fake, None, None,
                                      None, None, None) == 1


def test_decode_and_transform_argument_checks():
    L = gsc.lib()
    fake = ctypes.c_void_p(0x1000)
    ws = gsc.workspace_size(100, 8, 3)
    assert L.gsc_decode_frame(fake, 4096, 0, 3, 100, fake, None, fake, None, fake, ws, fake, None) == 2
    assert L.gsc_decode_frame(fake, 4096, 8, 3, 100, None, None, fake, None, fake, ws, fake, None) == 1
    assert L.gsc_decode_frame(fake, 4096, 8, 3, 100, fake, None, fake, None, fake, 10, fake, None) == 3
    assert L.gsc_raht_forward(fake, 100, 8, 3, fake, fake, fake, ws, fake, None) == 1  # aliasing
    assert L.gsc_raht_adjoint(fake, 100, 8, 70, fake, ctypes.c_void_p(0x2000), fake, ws, fake,
                              None) == 2
    descs = (gsc.FrameDescC * 1)()
    assert L.gsc_encode_batch(descs, 0, None, None) == 1
    assert L.gsc_encode_batch(descs, 65, None, None) == 1


def test_straight_through_argument_checks():
    L = gsc.lib()
    a, b, c = (ctypes.c_void_p(x) for x in (0x1000, 0x2000, 0x3000))
    J, C, n = 8, 4, 100
    p = gsc.make_params(J, C, 0.1)
    ws = gsc.workspace_size(n, J, C)
    cap = gsc.stream_capacity(n, J, C)

    def fwd(yhat=b, ahat=c, ws_bytes=ws, attr=a, params=p):
        return L.gsc_ste_forward(a, attr, n, ctypes.byref(params), a, cap, a, ws_bytes, a, yhat,
                                 ahat, None, None, None)
    assert fwd(yhat=None) == 1
    assert fwd(ahat=b) == 1            # yhat and ahat alias
    assert fwd(attr=b) == 1            # input aliases yhat
    assert fwd(ws_bytes=10) == 3
    assert fwd(params=gsc.make_params(J, C, 0.0)) == 1
    assert L.gsc_ste_backward(n, J, C, a, b, a, c, ws, c, None) == 1   # output aliases input
    assert L.gsc_ste_backward(n, J, C, None, b, c, a, ws, a, None) == 1
    assert L.gsc_ste_backward(n, 0, C, a, b, c, a, ws, a, None) == 2
    assert L.gsc_ste_backward(n, J, C, a, b, c, a, 10, a, None) == 3


def test_header_layout_matches_c_struct():
    # offsets of gsc_header fields as laid out by a C compiler (natural alignment)
    d = gsc.HEADER_DTYPE
    assert d.fields["level_sizes"][1] == 24
    assert d.fields["error"][1] == 112
    assert d.fields["bbox_min"][1] == 120
    assert d.fields["quant_step"][1] == 152
    assert d.fields["occ_offset"][1] == 416
    assert d.itemsize == 456 <= gsc.HEADER_BYTES
    assert d.fields["flags"][1] == 116
    assert ctypes.sizeof(gsc.Params) == 312
    assert gsc.Params.flags.offset == 304


def test_batch_buffer_overlap_is_rejected():
    # a batch launch must never see two frames' buffers overlap (e.g. a workspace released
    # early and handed to another frame's output by the allocator)
    gsc.assert_disjoint([(0x1000, 0x100), (0x1100, 0x10), (0x2000, 0x1000)])
    with pytest.raises(ValueError):
        gsc.assert_disjoint([(0x1000, 0x200), (0x1100, 0x10)])


# ------------------------------------------------------------------ overlapping buffers
# Fake device addresses, far apart unless a case places two of them on purpose: every call
# below is rejected by the host-side range check before anything is enqueued.
_B = 1 << 36


def _addr(k, off=0):
    return ctypes.c_void_p(_B * (k + 1) + off)


def _encode_frame_rc(n=1000, J=8, C=4, **over):
    L = gsc.lib()
    p = gsc.make_params(J, C, 0.1)
    ws = gsc.workspace_size(n, J, C)
    cap = gsc.stream_capacity(n, J, C)
    a = dict(pos=_addr(0), attr=_addr(1), stream=_addr(2), ws=_addr(3), info=_addr(4),
             coef=None, codes=None, perm=None, vof=None)
    a.update(over)
    return L.gsc_encode_frame(a["pos"], a["attr"], n, ctypes.byref(p), a["stream"], cap, a["ws"],
                              ws, a["info"], a["coef"], a["codes"], a["perm"], a["vof"], None)


def test_encode_rejects_overlapping_buffers():
    n, C = 1000, 4
    ws = gsc.workspace_size(n, 8, C)
    # the workspace's last byte is the stream's first
    assert _encode_frame_rc(stream=_addr(3, ws - 1)) == 1
    # the info words inside the stream
    assert _encode_frame_rc(info=_addr(2, 4096)) == 1
    # an optional output over the attribute input
    assert _encode_frame_rc(coef=_addr(1, 64)) == 1
    assert _encode_frame_rc(perm=_addr(5), vof=_addr(5, 4 * n - 4)) == 1
    assert _encode_frame_rc(codes=_addr(0, 12 * n - 8)) == 1      # leaf codes over positions


def test_decode_and_transform_reject_overlapping_buffers():
    L = gsc.lib()
    n, J, C = 1000, 8, 4
    ws = gsc.workspace_size(n, J, C)
    # decoded attributes over the stream being decoded
    assert L.gsc_decode_frame(_addr(0), 8192, J, C, n, _addr(1), None, _addr(0, 1024), None,
                              _addr(3), ws, _addr(4), None) == 1
    # voxel coordinates over the positions
    assert L.gsc_decode_frame(_addr(0), 8192, J, C, n, _addr(1), _addr(1, 12 * n - 4), _addr(2),
                              None, _addr(3), ws, _addr(4), None) == 1
    # transform output over the workspace
    assert L.gsc_raht_forward(_addr(0), n, J, C, _addr(1), _addr(3, 16), _addr(3), ws, _addr(4),
                              None) == 1
    # transform output over the codes
    assert L.gsc_raht_adjoint(_addr(0), n, J, C, _addr(1), _addr(0, 8 * n - 8), _addr(3), ws,
                              _addr(4), None) == 1


def test_batch_rejects_buffers_shared_between_frames():
    L = gsc.lib()
    J, C, n = 8, 4, 500
    p = gsc.make_params(J, C, 0.1)
    ws = gsc.workspace_size(n, J, C)
    cap = gsc.stream_capacity(n, J, C)
    descs = (gsc.FrameDescC * 2)()
    for f in range(2):
        d = descs[f]
        d.d_pos, d.d_attr, d.n = _addr(10 * f).value, _addr(10 * f + 1).value, n
        d.d_stream, d.stream_cap = _addr(10 * f + 2).value, cap
        d.d_ws, d.ws_bytes, d.d_info = _addr(10 * f + 3).value, ws, _addr(10 * f + 4).value
    descs[1].d_ws = descs[0].d_ws           # two frames on one workspace
    assert L.gsc_encode_batch(descs, 2, ctypes.byref(p), None) == 1
    descs[1].d_ws = _addr(13).value
    descs[1].d_info = descs[0].d_stream + 100   # frame 1's info inside frame 0's stream
    assert L.gsc_encode_batch(descs, 2, ctypes.byref(p), None) == 1
    sd = (gsc.StreamDescC * 2)()
    for f in range(2):
        d = sd[f]
        d.d_stream, d.stream_bytes, d.n_cap = _addr(10 * f).value, cap, n
        d.d_pos_out, d.d_attr_out = _addr(10 * f + 1).value, _addr(10 * f + 2).value
        d.d_ws, d.ws_bytes, d.d_info = _addr(10 * f + 3).value, ws, _addr(10 * f + 4).value
    sd[1].d_attr_out = sd[0].d_stream + 8     # frame 1's output over frame 0's input stream
    assert L.gsc_decode_batch(sd, 2, J, C, None) == 1


def test_straight_through_rejects_overlapping_buffers():
    L = gsc.lib()
    J, C, n = 8, 4, 100
    p = gsc.make_params(J, C, 0.1)
    ws = gsc.workspace_size(n, J, C)
    cap = gsc.stream_capacity(n, J, C)
    # ahat starts inside yhat (not at the same address)
    assert L.gsc_ste_forward(_addr(0), _addr(1), n, ctypes.byref(p), _addr(2), cap, _addr(3), ws,
                             _addr(4), _addr(5), _addr(5, 16), None, None, None) == 1
    # the gradient output over the workspace
    assert L.gsc_ste_backward(n, J, C, _addr(0), _addr(1), _addr(3, ws - 4), _addr(3), ws,
                              _addr(4), None) == 1


def test_binding_validates_tensors():
    torch = pytest.importorskip("torch")
    p = gsc.make_params(8, 4, 0.1)
    with pytest.raises(ValueError):   # host tensors are refused before any call
        gsc.encode_frame(torch.zeros((10, 3)), torch.zeros((10, 4)), p)


def test_rlgr_sizes_and_argument_checks():
    # worst case: 68 bits per value, a partial word per block, the header and the block table
    nv, C, B = 1000, 56, 512
    nb = -(-nv // B) * C
    assert gsc.rlgr_capacity(nv, C, B) == 32 + 4 * (nb + 1) + 4 * ((nv * C * 68 + 31) // 32 + nb)
    assert gsc.rlgr_workspace_size(nv, B) == 8 * (-(-nv // B) + 1)
    L = gsc.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    ws = gsc.rlgr_workspace_size(nv, B)
    cap = gsc.rlgr_capacity(nv, C, B)
    enc = lambda n=nv, c=C, b=B, w=ws, k=cap, q=fake: L.gsc_rlgr_encode(q, n, c, b, fake, k, fake, w, fake, None)
    assert enc(c=0) == 2 and enc(c=65) == 2
    assert enc(b=0) == 1 and enc(b=65537) == 1 and enc(n=-1) == 1
    assert enc(w=8) == 3
    assert enc(k=32) == 4
    assert enc(q=None) == 1
    dec = lambda n=nv, c=C, b=B, k=cap: L.gsc_rlgr_decode(fake, k, n, c, b, fake, fake, 8, fake, None)
    assert dec(k=16) == 4 and dec(c=0) == 2 and dec(b=0) == 1
    with pytest.raises(gsc.GscError):
        gsc.rlgr_capacity(10, 0, 512)


def test_color_sizes_and_argument_checks():
    # at most 256 blocks of 768 FP64 partial sums, then 8 folded groups of them
    assert gsc.color_workspace_size(0) == 8 * 768 * 8
    assert gsc.color_workspace_size(1_000_000) <= (256 + 8) * 768 * 8
    L = gsc.lib()
    fake = [ctypes.c_void_p(0x1000000 * (i + 1)) for i in range(6)]  # disjoint, never dereferenced
    n, C = 1000, 56
    ws = gsc.color_workspace_size(n)
    fwd = lambda n=n, c=C, s0=8, w=ws, a=fake[0], o=fake[1], k=fake[2]: L.gsc_color_forward(
        a, n, c, s0, o, k, None, fake[3], w, fake[4], None)
    assert fwd(c=65) == 1 and fwd(c=47) == 1 and fwd(s0=9) == 1 and fwd(s0=-1) == 1 and fwd(n=-1) == 1
    assert fwd(w=ws - 1) == 3
    assert fwd(k=None) == 1 and fwd(a=None) == 1
    assert fwd(o=fake[0]) == 1                      # output over the input
    assert fwd(k=ctypes.c_void_p(0x1000000 + 8)) == 1  # basis inside the input rows
    inv = lambda n=n, c=C, s0=8, a=fake[0], k=fake[2], o=fake[1]: L.gsc_color_inverse(a, n, c, s0, k, o, None)
    assert inv(s0=9) == 1 and inv(k=None) == 1 and inv(o=fake[0]) == 1


def test_rans_sizes_and_argument_checks():
    n, K = 100_000, 512
    nc = -(-n // K)
    # header, table, offsets and at most 2 bytes per input byte plus 4 per chunk
    assert gsc.rans_capacity(n, K) == 32 + 512 + 4 * (nc + 1) + 2 * n + 4 * nc
    assert gsc.rans_capacity(0, K) == 32 + 512 + 4
    L = gsc.lib()
    fake = [ctypes.c_void_p(0x10000000 * (i + 1)) for i in range(4)]  # disjoint, never dereferenced
    ws = gsc.rans_workspace_size(n, K)
    cap = gsc.rans_capacity(n, K)
    enc = lambda n=n, k=K, w=ws, c=cap, a=fake[0], o=fake[1]: L.gsc_rans_encode(a, n, k, o, c, fake[2], w, fake[3], None)
    assert enc(k=0) == 1 and enc(k=(1 << 20) + 1) == 1 and enc(n=-1) == 1 and enc(a=None) == 1
    assert enc(w=ws - 1) == 3
    assert enc(c=32) == 4
    assert enc(o=fake[0]) == 1  # the stream over the input
    dec = lambda n=n, k=K, c=cap, w=8, o=fake[1]: L.gsc_rans_decode(fake[0], c, n, k, o, fake[2], w, fake[3], None)
    assert dec(c=100) == 4 and dec(w=4) == 3 and dec(k=0) == 1 and dec(o=fake[0]) == 1
    # the stream and the workspace 8-byte aligned; the raw bytes anywhere (no launch is reached
    # with a misaligned pointer; an aligned call would launch, so only rejections are tried here)
    odd = lambda p, d: ctypes.c_void_p(p.value + d)
    assert enc(o=odd(fake[1], 4)) == 1
    assert L.gsc_rans_encode(fake[0], n, K, fake[1], cap, odd(fake[2], 1), ws, fake[3], None) == 1
    assert L.gsc_rans_encode(fake[0], n, K, fake[1], cap, fake[2], ws, odd(fake[3], 2), None) == 1
    assert L.gsc_rans_decode(odd(fake[0], 2), cap, n, K, fake[1], fake[2], 8, fake[3], None) == 1
    assert L.gsc_rans_decode(fake[0], cap, n, K, fake[1], odd(fake[2], 4), 8, fake[3], None) == 1
    with pytest.raises(gsc.GscError):
        gsc.rans_capacity(10, 0)


def test_tuning_table_round_trips_through_a_file(tmp_path):
    """The autotuner's table (host memory only, no GPU needed): entries set, saved, cleared,
    loaded back; the sizes of one class share an entry."""
    # untuned sizes: 2048-key tiles up to 2^18 Gaussians, 4096-key tiles above
    assert gsc.tune_get(10, 100_000) == 1 and gsc.tune_get(12, 1_000_000) == 0
    assert gsc.sort_default_variant(1 << 18) == 1 and gsc.sort_default_variant((1 << 18) + 1) == 0
    gsc.tune_set(12, 1_000_000, 2)
    gsc.tune_set(14, 4_000_000, 3)
    gsc.tune_set(10, 100_000, gsc.sort_default_variant(100_000))  # the default: not listed
    try:
        t = gsc.tune_table()
        assert t[(12, 20)] == 2 and t[(14, 22)] == 3 and (10, 17) not in t
        assert gsc.tune_get(12, 600_000) == 2  # same size class (2^19 < n <= 2^20)
        path = tmp_path / "tune.json"
        gsc.save_tuning(str(path))
        gsc.tune_set(12, 1_000_000, -1)
        gsc.tune_set(14, 4_000_000, -1)
        assert gsc.tune_table() == {}
        gsc.load_tuning(str(path))
        assert gsc.tune_table() == t
    finally:
        gsc.tune_set(12, 1_000_000, -1)
        gsc.tune_set(14, 4_000_000, -1)
        gsc.tune_set(10, 100_000, -1)
