"""Python binding of libgsc (include/gsc.h): argument marshalling only.

Every step of the codec runs in the HIP kernels of libgsc.so; this module only allocates device
buffers with PyTorch, passes raw pointers and the current HIP stream through ctypes, and reads
back the device status words. It fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "gsc.h")

MAX_DEPTH = 21
MAX_CHANNELS = 64
MAX_BATCH = 64
HEADER_BYTES = 1024
VERSION = 1         # GSC_VERSION
INFO_WORDS = 8
STATIC_SCRATCH_BYTES = 64 << 20  # GSC_STATIC_SCRATCH_BYTES

STATUS = {0: "GSC_OK", 1: "GSC_ERR_INVALID_ARG", 2: "GSC_ERR_DEPTH", 3: "GSC_ERR_WORKSPACE",
          4: "GSC_ERR_CAPACITY", 5: "GSC_ERR_CORRUPT_STREAM", 6: "GSC_ERR_HIP",
          7: "GSC_ERR_INTERNAL", 8: "GSC_ERR_SCRATCH"}


class GscError(RuntimeError):
    def __init__(self, code, where):
        self.code = int(code)
        super().__init__(f"{where}: {STATUS.get(self.code, self.code)}")


class Params(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int32), ("C", ctypes.c_int32),
                ("quant_step", ctypes.c_float * MAX_CHANNELS), ("tau", ctypes.c_float),
                ("bbox_mode", ctypes.c_int32), ("bbox_min", ctypes.c_double * 3),
                ("cell", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


FLAG_FP64_WEIGHTS = 0x1


class FrameDescC(ctypes.Structure):
    _fields_ = [("d_pos", ctypes.c_void_p), ("d_attr", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("d_stream", ctypes.c_void_p), ("stream_cap", ctypes.c_size_t),
                ("d_ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("d_info", ctypes.c_void_p)]


class StreamDescC(ctypes.Structure):
    _fields_ = [("d_stream", ctypes.c_void_p), ("stream_bytes", ctypes.c_size_t),
                ("n_cap", ctypes.c_int64), ("d_pos_out", ctypes.c_void_p),
                ("d_attr_out", ctypes.c_void_p), ("d_ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("d_info", ctypes.c_void_p)]


# Byte layout of the stream header (gsc_header in include/gsc.h), little-endian.
HEADER_DTYPE = np.dtype([
    ("magic", "<u4"), ("version", "<u4"), ("J", "<u4"), ("C", "<u4"), ("n_in", "<u4"),
    ("n_vox", "<u4"), ("level_sizes", "<u4", (22,)), ("error", "<u4"), ("flags", "<u4"),
    ("bbox_min", "<f8", (3,)), ("cell", "<f8"), ("quant_step", "<f4", (64,)), ("tau", "<f4"),
    ("reserved1", "<u4"), ("occ_offset", "<u8"), ("occ_bytes", "<u8"), ("coef_offset", "<u8"),
    ("coef_bytes", "<u8"), ("total_bytes", "<u8")])

_lib = None


def lib():
    """The loaded libgsc.so. Raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgsc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.gsc_workspace_size.restype = i32
        L.gsc_workspace_size.argtypes = [i64, i32, i32, ctypes.POINTER(sz)]
        L.gsc_stream_capacity.restype = i32
        L.gsc_stream_capacity.argtypes = [i64, i32, i32, ctypes.POINTER(sz)]
        L.gsc_encode_frame.restype = i32
        L.gsc_encode_frame.argtypes = [vp, vp, i64, ctypes.POINTER(Params), vp, sz, vp, sz, vp, vp,
                                       vp, vp, vp, vp]
        L.gsc_encode_frame_noalloc.restype = i32
        L.gsc_encode_frame_noalloc.argtypes = [vp, vp, i64, ctypes.POINTER(Params), vp, sz, vp,
                                               vp, vp, vp, vp, vp]
        L.gsc_decode_frame.restype = i32
        L.gsc_decode_frame.argtypes = [vp, sz, i32, i32, i64, vp, vp, vp, vp, vp, sz, vp, vp]
        L.gsc_encode_batch.restype = i32
        L.gsc_encode_batch.argtypes = [ctypes.POINTER(FrameDescC), i32, ctypes.POINTER(Params), vp]
        L.gsc_decode_batch.restype = i32
        L.gsc_decode_batch.argtypes = [ctypes.POINTER(StreamDescC), i32, i32, i32, vp]
        L.gsc_autotune.restype = i32
        L.gsc_autotune.argtypes = [ctypes.POINTER(FrameDescC), i32, ctypes.POINTER(Params), i32,
                                   ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), vp]
        L.gsc_tune_set.restype = i32
        L.gsc_tune_set.argtypes = [i32, i64, i32]
        L.gsc_tune_get.restype = i32
        L.gsc_tune_get.argtypes = [i32, i64, ctypes.POINTER(i32)]
        L.gsc_ste_forward.restype = i32
        L.gsc_ste_forward.argtypes = [vp, vp, i64, ctypes.POINTER(Params), vp, sz, vp, sz, vp, vp,
                                      vp, vp, vp, vp]
        L.gsc_ste_backward.restype = i32
        L.gsc_ste_backward.argtypes = [i64, i32, i32, vp, vp, vp, vp, sz, vp, vp]
        L.gsc_raht_forward.restype = i32
        L.gsc_raht_forward.argtypes = [vp, i64, i32, i32, vp, vp, vp, sz, vp, vp]
        L.gsc_raht_adjoint.restype = i32
        L.gsc_raht_adjoint.argtypes = [vp, i64, i32, i32, vp, vp, vp, sz, vp, vp]
        L.gsc_rlgr_capacity.restype = i32
        L.gsc_rlgr_capacity.argtypes = [i64, i32, i32, ctypes.POINTER(sz)]
        L.gsc_rlgr_workspace_size.restype = i32
        L.gsc_rlgr_workspace_size.argtypes = [i64, i32, ctypes.POINTER(sz)]
        L.gsc_rlgr_encode.restype = i32
        L.gsc_rlgr_encode.argtypes = [vp, i64, i32, i32, vp, sz, vp, sz, vp, vp]
        L.gsc_rlgr_decode.restype = i32
        L.gsc_rlgr_decode.argtypes = [vp, sz, i64, i32, i32, vp, vp, sz, vp, vp]
        L.gsc_rans_capacity.restype = i32
        L.gsc_rans_capacity.argtypes = [i64, i32, ctypes.POINTER(sz)]
        L.gsc_rans_workspace_size.restype = i32
        L.gsc_rans_workspace_size.argtypes = [i64, i32, ctypes.POINTER(sz)]
        L.gsc_rans_encode.restype = i32
        L.gsc_rans_encode.argtypes = [vp, i64, i32, vp, sz, vp, sz, vp, vp]
        L.gsc_rans_decode.restype = i32
        L.gsc_rans_decode.argtypes = [vp, sz, i64, i32, vp, vp, sz, vp, vp]
        L.gsc_color_workspace_size.restype = i32
        L.gsc_color_workspace_size.argtypes = [i64, ctypes.POINTER(sz)]
        L.gsc_color_forward.restype = i32
        L.gsc_color_forward.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, sz, vp, vp]
        L.gsc_color_inverse.restype = i32
        L.gsc_color_inverse.argtypes = [vp, i64, i32, i32, vp, vp, vp]
        L.gsc_status_string.restype = ctypes.c_char_p
        L.gsc_status_string.argtypes = [i32]
        _lib = L
    return _lib


def declared_symbols(header_path=HEADER_PATH):
    """Names of the functions declared in include/gsc.h."""
    text = open(header_path).read()
    return sorted(set(re.findall(r"^(?:gsc_status|const char \*)\s*(gsc_\w+)\(", text, re.M)))


def status_string(code):
    return lib().gsc_status_string(int(code)).decode()


def _check(code, where):
    if code != 0:
        raise GscError(code, where)


def workspace_size(n, J, C):
    out = ctypes.c_size_t()
    _check(lib().gsc_workspace_size(int(n), int(J), int(C), ctypes.byref(out)), "workspace_size")
    return out.value


def stream_capacity(n, J, C):
    out = ctypes.c_size_t()
    _check(lib().gsc_stream_capacity(int(n), int(J), int(C), ctypes.byref(out)),
           "stream_capacity")
    return out.value


def make_params(J, C, steps, tau=0.5, bbox=None, flags=0):
    p = Params()
    p.J, p.C = int(J), int(C)
    p.flags = int(flags)
    steps = np.broadcast_to(np.asarray(steps, dtype=np.float32), (C,))
    for c in range(C):
        p.quant_step[c] = float(steps[c])
    p.tau = float(tau)
    if bbox is None:
        p.bbox_mode = 0
    else:
        p.bbox_mode = 1
        for a in range(3):
            p.bbox_min[a] = float(bbox[0][a])
        p.cell = float(bbox[1])
    return p


def parse_header(stream_bytes):
    """Decode the 1024-byte header of a stream held in host memory (bytes or uint8 array)."""
    buf = np.frombuffer(bytes(stream_bytes[:HEADER_BYTES]), dtype=np.uint8)
    return np.frombuffer(buf[:HEADER_DTYPE.itemsize].tobytes(), dtype=HEADER_DTYPE)[0]


# ------------------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def assert_disjoint(ranges):
    """Raise if any two device ranges (pointer, bytes) of one launch overlap."""
    rs = sorted((int(p), int(n)) for p, n in ranges if n > 0)
    for (p0, n0), (p1, _) in zip(rs, rs[1:]):
        if p0 + n0 > p1:
            raise ValueError(f"device buffers of one batch overlap at {p1:#x}")


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_tensor(t, name, dtype, rows=None, cols=None, numel=None):
    """Raise unless t (if given) is a contiguous CUDA tensor of the dtype the C ABI reads or
    writes through its pointer, with at least `rows` rows of exactly `cols` columns (or at
    least `numel` elements)."""
    if t is None:
        return
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: a CUDA tensor is required")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if rows is not None:
        if t.dim() < 1 or t.shape[0] < rows:
            raise ValueError(f"{name}: needs at least {rows} rows, has shape {tuple(t.shape)}")
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"{name}: needs {cols} columns, has shape {tuple(t.shape)}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")


def _dev_u8(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class Encoded:
    stream: "object"     # uint8 device tensor holding the stream (capacity bytes)
    info: "object"       # int32 device tensor [GSC_INFO_WORDS]
    J: int
    C: int
    ws: "object" = None  # the workspace the call used (kept alive with the result)

    def host_info(self):
        return self.info.cpu().numpy()

    def total_bytes(self):
        i = self.host_info()
        return int(np.uint32(i[2])) | (int(np.uint32(i[3])) << 32)

    def n_vox(self):
        return int(self.host_info()[1])

    def check(self):
        i = self.host_info()
        if i[0] != 0:
            raise GscError(i[0], "device")
        return self

    def to_bytes(self):
        """The stream's used bytes, copied to the host."""
        return self.stream[:self.total_bytes()].cpu().numpy().tobytes()


class Workspace:
    """A reusable device workspace sized for frames of up to n_max entries."""

    def __init__(self, n_max, J, C, device="cuda"):
        self.n_max, self.J, self.C = int(n_max), int(J), int(C)
        self.bytes = workspace_size(n_max, J, C)
        self.buf = _dev_u8(self.bytes, device)

    def fits(self, n, J, C):
        return n <= self.n_max and J == self.J and C == self.C


def encode_frame(pos, attr, params, *, ws=None, stream_buf=None, info=None, coef_f32=None,
                 leaf_codes=None, perm=None, voxel_of=None, stream=None):
    """Encode one frame. pos: [n,3] float32 cuda, attr: [n,C] float32 cuda (contiguous).
    Optional outputs: coef_f32 [n,C] float32, leaf_codes [n] int64 (uint64 codes), perm and
    voxel_of [n] int32 (the stable sorted order and each Gaussian's voxel)."""
    torch = _torch()
    n = int(pos.shape[0])
    C = int(params.C)
    dev = pos.device
    _check_tensor(pos, "pos", torch.float32, n, 3)
    _check_tensor(attr, "attr", torch.float32, n, C)
    if ws is None:
        ws = Workspace(max(n, 1), params.J, C, dev)
    cap = stream_capacity(n, params.J, C)
    if stream_buf is None:
        stream_buf = _dev_u8(cap, dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(stream_buf, "stream_buf", torch.uint8, numel=cap)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    _check_tensor(coef_f32, "coef_f32", torch.float32, n, C)
    _check_tensor(leaf_codes, "leaf_codes", torch.int64, n)
    _check_tensor(perm, "perm", torch.int32, n)
    _check_tensor(voxel_of, "voxel_of", torch.int32, n)
    rc = lib().gsc_encode_frame(_ptr(pos), _ptr(attr), n, ctypes.byref(params), _ptr(stream_buf),
                                stream_buf.numel(), _ptr(ws.buf), ws.bytes, _ptr(info),
                                _ptr(coef_f32), _ptr(leaf_codes), _ptr(perm), _ptr(voxel_of),
                                _stream(stream))
    _check(rc, "gsc_encode_frame")
    return Encoded(stream_buf, info, int(params.J), C, ws)


def encode_frame_noalloc(pos, attr, params, *, stream_buf=None, info=None, coef_f32=None,
                         leaf_codes=None, perm=None, voxel_of=None, stream=None):
    """encode_frame on the library's static per-device scratch instead of a workspace (for
    frames whose workspace fits GSC_STATIC_SCRATCH_BYTES). The outputs, when not given, are
    allocated here; the C call itself allocates nothing."""
    torch = _torch()
    n = int(pos.shape[0])
    C = int(params.C)
    dev = pos.device
    _check_tensor(pos, "pos", torch.float32, n, 3)
    _check_tensor(attr, "attr", torch.float32, n, C)
    cap = stream_capacity(n, params.J, C)
    if stream_buf is None:
        stream_buf = _dev_u8(cap, dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(stream_buf, "stream_buf", torch.uint8, numel=cap)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    _check_tensor(coef_f32, "coef_f32", torch.float32, n, C)
    _check_tensor(leaf_codes, "leaf_codes", torch.int64, n)
    _check_tensor(perm, "perm", torch.int32, n)
    _check_tensor(voxel_of, "voxel_of", torch.int32, n)
    rc = lib().gsc_encode_frame_noalloc(_ptr(pos), _ptr(attr), n, ctypes.byref(params),
                                        _ptr(stream_buf), stream_buf.numel(), _ptr(info),
                                        _ptr(coef_f32), _ptr(leaf_codes), _ptr(perm),
                                        _ptr(voxel_of), _stream(stream))
    _check(rc, "gsc_encode_frame_noalloc")
    return Encoded(stream_buf, info, int(params.J), C, None)


@dataclass
class Decoded:
    pos: "object"
    attr: "object"
    vox: "object"
    codes: "object"
    info: "object"
    ws: "object" = None

    def n_vox(self):
        return int(self.info[1].item())

    def check(self):
        i = self.info.cpu().numpy()
        if i[0] != 0:
            raise GscError(i[0], "device")
        return self


def decode_frame(stream_buf, J, C, n_cap, *, stream_bytes=None, ws=None, want_vox=False,
                 want_codes=False, pos_out=None, attr_out=None, info=None, stream=None):
    """Decode one device stream into voxel centres and attributes (Morton order)."""
    torch = _torch()
    dev = stream_buf.device
    n_cap = int(n_cap)
    if ws is None:
        ws = Workspace(max(n_cap, 1), J, C, dev)
    if pos_out is None:
        pos_out = torch.empty((max(n_cap, 1), 3), dtype=torch.float32, device=dev)
    if attr_out is None:
        attr_out = torch.empty((max(n_cap, 1), C), dtype=torch.float32, device=dev)
    vox = torch.empty((max(n_cap, 1), 3), dtype=torch.int32, device=dev) if want_vox else None
    codes = torch.empty(max(n_cap, 1), dtype=torch.int64, device=dev) if want_codes else None
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    nbytes = stream_buf.numel() if stream_bytes is None else int(stream_bytes)
    _check_tensor(stream_buf, "stream_buf", torch.uint8, numel=nbytes)
    _check_tensor(pos_out, "pos_out", torch.float32, n_cap, 3)
    _check_tensor(attr_out, "attr_out", torch.float32, n_cap, C)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_decode_frame(_ptr(stream_buf), nbytes, int(J), int(C), n_cap, _ptr(pos_out),
                                _ptr(vox), _ptr(attr_out), _ptr(codes), _ptr(ws.buf), ws.bytes,
                                _ptr(info), _stream(stream))
    _check(rc, "gsc_decode_frame")
    return Decoded(pos_out, attr_out, vox, codes, info, ws)


def _encode_descs(frames, params, workspaces):
    torch = _torch()
    F = len(frames)
    if F < 1 or F > MAX_BATCH:
        raise ValueError("1..64 frames per batch")
    descs = (FrameDescC * F)()
    outs = []
    # Every buffer of every frame stays referenced (in `outs`) until after the launch: a
    # workspace released inside this loop could be handed by the caching allocator to the next
    # frame's buffers of the same batch, and one launch would then see overlapping buffers.
    for f, (pos, attr) in enumerate(frames):
        n = int(pos.shape[0])
        dev = pos.device
        _check_tensor(pos, f"frames[{f}] pos", torch.float32, n, 3)
        _check_tensor(attr, f"frames[{f}] attr", torch.float32, n, int(params.C))
        ws = workspaces[f] if workspaces is not None else Workspace(max(n, 1), params.J, params.C,
                                                                    dev)
        cap = stream_capacity(n, params.J, params.C)
        sb = _dev_u8(cap, dev)
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
        d = descs[f]
        d.d_pos, d.d_attr, d.n = pos.data_ptr(), attr.data_ptr(), n
        d.d_stream, d.stream_cap = sb.data_ptr(), sb.numel()
        d.d_ws, d.ws_bytes, d.d_info = ws.buf.data_ptr(), ws.bytes, info.data_ptr()
        outs.append(Encoded(sb, info, int(params.J), int(params.C), ws))
    assert_disjoint([(o.stream.data_ptr(), _nbytes(o.stream)) for o in outs] +
                    [(o.info.data_ptr(), _nbytes(o.info)) for o in outs] +
                    [(o.ws.buf.data_ptr(), o.ws.bytes) for o in outs])
    return descs, outs


def encode_batch(frames, params, *, workspaces=None, stream=None):
    """frames: list of (pos, attr) device tensors. Returns a list of Encoded."""
    descs, outs = _encode_descs(frames, params, workspaces)
    _check(lib().gsc_encode_batch(descs, len(frames), ctypes.byref(params), _stream(stream)),
           "gsc_encode_batch")
    return outs


SORT_VARIANTS = 4


def autotune(frames, params, *, reps=3, workspaces=None, stream=None):
    """Times every sort tiling on this batch and keeps the fastest for batches of its size
    class and depth. Synchronous. Returns (chosen variant, mean ms per variant, outputs)."""
    descs, outs = _encode_descs(frames, params, workspaces)
    chosen = ctypes.c_int32(-1)
    times = (ctypes.c_float * SORT_VARIANTS)()
    _check(lib().gsc_autotune(descs, len(frames), ctypes.byref(params), int(reps),
                              ctypes.byref(chosen), times, _stream(stream)), "gsc_autotune")
    return chosen.value, [float(t) for t in times], outs


def tune_set(J, n, variant):
    """Sets (variant >= 0) or clears (-1) the sort tiling used for depth J and frames of n."""
    _check(lib().gsc_tune_set(int(J), int(n), int(variant)), "gsc_tune_set")


def tune_get(J, n):
    v = ctypes.c_int32(-1)
    _check(lib().gsc_tune_get(int(J), int(n), ctypes.byref(v)), "gsc_tune_get")
    return v.value


SORT_DEFAULT_VARIANT = 0  # untuned tiling above 2^18 Gaussians (2048-key tiles, variant 1, below)
SORT_SMALL_VARIANT, SORT_SMALL_MAX = 1, 1 << 18
SORT_TUNE_MARGIN = 0.02  # autotune keeps the default unless another tiling is this much faster


def sort_default_variant(n):
    """The sort tiling used for frames of n Gaussians when nothing is tuned."""
    return SORT_SMALL_VARIANT if n <= SORT_SMALL_MAX else SORT_DEFAULT_VARIANT
_N_LIMIT = (1 << 30) - 1  # the largest frame the library takes
_MAX_DEPTH = 21


def tune_table():
    """The process's tuned sort tilings: {(J, size class c): variant} for every depth and frame
    size class (frames of 2^(c-1) < n <= 2^c Gaussians) whose tiling differs from the default."""
    out = {}
    for J in range(1, _MAX_DEPTH + 1):
        for c in range(0, 31):
            n = min(1 << c, _N_LIMIT)
            if c > 0 and n <= (1 << (c - 1)):
                break
            v = tune_get(J, n)
            if v != sort_default_variant(n):
                out[(J, c)] = v
    return out


def save_tuning(path):
    """Writes tune_table() to a JSON file (a list of {"J", "size_class", "variant"})."""
    import json
    rows = [{"J": J, "size_class": c, "variant": v} for (J, c), v in sorted(tune_table().items())]
    with open(path, "w") as f:
        json.dump({"version": VERSION, "sort_variants": SORT_VARIANTS, "entries": rows}, f, indent=1)


def load_tuning(path):
    """Sets the sort tilings saved by save_tuning (entries of another library version or variant
    count are refused)."""
    import json
    with open(path) as f:
        d = json.load(f)
    if d.get("version") != VERSION or d.get("sort_variants") != SORT_VARIANTS:
        raise ValueError("tuning file of another library version or variant set")
    for e in d["entries"]:
        tune_set(int(e["J"]), min(1 << int(e["size_class"]), _N_LIMIT), int(e["variant"]))


def decode_batch(encoded, n_caps, *, workspaces=None, stream=None):
    """encoded: list of Encoded. Returns a list of Decoded (pos, attr only)."""
    torch = _torch()
    F = len(encoded)
    descs = (StreamDescC * F)()
    outs = []
    J, C = encoded[0].J, encoded[0].C
    # buffers stay referenced until after the launch (see encode_batch)
    for f, e in enumerate(encoded):
        dev = e.stream.device
        n_cap = int(n_caps[f])
        ws = workspaces[f] if workspaces is not None else Workspace(max(n_cap, 1), J, C, dev)
        pos = torch.empty((max(n_cap, 1), 3), dtype=torch.float32, device=dev)
        attr = torch.empty((max(n_cap, 1), C), dtype=torch.float32, device=dev)
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
        d = descs[f]
        d.d_stream, d.stream_bytes, d.n_cap = e.stream.data_ptr(), e.stream.numel(), n_cap
        d.d_pos_out, d.d_attr_out = pos.data_ptr(), attr.data_ptr()
        d.d_ws, d.ws_bytes, d.d_info = ws.buf.data_ptr(), ws.bytes, info.data_ptr()
        outs.append(Decoded(pos, attr, None, None, info, ws))
    assert_disjoint([(o.pos.data_ptr(), _nbytes(o.pos)) for o in outs] +
                    [(o.attr.data_ptr(), _nbytes(o.attr)) for o in outs] +
                    [(o.info.data_ptr(), _nbytes(o.info)) for o in outs] +
                    [(o.ws.buf.data_ptr(), o.ws.bytes) for o in outs])
    _check(lib().gsc_decode_batch(descs, F, int(J), int(C), _stream(stream)), "gsc_decode_batch")
    return outs


def raht_forward(codes, A, J, *, ws=None, out=None, info=None, stream=None):
    """Y = T A for float rows A [nv, C] of voxels with sorted codes [nv] (int64 view of u64)."""
    return _raht(codes, A, J, ws, out, info, stream, adjoint=False)


def raht_adjoint(codes, Y, J, *, ws=None, out=None, info=None, stream=None):
    """A = T^T Y (the inverse transform)."""
    return _raht(codes, Y, J, ws, out, info, stream, adjoint=True)


def _raht(codes, X, J, ws, out, info, stream, adjoint):
    torch = _torch()
    nv, C = int(X.shape[0]), int(X.shape[1])
    dev = X.device
    _check_tensor(X, "input rows", torch.float32, nv, C)
    _check_tensor(codes, "codes", torch.int64, nv)
    if ws is None:
        ws = Workspace(max(nv, 1), J, C, dev)
    if out is None:
        out = torch.empty_like(X)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(out, "out", torch.float32, nv, C)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    fn = lib().gsc_raht_adjoint if adjoint else lib().gsc_raht_forward
    rc = fn(_ptr(codes), nv, int(J), C, _ptr(X), _ptr(out), _ptr(ws.buf), ws.bytes, _ptr(info),
            _stream(stream))
    _check(rc, "gsc_raht_adjoint" if adjoint else "gsc_raht_forward")
    return out, info


@dataclass
class SteForward:
    """Result of ste_forward: rows [:nv] of yhat, ahat, aref are valid once the call completes."""
    yhat: "object"       # [n, C] float32: dequantized coefficients q * step
    ahat: "object"       # [n, C] float32: T^T yhat, the decoded voxel attributes
    aref: "object"       # [n, C] float32: voxel means of the input rows
    encoded: Encoded     # the stream, info words and the workspace holding the schedule
    n: int


def ste_forward(pos, attr, params, *, ws=None, stream_buf=None, info=None, yhat=None, ahat=None,
                aref=None, leaf_codes=None, stream=None):
    """Straight-through forward: encode (stream written) + voxel means, dequantized
    coefficients and their synthesis."""
    torch = _torch()
    n = int(pos.shape[0])
    C = int(params.C)
    dev = pos.device
    if ws is None:
        ws = Workspace(max(n, 1), params.J, C, dev)
    cap = stream_capacity(n, params.J, C)
    if stream_buf is None:
        stream_buf = _dev_u8(cap, dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    rows = (max(n, 1), C)
    yhat = torch.empty(rows, dtype=torch.float32, device=dev) if yhat is None else yhat
    ahat = torch.empty(rows, dtype=torch.float32, device=dev) if ahat is None else ahat
    aref = torch.empty(rows, dtype=torch.float32, device=dev) if aref is None else aref
    _check_tensor(pos, "pos", torch.float32, n, 3)
    _check_tensor(attr, "attr", torch.float32, n, C)
    _check_tensor(stream_buf, "stream_buf", torch.uint8, numel=cap)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    for name, t in (("yhat", yhat), ("ahat", ahat), ("aref", aref)):
        _check_tensor(t, name, torch.float32, n, C)
    _check_tensor(leaf_codes, "leaf_codes", torch.int64, n)
    rc = lib().gsc_ste_forward(_ptr(pos), _ptr(attr), n, ctypes.byref(params), _ptr(stream_buf),
                               stream_buf.numel(), _ptr(ws.buf), ws.bytes, _ptr(info), _ptr(yhat),
                               _ptr(ahat), _ptr(aref), _ptr(leaf_codes), _stream(stream))
    _check(rc, "gsc_ste_forward")
    return SteForward(yhat, ahat, aref, Encoded(stream_buf, info, int(params.J), C, ws), n)


def ste_backward(fwd, grad_yhat, grad_ahat, *, out=None, info=None, stream=None):
    """dL/dattr [n, C] from dL/dyhat and dL/dahat ([nv, C] contiguous float32 each)."""
    torch = _torch()
    e = fwd.encoded
    dev = e.stream.device
    if out is None:
        out = torch.empty((max(fwd.n, 1), e.C), dtype=torch.float32, device=dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    # the gradients hold one row per occupied voxel (Nv <= n, known once the forward is done)
    _check_tensor(grad_yhat, "grad_yhat", torch.float32, 1, e.C)
    _check_tensor(grad_ahat, "grad_ahat", torch.float32, 1, e.C)
    _check_tensor(out, "out", torch.float32, fwd.n, e.C)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_ste_backward(fwd.n, e.J, e.C, _ptr(grad_yhat), _ptr(grad_ahat), _ptr(out),
                                _ptr(e.ws.buf), e.ws.bytes, _ptr(info), _stream(stream))
    _check(rc, "gsc_ste_backward")
    return out, info


# ----------------------------------------------------------------- block entropy coder
RLGR_MAGIC = 0x31474C52
RLGR_HEADER_DTYPE = np.dtype([("magic", "<u4"), ("version", "<u4"), ("nv", "<u4"), ("C", "<u4"),
                              ("B", "<u4"), ("nblocks", "<u4"), ("total_words", "<u4"),
                              ("reserved", "<u4")])


def rlgr_capacity(nv, C, B):
    out = ctypes.c_size_t()
    _check(lib().gsc_rlgr_capacity(int(nv), int(C), int(B), ctypes.byref(out)), "rlgr_capacity")
    return out.value


def rlgr_workspace_size(nv, B):
    out = ctypes.c_size_t()
    _check(lib().gsc_rlgr_workspace_size(int(nv), int(B), ctypes.byref(out)),
           "rlgr_workspace_size")
    return out.value


@dataclass
class RlgrStream:
    buf: "object"    # uint8 device tensor (capacity bytes)
    info: "object"   # int32 device tensor [GSC_INFO_WORDS]
    nv: int
    C: int
    B: int
    ws: "object" = None

    def check(self):
        i = self.info.cpu().numpy()
        if i[0] != 0:
            raise GscError(i[0], "device")
        return self

    def nbytes(self):
        i = self.info.cpu().numpy()
        return int(np.uint32(i[2])) | (int(np.uint32(i[3])) << 32)

    def to_bytes(self):
        return self.buf[:self.nbytes()].cpu().numpy().tobytes()


def rlgr_encode(q, B, *, out=None, ws=None, info=None, stream=None):
    """Block-parallel run-length / Golomb-Rice coding of q [nv, C] int32 (cuda, contiguous)
    with blocks of B values per channel."""
    torch = _torch()
    nv, C = int(q.shape[0]), int(q.shape[1])
    dev = q.device
    _check_tensor(q, "q", torch.int32, nv, C)
    cap = rlgr_capacity(nv, C, B)
    if out is None:
        out = _dev_u8(cap, dev)
    if ws is None:
        ws = _dev_u8(rlgr_workspace_size(nv, B), dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(out, "out", torch.uint8)
    _check_tensor(ws, "ws", torch.uint8, numel=rlgr_workspace_size(nv, B))
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_rlgr_encode(_ptr(q), nv, C, int(B), _ptr(out), out.numel(), _ptr(ws),
                               ws.numel(), _ptr(info), _stream(stream))
    _check(rc, "gsc_rlgr_encode")
    return RlgrStream(out, info, nv, C, int(B), ws)


def rlgr_decode(buf, nv, C, B, *, nbytes=None, q=None, ws=None, info=None, stream=None):
    """Inverse of rlgr_encode: the stream in `buf` (uint8 cuda) -> q [nv, C] int32."""
    torch = _torch()
    dev = buf.device
    nv, C = int(nv), int(C)
    if q is None:
        q = torch.empty((max(nv, 1), C), dtype=torch.int32, device=dev)
    if ws is None:
        ws = _dev_u8(8, dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(buf, "buf", torch.uint8)
    _check_tensor(q, "q", torch.int32, nv, C)
    _check_tensor(ws, "ws", torch.uint8, numel=8)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    n = buf.numel() if nbytes is None else int(nbytes)
    if n > buf.numel():
        raise ValueError("nbytes exceeds the buffer")
    rc = lib().gsc_rlgr_decode(_ptr(buf), n, nv, C, int(B), _ptr(q), _ptr(ws), ws.numel(),
                               _ptr(info), _stream(stream))
    _check(rc, "gsc_rlgr_decode")
    return q, info


# ----------------------------------------------------------------- colour decorrelation
COLOR_SH_CHANNELS = 48
COLOR_KLT_SHAPE = (3, 15, 15)


def color_workspace_size(n):
    out = ctypes.c_size_t()
    _check(lib().gsc_color_workspace_size(int(n), ctypes.byref(out)), "color_workspace_size")
    return out.value


@dataclass
class ColorForward:
    out: "object"    # [n, C] float32: YUV DC and KLT coefficients in the SH columns
    klt: "object"    # [3, 15, 15] float32: E[c][i][j], component i of basis vector j
    eig: "object"    # [3, 15] float64: the eigenvalues, decreasing
    info: "object"   # int32 [GSC_INFO_WORDS]


def color_forward(attr, sh0=8, *, out=None, klt=None, eig=None, ws=None, info=None, stream=None):
    """YUV on every SH function, then a per-frame KLT per YUV channel over the AC coefficients
    (attr: [n, C] float32 cuda, contiguous; the 48 SH channels start at column sh0)."""
    torch = _torch()
    n, C = int(attr.shape[0]), int(attr.shape[1])
    dev = attr.device
    _check_tensor(attr, "attr", torch.float32, n, C)
    if out is None:
        out = torch.empty((max(n, 1), C), dtype=torch.float32, device=dev)
    if klt is None:
        klt = torch.empty(COLOR_KLT_SHAPE, dtype=torch.float32, device=dev)
    if eig is None:
        eig = torch.empty((3, 15), dtype=torch.float64, device=dev)
    need = color_workspace_size(n)
    if ws is None:
        ws = _dev_u8(need, dev)
    if info is None:
        info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev)
    _check_tensor(out, "out", torch.float32, n, C)
    _check_tensor(klt, "klt", torch.float32, numel=3 * 15 * 15)
    _check_tensor(eig, "eig", torch.float64, numel=45)
    _check_tensor(ws, "ws", torch.uint8, numel=need)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_color_forward(_ptr(attr), n, C, int(sh0), _ptr(out), _ptr(klt), _ptr(eig),
                                 _ptr(ws), ws.numel(), _ptr(info), _stream(stream))
    _check(rc, "gsc_color_forward")
    return ColorForward(out, klt, eig, info)


def color_inverse(coef, klt, sh0=8, *, out=None, stream=None):
    """The decoder's side of color_forward: coef [n, C] and the frame's KLT matrices -> RGB rows."""
    torch = _torch()
    n, C = int(coef.shape[0]), int(coef.shape[1])
    _check_tensor(coef, "coef", torch.float32, n, C)
    _check_tensor(klt, "klt", torch.float32, numel=3 * 15 * 15)
    if out is None:
        out = torch.empty((max(n, 1), C), dtype=torch.float32, device=coef.device)
    _check_tensor(out, "out", torch.float32, n, C)
    rc = lib().gsc_color_inverse(_ptr(coef), n, C, int(sh0), _ptr(klt), _ptr(out), _stream(stream))
    _check(rc, "gsc_color_inverse")
    return out


# ----------------------------------------------------------------- occupancy-byte rANS coder
RANS_MAGIC = 0x314E4152
RANS_HEADER_DTYPE = np.dtype([("magic", "<u4"), ("version", "<u4"), ("n", "<u8"), ("K", "<u4"),
                              ("nchunks", "<u4"), ("total", "<u4"), ("reserved", "<u4")])


def rans_capacity(n, K):
    out = ctypes.c_size_t()
    _check(lib().gsc_rans_capacity(int(n), int(K), ctypes.byref(out)), "rans_capacity")
    return out.value


def rans_workspace_size(n, K):
    out = ctypes.c_size_t()
    _check(lib().gsc_rans_workspace_size(int(n), int(K), ctypes.byref(out)), "rans_workspace_size")
    return out.value


@dataclass
class RansStream:
    buf: "object"    # uint8 device tensor (capacity bytes)
    info: "object"   # int32 device tensor [GSC_INFO_WORDS]
    n: int
    K: int
    ws: "object" = None

    def check(self):
        i = self.info.cpu().numpy()
        if i[0] != 0:
            raise GscError(i[0], "device")
        return self

    def nbytes(self):
        i = self.info.cpu().numpy()
        return int(np.uint32(i[2])) | (int(np.uint32(i[3])) << 32)

    def to_bytes(self):
        return self.buf[:self.nbytes()].cpu().numpy().tobytes()


def rans_encode(data, K, *, out=None, ws=None, info=None, stream=None):
    """Range-ANS coding of a byte string (uint8 cuda tensor, contiguous) in chunks of K bytes."""
    torch = _torch()
    n = int(data.numel())
    dev = data.device
    _check_tensor(data, "data", torch.uint8, numel=n)
    cap = rans_capacity(n, K)
    need = rans_workspace_size(n, K)
    out = _dev_u8(cap, dev) if out is None else out
    ws = _dev_u8(need, dev) if ws is None else ws
    info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev) if info is None else info
    _check_tensor(out, "out", torch.uint8)
    _check_tensor(ws, "ws", torch.uint8, numel=need)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_rans_encode(_ptr(data), n, int(K), _ptr(out), out.numel(), _ptr(ws), ws.numel(),
                               _ptr(info), _stream(stream))
    _check(rc, "gsc_rans_encode")
    return RansStream(out, info, n, int(K), ws)


def rans_decode(buf, n, K, *, nbytes=None, out=None, ws=None, info=None, stream=None):
    """Inverse of rans_encode: the stream in `buf` (uint8 cuda) -> n bytes (uint8 cuda)."""
    torch = _torch()
    dev = buf.device
    n = int(n)
    out = torch.empty(max(n, 1), dtype=torch.uint8, device=dev) if out is None else out
    ws = torch.empty(8, dtype=torch.uint8, device=dev) if ws is None else ws
    info = torch.zeros(INFO_WORDS, dtype=torch.int32, device=dev) if info is None else info
    nb = buf.numel() if nbytes is None else int(nbytes)
    if nb > buf.numel():
        raise ValueError("nbytes exceeds the buffer")
    _check_tensor(buf, "buf", torch.uint8)
    _check_tensor(out, "out", torch.uint8, numel=n)
    _check_tensor(ws, "ws", torch.uint8, numel=8)
    _check_tensor(info, "info", torch.int32, numel=INFO_WORDS)
    rc = lib().gsc_rans_decode(_ptr(buf), nb, n, int(K), _ptr(out), _ptr(ws), ws.numel(), _ptr(info),
                               _stream(stream))
    _check(rc, "gsc_rans_decode")
    return out, info
