"""The allocation-free encode entry point (gsc_encode_frame_noalloc, workspace = the library's
static per-device scratch) against gsc_encode_frame with a caller workspace: the same stream
bytes, device info words and optional outputs, on two calls in a row, the second on a smaller
frame of another depth (the scratch still holds the first call's state)."""
import numpy as np
import pytest
import torch

from paper_2606_05650_amd import gsc, synth

pytestmark = pytest.mark.gpu


def _outputs(n, C, dev):
    return dict(coef_f32=torch.empty((n, C), dtype=torch.float32, device=dev),
                leaf_codes=torch.empty(n, dtype=torch.int64, device=dev),
                perm=torch.empty(n, dtype=torch.int32, device=dev),
                voxel_of=torch.empty(n, dtype=torch.int32, device=dev))


def test_noalloc_encode_matches_workspace_encode():
    dev = torch.device("cuda:0")
    steps = synth.quant_steps(synth.STEPS_GROUPED)
    for n, J, seed in [(500_000, 12, 71), (60_000, 10, 72)]:
        print(f"noalloc encode n={n} J={J} seed={seed}", flush=True)
        assert gsc.workspace_size(n, J, 56) <= gsc.STATIC_SCRATCH_BYTES
        pos, attr = synth.make_frame(n, seed=seed)
        tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
        p = gsc.make_params(J, attr.shape[1], steps)
        oa, ob = _outputs(n, attr.shape[1], dev), _outputs(n, attr.shape[1], dev)
        ref = gsc.encode_frame(tp, ta, p, **oa)
        got = gsc.encode_frame_noalloc(tp, ta, p, **ob)
        torch.cuda.synchronize()
        ref.check()
        got.check()
        assert np.array_equal(got.host_info(), ref.host_info())
        nv = ref.n_vox()
        assert 0 < nv <= n
        assert got.to_bytes() == ref.to_bytes(), "stream bytes differ"
        for k in ("perm", "voxel_of"):  # one entry per Gaussian
            assert torch.equal(ob[k], oa[k]), k
        for k in ("leaf_codes", "coef_f32"):  # one row per voxel
            assert torch.equal(ob[k][:nv], oa[k][:nv]), k
