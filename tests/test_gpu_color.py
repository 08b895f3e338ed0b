"""Parity of the colour decorrelation (Sec. 4: YUV on every SH function, one KLT per YUV channel
over the AC SH coefficients) on the GPU with the FP64 oracle.

Bars. The eigenvalues within 1e-5 of the largest one. Each basis vector within the perturbation
bound of its eigenvalue's gap: the GPU's covariance carries FP32 rounding (products summed in
FP32 over 64 rows before FP64), taken as at most 3e-5 of the largest eigenvalue in the 2-norm,
so vector j may turn by at most 2 * 3e-5 * lambda_max / gap_j (Davis-Kahan), plus 1e-5. The
canonical sign (largest-magnitude component positive) on the GPU's own basis. The forward
output: columns outside the SH range equal, the YUV DC within 1e-6 of the row scale, and every
KLT coefficient equal to the GPU's basis applied to the oracle's YUV values within 1e-5 of the
row scale (the basis is pinned by the first bar). The inverse applied to the oracle's forward
output with the oracle's basis returns the input rows within 1e-5 of the row scale.
"""
import numpy as np
import pytest

from oracle import color_oracle as co
from paper_2606_05650_amd import gsc, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SH0 = 8


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gpu_forward(attr, sh0=SH0):
    dev = _dev()
    r = gsc.color_forward(torch.from_numpy(np.ascontiguousarray(attr)).to(dev), sh0)
    torch.cuda.synchronize()
    info = r.info.cpu().numpy()
    assert info[0] == 0 and info[1] == attr.shape[0]
    n = attr.shape[0]
    return (r.out[:n].cpu().numpy().astype(np.float64), r.klt.cpu().numpy().astype(np.float64),
            r.eig.cpu().numpy())


def _yuv_ac(attr, sh0=SH0):
    M = co.yuv_matrix()
    return np.einsum("ck,nkf->ncf", M, attr[:, sh0 + 3:sh0 + 48].astype(np.float64).reshape(-1, 3, 15))


def _check_forward(attr, sh0=SH0):
    print(f"case n={attr.shape[0]} C={attr.shape[1]} sh0={sh0}", flush=True)
    out, E, eig = _gpu_forward(attr, sh0)
    ref = co.color_forward(attr, sh0)
    C = attr.shape[1]
    other = [j for j in range(C) if not sh0 <= j < sh0 + 48]
    assert np.array_equal(out[:, other], attr[:, other].astype(np.float64))
    scale = np.abs(attr[:, sh0:sh0 + 48]).max() + 1e-30
    assert np.abs(out[:, sh0:sh0 + 3] - ref["out"][:, sh0:sh0 + 3]).max() <= 1e-6 * scale
    x = _yuv_ac(attr, sh0)
    for c in range(3):
        lam = ref["eig"][c]
        lmax = max(lam[0], 1e-300)
        assert np.abs(eig[c] - lam).max() <= 1e-5 * lmax, f"channel {c} eigenvalues"
        gaps = np.minimum(np.r_[np.inf, -np.diff(lam)], np.r_[-np.diff(lam), np.inf])
        for j in range(15):
            tol = 2 * 3e-5 * lmax / max(gaps[j], 1e-300) + 1e-5
            assert np.linalg.norm(E[c][:, j] - ref["E"][c][:, j]) <= tol, f"channel {c} vector {j}"
            i = int(np.argmax(np.abs(E[c][:, j])))
            assert E[c][i, j] > 0
        a = out[:, sh0 + 3 + 15 * c:sh0 + 18 + 15 * c]
        assert np.abs(a - x[:, c, :] @ E[c]).max() <= 1e-5 * scale, f"channel {c} coefficients"
    return out, E


def _check_inverse(attr, sh0=SH0):
    dev = _dev()
    ref = co.color_forward(attr, sh0)
    coef = torch.from_numpy(ref["out"].astype(np.float32)).to(dev)
    klt = torch.from_numpy(ref["E"].astype(np.float32)).to(dev)
    got = gsc.color_inverse(coef, klt, sh0)
    torch.cuda.synchronize()
    got = got[:attr.shape[0]].cpu().numpy().astype(np.float64)
    scale = np.abs(attr).max()
    assert np.abs(got - attr).max() <= 1e-5 * scale


@pytest.mark.parametrize("n,seed", [(2_000, 1), (100_003, 2), (1_000_000, 3)])
def test_forward_and_inverse_match_oracle(n, seed):
    _, attr = synth.make_color_frame(n, seed)
    _check_forward(attr)
    _check_inverse(attr)


def test_round_trip_and_determinism():
    dev = _dev()
    _, attr = synth.make_color_frame(300_001, 4)
    ta = torch.from_numpy(attr).to(dev)
    r1 = gsc.color_forward(ta)
    r2 = gsc.color_forward(ta)
    back = gsc.color_inverse(r1.out, r1.klt)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out) and torch.equal(r1.klt, r2.klt)
    assert (back - ta).abs().max().item() <= 1e-5 * ta.abs().max().item()


def test_uncorrelated_sh_still_decorrelates():
    """The standard frames' SH coefficients are i.i.d., so their eigenvalues nearly coincide and
    the basis is not unique: the GPU's own basis must still be orthonormal and diagonalize the
    channel's covariance."""
    _, attr = synth.make_frame(200_000, 5)
    out, E, eig = _gpu_forward(attr)
    x = _yuv_ac(attr)
    for c in range(3):
        assert np.allclose(E[c].T @ E[c], np.eye(15), atol=1e-6)
        a = x[:, c, :] @ E[c]
        d = a - a.mean(axis=0)
        S = d.T @ d / len(a)
        off = S - np.diag(np.diag(S))
        assert np.abs(off).max() <= 1e-3 * S.diagonal().max()
        assert np.all(np.diff(eig[c]) <= 1e-12 * eig[c][0])


@pytest.mark.parametrize("n", [1, 2, 3, 63, 65, 257])
def test_small_and_ragged(n):
    _, attr = synth.make_color_frame(max(n, 2), 6)
    attr = attr[:n]
    if n < 2:
        out, E, eig = _gpu_forward(attr)
        assert np.array_equal(E, np.stack([np.eye(15)] * 3))
        ref = co.color_forward(attr)
        assert np.abs(out - ref["out"]).max() <= 1e-6 * np.abs(attr).max()
    else:
        _check_forward(attr)
    _check_inverse(attr)


def test_other_layouts():
    rng = np.random.default_rng(7)
    _, attr = synth.make_color_frame(5_000, 7)
    wide = np.concatenate([rng.normal(size=(5_000, 8)).astype(np.float32), attr], axis=1)  # C = 64, sh0 = 16
    _check_forward(wide, 16)
    _check_inverse(wide, 16)
    only = np.ascontiguousarray(attr[:, 8:56])  # C = 48, sh0 = 0
    _check_forward(only, 0)
    _check_inverse(only, 0)
    # C = 51 (not a multiple of 4: the kernels' scalar row path), SH at columns 3..50
    odd = np.ascontiguousarray(np.concatenate([attr[:, 5:8], attr[:, 8:56]], axis=1))
    _check_forward(odd, 3)
    _check_inverse(odd, 3)


def test_empty_frame():
    dev = _dev()
    r = gsc.color_forward(torch.empty((0, 56), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    assert np.array_equal(r.klt.cpu().numpy(), np.stack([np.eye(15)] * 3).astype(np.float32))
    assert r.info.cpu().numpy()[0] == 0
