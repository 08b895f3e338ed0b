"""Pins of the oracle's straight-through loss and gradient (the differentiable coder).

The gradient is pinned by central finite differences of the loss with the quantizer's rounding
residual r = Q(y0) - y0 frozen at the base point (the function whose derivative the
straight-through rule defines), evaluated here in FP64 from the transform alone; by the
adjoint identity of the transform; and by the codec it differentiates.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import synth

GROUPED = synth.quant_steps(synth.STEPS_GROUPED)


def _voxel_mean(attr64, voxel_of, nv):
    C = attr64.shape[1]
    s = np.zeros((nv, C))
    np.add.at(s, voxel_of, attr64)
    cnt = np.bincount(voxel_of, minlength=nv).astype(np.float64)
    return s / cnt[:, None]


def _surrogate(base, J, steps, lam):
    """L(attr) = mean((T^T(T a + r) - a_ref)^2) + lam sum log2(1 + |T a + r| / step), a the voxel
    means of attr, r and a_ref frozen at the base point."""
    leaf, vof, nv = base["leaf"], base["voxel_of"], base["nv"]
    y0 = orc.raht_forward(leaf, J, base["aref"])
    r = base["yhat"] - y0
    aref = base["aref"]
    C = aref.shape[1]

    def f(attr64):
        a = _voxel_mean(attr64, vof, nv)
        yh = orc.raht_forward(leaf, J, a) + r
        ah = orc.raht_inverse(leaf, J, yh)
        return ((ah - aref) ** 2).sum() / (nv * C) + lam * np.log2(1 + np.abs(yh) / steps).sum()
    return f


def test_adjoint_identity():
    rng = np.random.default_rng(0)
    J = 4
    codes = np.unique(rng.integers(0, 8 ** J, size=64).astype(np.uint64))
    x = rng.normal(size=(codes.size, 3))
    y = rng.normal(size=(codes.size, 3))
    lhs = (orc.raht_forward(codes, J, x) * y).sum()
    rhs = (x * orc.raht_inverse(codes, J, y)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(x).sum() * np.abs(y).sum()) ** 0.5


@pytest.mark.parametrize("n,J,lam,dups", [
    (2000, 11, 0.0, False),    # distortion term alone
    (2000, 11, 0.01, False),   # distortion + rate proxy at the lambda of the 500K workload
    (2000, 4, 0.01, True),     # ~4 Gaussians per voxel: the mean and the scatter
])
def test_gradient_matches_finite_differences(n, J, lam, dups):
    if dups:
        pos, attr = synth.make_duplicates_frame(n, seed=3, grid=8)
    else:
        pos, attr = synth.make_frame(n, seed=4)
    base = orc.ste_grad(pos, attr, J, GROUPED, 0.5, lam)
    f = _surrogate(base, J, GROUPED, lam)
    a0 = attr.astype(np.float64)
    assert abs(f(a0) - base["loss"]) <= 1e-12 * max(1.0, abs(base["loss"]))
    g = base["grad"]
    h = 1e-6
    rng = np.random.default_rng(5)
    gmax = np.abs(g).max()
    for _ in range(24):   # single coordinates
        i, c = rng.integers(0, n), rng.integers(0, attr.shape[1])
        d = np.zeros_like(a0)
        d[i, c] = 1.0
        fd = (f(a0 + h * d) - f(a0 - h * d)) / (2 * h)
        assert abs(fd - g[i, c]) <= 2e-6 * gmax + 1e-9, (i, c, fd, g[i, c])
    for _ in range(3):    # random directions
        d = rng.normal(size=a0.shape)
        fd = (f(a0 + h * d) - f(a0 - h * d)) / (2 * h)
        exact = (g * d).sum()
        assert abs(fd - exact) <= 1e-5 * np.abs(g * d).sum() + 1e-9, (fd, exact)


def test_gradient_orthonormal_form():
    """T^T (T g_ahat + g_yhat) = g_ahat + T^T g_yhat, since T^T T = I."""
    pos, attr = synth.make_duplicates_frame(3000, seed=6, grid=12)
    J, lam = 5, 0.01
    b = orc.ste_grad(pos, attr, J, GROUPED, 0.5, lam)
    nv, C = b["nv"], attr.shape[1]
    g_ahat = 2.0 / (nv * C) * (b["ahat"] - b["aref"])
    g_yhat = lam * np.sign(b["yhat"]) / (np.log(2) * (GROUPED + np.abs(b["yhat"])))
    gv = g_ahat + orc.raht_inverse(b["leaf"], J, g_yhat)
    cnt = np.bincount(b["voxel_of"], minlength=nv)
    want = gv[b["voxel_of"]] / cnt[b["voxel_of"], None]
    assert np.abs(b["grad"] - want).max() <= 1e-12 * np.abs(want).max()


def test_forward_is_the_codec():
    pos, attr = synth.make_frame(5000, seed=7)
    J = 9
    b = orc.ste_grad(pos, attr, J, GROUPED, 0.5, 0.01)
    e = orc.encode_frame(pos, attr, J, GROUPED, 0.5)
    assert b["nv"] == e["nv"] and np.array_equal(b["leaf"], e["leaf"])
    assert np.array_equal(b["aref"], e["vattr"])
    assert np.array_equal(b["yhat"], orc.dequantize(e["Q"], GROUPED))
    d = orc.decode_frame(e["occ"], e["level_sizes"], J, e["Q"], GROUPED, e["bbox_min"], e["cell"])
    assert np.array_equal(b["ahat"], d["attr"])
    dist = ((b["ahat"] - b["aref"]) ** 2).mean()
    rate = 0.01 * np.log2(1 + np.abs(e["Q"])).sum()
    assert abs(b["dist"] - dist) <= 1e-12 * dist and abs(b["rate"] - rate) <= 1e-12 * rate


def test_empty_frame():
    b = orc.ste_grad(np.zeros((0, 3), np.float32), np.zeros((0, 56), np.float32), 6, GROUPED)
    assert b["nv"] == 0 and b["loss"] == 0.0 and b["grad"].shape == (0, 56)
