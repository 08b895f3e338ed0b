"""Pins of the colour-decorrelation oracle (Sec. 4: YUV on every SH function, then one KLT per
YUV channel over the AC SH coefficients), against what the definitions fix: the BT.601 extremes,
an exactly constructed covariance with a known eigenbasis, orthonormality, energy, the degenerate
frame and the round trip."""
import numpy as np

from oracle import color_oracle as co

SH0 = 8


def test_yuv_definition_extremes():
    M = co.yuv_matrix()
    # white has luma 1 and no chroma; a pure primary's luma is its weight
    assert np.allclose(M @ [1.0, 1.0, 1.0], [1.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(M[0], [0.299, 0.587, 0.114], atol=1e-15)
    # the chroma ranges: U of pure blue is Umax, V of pure red is Vmax
    assert abs((M @ [0.0, 0.0, 1.0])[1] - 0.436) < 1e-15
    assert abs((M @ [1.0, 0.0, 0.0])[2] - 0.615) < 1e-15
    # the closed-form inverse undoes it
    rng = np.random.default_rng(0)
    rgb = rng.normal(size=(100, 3))
    assert np.allclose(co.yuv_to_rgb(rgb @ M.T), rgb, atol=1e-13)
    assert np.allclose(co.yuv_to_rgb(np.eye(3)) @ M.T, np.eye(3), atol=1e-13)


def _basis(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(15, 15)))
    return q * np.sign(np.diag(r))


def test_klt_recovers_a_constructed_eigenbasis():
    """Rows +-sqrt(15 s_k) q_k (k = 0..14) have mean 0 and covariance sum_k s_k q_k q_k^T
    exactly, so the KLT basis must be Q itself (columns in decreasing s, canonical signs)."""
    Q = _basis(1)
    s = np.linspace(2.0, 0.1, 15)
    rows = np.concatenate([np.sqrt(15 * s)[:, None] * Q.T, -np.sqrt(15 * s)[:, None] * Q.T])
    E, vals, m, S = co.klt_basis(rows)
    assert np.allclose(m, 0, atol=1e-14)
    assert np.allclose(S, Q @ np.diag(s) @ Q.T, atol=1e-13)
    assert np.allclose(vals, s, atol=1e-12)
    Qc = Q * np.where(Q[np.argmax(np.abs(Q), axis=0), np.arange(15)] < 0, -1.0, 1.0)
    assert np.allclose(E, Qc, atol=1e-10)
    # canonical: the largest-magnitude component of every column is positive
    assert np.all(E[np.argmax(np.abs(E), axis=0), np.arange(15)] > 0)


def _frame(n, seed):
    """56-channel rows whose SH coefficients are correlated across colours and functions."""
    rng = np.random.default_rng(seed)
    attr = rng.normal(size=(n, 56))
    mix = rng.normal(size=(48, 48)) * 0.2 + np.eye(48)
    attr[:, SH0:SH0 + 48] = attr[:, SH0:SH0 + 48] @ mix
    return attr


def test_forward_decorrelates_orders_and_keeps_energy():
    attr = _frame(5000, 2)
    r = co.color_forward(attr, SH0)
    out = r["out"]
    # untouched columns
    assert np.array_equal(out[:, :SH0], attr[:, :SH0])
    M = co.yuv_matrix()
    # DC: YUV only
    assert np.allclose(out[:, SH0:SH0 + 3], attr[:, SH0:SH0 + 3] @ M.T, atol=1e-12)
    for c in range(3):
        E = r["E"][c]
        assert np.allclose(E.T @ E, np.eye(15), atol=1e-12)
        a = out[:, SH0 + 3 + 15 * c:SH0 + 18 + 15 * c]
        # the coefficients are uncorrelated, with variances equal to the decreasing eigenvalues
        d = a - a.mean(axis=0)
        C = d.T @ d / a.shape[0]
        assert np.allclose(C, np.diag(r["eig"][c]), atol=1e-12 * r["eig"][c][0])
        assert np.all(np.diff(r["eig"][c]) <= 0)
        # an orthonormal change of basis keeps each row's energy in the channel
        x = np.einsum("k,nkf->nf", M[c], attr[:, SH0 + 3:SH0 + 48].reshape(-1, 3, 15))
        assert np.allclose((a ** 2).sum(axis=1), (x ** 2).sum(axis=1), rtol=1e-12)


def test_round_trip_and_single_row():
    attr = _frame(777, 3)
    r = co.color_forward(attr, SH0)
    assert np.allclose(co.color_inverse(r["out"], r["E"], SH0), attr, atol=1e-12)
    one = co.color_forward(attr[:1], SH0)
    assert np.array_equal(one["E"], np.stack([np.eye(15)] * 3))
    assert np.allclose(co.color_inverse(one["out"], one["E"], SH0), attr[:1], atol=1e-13)
    empty = co.color_forward(attr[:0], SH0)
    assert empty["out"].shape == (0, 56)


def test_a_planted_mistake_is_caught():
    """A transposed basis (E instead of E^T applied) breaks decorrelation: the pin above would
    fail for it."""
    attr = _frame(3000, 4)
    r = co.color_forward(attr, SH0)
    M = co.yuv_matrix()
    x = np.einsum("k,nkf->nf", M[0], attr[:, SH0 + 3:SH0 + 48].reshape(-1, 3, 15))
    wrong = x @ r["E"][0].T
    d = wrong - wrong.mean(axis=0)
    C = d.T @ d / len(wrong)
    assert not np.allclose(C, np.diag(np.diag(C)), atol=1e-6 * r["eig"][0][0])
