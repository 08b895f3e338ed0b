"""Plain FP64 CPU oracle of the colour decorrelation applied before RAHT (Sec. 4, "Improving
Compression"): every SH function's RGB triple goes to YUV, then each of the Y, U and V channels
gets its own per-frame Karhunen-Loeve transform (KLT) over its AC SH coefficients (degree > 0);
the DC coefficients get the YUV step only.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the benchmark's CPU-baseline
leg are the only callers. It shares no code with the HIP path and imports nothing from the
product package.

The paper names the two steps and where they apply, and gives no coefficients. The readings
taken here (also listed with the design notes):
  Y1  YUV: the BT.601 definition with luma weights Kr = 0.299, Kb = 0.114 (Kg = 1 - Kr - Kb) and
      chroma ranges Umax = 0.436, Vmax = 0.615:
          Y = Kr R + Kg G + Kb B,  U = Umax (B - Y) / (1 - Kb),  V = Vmax (R - Y) / (1 - Kr);
      its inverse B = Y + U (1 - Kb) / Umax, R = Y + V (1 - Kr) / Vmax, G = (Y - Kr R - Kb B) / Kg.
  Y2  Attribute layout: the 48 SH channels start at column sh0 (8 for the 56-channel frames:
      log-scale 3, rotation 4, opacity 1 before them): columns sh0 .. sh0 + 2 hold the DC of R,
      G, B, and column sh0 + 3 + 15 c + k holds AC function k (k = 0..14) of colour c (the
      storage order of degree-3 Gaussian splats: all of R's AC coefficients, then G's, then B's).
      After the transform column sh0 + c holds the DC of YUV channel c and column
      sh0 + 3 + 15 c + j the j-th KLT coefficient of channel c; other columns are unchanged.
  Y3  KLT of channel c: over the frame's n input rows (the transform is linear per row, so it
      commutes with the mean over a voxel's Gaussians), the mean m and the covariance
      S = (1/n) sum_r (x_r - m)(x_r - m)^T of the channel's 15 AC coefficients x_r. Its
      eigenvectors, in order of decreasing eigenvalue, each with its largest-magnitude component
      positive (the first one on a tie), are the columns of E_c. Coefficients a = E_c^T x (no
      centring: the mean goes through the transform like any other content); inverse x = E_c a.
  Y4  n < 2: S is zero and E_c is the identity.
"""
from __future__ import annotations

import numpy as np

KR, KB = 0.299, 0.114
UMAX, VMAX = 0.436, 0.615
N_AC = 15          # AC SH functions per colour (degree 1..3)
N_SH = 3 + 3 * N_AC  # 48 SH channels: 3 DC + 45 AC


def yuv_matrix() -> np.ndarray:
    """Y1: the 3x3 matrix M with (Y, U, V) = M (R, G, B), written out from its definition."""
    kg = 1.0 - KR - KB
    y = np.array([KR, kg, KB])
    u = UMAX / (1.0 - KB) * (np.array([0.0, 0.0, 1.0]) - y)
    v = VMAX / (1.0 - KR) * (np.array([1.0, 0.0, 0.0]) - y)
    return np.stack([y, u, v])


def yuv_to_rgb(yuv: np.ndarray) -> np.ndarray:
    """Y1 inverse, by its closed form (not a matrix inverse): yuv [..., 3] -> rgb [..., 3]."""
    Y, U, V = yuv[..., 0], yuv[..., 1], yuv[..., 2]
    B = Y + U * (1.0 - KB) / UMAX
    R = Y + V * (1.0 - KR) / VMAX
    G = (Y - KR * R - KB * B) / (1.0 - KR - KB)
    return np.stack([R, G, B], axis=-1)


def _split(attr: np.ndarray, sh0: int):
    """Y2: (DC [n, 3 colours], AC [n, 3 colours, 15 functions]) of the attribute rows."""
    sh = attr[:, sh0:sh0 + N_SH].astype(np.float64)
    return sh[:, :3], sh[:, 3:].reshape(-1, 3, N_AC)


def _canonical(vals: np.ndarray, vecs: np.ndarray):
    """Y3: eigenpairs in decreasing eigenvalue order, each vector's largest-magnitude component
    positive (the first on a tie)."""
    order = np.argsort(-vals, kind="stable")
    vals, vecs = vals[order], vecs[:, order].copy()
    for j in range(vecs.shape[1]):
        i = int(np.argmax(np.abs(vecs[:, j])))
        if vecs[i, j] < 0:
            vecs[:, j] = -vecs[:, j]
    return vals, vecs


def klt_basis(x: np.ndarray):
    """Y3/Y4: (E [15, 15] with the basis vectors as columns, eigenvalues [15], mean [15],
    covariance [15, 15]) of the rows x [n, 15]."""
    n = x.shape[0]
    if n < 2:
        return np.eye(N_AC), np.zeros(N_AC), (x.mean(axis=0) if n else np.zeros(N_AC)), np.zeros((N_AC, N_AC))
    m = x.mean(axis=0)
    d = x - m
    S = d.T @ d / n
    vals, vecs = np.linalg.eigh(S)
    vals, vecs = _canonical(vals, vecs)
    return vecs, vals, m, S


def color_forward(attr: np.ndarray, sh0: int = 8):
    """Sec. 4: YUV on every SH function, then each channel's KLT on its AC coefficients.
    Returns dict(out [n, C] FP64, E [3, 15, 15], eig [3, 15], mean [3, 15], cov [3, 15, 15])."""
    attr = np.asarray(attr)
    M = yuv_matrix()
    dc, ac = _split(attr, sh0)
    dc_yuv = dc @ M.T                                 # [n, 3]
    ac_yuv = np.einsum("ck,nkf->ncf", M, ac)          # [n, 3 channels, 15]
    out = attr.astype(np.float64).copy()
    out[:, sh0:sh0 + 3] = dc_yuv
    E = np.zeros((3, N_AC, N_AC))
    eig = np.zeros((3, N_AC))
    mean = np.zeros((3, N_AC))
    cov = np.zeros((3, N_AC, N_AC))
    for c in range(3):
        E[c], eig[c], mean[c], cov[c] = klt_basis(ac_yuv[:, c, :])
        out[:, sh0 + 3 + N_AC * c:sh0 + 3 + N_AC * (c + 1)] = ac_yuv[:, c, :] @ E[c]
    return dict(out=out, E=E, eig=eig, mean=mean, cov=cov)


def color_inverse(coef: np.ndarray, E: np.ndarray, sh0: int = 8) -> np.ndarray:
    """The decoder's side: each channel's KLT undone (x = E a), then YUV back to RGB."""
    coef = np.asarray(coef, dtype=np.float64)
    out = coef.copy()
    ac_yuv = np.stack([coef[:, sh0 + 3 + N_AC * c:sh0 + 3 + N_AC * (c + 1)] @ np.asarray(E[c]).T
                       for c in range(3)], axis=1)   # [n, 3, 15]
    out[:, sh0:sh0 + 3] = yuv_to_rgb(coef[:, sh0:sh0 + 3])
    rgb = yuv_to_rgb(np.transpose(ac_yuv, (0, 2, 1)))  # [n, 15, 3]
    for c in range(3):
        out[:, sh0 + 3 + N_AC * c:sh0 + 3 + N_AC * (c + 1)] = rgb[:, :, c]
    return out
