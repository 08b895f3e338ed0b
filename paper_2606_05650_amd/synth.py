"""Seeded synthetic Gaussian frames shaped like the dynamic-3DGS frames the codec is built for.

This module only draws inputs. It holds none of the codec's arithmetic (no voxelization, Morton
coding, octree or transform), so both the CPU oracle's tests and the GPU path can take their
inputs from it without sharing any of the method.

Frame recipe (stand-in for HiFi4G / N3DV frames, which trained Gaussians the paper evaluates on,
Sec. 5.1; a frame holds 120K-400K Gaussians there and 2-4M for static scenes):
  * 20 surfaces in the unit cube, each a sphere (probability 1/2; centre U(0.2,0.8)^3, radius
    U(0.05,0.2)) or a square planar patch (centre U(0.2,0.8)^3, random orthonormal frame,
    half-side U(0.1,0.3)).
  * Gaussians are assigned to surfaces multinomially by area, sampled uniformly on the
    surface, jittered by N(0, 0.002) per axis, clipped to [0,1]^3 and stored as float32.
  * 56 attribute channels per Gaussian (degree-3 spherical harmonics, Sec. 1.1 and Table 4):
    log-scale 3 ~ N(-4, 0.5), rotation quaternion 4 = normalized N(0,1)^4, opacity logit
    1 ~ N(0, 2), SH DC 3 ~ N(0, 0.5), SH rest 45 ~ N(0, 0.05).
"""
from __future__ import annotations

import numpy as np

# (name, channel count) in storage order; 3 + 4 + 1 + 3 + 45 = 56.
CHANNEL_GROUPS = (("scale", 3), ("rot", 4), ("opacity", 1), ("sh_dc", 3), ("sh_rest", 45))
NUM_CHANNELS = 56

# Quantization steps per channel group.
STEPS_UNIFORM_64 = {"scale": 1 / 64, "rot": 1 / 64, "opacity": 1 / 64, "sh_dc": 1 / 64,
                    "sh_rest": 1 / 64}
STEPS_GROUPED = {"scale": 1 / 32, "rot": 1 / 128, "opacity": 1 / 32, "sh_dc": 1 / 64,
                 "sh_rest": 1 / 16}

# The five workloads: name -> (Gaussians per frame, octree depth J, step table).
WORKLOADS = {
    "frame100k_J10": (100_000, 10, STEPS_UNIFORM_64),
    "frame1M_J12": (1_000_000, 12, STEPS_GROUPED),
    "seq30_J12": (None, 12, STEPS_GROUPED),
    "diff500k_J11": (500_000, 11, STEPS_GROUPED),
    "frame4M_J14": (4_000_000, 14, STEPS_GROUPED),
}


def channel_group_slices():
    """Return {group name: slice of channels}."""
    out, c0 = {}, 0
    for name, k in CHANNEL_GROUPS:
        out[name] = slice(c0, c0 + k)
        c0 += k
    return out


def quant_steps(table) -> np.ndarray:
    """Per-channel float32 quantization steps from a {group: step} table."""
    steps = np.empty(NUM_CHANNELS, dtype=np.float32)
    for name, sl in channel_group_slices().items():
        steps[sl] = table[name]
    return steps


def _draw_surfaces(rng, n_surf=20):
    surfs = []
    for _ in range(n_surf):
        if rng.random() < 0.5:
            c = rng.uniform(0.2, 0.8, 3)
            r = rng.uniform(0.05, 0.2)
            surfs.append(("sphere", c, r, None, 4.0 * np.pi * r * r))
        else:
            c = rng.uniform(0.2, 0.8, 3)
            q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            h = rng.uniform(0.1, 0.3)
            surfs.append(("patch", c, h, q[:, :2], (2.0 * h) ** 2))
    return surfs


def _sample_on_surfaces(rng, n, surfs, jitter=0.002):
    if n == 0:
        return np.zeros((0, 3), dtype=np.float32)
    areas = np.array([s[4] for s in surfs])
    counts = rng.multinomial(n, areas / areas.sum())
    parts = []
    for (kind, c, r, basis, _), k in zip(surfs, counts):
        if k == 0:
            continue
        if kind == "sphere":
            d = rng.normal(size=(k, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            p = c + r * d
        else:
            uv = rng.uniform(-r, r, size=(k, 2))
            p = c + uv @ basis.T
        parts.append(p)
    p = np.concatenate(parts, axis=0)
    p = p[rng.permutation(n)]
    p = p + rng.normal(0.0, jitter, size=p.shape)
    return np.clip(p, 0.0, 1.0).astype(np.float32)


def sample_attributes(rng, n) -> np.ndarray:
    """n x 56 float32 attributes with the distributions listed in the module docstring."""
    a = np.empty((n, NUM_CHANNELS), dtype=np.float64)
    sl = channel_group_slices()
    a[:, sl["scale"]] = rng.normal(-4.0, 0.5, size=(n, 3))
    q = rng.normal(size=(n, 4))
    nrm = np.linalg.norm(q, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    a[:, sl["rot"]] = q / nrm
    a[:, sl["opacity"]] = rng.normal(0.0, 2.0, size=(n, 1))
    a[:, sl["sh_dc"]] = rng.normal(0.0, 0.5, size=(n, 3))
    a[:, sl["sh_rest"]] = rng.normal(0.0, 0.05, size=(n, 45))
    return a.astype(np.float32)


def sample_correlated_sh(rng, n) -> np.ndarray:
    """n x 48 float32 SH coefficients whose colours and functions are correlated, as in trained
    splats (the correlation the colour decorrelation of Sec. 4 removes): per SH function f a
    shared luminance value with standard deviation s_f (0.5 for the DC; 0.08, 0.05, 0.03 for the
    AC functions of degree 1, 2, 3) plus per-colour deviations of 0.3 s_f; the AC luminances
    and the per-colour deviations are mixed across functions by fixed (seed 12345) 15 x 15
    matrices with decaying spectra (one for the luminance, one per colour), so each YUV
    channel's AC covariance has well separated eigenvalues. Columns: DC of R, G, B, then the 15
    AC functions of R, of G and of B."""
    deg = np.array([1] * 3 + [2] * 5 + [3] * 7)
    s_ac = np.array([0.08, 0.05, 0.03])[deg - 1]
    mrng = np.random.default_rng(12345)

    def mixing(hi, lo):
        q, _ = np.linalg.qr(mrng.normal(size=(15, 15)))
        return q @ np.diag(np.geomspace(hi, lo, 15)) @ q.T

    mix = mixing(2.0, 0.3)
    mix_c = [mixing(1.5, 0.2) for _ in range(3)]
    lum_dc = rng.normal(0.0, 0.5, size=(n, 1))
    lum_ac = (rng.normal(size=(n, 15)) * s_ac) @ mix.T
    sh = np.empty((n, 48))
    sh[:, 0:3] = lum_dc + rng.normal(0.0, 0.15, size=(n, 3))
    for c in range(3):
        sh[:, 3 + 15 * c:18 + 15 * c] = lum_ac + (rng.normal(size=(n, 15)) * (0.3 * s_ac)) @ mix_c[c].T
    return sh.astype(np.float32)


def make_color_frame(n: int, seed, n_surf: int = 20):
    """make_frame with correlated SH coefficients (sample_correlated_sh) in columns 8..55."""
    pos, attr = make_frame(n, seed, n_surf)
    attr[:, 8:56] = sample_correlated_sh(np.random.default_rng((seed, 1)), n)
    return pos, attr


def make_frame(n: int, seed, n_surf: int = 20):
    """One frame: (positions n x 3 float32 in [0,1]^3, attributes n x 56 float32)."""
    rng = np.random.default_rng(seed)
    surfs = _draw_surfaces(rng, n_surf)
    pos = _sample_on_surfaces(rng, n, surfs)
    attr = sample_attributes(rng, n)
    return np.ascontiguousarray(pos), np.ascontiguousarray(attr)


def make_sequence(num_frames: int = 30, n_min: int = 200_000, n_max: int = 1_500_000,
                  seed: int = 3, drift: float = 0.001, replace_frac: float = 0.05):
    """A dynamic sequence: frame t = frame t-1 + N(0, drift) per axis, replace_frac of the
    Gaussians replaced by fresh surface samples, then random drops or appends to reach a count
    drawn from U[n_min, n_max]. Frame t draws from the seed (seed, t). Yields (pos, attr)."""
    rng0 = np.random.default_rng([seed, 0])
    counts = rng0.integers(n_min, n_max + 1, size=num_frames)
    surfs = _draw_surfaces(rng0)
    pos = _sample_on_surfaces(rng0, int(counts[0]), surfs)
    attr = sample_attributes(rng0, int(counts[0]))
    yield pos, attr
    for t in range(1, num_frames):
        rng = np.random.default_rng([seed, t])
        n_prev = pos.shape[0]
        pos = pos.astype(np.float64) + rng.normal(0.0, drift, size=pos.shape)
        k = int(round(replace_frac * n_prev))
        idx = rng.choice(n_prev, size=k, replace=False)
        pos[idx] = _sample_on_surfaces(rng, k, surfs)
        attr = attr.copy()
        attr[idx] = sample_attributes(rng, k)
        pos = np.clip(pos, 0.0, 1.0).astype(np.float32)
        n_t = int(counts[t])
        if n_t < n_prev:
            keep = np.sort(rng.choice(n_prev, size=n_t, replace=False))
            pos, attr = pos[keep], attr[keep]
        elif n_t > n_prev:
            extra = n_t - n_prev
            pos = np.concatenate([pos, _sample_on_surfaces(rng, extra, surfs)], axis=0)
            attr = np.concatenate([attr, sample_attributes(rng, extra)], axis=0)
        yield np.ascontiguousarray(pos), np.ascontiguousarray(attr)


def sequence_counts(num_frames: int = 30, n_min: int = 200_000, n_max: int = 1_500_000,
                    seed: int = 3):
    """Gaussian counts of make_sequence's frames, without generating them."""
    rng0 = np.random.default_rng([seed, 0])
    return rng0.integers(n_min, n_max + 1, size=num_frames)


def make_duplicates_frame(n: int, seed, grid: int = 8):
    """A frame whose positions sit on a coarse lattice (grid^3 sites), so that many Gaussians
    share a voxel at any depth >= log2(grid): exercises the merge of duplicates."""
    rng = np.random.default_rng(seed)
    site = rng.integers(0, grid, size=(n, 3))
    pos = ((site + 0.5) / grid).astype(np.float32)
    attr = sample_attributes(rng, n)
    return np.ascontiguousarray(pos), np.ascontiguousarray(attr)
