"""Seeded synthetic anchor patches for the inpainting affinity (Sec. III-B).

Each patch pair holds P target and Q source anchors on a ground patch of side
`side` metres (8, 4 or 2 at the three levels).  An anchor row is its 32-wide
bf16 feature followed by a sinusoidal encoding of its location (x, y relative
to the patch centre, at `n_freq` octaves), zero-padded to `d` columns and
rounded to bf16: the encoded matrices X_T, X_S that the affinity consumes.
Source patches reuse the target's feature statistics with noise, as
candidate patches cut from a repetitive road would.
"""
from __future__ import annotations

import numpy as np

from gen.scenes import bf16_bits_to_f32, bf16_round_bits


def encode(feat: np.ndarray, loc: np.ndarray, side: float, n_freq: int, d: int) -> np.ndarray:
    """[n][32] features, [n][2] locations -> [n][d] bf16 bit patterns."""
    n = feat.shape[0]
    cols = [feat.astype(np.float64)]
    u = loc / side  # about [-0.5, 0.5]
    for k in range(n_freq):
        w = np.pi * (2.0 ** k)
        cols += [np.sin(w * u), np.cos(w * u)]
    x = np.concatenate(cols, axis=1)
    if x.shape[1] > d:
        raise ValueError("encoded row wider than d")
    out = np.zeros((n, d), np.float64)
    out[:, :x.shape[1]] = x
    return bf16_round_bits(out.astype(np.float32))


def patch_pairs(seed: int, batch: int, p: int, q: int, side: float = 8.0, n_freq: int = 4, d: int = 64,
                feat_scale: float = 0.35):
    """(xt_bits [B][P][d] uint16, xs_bits [B][Q][d] uint16)."""
    rng = np.random.default_rng(seed)
    xt = np.empty((batch, p, d), np.uint16)
    xs = np.empty((batch, q, d), np.uint16)
    for b in range(batch):
        base = rng.normal(0, feat_scale, 32)
        ft = base + rng.normal(0, feat_scale, (p, 32))
        fs = base + rng.normal(0, feat_scale, (q, 32))
        lt = rng.uniform(-side / 2, side / 2, (p, 2))
        ls = rng.uniform(-side / 2, side / 2, (q, 2))
        xt[b] = encode(ft, lt, side, n_freq, d)
        xs[b] = encode(fs, ls, side, n_freq, d)
    return xt, xs


def as_f32(bits: np.ndarray) -> np.ndarray:
    return bf16_bits_to_f32(bits)
