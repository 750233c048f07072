"""Inpainting patch affinity in FP64 -- TEST INFRASTRUCTURE ONLY.

Sec. III-B, Eq. 6: the affinity between a target patch T and a candidate
source patch S is the softmax of the product of their anchor matrices, each
anchor row being the anchor's feature vector concatenated with a positional
encoding of its location: A = softmax(X_T X_S^T), X = F (+) PE(L).

Readings (the paper leaves these open):
  * the softmax runs along each row, i.e. over the source anchors, so that row
    i is a distribution of target anchor i over the source patch's anchors;
  * no temperature or 1/sqrt(D) scale (none is written);
  * the encoded rows X are the operation's inputs, given in bfloat16 (the
    features are bf16 parameters; the encoding is rounded to bf16 by whoever
    builds X), so both sides start from the same exact values;
  * the nearest-neighbour distance-field term and the patch search around the
    score are not part of this operation.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may use this.
"""
from __future__ import annotations

import numpy as np


def logits(xt: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """X_T X_S^T for one patch pair: xt [P][D], xs [Q][D] -> [P][Q] (FP64)."""
    return np.asarray(xt, np.float64) @ np.asarray(xs, np.float64).T


def row_softmax(z: np.ndarray) -> np.ndarray:
    """softmax along the last axis, with the row maximum subtracted first."""
    z = np.asarray(z, np.float64)
    if z.shape[-1] == 0:
        return z.copy()
    e = np.exp(z - z.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def affinity(xt: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """Eq. 6 for a batch of patch pairs: xt [B][P][D], xs [B][Q][D] -> A [B][P][Q]."""
    xt = np.asarray(xt, np.float64)
    xs = np.asarray(xs, np.float64)
    out = np.empty((xt.shape[0], xt.shape[1], xs.shape[1]), np.float64)
    for b in range(xt.shape[0]):
        out[b] = row_softmax(logits(xt[b], xs[b]))
    return out
