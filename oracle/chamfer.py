"""Chamfer distance transform T(X) of a binary lattice image (Section 5).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it, and it
imports nothing from the product.

Section 5 weights the pixels of a binary shape by a distance transform so that
interior pixels count more, P = T(X) * G_xi, and names Borgefors' chamfer
transforms for T. This is Borgefors' two-pass propagation with a 3x3 mask:
orthogonal steps cost `a`, diagonal steps cost `b` (3 and 4 for the usual
3-4 chamfer; T/a approximates the Euclidean distance in pixels).

Readings (listed with the design notes):
* T is the distance from each foreground pixel (X != 0) to the nearest
  background pixel; background pixels get 0;
* everything outside the H x W lattice is background, so a shape that
  touches the image border is measured to the border;
* the result is in chamfer units (integers); weight images use T / a.
"""
from __future__ import annotations

import numpy as np

__all__ = ["chamfer_transform"]


def chamfer_transform(X: np.ndarray, a: int = 3, b: int = 4) -> np.ndarray:
    """Borgefors' sequential two-pass chamfer transform (int64, chamfer units).

    The image is padded with one ring of background pixels (the outside of
    the lattice). The forward raster pass (rows top to bottom, columns left
    to right) relaxes every foreground pixel against its four already-visited
    neighbours (upper-left, up, upper-right, left); the backward pass (rows
    bottom to top, columns right to left) against the mirrored four.
    """
    X = np.asarray(X)
    H, W = X.shape
    big = (a + b) * (H + W + 2)  # larger than any distance on the lattice
    d = np.zeros((H + 2, W + 2), dtype=np.int64)
    d[1:-1, 1:-1] = np.where(X != 0, big, 0)
    for i in range(1, H + 1):
        for j in range(1, W + 1):
            if d[i, j]:
                d[i, j] = min(d[i, j], d[i - 1, j - 1] + b, d[i - 1, j] + a, d[i - 1, j + 1] + b,
                              d[i, j - 1] + a)
    for i in range(H, 0, -1):
        for j in range(W, 0, -1):
            if d[i, j]:
                d[i, j] = min(d[i, j], d[i + 1, j + 1] + b, d[i + 1, j] + a, d[i + 1, j - 1] + b,
                              d[i, j + 1] + a)
    return d[1:-1, 1:-1].copy()
