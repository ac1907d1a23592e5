"""Line objects of an embedded boundary (Sec. 4.3), test infrastructure.

The x- and y-convolutions act on line objects: the inside nodes of one grid
line between two crossings of the boundary curve, closed by the two boundary
points at the crossings.  Reading of the paper: every maximal run of inside
nodes is one line object (the paper's ellipse is convex and never needs more
than one per line; a star-shaped domain can).

Inputs: ``mask`` (n_y, n_x) uint8, 1 = inside; ``cross`` (4, n_y, n_x)
float64 or None: at an inside node next to an outside node, the distance to
the crossing in units of h toward -x, +x, -y, +y (0 < theta <= 1).  None puts
the boundary point on the first outside node (theta = 1).
"""
from __future__ import annotations

import numpy as np


def extract(mask, cross=None, axis=0):
    """Returns (seg_idx[n,3] int64 = (line, first, last inside node),
    seg_th[n,2] float64 = (theta_lo, theta_hi)) for grid axis 0 (x) or 1 (y)."""
    m = np.asarray(mask).astype(bool)
    ny, nx = m.shape
    if m[0, :].any() or m[-1, :].any() or m[:, 0].any() or m[:, -1].any():
        raise ValueError("the outer ring of the grid must lie outside the domain")
    idx, th = [], []
    lines = m if axis == 0 else m.T
    for line in range(lines.shape[0]):
        row = lines[line]
        i = 0
        n = len(row)
        while i < n:
            if not row[i]:
                i += 1
                continue
            j = i
            while j + 1 < n and row[j + 1]:
                j += 1
            if cross is None:
                tl = tr = 1.0
            elif axis == 0:
                tl, tr = cross[0, line, i], cross[1, line, j]
            else:
                tl, tr = cross[2, i, line], cross[3, j, line]
            if not (0.0 < tl <= 1.0 and 0.0 < tr <= 1.0):
                raise ValueError("crossing offsets must lie in (0, 1]")
            idx.append((line, i, j))
            th.append((float(tl), float(tr)))
            i = j + 1
    return (np.array(idx, dtype=np.int64).reshape(-1, 3),
            np.array(th, dtype=np.float64).reshape(-1, 2))


def segments(mask, cross=None):
    """Both axes: [(x line objects), (y line objects)]."""
    return [extract(mask, cross, 0), extract(mask, cross, 1)]
