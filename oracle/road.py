"""CPU oracle of the road profile in v-disparity space and of the u-disparity image —
TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this module;
the product library never does. Plain numpy, integer throughout.

Section 3.5 of the paper:
* eq. disp_map: H_x{U}(i, j) = the number of pixels of image row j whose disparity is i
  (the v-disparity image). Invalid disparities (-1) and values outside [0, D) are not
  counted.
* eq. hy: H_y{U}(i, j) = the number of pixels of image column j whose disparity is i (the
  u-disparity image); its second Kronecker delta is printed on the column index again and is
  read as the disparity's, the column-wise counterpart of eq. disp_map.
* eqs. P_hat and e: every (i, j) of H_x is a Viterbi node; a road profile is a path
  j = P(i) over all disparities i = 0 .. D-1 with e(0, j) = H_x(0, j) and
  e(i, j) = H_x(i, j) + max over 0 < j - j' < eta of e(i-1, j'), so the row grows by 1 to
  eta-1 per disparity step (nearer road lies lower in the image). The profile ends at the
  row maximising e(D-1, .) and is traced back through the maximising predecessors.

Readings: nodes without a predecessor (j - j' >= 1 needs j' >= 0) are unreachable for
i > 0; ties take the smallest row, both at the end and for each predecessor; when no row
is reachable at i = D-1 the profile is all -1 and the energy -1.
"""
from __future__ import annotations

import numpy as np

NEG = -1  # unreachable (every reachable energy is >= 0)


def vdisparity(disp: np.ndarray, num_disp: int) -> np.ndarray:
    """hist[i][j] (uint32 [D][H]): pixels of row j with disparity i (eq. disp_map)."""
    disp = np.asarray(disp)
    h = disp.shape[0]
    hist = np.zeros((num_disp, h), np.uint32)
    for j in range(h):
        row = disp[j]
        ok = (row >= 0) & (row < num_disp)
        hist[:, j] = np.bincount(row[ok].astype(np.int64), minlength=num_disp)[:num_disp]
    return hist


def road(hist: np.ndarray, eta: int):
    """Road profile (eqs. P_hat, e): returns (path int16 [D] of rows, energy int).
    The recurrence over the predecessor window is written out node by node."""
    hist = np.asarray(hist, np.int64)
    D, H = hist.shape
    e = np.full((D, H), NEG, np.int64)
    back = np.full((D, H), -1, np.int64)
    e[0] = hist[0]
    for i in range(1, D):
        for j in range(H):
            best, arg = NEG, -1
            for jp in range(max(0, j - eta + 1), j):  # 0 < j - jp < eta
                if e[i - 1, jp] > best:               # strict: the smallest row wins ties
                    best, arg = e[i - 1, jp], jp
            if arg >= 0:
                e[i, j] = hist[i, j] + best
                back[i, j] = arg
    end = int(np.argmax(e[D - 1]))  # first maximum: the smallest row
    if e[D - 1, end] == NEG:
        return np.full(D, -1, np.int16), NEG
    path = np.empty(D, np.int16)
    path[D - 1] = end
    for i in range(D - 1, 0, -1):
        path[i - 1] = back[i, path[i]]
    return path, int(e[D - 1, end])


def udisparity(disp: np.ndarray, num_disp: int) -> np.ndarray:
    """hist[i][j] (uint32 [D][W]): pixels of column j with disparity i (eq. hy, read with
    its second Kronecker delta on the disparity, the column-wise counterpart of eq.
    disp_map). Invalid (-1) and out-of-range disparities are not counted."""
    disp = np.asarray(disp)
    w = disp.shape[1]
    hist = np.zeros((num_disp, w), np.uint32)
    for j in range(w):
        col = disp[:, j]
        ok = (col >= 0) & (col < num_disp)
        hist[:, j] = np.bincount(col[ok].astype(np.int64), minlength=num_disp)[:num_disp]
    return hist
