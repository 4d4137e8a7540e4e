"""Sampled-cell parity at sizes the oracle cannot run whole.

A substage right-hand side at a cell depends only on the cells at most three
away along each axis (the parabola of a face's far cell reaches two cells
beyond it; the edge fields of the face-field update take faces of the next
rows, whose cell-centre fields reach one row further), and on dt and the
cell size h only through dt / h.  So the oracle's right-hand side on a
periodic window of 13^3 cells cut around a cell, with dt scaled by the ratio
of the cell sizes (h = 1 / nx on both sides), is the whole box's right-hand
side at the window's central 5^3 cells, one cell of margin to spare (the
cells nearer the window's faces see the wrapped window instead).
"""
import numpy as np

import oracle

HALF = 6      # window cells on each side of its centre cell
CORE = 2      # compared cells on each side of the centre


def cut(U, centre):
    """The periodic window of U (fields, nz, ny, nx) around centre (z, y, x)."""
    n = U.shape[1:]
    idx = [(c + np.arange(-HALF, HALF + 1)) % m for c, m in zip(centre, n)]
    return np.ascontiguousarray(U[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]])


def core_of_box(A, centre):
    """The central cells of the window around centre, taken from a whole-box array."""
    n = A.shape[1:]
    idx = [(c + np.arange(-CORE, CORE + 1)) % m for c, m in zip(centre, n)]
    return A[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]


def core_of_window(Aw):
    s = slice(HALF - CORE, HALF + CORE + 1)
    return Aw[:, s, s, s]


def window_rhs(stage_rhs, U, centre, dt, **params):
    """stage_rhs (oracle.nonadv_rhs or oracle.adv_rhs) at the central cells
    of the window around centre, for a box U of cell size 1 / nx."""
    m = 2 * HALF + 1
    Pw = oracle.make_params((m, m, m), **params)
    dtw = dt * U.shape[3] / m
    return core_of_window(stage_rhs(Pw, cut(U, centre), dtw))
