"""Shared assertion for UOT mask parity: every bit must match; a failure
names each differing position with its distance |U - p*| / p* to the keep
boundary, which separates a rounding-level disagreement (U within ~1e-15 of
p*) from a wrong decision."""
import numpy as np

from oracle import sparsink_oracle as O


def assert_mask_equal(g_mask, o_mask, p, prob, rows=None):
    """g_mask, o_mask: uint64 words (rows x words); `rows` names the rows of
    the problem they hold (all rows when None)."""
    diff = g_mask ^ o_mask
    if not diff.any():
        return
    bits = np.unpackbits(diff.view(np.uint8), axis=1, bitorder="little")[:, : p.m]
    rr, cc = np.nonzero(bits)
    if rows is not None:
        rr = np.asarray(rows)[rr]
    u = O.uniform01(rr, cc, p.problem_index, p.seed)
    pst = np.array([prob.pstar(np.array([r]), np.array([c]))[0, 0] for r, c in zip(rr, cc)])
    where = [(int(r), int(c), float(abs(uu - pp) / pp)) for r, c, uu, pp in zip(rr, cc, u, pst)]
    raise AssertionError(f"{len(rr)} differing mask bits (row, col, |U - p*|/p*): {where[:16]}")
