"""Comparison helpers of the GPU parity tests (evaluation chapter,
"Functional correctness": results against a reference, here the FP64
oracle, beside the bitwise comparisons between schedules).

A field is compared through its relative L2 error (the stated tolerance) and
element by element (no point off by more than the tolerance times the
field's largest magnitude), so that an error confined to a face, a plane or
a few points cannot hide in the norm of the whole field.  Receiver traces are
compared as a set and one by one: every trace carrying at least `floor` of
the largest trace's energy must meet ten times the tolerance on its own
(FP32 rounding grows relative to a weak trace's norm).
"""
import numpy as np


def rel(a, b):
    a = np.ravel(a).astype(np.float64)
    b = np.ravel(b).astype(np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def assert_field(got, ref, tol, what=""):
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    e = rel(g, r)
    assert e <= tol, "%s relative L2 %.3e > %.1e" % (what, e, tol)
    m = np.abs(g - r).max()
    assert m <= tol * np.abs(r).max(), "%s max |error| %.3e > %.1e x max |ref| %.3e" % (what, m, tol, np.abs(r).max())


def assert_traces(got, ref, tol, floor=1e-2, what="traces"):
    """got, ref: [nt][nrec]."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    e = rel(g, r)
    assert e <= tol, "%s relative L2 %.3e > %.1e" % (what, e, tol)
    norms = np.linalg.norm(r, axis=0)
    strong = norms >= floor * norms.max()
    per = np.linalg.norm(g - r, axis=0)[strong] / norms[strong]
    assert per.max() <= 10 * tol, "%s: worst trace relative L2 %.3e > %.1e" % (what, per.max(), 10 * tol)
