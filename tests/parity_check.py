"""Element-by-element comparison of GPU outputs with the oracle's (imported by the GPU tests).

Every map is held to two bounds: the relative L2 error of each map (the per-output tolerance of
the parity table) and the largest error of any single element, measured against the map's natural
scale (sqrt(xi(0)) for a Gaussian field, 1 + |delta| for the lognormal contrast), so that a few
wrong cells cannot hide inside a norm over a million of them.
"""

import numpy as np


def _stack(a, nmaps):
    return np.asarray(a, dtype=np.float64).reshape(nmaps, -1)


def check_maps(got, ref, tol, scale, what="field"):
    """Stacks of maps (count, ...): assert, for every map k, ||got_k - ref_k|| <= tol ||ref_k||
    and max_i |got_ki - ref_ki| <= tol * scale.  Returns (worst relative L2, worst max |d| / scale)."""
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[0]
    g, r = _stack(got, n), _stack(ref, n)
    d = g - r
    l2 = np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)
    mx = np.max(np.abs(d), axis=1) / scale
    print("%s: rel L2 %.3e, max |d| / scale %.3e (tol %.0e)" % (what, l2.max(), mx.max(), tol), flush=True)
    assert l2.max() <= tol, (what, l2)
    assert mx.max() <= tol, (what, mx, int(np.argmax(np.abs(d)) % g.shape[1]))
    return float(l2.max()), float(mx.max())


def check_delta(got, ref, tol, what="delta"):
    """Stacks of lognormal contrasts (count, ...): relative L2 per map <= tol and
    |got - ref| <= tol (1 + |ref|) per cell."""
    ref = np.asarray(ref, dtype=np.float64)
    n = ref.shape[0]
    g, r = _stack(got, n), _stack(ref, n)
    d = g - r
    l2 = np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)
    mx = np.max(np.abs(d) / (1.0 + np.abs(r)), axis=1)
    print("%s: rel L2 %.3e, max |d| / (1 + |ref|) %.3e (tol %.0e)" % (what, l2.max(), mx.max(), tol), flush=True)
    assert l2.max() <= tol, (what, l2)
    assert mx.max() <= tol, (what, mx)
    return float(l2.max()), float(mx.max())
