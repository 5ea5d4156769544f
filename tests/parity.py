"""Error statistics of a GPU grid against the FP64 oracle's grid (helper of
the GPU parity tests; not a test module).

The bar (FP32 grids): max |gpu - oracle| <= 1e-5 * max(oracle).  Beside it
the tests report the RMS error over the support (voxels where either side is
nonzero) relative to the peak, and the support mismatch: voxels where exactly
one side is nonzero.  A mismatch can only come from a (voxel, point) pair
whose FP32 support test disagrees with FP64 -- 1 - u^2 - v^2 or 1 - w^2 within
about 1e-6 of zero, where the Epanechnikov pair is about 1e-6 of its peak --
so the value on the nonzero side must be tiny.
"""
import numpy as np

TOL = 1e-5
MISMATCH_VALUE = 1e-6  # largest value (relative to the peak) a mismatched voxel may hold


def error_stats(gpu, ref):
    """dict(max_rel, rms_rel, peak, mismatch, mismatch_max_rel) of FP32 `gpu`
    against FP64 `ref` (same shape)."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    if g.shape != r.shape:
        raise ValueError(f"shapes differ: {g.shape} vs {r.shape}")
    peak = float(np.max(np.abs(r))) if r.size else 0.0
    scale = max(peak, 1e-300)
    d = np.abs(g - r)
    supp = (g != 0.0) | (r != 0.0)
    nsupp = int(np.count_nonzero(supp))
    mism = (g != 0.0) != (r != 0.0)
    nm = int(np.count_nonzero(mism))
    return {
        "max_rel": float(np.max(d)) / scale if d.size else 0.0,
        "rms_rel": float(np.sqrt(np.mean(d[supp] ** 2))) / scale if nsupp else 0.0,
        "peak": peak,
        "support": nsupp,
        "mismatch": nm,
        "mismatch_max_rel": float(np.max(np.abs(g[mism]) + np.abs(r[mism]))) / scale if nm else 0.0,
    }


def assert_parity(gpu, ref, tol=TOL, what=""):
    """Assert the bar and the mismatch bound; return the statistics."""
    st = error_stats(gpu, ref)
    assert st["max_rel"] <= tol, f"{what}: max rel err {st['max_rel']:.3e} > {tol:g}"
    assert st["mismatch_max_rel"] <= MISMATCH_VALUE, \
        f"{what}: {st['mismatch']} support mismatches up to {st['mismatch_max_rel']:.3e} of the peak"
    return st
