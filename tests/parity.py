"""Per-cell comparison metric of the GPU path against the oracle.

Relative error per variable and cell, |a - b| / max(|b|, s_q), with s_q = 0
for density, total and auxiliary energy (positive quantities) and
s_q = 1e-8 max|m_q| for momentum components (which change sign).
"""
import numpy as np

TOL = 1e-11


def rel_err(nv, mesh, a, b):
    off = mesh.offsets(nv)
    errs = np.zeros(nv)
    scale = np.zeros(nv)
    for v in (1, 2, 3):
        for blk in range(mesh.nblocks):
            x = b[off[blk]:off[blk + 1]].reshape(nv, -1)[v]
            scale[v] = max(scale[v], np.abs(x).max())
    scale = 1e-8 * scale
    for blk in range(mesh.nblocks):
        A = a[off[blk]:off[blk + 1]].reshape(nv, -1)
        B = b[off[blk]:off[blk + 1]].reshape(nv, -1)
        for v in range(nv):
            den = np.maximum(np.abs(B[v]), scale[v]) if v in (1, 2, 3) else np.abs(B[v])
            with np.errstate(divide="ignore", invalid="ignore"):
                r = np.where(den > 0, np.abs(A[v] - B[v]) / den, np.abs(A[v] - B[v]))
            errs[v] = max(errs[v], float(np.max(r)))
    return errs
