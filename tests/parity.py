"""Per-cell comparison metric of the GPU path against the oracle.

Relative error per variable and cell, |a - b| / s, with
  s = |b|                         for density, total and auxiliary energy
                                  (positive quantities);
  s = max(|b|, sqrt(rho_b E_b))   for each momentum component.
A momentum component changes sign, so its own magnitude is no scale near a
zero crossing; sqrt(rho E) is the cell's momentum scale (it bounds rho|v|/sqrt(2)
from above and is of order rho c_s in a gas at rest), and round-off in a
momentum flux is a fraction of exactly that.
"""
import numpy as np

TOL = 1e-11


def rel_err(nv, mesh, a, b):
    if not (np.all(np.isfinite(a)) and np.all(np.isfinite(b))):
        return np.full(nv, np.inf)  # a non-finite state never passes
    off = mesh.offsets(nv)
    errs = np.zeros(nv)
    for blk in range(mesh.nblocks):
        A = a[off[blk]:off[blk + 1]].reshape(nv, -1)
        B = b[off[blk]:off[blk + 1]].reshape(nv, -1)
        mscale = np.sqrt(np.abs(B[0])) * np.sqrt(np.abs(B[4]))
        for v in range(nv):
            den = np.maximum(np.abs(B[v]), mscale) if v in (1, 2, 3) else np.abs(B[v])
            with np.errstate(divide="ignore", invalid="ignore"):
                r = np.where(den > 0, np.abs(A[v] - B[v]) / den, np.abs(A[v] - B[v]))
            errs[v] = max(errs[v], float(np.max(r)))
    return errs
