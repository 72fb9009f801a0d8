"""Per-cell comparison metric of the GPU path against the oracle.

Relative error per variable and cell, |a - b| / s, with the scale s of each
variable the magnitude its rounding error is a fraction of:
  density:            s = |rho|
  total energy:       s = E_hat = max(|E|, K + |U|), K the kinetic energy density
                      and U the internal energy (U_aux with dual energy, else
                      E - K).  Where gravity work has driven E far below its
                      kinetic and thermal parts, E is a small difference of
                      large terms and its error is a fraction of E_hat.
  momentum component: s = max(|m_q|, sqrt(rho E_hat)) (a component changes
                      sign; sqrt(rho E_hat) is the cell's momentum scale).
  U_aux:              s = |U_aux|, except in cells where resynchronisation can
                      copy E - K into it (U_aux >= eta2 |E|): there
                      s = max(|U_aux|, 1e-2 E_hat), since U_aux then carries the
                      rounding of E - K.  Cold cells (U_aux << eta2 E, where the
                      dual energy matters) are measured strictly against U_aux.
Non-finite values fail.
"""
import numpy as np

TOL = 1e-11
ETA2 = 1e-4


def rel_err(nv, mesh, a, b, with_counts=False):
    if not (np.all(np.isfinite(a)) and np.all(np.isfinite(b))):
        return np.full(nv, np.inf)  # a non-finite state never passes
    off = mesh.offsets(nv)
    errs = np.zeros(nv)
    ill = 0
    for blk in range(mesh.nblocks):
        A = a[off[blk]:off[blk + 1]].reshape(nv, -1)
        B = b[off[blk]:off[blk + 1]].reshape(nv, -1)
        K = 0.5 * (B[1] ** 2 + B[2] ** 2 + B[3] ** 2) / B[0]
        U = B[5] if nv > 5 else B[4] - K
        Ehat = np.maximum(np.abs(B[4]), K + np.abs(U))
        ill += int(np.sum(Ehat > 100.0 * np.abs(B[4])))
        mscale = np.sqrt(np.abs(B[0])) * np.sqrt(Ehat)
        for v in range(nv):
            if v in (1, 2, 3):
                den = np.maximum(np.abs(B[v]), mscale)
            elif v == 4:
                den = Ehat
            elif v == 5:
                den = np.where(np.abs(B[5]) >= ETA2 * np.abs(B[4]), np.maximum(np.abs(B[5]), 1e-2 * Ehat),
                               np.abs(B[5]))
            else:
                den = np.abs(B[v])
            with np.errstate(divide="ignore", invalid="ignore"):
                r = np.where(den > 0, np.abs(A[v] - B[v]) / den, np.abs(A[v] - B[v]))
            errs[v] = max(errs[v], float(np.max(r)))
    if with_counts:
        return errs, ill
    return errs
