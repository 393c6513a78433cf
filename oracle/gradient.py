"""Gradients of a loss of the transform, written out from their definitions.

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

For g = A c with A(j,k) = J_nu(w_j r_k) (Sec. 1, eq. DHT) and gbar = dL/dg:

  dL/dc_k = sum_j gbar_j J_nu(w_j r_k)                 (the transposed sum)
  dL/dr_k = c_k sum_j gbar_j w_j J_nu'(w_j r_k)        (chain rule in r_k)
  dL/dw_j = gbar_j sum_k c_k r_k J_nu'(w_j r_k)        (chain rule in w_j)

with the derivative from the recurrence J_nu' = (J_{nu-1} - J_{nu+1}) / 2
(DLMF 10.6.1; J_{-n} = (-1)^n J_n).  Every sum is the O1 direct sum of
``direct.dht`` (exact arguments, compensated summation) at order nu or nu -+ 1.
"""
import numpy as np

from oracle import direct


def besselj_prime(nu: int, x) -> np.ndarray:
    """J_nu'(x) = (J_{nu-1}(x) - J_{nu+1}(x)) / 2."""
    return 0.5 * (direct.besselj(nu - 1, x) - direct.besselj(nu + 1, x))


def gradient(nu: int, r, c, w, gbar):
    """(dL/dc, dL/dr, dL/dw) for g = A c and dL/dg = gbar (caller order)."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    # sum_j gbar_j J_nu(r_k w_j): the direct sum with the roles of r and w exchanged
    dc = direct.dht(nu, w, gbar, r)
    gw = gbar * w
    dr = 0.5 * c * (direct.dht(nu - 1, w, gw, r) - direct.dht(nu + 1, w, gw, r))
    cr = c * r
    dw = 0.5 * gbar * (direct.dht(nu - 1, r, cr, w) - direct.dht(nu + 1, r, cr, w))
    return dc, dr, dw


def gradient_at(nu: int, r, c, w, gbar, idx_c, idx_r, idx_w):
    """The same derivatives at selected entries only (O(n m) per entry set)."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    dc = direct.dht(nu, w, gbar, r[idx_c])
    gw = gbar * w
    rk = r[idx_r]
    dr = 0.5 * c[idx_r] * (direct.dht(nu - 1, w, gw, rk) - direct.dht(nu + 1, w, gw, rk))
    cr = c * r
    wj = w[idx_w]
    dw = 0.5 * gbar[idx_w] * (direct.dht(nu - 1, r, cr, wj) - direct.dht(nu + 1, r, cr, wj))
    return dc, dr, dw
