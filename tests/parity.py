"""Tolerance checks shared by the GPU parity tests (not collected by pytest).

The contract is "from the same x": the GPU sweep and the oracle sweep take the
same point and the same stored data.  Because cancellation in r_i and mask
flips at r_i ~ 0 make plain relative error meaningless near feasibility, each
quantity is compared on its own rounding-error scale (Higham, Accuracy and
Stability of Numerical Algorithms, ch. 3):

  r:     |r_G - r_O| <= tol * t_i,   t_i = sum_j |a_ij x_j| + |b_i|
  h:     equal up to rows in the ambiguous band |r_O| <= tol * t_i
  y:     ||y_G - y_O|| <= tol * max(||y_O||, s_y),
         s_y = || sum over rows with r_O > -tol t_i of (t_i/||a_i||^2) |a_i| ||
  dmax:  |dmax_G - dmax_O| <= tol * max over the same rows of t_i/||a_i||

The plain normwise relative error of y is logged but not required: a
residual outside the ambiguous band can still be small against its rounding
scale (r_i << t_i), and its weight r_i/||a_i||^2 then carries a relative error
up to about u t_i / r_i (u the unit roundoff of the accumulation), which the
bound on the scale s_y covers and a plain relative bound does not.  Without
such cancellation s_y is close to ||y|| and the two bounds agree.
"""
from __future__ import annotations

import json
import os

import numpy as np

import workloads as W

# tolerances per storage type (FP64 dot products for f64, FP32 for f32/bf16)
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}
# BF16-stored system against the FP64 system it was rounded from (quantisation)
TOL_BF16_VS_F64 = 5e-3


def weighted_abs_rows(A, dtype, w, chunk=8192):
    """sum_i w_i |a_i| over the stored rows, in row chunks (bounded memory)."""
    out = np.zeros(A.shape[1])
    for r0 in range(0, A.shape[0], chunk):
        ww = w[r0:r0 + chunk]
        if np.any(ww != 0):
            out += ww @ np.abs(W.stored_to_f64(A[r0:r0 + chunk], dtype))
    return out


def check_sweep(A, dtype, o, y_g, h_g, dmax_g, r_g=None, tol=None, label=""):
    """Compare one GPU sweep with the oracle sweep `o`; returns a dict of errors."""
    tol = TOL[dtype] if tol is None else tol
    band = np.abs(o.r) <= tol * o.t
    near = o.r > -tol * o.t
    w = np.where(near, o.t / o.nu, 0.0)
    s_y = float(np.linalg.norm(weighted_abs_rows(A, dtype, w)))
    ynorm = float(np.linalg.norm(o.y))
    dy = float(np.linalg.norm(np.asarray(y_g) - o.y))
    err = {"y_scaled": dy / max(ynorm, s_y, 1e-300),
           "y_rel": dy / ynorm if ynorm > 0 else dy,
           "band_rows": int(band.sum())}
    assert err["y_scaled"] <= tol, (label, err)
    # h: equal up to the ambiguous rows
    assert abs(int(h_g) - o.h) <= int(band.sum()), (label, h_g, o.h, int(band.sum()))
    if band.sum() == 0:
        assert int(h_g) == o.h, (label, h_g, o.h)
    dscale = float(np.max(np.where(near, o.t / np.sqrt(o.nu), 0.0), initial=0.0))
    err["dmax"] = abs(dmax_g - o.dmax) / max(dscale, 1e-300)
    assert abs(dmax_g - o.dmax) <= tol * max(dscale, 1e-300) + 1e-300, (label, dmax_g, o.dmax, dscale)
    if r_g is not None:
        rerr = np.abs(np.asarray(r_g) - o.r) / np.maximum(o.t, 1e-300)
        err["r_scaled"] = float(rerr.max())
        assert err["r_scaled"] <= tol, (label, err)
    log = os.environ.get("MODAP_PARITY_LOG")
    if log:
        with open(log, "a") as f:
            f.write(json.dumps({"case": label, "dtype": dtype, "tol": tol, **err}) + "\n")
    return err


def fejer_gap(A, dtype, x, z, y, r, chunk=8192):
    """<x - z, y> - sum_{r_i>0} r_i^2/||a_i||^2 (>= 0 for a feasible z, any size)."""
    tot = 0.0
    for r0 in range(0, A.shape[0], chunk):
        A64 = W.stored_to_f64(A[r0:r0 + chunk], dtype)
        nu = np.einsum("ij,ij->i", A64, A64)
        rr = r[r0:r0 + chunk]
        viol = rr > 0
        tot += np.sum(rr[viol] ** 2 / nu[viol])
    return float((x - z) @ y - tot)
