"""Learned normalised/offset min-sum, unrolled: binary64 forward and adjoint
-- TEST INFRASTRUCTURE (same rules as the rest of ``oracle/``: only tests,
``smoke()`` and the CPU baseline may use it; the library never does).

Decoder (the check update of Sec. III with its constant lambda and beta
generalised to one pair per iteration t and check-degree class c):
    Z^(0) = y,  L^(0) = 0
    t_mn  = Z^(t-1)_n - L^(t-1)_mn
    L^(t)_mn = prod_{n' != n} sgn(t_mn') * max(a[t,c_m] * min_{n' != n} |t_mn'| - b[t,c_m], 0)
    Z^(t)_n = Z^(0)_n + sum_{m in M(n)} L^(t)_mn              (t = 1..T)
Classes: the distinct row degrees of H in ascending order.  sgn(x) = -1 iff
x < 0; the minimum's position is the lowest index among equal values.

Loss: BCE of the posteriors against the transmitted bits x, summed over
iterations, frames and bits:  sum_t sum_f sum_n softplus(s * Z^(t)_n) with
s = 2x - 1 (bit 0 wants Z > 0).  The adjoint also takes a weight w_t per
iteration (the objective sum_t w_t loss_t; all ones by default), for
objectives that favour decoding in fewer iterations.

Adjoint: reverse mode through the unrolled graph.  L^(t)_mn depends on the
extrinsics only through the minimising position k(n) (away from ties and
from the kink of max(., 0)), with d|t|/dt = sgn(t); the sign product is
piecewise constant.  Written out per position from the exclusion form above,
without the min1/min2 shortcut of the kernels.
"""
from __future__ import annotations

import numpy as np


def degree_classes(code):
    """(row degrees, class index of each row, ascending distinct degrees)."""
    rp = np.asarray(code.row_ptr)
    deg = np.diff(rp)
    levels = np.unique(deg)
    cls = np.searchsorted(levels, deg)
    return deg, cls, levels


def _softplus(x):
    return np.logaddexp(0.0, x)


def _sigmoid(x):
    return np.exp(-np.logaddexp(0.0, -x))


def _row_groups(code):
    """Rows grouped by degree: (d, rows, edge index matrix [R, d], column matrix [R, d])."""
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    deg = np.diff(rp)
    out = []
    for d in np.unique(deg):
        rows = np.nonzero(deg == d)[0]
        e = rp[rows][:, None] + np.arange(d)[None, :]
        out.append((int(d), rows, e, ci[e]))
    return out


def _pair(W, t, cls_rows):
    """The (a, b) pair of iteration t (1-based) for rows of classes ``cls_rows``:
    row t - 1 of the table, column = the row's class."""
    return W[t - 1, cls_rows, 0], W[t - 1, cls_rows, 1]


def _check_update(tm, a, b):
    """Exclusion-form check update of one degree group.
    tm [F, R, d] extrinsics, a/b [R] weights.  Returns L [F, R, d] and, per
    position j, the minimising other position k [F, R, d], the minimum mn,
    the sign product sg and the active flag (a*mn - b > 0)."""
    F, R, d = tm.shape
    L = np.empty_like(tm)
    K = np.empty((F, R, d), dtype=np.int64)
    MN = np.empty_like(tm)
    SG = np.empty_like(tm)
    zero = tm.dtype.type(0)
    ACT = np.empty(tm.shape, dtype=bool)
    for j in range(d):
        others = np.array([k for k in range(d) if k != j])
        ab = np.abs(tm[:, :, others])
        pos = np.argmin(ab, axis=2)                       # first of equal minima
        mn = np.take_along_axis(ab, pos[:, :, None], axis=2)[:, :, 0]
        sg = np.prod(np.where(tm[:, :, others] < 0, -1.0, 1.0), axis=2).astype(tm.dtype)
        v = a[None, :] * mn - b[None, :]
        act = v > 0
        L[:, :, j] = sg * np.where(act, v, zero)
        K[:, :, j] = others[pos]
        MN[:, :, j] = mn
        SG[:, :, j] = sg
        ACT[:, :, j] = act
    return L, K, MN, SG, ACT


def forward(code, llr, weights, target=None, dtype=np.float64):
    """Unrolled decoder.  llr [F, N]; weights [T, C, 2] (a, b); target [F, N]
    bits or None (all-zero word).  Returns dict with per-iteration losses
    ``loss`` [T], posteriors ``Z`` [T+1, F, N] and messages ``L`` [T+1, F, E]
    (CSR edge order).  ``dtype=np.float32`` runs every decoder operation in
    binary32 (a*m rounded before b is subtracted, posterior sums in ascending
    check order); the loss is then still summed in binary64."""
    llr = np.asarray(llr, dtype=dtype)
    W = np.asarray(weights, dtype=dtype)
    T = W.shape[0]
    F, N = llr.shape
    ci = np.asarray(code.col_idx)
    E = ci.size
    _, cls, _ = degree_classes(code)
    groups = _row_groups(code)
    x = np.zeros((F, N)) if target is None else np.asarray(target, dtype=np.float64)
    s = 2.0 * x - 1.0
    Zs = [llr.copy()]
    Ls = [np.zeros((F, E), dtype=dtype)]
    losses = []
    for t in range(1, T + 1):
        Zp, Lp = Zs[-1], Ls[-1]
        Ln = np.zeros((F, E), dtype=dtype)
        for d, rows, e, cols in groups:
            tm = Zp[:, cols] - Lp[:, e]
            a, b = _pair(W, t, cls[rows])
            L, *_ = _check_update(tm, a, b)
            Ln[:, e] = L
        Zn = llr.copy()
        # posterior sums in ascending check order (CSR edge order)
        for k in range(E):
            Zn[:, ci[k]] += Ln[:, k]
        Zs.append(Zn)
        Ls.append(Ln)
        losses.append(float(np.sum(_softplus(s * Zn.astype(np.float64)))))
    return {"loss": np.array(losses), "Z": np.stack(Zs), "L": np.stack(Ls)}


def adjoint(code, llr, weights, target=None, loss_weights=None):
    """Gradient of sum_t w_t loss_t with respect to the weights, [T, C, 2]
    (w_t = loss_weights[t - 1], all ones if None)."""
    fw = forward(code, llr, weights, target)
    W = np.asarray(weights, dtype=np.float64)
    T, C = W.shape[0], W.shape[1]
    lw = np.ones(T) if loss_weights is None else np.asarray(loss_weights, dtype=np.float64)
    Zs, Ls = fw["Z"], fw["L"]
    F, N = Zs.shape[1], Zs.shape[2]
    ci = np.asarray(code.col_idx)
    E = ci.size
    _, cls, _ = degree_classes(code)
    groups = _row_groups(code)
    x = np.zeros((F, N)) if target is None else np.asarray(target, dtype=np.float64)
    s = 2.0 * x - 1.0
    grad = np.zeros((T, C, 2))
    tbar_next = np.zeros((F, E))   # adjoint of t^(t+1) per edge
    for t in range(T, 0, -1):
        # Z^(t): its own loss term, and every t^(t+1)_mn = Z^(t)_n - L^(t)_mn
        Zbar = lw[t - 1] * s * _sigmoid(s * Zs[t])
        np.add.at(Zbar.T, ci, tbar_next.T)
        # L^(t)_mn feeds Z^(t)_n (+) and t^(t+1)_mn (-)
        Lbar = Zbar[:, ci] - tbar_next
        tbar = np.zeros((F, E))
        for d, rows, e, cols in groups:
            tm = Zs[t - 1][:, cols] - Ls[t - 1][:, e]
            a, b = _pair(W, t, cls[rows])
            _, K, MN, SG, ACT = _check_update(tm, a, b)
            lb = Lbar[:, e]                                    # [F, R, d]
            live = lb * SG * ACT                               # dL_j / d(a*mn - b)
            np.add.at(grad[t - 1, :, 0], cls[rows], np.sum(live * MN, axis=(0, 2)))
            np.add.at(grad[t - 1, :, 1], cls[rows], -np.sum(live, axis=(0, 2)))
            tk = np.take_along_axis(tm, K, axis=2)
            contrib = live * a[None, :, None] * np.where(tk < 0, -1.0, 1.0)
            g = np.zeros_like(tm)
            for j in range(d):
                np.put_along_axis(g, K[:, :, j:j + 1],
                                  np.take_along_axis(g, K[:, :, j:j + 1], axis=2) + contrib[:, :, j:j + 1],
                                  axis=2)
            tbar[:, e] = g
        tbar_next = tbar
    return grad, fw
