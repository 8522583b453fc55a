"""Preconditioned MINRES (Paige & Saunders 1975) -- oracle.

Solves K x = b for symmetric (possibly singular but consistent) K with an SPD
preconditioner M^{-1} = K-hat^{-1}.  Starting from x_0 = 0, it runs the
preconditioned Lanczos process: with z_1 = M^{-1} b, beta_1 = sqrt(b . z_1)
and v_j = z_j / beta_j,

    K v_j = beta_j r_{j-1} + alpha_j r_j + beta_{j+1} r_{j+1}  (in the M-metric),

giving a symmetric tridiagonal T_j.  A QR factorisation of T_j by Givens
rotations is updated one column at a time; the iterate is
x_j = x_{j-1} + tau_j w_j with search directions w_j obtained from the
three-term recurrence of the rotated tridiagonal.  The M^{-1}-norm of the
residual equals |phi_bar_j| = beta_1 * prod |s_i| and is the stopping test:

    stop when phi_bar_j <= tol * beta_1   (preconditioned relative residual).
"""
from __future__ import annotations

import math

import numpy as np


def minres(apply_K, apply_Minv, b, tol=1e-10, max_it=1000, callback=None):
    n = b.shape[0]
    x = np.zeros(n)
    r_prev = np.zeros(n)
    r_cur = b.copy()
    z = apply_Minv(r_cur)
    beta1 = math.sqrt(float(r_cur @ z))
    info = dict(iterations=0, converged=False, phibar=beta1, beta1=beta1, history=[])
    if beta1 == 0.0:
        info["converged"] = True
        return x, info
    beta = beta1
    beta_old = 0.0
    # rotation state
    c_prev, s_prev = -1.0, 0.0
    dbar = 0.0
    eps = 0.0
    phibar = beta1
    w_prev2 = np.zeros(n)
    w_prev = np.zeros(n)
    for it in range(1, max_it + 1):
        # --- Lanczos step
        v = z / beta
        y = apply_K(v)
        if it > 1:
            y = y - (beta / beta_old) * r_prev
        alpha = float(v @ y)
        y = y - (alpha / beta) * r_cur
        r_prev, r_cur = r_cur, y
        z = apply_Minv(r_cur)
        beta_old = beta
        beta2 = float(r_cur @ z)
        if beta2 < 0.0:
            info["breakdown"] = True
            break
        beta = math.sqrt(beta2)
        # --- apply the previous rotation to the new column (entries eps, delta, gbar)
        eps_old = eps
        delta = c_prev * dbar + s_prev * alpha
        gbar = s_prev * dbar - c_prev * alpha
        eps = s_prev * beta
        dbar = -c_prev * beta
        # --- new rotation annihilating beta
        gamma = math.hypot(gbar, beta)
        if gamma == 0.0:
            gamma = np.finfo(float).tiny
        c_prev = gbar / gamma
        s_prev = beta / gamma
        phi = c_prev * phibar
        phibar = s_prev * phibar
        # --- direction and solution update
        w = (v - eps_old * w_prev2 - delta * w_prev) / gamma
        w_prev2, w_prev = w_prev, w
        x = x + phi * w
        info["history"].append(phibar / beta1)
        if callback is not None:
            callback(it, x, phibar / beta1)
        info["iterations"] = it
        info["phibar"] = phibar
        if phibar <= tol * beta1:
            info["converged"] = True
            break
    return x, info
