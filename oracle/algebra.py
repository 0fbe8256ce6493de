"""Rake fold and compress composition of Sec. IV-A, written out literally.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Used by the pins of
Lemma 1 (elimination identities), Prop. 3's PSD increments and the
node-aware associativity of eq. (node-aware-associativity).

  tau(alpha, U) = P + A^T U (I + C U)^{-1} A                  eq. (terminal-fold)
  Pt = P_r + U_j,  S = I + C_l Pt                             eq. (compress-intermediates)
  A_lr = A_r S^{-1} A_l
  C_lr = C_r + A_r S^{-1} C_l A_r^T
  P_lr = P_l + A_l^T Pt S^{-1} A_l                            eq. (composition)
"""
from __future__ import annotations

import numpy as np


def tau(A, C, P, U):
    n = A.shape[0]
    return P + A.T @ U @ np.linalg.solve(np.eye(n) + C @ U, A)


def compose(right, left, Uj):
    """alpha_r o_{U_j} alpha_l, each alpha = (A, C, P)."""
    Ar, Cr, Pr = right
    Al, Cl, Pl = left
    n = Al.shape[0]
    Pt = Pr + Uj
    S = np.eye(n) + Cl @ Pt
    return (Ar @ np.linalg.solve(S, Al),
            Cr + Ar @ np.linalg.solve(S, Cl @ Ar.T),
            Pl + Al.T @ Pt @ np.linalg.solve(S, Al))


def condense(A, B, R, M, Delta_j):
    """Edge triple of eq. (edge-components)."""
    Ri = np.linalg.inv(R)
    return (A - B @ Ri @ M.T, Delta_j + B @ Ri @ B.T, -M @ Ri @ M.T)
