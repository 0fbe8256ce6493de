"""Gradients of a scalar loss through the tree-LQR solve (the adjoint system).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The solution z = (x, u, y) of eq. (kkt) satisfies M z = -(q, r, c), where the
rows of M are the node stationarity eq. (kkt-x), the control stationarity
eq. (kkt-u) and the root and dynamics equations eqs. (kkt-root), (kkt-dyn),
and M = [[H, C^T], [C, -D]] is symmetric (proof of Prop. 1).  For a loss
L(z) with seed g = dL/dz:

  dL/d(q, r, c) = -M^{-1} g,

which is the solution of the same system with the seeds in place of
(q, r, c): the oracle solve with right-hand side (q, r, c) := (g_x, g_u, g_y).
Call that solution a = (a_x, a_u, a_y).  Differentiating M z = b gives
dL = a^T dM z for a change dM of the matrix blocks, and each block's place in
eq. (kkt) gives its gradient (for the edge e = (i, j), edge slot j):

  Q_i      in  Q_i x_i                   ->  a_x,i x_i^T
  Delta_j  in  -Delta_j y_j              ->  -a_y,j y_j^T
  R_e      in  R_e u_e                   ->  a_u,e u_e^T
  M_e (S)  in  M_e u_e and M_e^T x_i     ->  a_x,i u_e^T + x_i a_u,e^T
  A_e      in  A_e x_i and A_e^T y_j     ->  a_y,j x_i^T + y_j a_x,i^T
  B_e      in  B_e u_e and B_e^T y_j     ->  a_y,j u_e^T + y_j a_u,e^T

The root's edge slot (no edge) gets zero gradients.  The gradients are the
raw (unsymmetrised) ones; the pins compare them with finite differences of
the dense KKT solve.
"""
from __future__ import annotations

import numpy as np

from . import riccati


def adjoint(parent, data: dict, sol: dict, seed: dict) -> dict:
    """Gradients of L with dL/dx = seed['x'], dL/du = seed['u'], dL/dy = seed['lam']
    at the forward solution sol (x, u, lam) of problem data.  Returns a dict with
    the fields of the problem (Q, q, c, Delta, R, S, r, A, B)."""
    parent = np.asarray(parent, dtype=np.int64)
    rhs = dict(data)
    rhs["q"] = seed["x"]
    rhs["r"] = seed["u"]
    rhs["c"] = seed["lam"]
    a = riccati.tree_riccati(parent, rhs)
    ax, au, ay = a["x"], a["u"], a["lam"]
    x, u, y = sol["x"], sol["u"], sol["lam"]
    N = parent.shape[0]
    n = data["Q"].shape[-1]
    m = data["R"].shape[-1]
    g = {"q": ax.copy(), "r": au.copy(), "c": ay.copy(),
         "Q": np.einsum("ia,ib->iab", ax, x), "Delta": -np.einsum("ia,ib->iab", ay, y),
         "R": np.zeros((N, m, m)), "S": np.zeros((N, n, m)), "A": np.zeros((N, n, n)),
         "B": np.zeros((N, n, m))}
    for j in range(N):
        i = parent[j]
        if i < 0:
            g["r"][j] = 0.0
            continue
        g["R"][j] = np.outer(au[j], u[j])
        g["S"][j] = np.outer(ax[i], u[j]) + np.outer(x[i], au[j])
        g["A"][j] = np.outer(ay[j], x[i]) + np.outer(y[j], ax[i])
        g["B"][j] = np.outer(ay[j], u[j]) + np.outer(y[j], au[j])
    return g
