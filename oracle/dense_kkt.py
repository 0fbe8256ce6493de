"""Dense KKT assembly and solve, and brute-force Riccati coefficients.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Tiny trees only: the
KKT matrix is dense.

* `solve_kkt` writes out the KKT equations eq. (kkt) (Sec. II-A) row by row,
  with unknowns ordered [x_0..x_{N-1}, u_e for non-root slots, y_0..y_{N-1}],
  and solves them with LAPACK (numpy.linalg.solve).  By Prop. 1 the solution
  is unique, so it is the definition of (x, u, y).
* `kkt_residual` evaluates the four residual blocks of eq. (kkt).
* `subtree_P_K` computes P_i and K_e straight from their definitions: P_i is
  the Hessian of the homogeneous subtree value V_i^0 with x_i fixed
  (eq. (homogeneous-subtree-value-definition), Thm. 1) and K_e the map
  x_i -> u_e of that subtree problem (eq. (eliminated-edge-affine)).  Each
  column comes from one dense solve of the subtree's KKT equations with
  x_i = unit vector, evaluating the envelope gradient
  Q_i x_i + sum_out (M_e u_e + A_e^T y_j) (proof of Thm. 2).
"""
from __future__ import annotations

import numpy as np


def _children(parent):
    N = len(parent)
    ch = [[] for _ in range(N)]
    for j in range(N):
        if parent[j] >= 0:
            ch[parent[j]].append(j)
    return ch


def _assemble(parent, d, nodes, fixed=None):
    """Rows/cols of the KKT equations restricted to the subtree `nodes` (a set,
    containing its top node t).  If `fixed` is not None, x_t is a parameter
    (moved to the right-hand side as x_t = fixed), node stationarity at t and
    the constraint entering t are dropped.  Returns (Kmat, rhs, index maps)."""
    n = d["Q"].shape[-1]
    m = d["R"].shape[-1]
    nodes = sorted(nodes)
    top = [v for v in nodes if parent[v] < 0 or parent[v] not in set(nodes)]
    assert len(top) == 1
    t = top[0]
    edges = [j for j in nodes if j != t]          # edge slot j = (parent[j], j)
    xs = [v for v in nodes if not (fixed is not None and v == t)]
    ys = [v for v in nodes if not (fixed is not None and v == t)]
    ix = {v: k * n for k, v in enumerate(xs)}
    off_u = len(xs) * n
    iu = {j: off_u + k * m for k, j in enumerate(edges)}
    off_y = off_u + len(edges) * m
    iy = {v: off_y + k * n for k, v in enumerate(ys)}
    dim = off_y + len(ys) * n
    Km = np.zeros((dim, dim))
    rhs = np.zeros(dim)  # equations are  Km z + const = 0  ->  rhs = -const
    xfix = np.zeros(n) if fixed is None else np.asarray(fixed, dtype=float)
    ch = _children(parent)

    def add_x(row, v, M):       # contribution M x_v to rows `row`
        if v in ix:
            Km[row:row + M.shape[0], ix[v]:ix[v] + n] += M
        else:                   # fixed top state
            rhs[row:row + M.shape[0]] -= M @ xfix

    # node stationarity eq. (kkt-x): Q_i x_i + q_i - y_i + sum_out (M_e u_e + A_e^T y_j) = 0
    for v in xs:
        r0 = ix[v]
        add_x(r0, v, d["Q"][v])
        rhs[r0:r0 + n] -= d["q"][v]
        Km[r0:r0 + n, iy[v]:iy[v] + n] -= np.eye(n)
        for j in ch[v]:
            Km[r0:r0 + n, iu[j]:iu[j] + m] += d["S"][j]
            Km[r0:r0 + n, iy[j]:iy[j] + n] += d["A"][j].T
    # control stationarity eq. (kkt-u): M_e^T x_i + R_e u_e + r_e + B_e^T y_j = 0
    for j in edges:
        r0 = iu[j]
        i = parent[j]
        add_x(r0, i, d["S"][j].T)
        Km[r0:r0 + m, iu[j]:iu[j] + m] += d["R"][j]
        rhs[r0:r0 + m] -= d["r"][j]
        Km[r0:r0 + m, iy[j]:iy[j] + n] += d["B"][j].T
    # root eq. (kkt-root): c_rho - x_rho - Delta_rho y_rho = 0  (only for the full tree)
    for v in ys:
        r0 = iy[v]
        if v == t:
            Km[r0:r0 + n, ix[v]:ix[v] + n] -= np.eye(n)
            Km[r0:r0 + n, iy[v]:iy[v] + n] -= d["Delta"][v]
            rhs[r0:r0 + n] -= d["c"][v]
        else:
            # dynamics eq. (kkt-dyn): A_e x_i + B_e u_e + c_j - x_j - Delta_j y_j = 0
            i = parent[v]
            add_x(r0, i, d["A"][v])
            Km[r0:r0 + n, iu[v]:iu[v] + m] += d["B"][v]
            rhs[r0:r0 + n] -= d["c"][v]
            Km[r0:r0 + n, ix[v]:ix[v] + n] -= np.eye(n)
            Km[r0:r0 + n, iy[v]:iy[v] + n] -= d["Delta"][v]
    return Km, rhs, ix, iu, iy


def kkt_matrix(parent, d):
    """The dense KKT matrix and right-hand side of eq. (kkt) for the whole tree."""
    parent = list(map(int, parent))
    Km, rhs, ix, iu, iy = _assemble(parent, d, set(range(len(parent))))
    return Km, rhs


def solve_kkt(parent, d):
    """Unique solution (x, u, y) of eq. (kkt) by a dense LAPACK solve."""
    parent = list(map(int, parent))
    N = len(parent)
    n = d["Q"].shape[-1]
    m = d["R"].shape[-1]
    Km, rhs, ix, iu, iy = _assemble(parent, d, set(range(N)))
    z = np.linalg.solve(Km, rhs)
    x = np.zeros((N, n))
    u = np.zeros((N, m))
    y = np.zeros((N, n))
    for v in range(N):
        x[v] = z[ix[v]:ix[v] + n]
        y[v] = z[iy[v]:iy[v] + n]
    for j, o in iu.items():
        u[j] = z[o:o + m]
    return x, u, y


def kkt_residual(parent, d, x, u, y):
    """Residual blocks of eq. (kkt): (r_x [N,n], r_u [N,m], r_root [n], r_dyn [N,n]).
    Root slots of r_u and r_dyn are zero."""
    parent = np.asarray(parent)
    N = len(parent)
    n = d["Q"].shape[-1]
    m = d["R"].shape[-1]
    rx = np.einsum("nij,nj->ni", d["Q"], x) + d["q"] - y
    ru = np.zeros((N, m))
    rdyn = np.zeros((N, n))
    for j in range(N):
        i = parent[j]
        if i < 0:
            root = j
            continue
        rx[i] += d["S"][j] @ u[j] + d["A"][j].T @ y[j]
        ru[j] = d["S"][j].T @ x[i] + d["R"][j] @ u[j] + d["r"][j] + d["B"][j].T @ y[j]
        rdyn[j] = d["A"][j] @ x[i] + d["B"][j] @ u[j] + d["c"][j] - x[j] - d["Delta"][j] @ y[j]
    rroot = d["c"][root] - x[root] - d["Delta"][root] @ y[root]
    return rx, ru, rroot, rdyn


def subtree_P_K(parent, d):
    """P_i (all nodes) and K_e (all non-root slots) from their definitions by
    dense solves of homogeneous subtree problems with x_i fixed."""
    parent = list(map(int, parent))
    N = len(parent)
    n = d["Q"].shape[-1]
    m = d["R"].shape[-1]
    hom = dict(d)
    hom["q"] = np.zeros_like(d["q"])
    hom["r"] = np.zeros_like(d["r"])
    hom["c"] = np.zeros_like(d["c"])
    ch = _children(parent)
    P = np.zeros((N, n, n))
    K = np.zeros((N, m, n))
    for i in range(N):
        sub = set()
        stack = [i]
        while stack:
            v = stack.pop()
            sub.add(v)
            stack.extend(ch[v])
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            if len(sub) == 1:
                P[i][:, k] = d["Q"][i] @ e
                continue
            Km, rhs, ix, iu, iy = _assemble(parent, hom, sub, fixed=e)
            z = np.linalg.solve(Km, rhs)
            grad = d["Q"][i] @ e
            for j in ch[i]:
                uj = z[iu[j]:iu[j] + m]
                yj = z[iy[j]:iy[j] + n]
                grad = grad + d["S"][j] @ uj + d["A"][j].T @ yj
                K[j][:, k] = uj
            P[i][:, k] = grad
    return P, K
