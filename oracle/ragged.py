"""Tree LQR with per-node state and per-edge control dimensions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The problem of Sec. II-A does not need uniform dimensions (the paper says
so there): node i has a state of dimension n_i and the edge e = (i, j) a
control of dimension m_e, so A_e is n_j x n_i, B_e n_j x m_e, M_e (S) n_i x m_e,
R_e m_e x m_e.  Data are lists of per-node (or per edge slot) numpy blocks;
the root's edge blocks are empty and ignored.

* `solve_kkt_ragged` writes out eq. (kkt) with these block sizes and solves it
  densely (LAPACK); by Prop. 1 its solution is the definition of (x, u, y).
* `tree_riccati_ragged` is the sequential dual-regularised tree Riccati
  recursion (the CPU baseline of Sec. XI-A) with rectangular blocks, in plain
  numpy: for every child edge e = (i, j), with the formulas of eqs. (FW),
  (factor-local), (local-affine-solve) and the message of Lemma 5,
    F_j = I + Delta_j P_j, W_j = P_j F_j^{-1}, f_j = Delta_j p_j - c_j,
    g_j = p_j - W_j f_j, G = R + B^T W_j B, H = B^T W_j A + M^T,
    K = -G^{-1} H, k = -G^{-1} (r + B^T g_j), A^cl = A + B K,
    P_i += A^T W_j A - H^T G^{-1} H, p_i += K^T r + (A^cl)^T g_j;
  the root state of eq. (xroot) and the forward pass of eq. (recover).
"""
from __future__ import annotations

import numpy as np


def _children(parent):
    ch = [[] for _ in range(len(parent))]
    for j, p in enumerate(parent):
        if p >= 0:
            ch[p].append(j)
    return ch


def _bfs(parent):
    ch = _children(parent)
    root = [v for v, p in enumerate(parent) if p < 0]
    assert len(root) == 1
    order = [root[0]]
    for v in order:
        order.extend(ch[v])
    assert len(order) == len(parent)
    return order, ch


def solve_kkt_ragged(parent, n_node, m_edge, d):
    """Dense solve of eq. (kkt) with per-node/per-edge block sizes.  Returns lists
    x (n_i), u (m_e; empty at the root), y (n_i)."""
    parent = [int(p) for p in parent]
    N = len(parent)
    edges = [j for j in range(N) if parent[j] >= 0]
    ix, iu, iy, k = {}, {}, {}, 0
    for v in range(N):
        ix[v] = k
        k += n_node[v]
    for j in edges:
        iu[j] = k
        k += m_edge[j]
    for v in range(N):
        iy[v] = k
        k += n_node[v]
    M = np.zeros((k, k))
    rhs = np.zeros(k)
    ch = _children(parent)
    for i in range(N):  # eq. (kkt-x): Q x + q - y + sum_out (M_e u_e + A_e^T y_j) = 0
        a, ni = ix[i], n_node[i]
        M[a:a + ni, a:a + ni] += d["Q"][i]
        M[a:a + ni, iy[i]:iy[i] + ni] -= np.eye(ni)
        rhs[a:a + ni] -= d["q"][i]
        for j in ch[i]:
            M[a:a + ni, iu[j]:iu[j] + m_edge[j]] += d["S"][j]
            M[a:a + ni, iy[j]:iy[j] + n_node[j]] += d["A"][j].T
    for j in edges:  # eq. (kkt-u): M^T x_i + R u + r + B^T y_j = 0
        i, a, mj = parent[j], iu[j], m_edge[j]
        M[a:a + mj, ix[i]:ix[i] + n_node[i]] += d["S"][j].T
        M[a:a + mj, a:a + mj] += d["R"][j]
        M[a:a + mj, iy[j]:iy[j] + n_node[j]] += d["B"][j].T
        rhs[a:a + mj] -= d["r"][j]
    for v in range(N):  # eqs. (kkt-root), (kkt-dyn): (A x_i + B u +) c - x - Delta y = 0
        a, nv = iy[v], n_node[v]
        M[a:a + nv, ix[v]:ix[v] + nv] -= np.eye(nv)
        M[a:a + nv, a:a + nv] -= d["Delta"][v]
        rhs[a:a + nv] -= d["c"][v]
        if parent[v] >= 0:
            i = parent[v]
            M[a:a + nv, ix[i]:ix[i] + n_node[i]] += d["A"][v]
            M[a:a + nv, iu[v]:iu[v] + m_edge[v]] += d["B"][v]
    z = np.linalg.solve(M, rhs)
    x = [z[ix[v]:ix[v] + n_node[v]] for v in range(N)]
    y = [z[iy[v]:iy[v] + n_node[v]] for v in range(N)]
    u = [z[iu[j]:iu[j] + m_edge[j]] if parent[j] >= 0 else np.zeros(0) for j in range(N)]
    return x, u, y


def tree_riccati_ragged(parent, n_node, m_edge, d):
    """The sequential recursion with rectangular blocks.  Returns dict of lists:
    K (m_e x n_i; empty at the root), P (n_i x n_i), x, u, lam."""
    parent = [int(p) for p in parent]
    N = len(parent)
    order, ch = _bfs(parent)
    P = [None] * N
    p = [None] * N
    K = [np.zeros((0, 0))] * N
    kf = [np.zeros(0)] * N
    Finv = [None] * N
    f = [None] * N
    for i in reversed(order):
        Pi = np.array(d["Q"][i], dtype=float)
        pi = np.array(d["q"][i], dtype=float)
        for j in ch[i]:
            nj = n_node[j]
            F = np.eye(nj) + d["Delta"][j] @ P[j]
            Fi = np.linalg.inv(F)
            W = P[j] @ Fi
            fj = d["Delta"][j] @ p[j] - d["c"][j]
            g = p[j] - W @ fj
            A, B, S, R, r = d["A"][j], d["B"][j], d["S"][j], d["R"][j], d["r"][j]
            G = R + B.T @ W @ B
            H = B.T @ W @ A + S.T
            Ke = -np.linalg.solve(G, H)
            ke = -np.linalg.solve(G, r + B.T @ g)
            Acl = A + B @ Ke
            Pi = Pi + A.T @ W @ A - H.T @ np.linalg.solve(G, H)
            pi = pi + Ke.T @ r + Acl.T @ g
            K[j], kf[j], Finv[j], f[j] = Ke, ke, Fi, fj
        P[i], p[i] = Pi, pi
    root = order[0]
    Fr = np.eye(n_node[root]) + d["Delta"][root] @ P[root]
    fr = d["Delta"][root] @ p[root] - d["c"][root]
    x = [None] * N
    u = [np.zeros(0)] * N
    x[root] = -np.linalg.solve(Fr, fr)
    for v in order:
        for j in ch[v]:
            u[j] = K[j] @ x[v] + kf[j]
            x[j] = Finv[j] @ (d["A"][j] @ x[v] + d["B"][j] @ u[j] - f[j])
    lam = [P[v] @ x[v] + p[v] for v in range(N)]
    return {"K": K, "P": P, "x": x, "u": u, "lam": lam}
