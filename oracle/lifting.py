"""Node-control scenario MPC: native dense KKT and the lifting of Sec. II-B.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Native problem (eq. (node-lagrangian), eq. (node-control)): one control v_i
per non-leaf node, shared by all outgoing transitions
    x_j = A_ij x_i + B_ij v_i + c_j,  j a child of i.
Native data (row-major float64): per node Q[N,n,n], q[N,n], c[N,n],
Delta[N,n,n]; per node (non-leaf rows used) M[N,n,m], R[N,m,m], r[N,m]; per
edge slot j (edge (parent[j], j)) A[N,n,n], B[N,n,m].

`solve_native` writes out the stationarity and dynamics equations of the
native saddle function and solves them densely.  `lift` builds the lifted
edge-control tree of Prop. 2: every node i becomes a predecision node i^-
(keeping id i) and, if non-terminal, a decision node i^+ (id N + rank among
non-leaves), with state s = (x, v) of dimension n + m:
    decision edge i^- -> i^+:   A = [[I,0],[0,0]], B = [0; I], R = R_i,
                                S = [M_i; 0], r = r_i                 eq. (decision-edge)
    uncertainty edge i^+ -> j^-: A = [[A_ij, B_ij],[0,0]], B = 0,
                                dummy R = I, S = 0, r = 0             eq. (uncertainty-edge)
    costs at i^-: diag(Q_i, 0), (q_i, 0); regulariser diag(Delta_i, 0) and
    offset (c_i, 0) on the constraint entering i^-; all else zero.
`project` maps a lifted solution back: x_i = upper(s_{i^-}), v_i = the
decision-edge control, y_i = upper(y_{i^-}).
"""
from __future__ import annotations

import numpy as np


def nonleaves(parent):
    N = len(parent)
    isleaf = np.ones(N, dtype=bool)
    for j in range(N):
        if parent[j] >= 0:
            isleaf[parent[j]] = False
    return np.nonzero(~isleaf)[0]


def solve_native(parent, nd):
    parent = list(map(int, parent))
    N = len(parent)
    n = nd["Q"].shape[-1]
    m = nd["R"].shape[-1]
    nl = list(nonleaves(parent))
    ch = [[] for _ in range(N)]
    for j in range(N):
        if parent[j] >= 0:
            ch[parent[j]].append(j)
    ix = {v: v * n for v in range(N)}
    off_v = N * n
    iv = {i: off_v + k * m for k, i in enumerate(nl)}
    off_y = off_v + len(nl) * m
    iy = {v: off_y + v * n for v in range(N)}
    dim = off_y + N * n
    K = np.zeros((dim, dim))
    rhs = np.zeros(dim)
    for i in range(N):
        r0 = ix[i]
        K[r0:r0 + n, ix[i]:ix[i] + n] += nd["Q"][i]
        rhs[r0:r0 + n] -= nd["q"][i]
        K[r0:r0 + n, iy[i]:iy[i] + n] -= np.eye(n)
        if i in iv:
            K[r0:r0 + n, iv[i]:iv[i] + m] += nd["M"][i]
        for j in ch[i]:
            K[r0:r0 + n, iy[j]:iy[j] + n] += nd["A"][j].T
    for i in nl:
        r0 = iv[i]
        K[r0:r0 + m, ix[i]:ix[i] + n] += nd["M"][i].T
        K[r0:r0 + m, iv[i]:iv[i] + m] += nd["R"][i]
        rhs[r0:r0 + m] -= nd["r"][i]
        for j in ch[i]:
            K[r0:r0 + m, iy[j]:iy[j] + n] += nd["B"][j].T
    for v in range(N):
        r0 = iy[v]
        i = parent[v]
        if i < 0:
            K[r0:r0 + n, ix[v]:ix[v] + n] -= np.eye(n)
        else:
            K[r0:r0 + n, ix[i]:ix[i] + n] += nd["A"][v]
            K[r0:r0 + n, iv[i]:iv[i] + m] += nd["B"][v]
            K[r0:r0 + n, ix[v]:ix[v] + n] -= np.eye(n)
        K[r0:r0 + n, iy[v]:iy[v] + n] -= nd["Delta"][v]
        rhs[r0:r0 + n] -= nd["c"][v]
    z = np.linalg.solve(K, rhs)
    x = np.stack([z[ix[v]:ix[v] + n] for v in range(N)])
    y = np.stack([z[iy[v]:iy[v] + n] for v in range(N)])
    vv = np.zeros((N, m))
    for i in nl:
        vv[i] = z[iv[i]:iv[i] + m]
    return x, vv, y


def lift(parent, nd):
    """Lifted (parent', data') of Prop. 2 and the decision-node id map."""
    parent = np.asarray(parent, dtype=np.int64)
    N = len(parent)
    n = nd["Q"].shape[-1]
    m = nd["R"].shape[-1]
    nl = nonleaves(parent)
    plus = -np.ones(N, dtype=np.int64)
    plus[nl] = N + np.arange(len(nl))
    NL = N + len(nl)
    d = n + m
    lp = np.empty(NL, dtype=np.int64)
    for i in range(N):
        lp[i] = -1 if parent[i] < 0 else plus[parent[i]]
    for i in nl:
        lp[plus[i]] = i
    Q = np.zeros((NL, d, d)); q = np.zeros((NL, d)); c = np.zeros((NL, d)); De = np.zeros((NL, d, d))
    R = np.zeros((NL, m, m)); S = np.zeros((NL, d, m)); r = np.zeros((NL, m))
    A = np.zeros((NL, d, d)); B = np.zeros((NL, d, m))
    for i in range(N):
        Q[i, :n, :n] = nd["Q"][i]
        q[i, :n] = nd["q"][i]
        c[i, :n] = nd["c"][i]
        De[i, :n, :n] = nd["Delta"][i]
        if parent[i] >= 0:   # uncertainty edge (pa(i))^+ -> i^-
            A[i, :n, :n] = nd["A"][i]
            A[i, :n, n:] = nd["B"][i]
            R[i] = np.eye(m)
        else:
            R[i] = np.eye(m)
    for i in nl:
        k = plus[i]          # decision edge i^- -> i^+
        A[k, :n, :n] = np.eye(n)
        B[k, n:, :] = np.eye(m)
        R[k] = nd["R"][i]
        S[k, :n, :] = nd["M"][i]
        r[k] = nd["r"][i]
    data = {"Q": Q, "q": q, "c": c, "Delta": De, "R": R, "S": S, "r": r, "A": A, "B": B}
    return lp, data, plus


def project(n, plus, x_l, u_l, y_l):
    N = plus.shape[0]
    x = x_l[:N, :n].copy()
    y = y_l[:N, :n].copy()
    m = u_l.shape[-1]
    v = np.zeros((N, m))
    has = plus >= 0
    v[has] = u_l[plus[has]]
    return x, v, y
