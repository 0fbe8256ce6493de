"""Seeded synthetic inputs: tree topologies and tree-LQR data.

This module only draws random numbers and builds arrays.  It contains none of
the solver's arithmetic, so both the GPU path and the CPU checker can consume
the same inputs without sharing any part of the method.

Data layout (the one the C-ABI takes, all float64, row-major):
  per node i      Q[N,n,n]  q[N,n]  c[N,n]  Delta[N,n,n]
  per edge slot j R[N,m,m]  S[N,n,m]  r[N,m]  A[N,n,n]  B[N,n,m]
The edge (parent[j], j) lives in slot j; the root's edge slot is unused and
filled with harmless values (R = I, everything else zero).

The data model is the edge-control normal form of Sec. II-A (Lagrangian
eq. (lagrangian)); `S` is the paper's cross term M_e and `Delta` the node dual
regulariser.  Distributions follow the benchmark configurations:
  Q = G G^T / n + 0.1 I,  G iid N(0,1)          q ~ N(0,1)
  A = I + 0.1 G / sqrt(n)                        B ~ N(0,1) / sqrt(n)
  R = W W^T / m + I                              r ~ N(0,1)
  c ~ N(0, 0.01) (variance 0.01, sigma 0.1)      S = 0 unless requested
  Delta = 0, or rank-k PSD  V diag(lam) V^T with V from a QR of an n x k
  Gaussian and lam ~ U(0, delta_scale).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FIELDS_NODE = ("Q", "q", "c", "Delta")
FIELDS_EDGE = ("R", "S", "r", "A", "B")
FIELDS = FIELDS_NODE + FIELDS_EDGE


def config_seed(config: int, resolve: int = 0, tree: int = 0) -> int:
    """Seed of tree `tree`, re-solve `resolve` of benchmark configuration `config`."""
    return 20260000 + 100000 * config + 1000 * resolve + tree


# --------------------------------------------------------------------------- trees
def tree_chainprob(N: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """parent[0] = -1; for i >= 1, parent[i] = i-1 with probability p, else
    uniform on {0, ..., i-1} (inclusive)."""
    parent = np.empty(N, dtype=np.int64)
    parent[0] = -1
    if N == 1:
        return parent
    i = np.arange(1, N, dtype=np.int64)
    chain = rng.random(N - 1) < p
    unif = np.floor(rng.random(N - 1) * i).astype(np.int64)
    unif = np.minimum(unif, i - 1)
    parent[1:] = np.where(chain, i - 1, unif)
    return parent


def tree_chain(N: int) -> np.ndarray:
    parent = np.arange(-1, N - 1, dtype=np.int64)
    return parent


def tree_star(N: int) -> np.ndarray:
    parent = np.zeros(N, dtype=np.int64)
    parent[0] = -1
    return parent


def tree_balanced(N: int) -> np.ndarray:
    """Complete binary tree in heap order: parent(i) = (i-1)//2."""
    parent = (np.arange(N, dtype=np.int64) - 1) // 2
    parent[0] = -1
    return parent


def tree_comb(N: int) -> np.ndarray:
    """A trunk 0 -> 2 -> 4 -> ... with one side leaf 2k+1 hanging off trunk node 2k."""
    parent = np.empty(N, dtype=np.int64)
    parent[0] = -1
    for i in range(1, N):
        parent[i] = i - 1 if i % 2 == 1 else i - 2
    return parent


def tree_caterpillar(trunk: int, legs: int) -> np.ndarray:
    """Trunk 0 -> 1 -> ... -> trunk-1; every trunk node carries `legs` leaves."""
    N = trunk * (1 + legs)
    parent = np.empty(N, dtype=np.int64)
    parent[0] = -1
    parent[1:trunk] = np.arange(0, trunk - 1)
    parent[trunk:] = np.repeat(np.arange(trunk, dtype=np.int64), legs)
    return parent


def tree_star_heavy(chains: int, lengths: np.ndarray) -> np.ndarray:
    """Root with `chains` children, child c heading a chain of lengths[c] nodes."""
    lengths = np.asarray(lengths, dtype=np.int64)
    assert lengths.shape == (chains,)
    N = 1 + int(lengths.sum())
    parent = np.empty(N, dtype=np.int64)
    parent[0] = -1
    pos = 1
    for c in range(chains):
        L = int(lengths[c])
        parent[pos] = 0
        if L > 1:
            parent[pos + 1:pos + L] = np.arange(pos, pos + L - 1)
        pos += L
    return parent


def star_heavy_1m() -> np.ndarray:
    """Root + 10,000 chains: 8,575 chains of 105 nodes and 1,425 of 104 (N = 1,048,576)."""
    lengths = np.array([105] * 8575 + [104] * 1425, dtype=np.int64)
    return tree_star_heavy(10000, lengths)


def lemma2_tight_tree(k: int) -> np.ndarray:
    """Unary root above a full binary tree with k leaves (k a power of two), each
    of those leaves given one extra child; 3k nodes in total (Lemma 2)."""
    assert k >= 1 and (k & (k - 1)) == 0
    # node 0: root; node 1..(2k-1): heap-ordered full binary tree, node 1 its root
    nb = 2 * k - 1
    parent = [-1]
    for h in range(1, nb + 1):
        parent.append(0 if h == 1 else h // 2)
    first_leaf = k  # heap leaves are k..2k-1
    for leaf in range(first_leaf, 2 * k):
        parent.append(leaf)
    return np.asarray(parent, dtype=np.int64)


def permute_labels(parent: np.ndarray, rng: np.random.Generator):
    """Relabel nodes by a random permutation; returns (new_parent, perm) with
    new id = perm[old id]."""
    N = parent.shape[0]
    perm = rng.permutation(N).astype(np.int64)
    newp = np.empty(N, dtype=np.int64)
    old = np.arange(N)
    newp[perm[old]] = np.where(parent >= 0, perm[np.maximum(parent, 0)], -1)
    return newp, perm


def tree_stats(parent: np.ndarray) -> dict:
    """Height, leaf fraction and maximum out-degree of a parent array (integer work only)."""
    N = parent.shape[0]
    deg = np.bincount(parent[parent >= 0], minlength=N)
    # depth by repeated parent lookups over a topological order (BFS)
    order = bfs_order(parent)
    depth = np.zeros(N, dtype=np.int64)
    for v in order[1:]:
        depth[v] = depth[parent[v]] + 1
    return {"N": int(N), "height": int(depth.max()) if N else 0,
            "leaves": int((deg == 0).sum()), "max_degree": int(deg.max()) if N else 0}


def bfs_order(parent: np.ndarray) -> np.ndarray:
    N = parent.shape[0]
    roots = np.nonzero(parent < 0)[0]
    assert roots.shape[0] == 1
    kids = np.argsort(np.where(parent < 0, -1, parent), kind="stable")
    counts = np.bincount(parent[parent >= 0], minlength=N)
    start = np.zeros(N + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    kids = kids[1:]  # drop the root (its key -1 sorts first)
    order = np.empty(N, dtype=np.int64)
    order[0] = roots[0]
    head, tail = 0, 1
    while head < tail:
        v = order[head]
        head += 1
        ch = kids[start[v]:start[v + 1]]
        order[tail:tail + ch.shape[0]] = ch
        tail += ch.shape[0]
    assert tail == N, "parent array is not a single rooted tree"
    return order


# --------------------------------------------------------------------------- data
@dataclass
class DataSpec:
    n: int
    m: int
    delta_rank: int = 0          # 0: Delta = 0; k: rank-k PSD Delta at every node
    delta_scale: float = 1e-2    # eigenvalues of Delta ~ U(0, delta_scale)
    cross: bool = False          # S != 0 (kept within the convexity assumptions)


def _spd_sym(G: np.ndarray, scale: float, shift: float) -> np.ndarray:
    return np.einsum("nij,nkj->nik", G, G) * scale + shift * np.eye(G.shape[-1])


def lqr_data(parent: np.ndarray, spec: DataSpec, rng: np.random.Generator) -> dict:
    """Random tree-LQR data satisfying the standing convexity assumptions
    (Definition 1): R > 0, Delta >= 0, Q_i - sum_out S R^-1 S^T >= 0."""
    N = parent.shape[0]
    n, m = spec.n, spec.m
    G = rng.standard_normal((N, n, n))
    Q = _spd_sym(G, 1.0 / n, 0.1)
    q = rng.standard_normal((N, n))
    c = rng.standard_normal((N, n)) * 0.1
    A = np.eye(n)[None] + 0.1 * rng.standard_normal((N, n, n)) / math.sqrt(n)
    B = rng.standard_normal((N, n, m)) / math.sqrt(n)
    Wm = rng.standard_normal((N, m, m))
    R = _spd_sym(Wm, 1.0 / m, 1.0)
    r = rng.standard_normal((N, m))
    Delta = np.zeros((N, n, n))
    k = spec.delta_rank
    if k > 0:
        V, _ = np.linalg.qr(rng.standard_normal((N, n, k)))
        lam = rng.random((N, k)) * spec.delta_scale
        Delta = np.einsum("nik,nk,njk->nij", V, lam, V)
    S = np.zeros((N, n, m))
    if spec.cross:
        # S_e = L_Q(i) Xi L_R(e)^T / (2 sqrt(deg i)), ||Xi||_2 <= 1, so that
        # sum over the deg(i) children of S R^-1 S^T <= Q_i / 4.
        deg = np.bincount(parent[parent >= 0], minlength=N)
        LQ = np.linalg.cholesky(Q)
        LR = np.linalg.cholesky(R)
        Xi = rng.standard_normal((N, n, m))
        Xi /= np.linalg.norm(Xi, ord=2, axis=(1, 2))[:, None, None]
        par = np.maximum(parent, 0)
        S = np.einsum("nij,njk,nlk->nil", LQ[par], Xi, LR)
        S /= (2.0 * np.sqrt(np.maximum(deg[par], 1)))[:, None, None]
    root = int(np.nonzero(parent < 0)[0][0])
    # root edge slot is unused: make it inert
    R[root] = np.eye(m)
    S[root] = 0.0
    r[root] = 0.0
    A[root] = 0.0
    B[root] = 0.0
    return {"Q": Q, "q": q, "c": c, "Delta": Delta,
            "R": R, "S": S, "r": r, "A": A, "B": B}


def table2_data(parent: np.ndarray, n: int, m: int, rng: np.random.Generator) -> dict:
    """The synthetic-benchmark data of Sec. XI-A: Q = 2I, R = I, Delta = 0.02 I,
    remaining arrays pseudorandom (here: the lqr_data distributions)."""
    d = lqr_data(parent, DataSpec(n, m), rng)
    N = parent.shape[0]
    d["Q"] = np.broadcast_to(2.0 * np.eye(n), (N, n, n)).copy()
    d["R"] = np.broadcast_to(np.eye(m), (N, m, m)).copy()
    d["Delta"] = np.broadcast_to(0.02 * np.eye(n), (N, n, n)).copy()
    return d


def config_instance(config: int, resolve: int = 0, tree: int = 0):
    """(parent, data, spec) of one synthetic benchmark instance.

    1: N=255,  p=0.9,  n=4,  m=2, Delta = 0
    2: N=65,536, p=0.95, n=12, m=4, Delta rank 6, eigenvalues U(0, 1e-2)
    3: tree t of 512: N log-uniform in [256, 16384], p ~ U(0.8, 0.98), n=8, m=3
    4: a/b/c shape extremes at N=1,048,576, n=6, m=2 (use shape_extreme())
    """
    seed = config_seed(config, resolve, tree)
    rng = np.random.default_rng(seed)
    if config == 1:
        parent = tree_chainprob(255, 0.9, rng)
        spec = DataSpec(4, 2)
    elif config == 2:
        parent = tree_chainprob(65536, 0.95, rng)
        spec = DataSpec(12, 4, delta_rank=6, delta_scale=1e-2)
    elif config == 3:
        N = int(round(math.exp(rng.uniform(math.log(256), math.log(16384)))))
        p = rng.uniform(0.8, 0.98)
        parent = tree_chainprob(N, p, rng)
        spec = DataSpec(8, 3)
    else:
        raise ValueError("config 4 instances come from shape_extreme(); 5 from the serving workload")
    # data for a re-solve is drawn from its own stream so the topology can be reused
    drng = np.random.default_rng(seed + 7919)
    return parent, lqr_data(parent, spec, drng), spec


def shape_extreme(kind: str) -> np.ndarray:
    """Topologies of the N = 1,048,576 shape-extreme workload."""
    if kind == "caterpillar":
        return tree_caterpillar(262144, 3)
    if kind == "star_heavy":
        return star_heavy_1m()
    if kind == "chainprob":
        return tree_chainprob(1048576, 0.9, np.random.default_rng(config_seed(4, 0, 2)))
    raise ValueError(kind)


def native_node_control_data(parent: np.ndarray, spec: DataSpec, rng: np.random.Generator) -> dict:
    """Data of the native node-control problem of Sec. II-B (eq. (node-lagrangian)).

    Per node: Q, q, c, Delta (as in lqr_data) and, used at non-leaf nodes only,
    the control cost M[N,n,m], R[N,m,m], r[N,m]; per edge slot j: A, B of the
    transition x_j = A_ij x_i + B_ij v_i + c_j.  M = 0 unless spec.cross, in
    which case M_i = L_Q Xi L_R^T / 2 keeps Q_i - M_i R_i^-1 M_i^T >= 0
    (eq. (native-assumptions))."""
    d = lqr_data(parent, DataSpec(spec.n, spec.m, spec.delta_rank, spec.delta_scale, False), rng)
    N = parent.shape[0]
    n, m = spec.n, spec.m
    M = np.zeros((N, n, m))
    if spec.cross:
        LQ = np.linalg.cholesky(d["Q"])
        LR = np.linalg.cholesky(d["R"])
        Xi = rng.standard_normal((N, n, m))
        Xi /= np.linalg.norm(Xi, ord=2, axis=(1, 2))[:, None, None]
        M = np.einsum("nij,njk,nlk->nil", LQ, Xi, LR) / 2.0
    return {"Q": d["Q"], "q": d["q"], "c": d["c"], "Delta": d["Delta"],
            "M": M, "R": d["R"], "r": d["r"], "A": d["A"], "B": d["B"]}


# --------------------------------------------------------------------------- serving stream
def serve_requests(count: int, rate: float, seed: int, n_choices=(4, 8, 12, 16), m_choices=(2, 4),
                   N_range=(1024, 131072), p_range=(0.85, 0.97), reuse: float = 0.3) -> list:
    """A stream of tree-LQR solve requests with Poisson arrivals at `rate` per
    second.  A fresh request draws N log-uniform in N_range, n and m uniformly
    from their choices and a chain probability p ~ U(p_range); with
    probability `reuse` a request instead resends the topology (and n, m) of an
    earlier request, uniformly chosen, with new data.  Each entry: rid,
    arrival (s), topo (topology id), N, n, m, p, tree_seed, variant (which data
    variant of its (n, m) class it uses; a resend takes the other variant than
    the request it resends), resend_of (that request's rid, or -1)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(count):
        if out and rng.random() < reuse:
            prev = out[int(rng.integers(0, len(out)))]
            e = dict(prev)
            e.update(rid=k, arrival=float(t[k]), variant=1 - prev["variant"], resend_of=prev["rid"])
        else:
            N = int(round(math.exp(rng.uniform(math.log(N_range[0]), math.log(N_range[1])))))
            e = {"rid": k, "arrival": float(t[k]), "topo": k, "N": N,
                 "n": int(rng.choice(n_choices)), "m": int(rng.choice(m_choices)),
                 "p": float(rng.uniform(*p_range)), "tree_seed": seed * 1000003 + k, "variant": 0,
                 "resend_of": -1}
        out.append(e)
    return out


def serve_tree(e: dict) -> np.ndarray:
    """The parent array of a serving request (root 0)."""
    return tree_chainprob(e["N"], e["p"], np.random.default_rng(e["tree_seed"]))


def serve_data_block(N: int, n: int, m: int, variant: int, seed: int) -> dict:
    """Data of the (n, m) class, variant `variant`, for N nodes with root 0: a
    request of N' <= N nodes whose root is node 0 uses rows [0, N').  Rank n/2
    PSD dual regularisation with eigenvalues U(0, 1e-2), S = 0; the root's edge
    slot is inert.  Rows of an edge slot do not depend on the topology, so one
    block serves every tree of the class."""
    par = np.arange(-1, N - 1, dtype=np.int64)  # any tree with root 0: only the root row is special
    return lqr_data(par, DataSpec(n, m, delta_rank=max(1, n // 2)),
                    np.random.default_rng(seed * 97 + 13 * n + m + 1000 * variant))


def config2_lift_instance(resolve: int = 0):
    """The one-control-per-information-node variant of the 65,536-node instance:
    the same tree (p = 0.95) and distributions (n = 12, m = 4, rank-6 PSD
    Delta), as a native node-control problem with M_i = 0, lifted to state 16."""
    seed = config_seed(2, resolve, 0)
    parent = tree_chainprob(65536, 0.95, np.random.default_rng(seed))
    data = native_node_control_data(parent, DataSpec(12, 4, delta_rank=6, delta_scale=1e-2),
                                    np.random.default_rng(seed + 104729))
    return parent, data


# --------------------------------------------------------------------------- ragged
def ragged_instance(N: int, nmax: int, mmax: int, rng: np.random.Generator, p: float = 0.9, delta: bool = True,
                    cross: bool = True, nmin: int = 1, mmin: int = 1):
    """A tree with per-node state dimensions n_v in [nmin, nmax] and per-edge
    control dimensions m_v in [mmin, mmax] (m at the root: 0), and data as lists
    of per-node blocks with the distributions of lqr_data (A_e = the n_j x n_i
    corner of I plus 0.1 G / sqrt(n_i); S_e = L_Q Xi L_R^T / (2 sqrt(deg)) keeps
    Definition 1).  Returns (parent, n_node, m_edge, blocks)."""
    parent = tree_chainprob(N, p, rng)
    n_node = rng.integers(nmin, nmax + 1, size=N).astype(np.int32)
    m_edge = rng.integers(mmin, mmax + 1, size=N).astype(np.int32)
    m_edge[parent < 0] = 0
    deg = np.bincount(parent[parent >= 0], minlength=N)
    d = {k: [] for k in ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")}
    for v in range(N):
        nv, mv = int(n_node[v]), int(m_edge[v])
        pv = int(parent[v])
        npar = int(n_node[pv]) if pv >= 0 else 0
        G = rng.standard_normal((nv, nv))
        d["Q"].append(G @ G.T / nv + 0.1 * np.eye(nv))
        d["q"].append(rng.standard_normal(nv))
        d["c"].append(rng.standard_normal(nv) * 0.1)
        if delta and nv > 1:
            k = nv // 2
            V, _ = np.linalg.qr(rng.standard_normal((nv, k)))
            d["Delta"].append(V @ np.diag(rng.random(k) * 1e-2) @ V.T)
        else:
            d["Delta"].append(np.zeros((nv, nv)))
        d["A"].append(np.eye(nv, npar) + 0.1 * rng.standard_normal((nv, npar)) / np.sqrt(max(npar, 1)))
        d["B"].append(rng.standard_normal((nv, mv)) / np.sqrt(nv))
        Wm = rng.standard_normal((mv, mv))
        d["R"].append(Wm @ Wm.T / max(mv, 1) + np.eye(mv))
        d["r"].append(rng.standard_normal(mv))
        d["S"].append(np.zeros((npar, mv)))
    if cross:
        for v in range(N):
            pv = int(parent[v])
            if pv < 0:
                continue
            LQ = np.linalg.cholesky(d["Q"][pv])
            LR = np.linalg.cholesky(d["R"][v])
            Xi = rng.standard_normal((LQ.shape[0], LR.shape[0]))
            Xi /= np.linalg.norm(Xi, ord=2)
            d["S"][v] = LQ @ Xi @ LR.T / (2.0 * np.sqrt(max(deg[pv], 1)))
    return parent, n_node, m_edge, d


def pack_ragged(blocks: dict) -> dict:
    """Packed arrays of a ragged problem (the blocks of every node, row-major, one
    after another in node order: the layout of rcr_ragged_solve)."""
    return {k: (np.concatenate([np.ravel(b) for b in v]) if v else np.zeros(0)) for k, v in blocks.items()}


def unpack_ragged(flat: np.ndarray, shapes) -> list:
    """The per-node blocks of a packed array, given each block's shape."""
    out, at = [], 0
    for sh in shapes:
        size = int(np.prod(sh)) if len(sh) else 1
        out.append(flat[at:at + size].reshape(sh))
        at += size
    return out
