"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def colrel(a, b):
    """max over columns of |a_j - b_j| / |b_j|"""
    a = np.asarray(a).reshape(len(a), -1); b = np.asarray(b).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))


def oracle_skeletons(o, rank, cmax):
    """Oracle skeletons in the exchange format of askit_skeletons_import."""
    nn = o.nnodes
    ids = np.full(nn * rank, -1, dtype=np.int32)
    P = np.zeros(nn * rank * cmax)
    sizes = np.zeros(2 * nn, dtype=np.int32)
    for node in range(1, nn):
        pos, Pn, _ = o.skeleton(node)
        sr, nc = Pn.shape
        ids[node * rank: node * rank + sr] = pos
        P[node * rank * cmax: node * rank * cmax + sr * nc] = Pn.ravel()
        sizes[2 * node] = sr
        sizes[2 * node + 1] = nc
    return ids, P, sizes


def skeleton_agreement(o, ids, P, sizes, rank, cmax):
    """(#nodes with identical skeletons, #nodes, max |P - P_oracle| over those nodes)"""
    same, worst = 0, 0.0
    for node in range(1, o.nnodes):
        pos, Pn, _ = o.skeleton(node)
        sr, nc = Pn.shape
        if sizes[2 * node] != sr or sizes[2 * node + 1] != nc:
            continue
        if not np.array_equal(ids[node * rank: node * rank + sr], pos):
            continue
        same += 1
        Pg = P[node * rank * cmax: node * rank * cmax + sr * nc].reshape(sr, nc)
        worst = max(worst, float(np.max(np.abs(Pg - Pn))) if Pn.size else 0.0)
    return same, o.nnodes - 1, worst


def id_residual(orc_mod, o, X, h, node, P, seed, problem=0):
    """|M - M[:, skel] P|_F / |M|_F for the oracle's sampled block M = K(X_S', X_C)
    of `node` and a projection P (s_alpha x |C|) whose skeleton columns are the
    candidates where P has an identity column."""
    b, e = o.node_range(node)
    q = orc_mod.sample(seed, problem, node, o.N, b, e, o.nsamp)
    perm = o.perm()
    cand = o.candidates(node)
    M = orc_mod.kernel_matrix(X, h, perm[q], perm[cand])
    pos, _, _ = o.skeleton(node)
    cols = [int(np.where(cand == p)[0][0]) for p in pos]
    return float(np.linalg.norm(M - M[:, cols] @ P) / np.linalg.norm(M))
