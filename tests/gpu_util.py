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


EPS = 2.0 ** -52


def skeleton_parity(orc_mod, o, X, h, seed, ids, P, sizes, rank, cmax, problem=0, tau=0.0, sampler=None):
    """Node-by-node comparison of exported GPU skeletons with the oracle's,
    from the leaves up.  A node is compared when its candidates agree (a leaf,
    or an internal node whose children both matched).  On each such node the
    oracle's sampled block M is formed again (oracle sampling and kernel, no
    GPU value) and factored by the oracle's pivoted QR; then:
      - identical skeletons: the GPU's P leaves the ID residual
        |M - M[:, skel] P|_F of the oracle's P (the two differ only through
        the rounding of T = R11^-1 R12, and |R11 dT| is at rounding level
        whatever cond(R11) is); where cond(R11) is moderate, P must also agree
        element by element within 256 u cond(R11) (1 + max|T|);
      - different skeletons: the first differing pivot must be a near-tie,
        its column's trailing norm (orthogonal to the earlier pivots) within
        1e-12 |M|_F of the oracle's pivot's, or the ranks differ at a
        diagonal entry that lies within 1e-12 |M|_F of the stopping
        threshold.
    sampler(node), if given, returns the oracle's sampled rows of a node
    (neighbour sampling); else the uniform sampler is used.
    Returns a report; failures lists the nodes that break these rules."""
    perm = o.perm()
    nn, D = o.nnodes, o.D
    ok = np.zeros(nn, dtype=bool)
    rep = dict(compared=0, identical=0, near_tie=0, elementwise=0, worst_dP_over_bar=0.0,
               worst_resid_excess=0.0, failures=[])
    for node in range(nn - 1, 0, -1):
        leaf = node >= (1 << D) - 1
        if not leaf and not (ok[2 * node + 1] and ok[2 * node + 2]):
            continue
        rep["compared"] += 1
        pos_o, P_o, _ = o.skeleton(node)
        sr_o, nc = P_o.shape
        sr_g, nc_g = int(sizes[2 * node]), int(sizes[2 * node + 1])
        if nc_g != nc:
            rep["failures"].append((node, "candidate count", nc_g, nc))
            continue
        ids_g = np.asarray(ids[node * rank: node * rank + sr_g], dtype=np.int64)
        Pg = np.asarray(P[node * rank * cmax: node * rank * cmax + sr_g * nc]).reshape(sr_g, nc)
        cand = o.candidates(node)
        if nc <= rank:  # P = I, no QR
            same = sr_g == nc and np.array_equal(ids_g, cand) and np.array_equal(Pg, np.eye(nc))
            ok[node] = same
            rep["identical"] += int(same)
            if not same:
                rep["failures"].append((node, "identity skeleton differs"))
            continue
        b, e = o.node_range(node)
        q = sampler(node) if sampler else orc_mod.sample(seed, problem, node, o.N, b, e, o.nsamp)
        M = orc_mod.kernel_matrix(X, h, perm[q], perm[cand])
        nM = np.linalg.norm(M)
        rk, piv, rd, T, R, tr = orc_mod.qrcp(M, min(rank, nc), tau)
        assert rk == sr_o and np.array_equal(cand[piv[:rk]], pos_o)  # the oracle reproduces itself
        if sr_g == sr_o and np.array_equal(ids_g, pos_o):
            ok[node] = True
            rep["identical"] += 1
            sk = piv[:rk]
            eo = np.linalg.norm(M - M[:, sk] @ P_o)
            eg = np.linalg.norm(M - M[:, sk] @ Pg)
            excess = (eg - eo) / nM
            rep["worst_resid_excess"] = max(rep["worst_resid_excess"], excess)
            if excess > 1e-12:
                rep["failures"].append((node, "ID residual", eg / nM, eo / nM))
            kap = np.linalg.cond(R[:rk, :rk])
            bar = 256 * EPS * kap * (1.0 + (np.abs(T).max() if T.size else 0.0))
            if bar <= 1e-6:
                rep["elementwise"] += 1
                dP = np.abs(Pg - P_o).max()
                rep["worst_dP_over_bar"] = max(rep["worst_dP_over_bar"], dP / bar)
                if dP > bar:
                    rep["failures"].append((node, "P elementwise", dP, bar))
            continue
        # first differing step
        m = min(sr_g, sr_o)
        diff = np.nonzero(ids_g[:m] != pos_o[:m])[0]
        j = int(diff[0]) if diff.size else m
        rep["near_tie"] += 1
        if j < m:
            Qj = np.linalg.qr(M[:, piv[:j]])[0] if j else np.zeros((M.shape[0], 0))
            col = {int(c): k for k, c in enumerate(cand)}
            co, cg = col[int(pos_o[j])], col.get(int(ids_g[j]), -1)
            if cg < 0:
                rep["failures"].append((node, "GPU pivot not a candidate", int(ids_g[j])))
                continue
            rn = lambda c: np.linalg.norm(M[:, c] - Qj @ (Qj.T @ M[:, c]))
            gap = abs(rn(co) - rn(cg))
            if gap > 1e-12 * nM:
                rep["failures"].append((node, "pivot", j, gap / nM))
        else:
            # one rank is a prefix of the other: the stopping rule decided
            # differently at step m; |R_mm| must sit at the threshold
            Qj = np.linalg.qr(M[:, piv[:m]])[0]
            nxt = pos_o[m] if sr_o > m else ids_g[m]
            c = {int(cc): k for k, cc in enumerate(cand)}[int(nxt)]
            rmm = np.linalg.norm(M[:, c] - Qj @ (Qj.T @ M[:, c]))
            thr = max(1e-14, tau) * abs(rd[0])
            if abs(rmm - thr) > 1e-12 * nM:
                rep["failures"].append((node, "rank", sr_g, sr_o, rmm / nM, thr / nM))
    return rep
