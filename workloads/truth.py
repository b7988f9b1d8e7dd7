"""Exact nearest neighbours by brute force, for recall (not for parity).

Cosine for dense rows (FP64), Jaccard for item sets through an inverted index
over items (the paper computed its URL and genome ground truth the same way,
Appendix "Hyperparameters").  Ties break by ascending id.
"""
import numpy as np


def cosine_topk(X, Q, k, chunk=65536):
    """Top-k ids by cosine similarity.  X, Q: float arrays (FP64 math)."""
    Qn = np.asarray(Q, dtype=np.float64)
    Qn = Qn / np.maximum(np.linalg.norm(Qn, axis=1, keepdims=True), 1e-300)
    nq = Qn.shape[0]
    best_s = np.full((nq, 0), -np.inf)
    best_i = np.zeros((nq, 0), dtype=np.int64)
    for s in range(0, X.shape[0], chunk):
        Xc = np.asarray(X[s:s + chunk], dtype=np.float64)
        Xc = Xc / np.maximum(np.linalg.norm(Xc, axis=1, keepdims=True), 1e-300)
        S = Qn @ Xc.T
        ids = np.broadcast_to(np.arange(s, s + Xc.shape[0]), S.shape)
        allS = np.concatenate([best_s, S], axis=1)
        allI = np.concatenate([best_i, ids], axis=1)
        o = np.lexsort((allI, -allS), axis=1)[:, :k]
        best_s = np.take_along_axis(allS, o, axis=1)
        best_i = np.take_along_axis(allI, o, axis=1)
    return best_i, best_s


class JaccardIndex:
    """Inverted index over items for exact Jaccard search."""

    def __init__(self, items, offsets):
        offsets = np.asarray(offsets, dtype=np.int64)
        self.sizes = np.diff(offsets)
        owner = np.repeat(np.arange(len(self.sizes), dtype=np.int64), self.sizes)
        order = np.argsort(items, kind="stable")
        self.items = np.asarray(items)[order]
        self.owner = owner[order]

    def topk(self, qitems, qoffsets, k):
        qoffsets = np.asarray(qoffsets, dtype=np.int64)
        nq = len(qoffsets) - 1
        out_i = np.full((nq, k), -1, dtype=np.int64)
        out_s = np.zeros((nq, k))
        for q in range(nq):
            its = np.asarray(qitems[qoffsets[q]:qoffsets[q + 1]])
            lo = np.searchsorted(self.items, its, side="left")
            hi = np.searchsorted(self.items, its, side="right")
            if len(its) == 0 or (hi - lo).sum() == 0:
                continue
            cand = np.concatenate([self.owner[a:b] for a, b in zip(lo, hi)])
            u, inter = np.unique(cand, return_counts=True)
            J = inter / (len(its) + self.sizes[u] - inter)
            o = np.lexsort((u, -J))[:k]
            out_i[q, :len(o)] = u[o]
            out_s[q, :len(o)] = J[o]
        return out_i, out_s


def recall_at(found, truth_top1):
    """R1@k: fraction of queries whose exact nearest neighbour is among the k
    returned ids."""
    found = np.asarray(found)
    t = np.asarray(truth_top1).reshape(-1, 1)
    return float(np.mean(np.any(found == t, axis=1)))
