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


def cosine_topk_gpu(X, Q, k, chunk=65536, dense_bf16=False, X_dev=None):
    """Top-k ids by cosine similarity for large dense sets: candidates by a
    chunked fp32 scan on the GPU (torch), re-scored exactly in FP64 on the
    host.  X, Q are host arrays (fp32, or bf16 bit patterns if dense_bf16);
    X_dev, if given, is the same data already on the device (the scan then
    reads it there)."""
    import torch

    def dev_chunk(s):
        if X_dev is None:
            return torch.from_numpy(to_f32(X[s:s + chunk])).cuda()
        c = X_dev[s:s + chunk]
        if dense_bf16:
            return ((c.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)
        return c.float()

    def to_f32(a):
        a = np.ascontiguousarray(a)
        if dense_bf16:
            return (a.astype(np.uint32) << np.uint32(16)).view(np.float32)
        return a.astype(np.float32)

    Qh = to_f32(Q).astype(np.float64)
    Qd = torch.from_numpy(to_f32(Q)).cuda()
    Qd = Qd / Qd.norm(dim=1, keepdim=True).clamp_min(1e-30)
    kk = k + 16
    best_s = torch.full((Qd.shape[0], 0), -2.0, device="cuda")
    best_i = torch.zeros((Qd.shape[0], 0), dtype=torch.int64, device="cuda")
    for s in range(0, X.shape[0], chunk):
        Xc = dev_chunk(s)
        Xc = Xc / Xc.norm(dim=1, keepdim=True).clamp_min(1e-30)
        S = Qd @ Xc.T
        v, i = torch.topk(S, min(kk, S.shape[1]), dim=1)
        best_s = torch.cat([best_s, v], dim=1)
        best_i = torch.cat([best_i, i + s], dim=1)
        v, o = torch.topk(best_s, min(kk, best_s.shape[1]), dim=1)
        best_s, best_i = v, torch.gather(best_i, 1, o)
    cand = best_i.cpu().numpy()
    out_i = np.zeros((Qh.shape[0], k), dtype=np.int64)
    out_s = np.zeros((Qh.shape[0], k))
    qn = Qh / np.maximum(np.linalg.norm(Qh, axis=1, keepdims=True), 1e-300)
    for q in range(Qh.shape[0]):
        C = to_f32(X[cand[q]]).astype(np.float64)
        sc = (C / np.maximum(np.linalg.norm(C, axis=1, keepdims=True), 1e-300)) @ qn[q]
        o = np.lexsort((cand[q], -sc))[:k]
        out_i[q], out_s[q] = cand[q][o], sc[o]
    return out_i, out_s


def recall_at(found, truth_top1):
    """R1@k: fraction of queries whose exact nearest neighbour is among the k
    returned ids."""
    found = np.asarray(found)
    t = np.asarray(truth_top1).reshape(-1, 1)
    return float(np.mean(np.any(found == t, axis=1)))
