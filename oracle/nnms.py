"""FP64 reference for the learned (neural) normalized-offset min-sum decoder.

TEST INFRASTRUCTURE ONLY (imported by the tests and the benchmark's CPU leg,
never by the product).

The decoder keeps the flooding schedule of Algorithm 1 and replaces the
check-node rule (Eq. 3) by a scaled and offset minimum, with one scale w and
one offset b per iteration t and per edge class e -- the neural normalized /
offset min-sum of Nachmani et al. (2016, 2018) and Lugosch & Gross (2017),
with weights shared by the edges of a class:

    alpha_mn = w[t, e] * prod_{n' != n} sgn(beta_mn') * max(min_{n' != n} |beta_mn'| - b[t, e], 0)

where e is the class of edge (m, n) and sgn(x) = -1 for x < 0 and +1
otherwise.  For a QC code (Eq. 2) the class of an edge is its circulant
block: the nonzero blocks of the base matrix numbered row by row, left to
right (18 classes for a full 3 x 6 base).  The variable-node step (Eq. 4,
a direct sum over the other edges), the posterior (Eq. 5), the hard decision
(Eq. 6) and the clip of beta at +-30 are those of the sum-product decoder.
Training loss: binary cross-entropy of every iteration's posterior against the
transmitted bits, averaged over iterations, frames and bits:
    loss = mean_t mean_{g, n} softplus(-x_gn * L_gn^(t)),  x = 1 - 2c.

Written with plain torch operations in float64 on the CPU (gather, scatter,
sort) so that torch's autograd gives the reference gradient; finite
differences pin that gradient in the tests.
"""
from __future__ import annotations

import numpy as np
import torch

LMAX = 30.0


class EdgeGraph:
    """Edges of an explicit parity-check matrix (row-major) with tables of the
    edges of every row and of every column, and each edge's class (edge ids
    in row-major order; default: one class)."""

    def __init__(self, H, edge_class=None):
        rp = np.asarray(H.row_ptr, dtype=np.int64)
        ci = np.asarray(H.col_idx, dtype=np.int64)
        self.n, self.m = H.n, H.m
        self.E = int(rp[-1])
        rows = np.repeat(np.arange(H.m), np.diff(rp))
        self.col = torch.from_numpy(ci)
        # rows: [m, dc] edge ids, -1 padded
        dc = max(int(np.diff(rp).max()) if H.m else 1, 1)
        pos = np.arange(self.E) - np.repeat(rp[:-1], np.diff(rp))
        rt = -np.ones((H.m, dc), dtype=np.int64)
        rt[rows, pos] = np.arange(self.E)
        self.rowtab = torch.from_numpy(rt)
        # columns: [n, dv] edge ids in ascending row order, -1 padded
        order = np.lexsort((rows, ci))
        cnt = np.bincount(ci, minlength=H.n)
        dv = max(int(cnt.max()) if H.n else 1, 1)
        cstart = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        cpos = np.arange(self.E) - np.repeat(cstart, cnt)
        ct = -np.ones((H.n, dv), dtype=np.int64)
        ct[ci[order], cpos] = order
        self.coltab = torch.from_numpy(ct)
        ec = np.zeros(self.E, dtype=np.int64) if edge_class is None else np.asarray(edge_class, dtype=np.int64)
        if ec.shape != (self.E,):
            raise ValueError("one class per edge")
        self.edge_class = torch.from_numpy(ec)


def qc_edge_class(shifts, p: int) -> np.ndarray:
    """Class of every edge of the QC code of `shifts` (row-major edge order,
    as qc_parity_check lays it out): the index of its circulant block among
    the base's nonzero blocks, numbered row by row, left to right.  Row
    (j, s) meets its blocks in increasing base column, which is also the
    order of its columns."""
    a = np.asarray(shifts)
    J, L = a.shape
    block = -np.ones((J, L), dtype=np.int64)
    nz = a >= 0
    block[nz] = np.arange(int(nz.sum()))
    out = []
    for j in range(J):
        row = block[j][block[j] >= 0]
        out.append(np.tile(row, p))
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def check_step(G: EdgeGraph, beta: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """alpha [F, E] from beta [F, E]; w, b [edge classes]."""
    F = beta.shape[0]
    pad = G.rowtab < 0
    mag = beta.abs()[:, G.rowtab.clamp(min=0)]                   # [F, m, dc]
    mag = torch.where(pad, torch.full_like(mag, float("inf")), mag)
    neg = (beta < 0)[:, G.rowtab.clamp(min=0)] & ~pad
    dc = mag.shape[-1]
    other = ~torch.eye(dc, dtype=torch.bool)                     # [dc, dc]: k' != k
    # minimum and sign product over the other edges of the row, taken directly
    excl_min = torch.where(other, mag.unsqueeze(-2), torch.full_like(mag.unsqueeze(-2), float("inf"))).amin(-1)
    excl_neg = (neg.unsqueeze(-2) & other).sum(-1) % 2
    sgn = 1.0 - 2.0 * excl_neg.to(beta.dtype)
    cls = G.edge_class[G.rowtab.clamp(min=0)]                    # [m, dc]
    wr = w[cls].unsqueeze(0)
    br = b[cls].unsqueeze(0)
    a_rows = wr * sgn * torch.clamp(excl_min - br, min=0.0)     # [F, m, dc]
    alpha = torch.zeros((F, G.E), dtype=beta.dtype)
    alpha = alpha.index_put((torch.arange(F).view(-1, 1), G.rowtab[~pad].view(1, -1)), a_rows[:, ~pad])
    return alpha


def variable_step(G: EdgeGraph, mu: torch.Tensor, alpha: torch.Tensor, lmax: float):
    """beta [F, E] (direct sums over the other edges, clipped) and the
    posterior L [F, n]."""
    F = mu.shape[0]
    pad = G.coltab < 0
    a_cols = torch.where(pad, torch.zeros(()), alpha[:, G.coltab.clamp(min=0)])   # [F, n, dv]
    dv = a_cols.shape[-1]
    other = (~torch.eye(dv, dtype=torch.bool)).to(mu.dtype)
    excl = (a_cols.unsqueeze(-2) * other).sum(-1)                # [F, n, dv]
    b_cols = torch.clamp(mu.unsqueeze(-1) + excl, -lmax, lmax)
    L = mu + a_cols.sum(-1)
    beta = torch.zeros((F, G.E), dtype=mu.dtype)
    beta = beta.index_put((torch.arange(F).view(-1, 1), G.coltab[~pad].view(1, -1)), b_cols[:, ~pad])
    return beta, L


def run(G: EdgeGraph, llr, w, b, T: int, lmax: float = LMAX):
    """T iterations of the learned min-sum decoder.  llr [F, n]; w, b [T,
    edge classes].
    Returns the posteriors L^(1..T), each [F, n]."""
    mu = torch.as_tensor(np.asarray(llr), dtype=torch.float64)
    beta = torch.clamp(mu[:, G.col], -lmax, lmax)
    posts = []
    for t in range(T):
        alpha = check_step(G, beta, w[t], b[t])
        beta, L = variable_step(G, mu, alpha, lmax)
        posts.append(L)
    return posts


def iteration_losses(G: EdgeGraph, llr, x, w, b, T: int, lmax: float = LMAX) -> torch.Tensor:
    """[T]: the BCE of each iteration's posterior, averaged over frames and
    bits; x [F, n] = 1 - 2c."""
    xs = torch.as_tensor(np.asarray(x), dtype=torch.float64)
    posts = run(G, llr, w, b, T, lmax)
    return torch.stack([torch.nn.functional.softplus(-xs * L).mean() for L in posts])


def loss(G: EdgeGraph, llr, x, w, b, T: int, lmax: float = LMAX, coef=None):
    """sum_t coef[t] * iteration_losses[t]; coef defaults to 1/T (the mean
    over iterations)."""
    per = iteration_losses(G, llr, x, w, b, T, lmax)
    c = torch.full((T,), 1.0 / T, dtype=torch.float64) if coef is None else \
        torch.as_tensor(np.asarray(coef), dtype=torch.float64)
    return (c * per).sum()


def grad(G: EdgeGraph, llr, x, w, b, T: int, lmax: float = LMAX, coef=None):
    """(loss, dloss/dw, dloss/db) by autograd in float64."""
    wt = torch.tensor(np.asarray(w), dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(np.asarray(b), dtype=torch.float64, requires_grad=True)
    val = loss(G, llr, x, wt, bt, T, lmax, coef)
    val.backward()
    return float(val.detach()), wt.grad.numpy().copy(), bt.grad.numpy().copy()


def decode(G: EdgeGraph, llr, w, b, T: int, lmax: float = LMAX):
    """Posterior (clipped) and hard decisions after T iterations."""
    with torch.no_grad():
        L = run(G, llr, torch.as_tensor(np.asarray(w), dtype=torch.float64),
                torch.as_tensor(np.asarray(b), dtype=torch.float64), T, lmax)[-1]
    L = L.numpy()
    return dict(post=np.clip(L, -lmax, lmax), bits=(L < 0).astype(np.uint8), raw=L)
