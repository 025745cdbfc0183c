"""FP64 reference for the batched LDPC / LDPC-convolutional-code decoder.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this package: only
the test suite, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the GPU library; the two meet only in the seeded inputs
from `synth`.

Contents
  * graph construction written from the paper:
      - `qc_parity_check` -- Eq. 2: H is a J x L array of p x p circulants,
        block (j, l) being the identity with its columns shifted cyclically to
        the right a[j][l] times (a = -1: zero block);
      - `unwrap_qc` -- Sec. II-D: partition H_QC into Lambda x Lambda
        sub-blocks (Lambda = gcd(J, L)), split it into the lower part (diagonal
        included) and the strictly upper part, paste the upper part below the
        lower part and repeat the pair down the diagonal; terminated after a
        number of code positions;
      - `edge_lookup_tables` -- the LUT_c / LUT_v index tables of Sec. IV-A
        for message packages stored row by row, left to right;
  * `decode_block` / `decode_window` / `decode_pipeline` -- ctypes wrappers of
    the C decoders in bp.c (Algorithm 1 in FP64; the sliding-window schedule
    and the pipelined schedule of Algorithm 2 for the terminated
    convolutional code);
  * `map_decode` -- bitwise MAP by enumerating every codeword (tiny codes).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

LMAX = 30.0


# ----------------------------------------------------------------------------
# graph construction
# ----------------------------------------------------------------------------

class SparseH:
    """Explicit parity-check matrix in compressed rows (ascending columns)."""

    def __init__(self, n: int, m: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        self.n, self.m = int(n), int(m)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.layer_of_row = None
        self.pos_of_col = None
        self.nlayers = 0
        self.npos = 0

    @property
    def ne(self) -> int:
        return int(self.row_ptr[-1])

    @classmethod
    def from_dense(cls, H) -> "SparseH":
        H = np.asarray(H, dtype=np.uint8)
        m, n = H.shape
        rows, cols = np.nonzero(H)
        rp = np.zeros(m + 1, dtype=np.int32)
        np.add.at(rp, rows + 1, 1)
        return cls(n, m, np.cumsum(rp).astype(np.int32), cols.astype(np.int32))

    def dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.uint8)
        for r in range(self.m):
            H[r, self.col_idx[self.row_ptr[r]:self.row_ptr[r + 1]]] = 1
        return H

    def syndrome(self, bits: np.ndarray) -> np.ndarray:
        """H c^T (mod 2) for bits [gamma, n] -> [gamma, m]."""
        b = np.asarray(bits, dtype=np.uint8)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        out = np.zeros((b.shape[0], self.m), dtype=np.int64)
        for g in range(b.shape[0]):
            np.add.at(out[g], rows, b[g, self.col_idx])
        return (out & 1).astype(np.uint8)


def circulant(a: int, p: int) -> np.ndarray:
    """p x p circulant permutation of Eq. 2: the identity with its columns
    shifted cyclically right a times (row r has its one at column (r+a) mod p);
    a = -1 is the zero matrix."""
    P = np.zeros((p, p), dtype=np.uint8)
    if a >= 0:
        P[np.arange(p), (np.arange(p) + a) % p] = 1
    return P


def qc_parity_check(shifts, p: int) -> SparseH:
    """Eq. 2, built sparsely: block (j, l) contributes rows j*p + r, columns
    l*p + (r + a[j][l]) mod p."""
    a = np.asarray(shifts, dtype=np.int64)
    J, L = a.shape
    if p < 1 or np.any(a < -1) or np.any(a >= p):
        raise ValueError("shifts must lie in {-1} U [0, p)")
    rows, cols = [], []
    r = np.arange(p)
    for j in range(J):
        for l in range(L):
            if a[j, l] >= 0:
                rows.append(j * p + r)
                cols.append(l * p + (r + a[j, l]) % p)
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = np.zeros(0, dtype=np.int64)
        cols = np.zeros(0, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(J * p + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return SparseH(L * p, J * p, np.cumsum(rp), cols)


def unwrap_qc(shifts, p: int, positions: int, terminate: bool = True):
    """Sec. II-D.  Returns (H, info) with H the explicit terminated parity-check
    matrix of the LDPC convolutional code unwrapped from the QC code.

    Step 1: Lambda = gcd(J, L); sub-block H_{i,j} is block rows
            [i J/L', (i+1) J/L') x block columns [j L/L', (j+1) L/L') of the base
            (L' = Lambda).
    Step 2: H^L keeps sub-blocks with j <= i, H^U those with j > i.
    Step 3: H_conv = [[H^L], [H^U, H^L], [H^U, H^L], ...] (copies of the
            Lambda x Lambda sub-block pair placed every Lambda sub-block rows
            and columns).
    A code position (frame) is one sub-block column (c = p L / Lambda bits), a
    check layer one sub-block row (c - b = p J / Lambda checks).  The chain is
    cut after `positions` positions; with terminate=True every check layer
    that still touches a kept position is kept (positions + m_s layers),
    otherwise only layers 0 .. positions-1.
    """
    a = np.asarray(shifts, dtype=np.int64)
    J, L = a.shape
    lam = math.gcd(J, L)
    Jb, Lb = J // lam, L // lam
    ms = lam - 1
    # step 1/2: base-level lower and strictly upper parts
    HL = np.full_like(a, -1)
    HU = np.full_like(a, -1)
    for i in range(lam):
        for j in range(lam):
            blk = a[i * Jb:(i + 1) * Jb, j * Lb:(j + 1) * Lb]
            if j <= i:
                HL[i * Jb:(i + 1) * Jb, j * Lb:(j + 1) * Lb] = blk
            else:
                HU[i * Jb:(i + 1) * Jb, j * Lb:(j + 1) * Lb] = blk
    # step 3: paste H^U below H^L and repeat down the diagonal
    copies = -(-positions // lam)
    big = np.full(((copies + 1) * J, copies * L), -1, dtype=np.int64)
    for u in range(copies):
        big[u * J:(u + 1) * J, u * L:(u + 1) * L] = HL
        big[(u + 1) * J:(u + 2) * J, u * L:(u + 1) * L] = HU
    big = big[:, :positions * Lb]
    nlayers = positions + ms if terminate else positions
    big = big[:nlayers * Jb, :]
    H = qc_parity_check(big, p)
    H.layer_of_row = (np.arange(H.m) // (Jb * p)).astype(np.int32)
    H.pos_of_col = (np.arange(H.n) // (Lb * p)).astype(np.int32)
    H.nlayers = nlayers
    H.npos = positions
    info = dict(Lambda=lam, ms=ms, T=lam, Jb=Jb, Lb=Lb, c=Lb * p, cb=Jb * p,
                nlayers=nlayers, positions=positions, base=big)
    return H, info


def edge_lookup_tables(H):
    """Sec. IV-A: message packages are numbered by the positions of the ones of
    H, row by row and left to right.  LUT_c[m] lists the package numbers of
    check m, LUT_v[n] those of variable n (ascending row order)."""
    H = np.asarray(H, dtype=np.uint8)
    num = -np.ones(H.shape, dtype=np.int64)
    rows, cols = np.nonzero(H)           # row-major order
    num[rows, cols] = np.arange(len(rows))
    lut_c = [list(num[r, H[r] == 1]) for r in range(H.shape[0])]
    lut_v = [list(num[H[:, c] == 1, c]) for c in range(H.shape[1])]
    return lut_c, lut_v


# ----------------------------------------------------------------------------
# C decoders
# ----------------------------------------------------------------------------

def build_lib(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               os.path.join(_HERE, "bp.c"), "-o", _LIB_PATH, "-lm"])
    return _LIB_PATH


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build_lib(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.oracle_decode_block.restype = ci
    lib.oracle_decode_block.argtypes = [ci, ci, vp, vp, vp, ci, ci, ci, cd, ci,
                                        vp, vp, vp, vp, vp, vp, cd, vp, vp]
    lib.oracle_decode_window.restype = ci
    lib.oracle_decode_window.argtypes = [ci, ci, vp, vp, vp, vp, ci, ci, vp, ci, ci, ci, cd, ci,
                                         vp, vp]
    lib.oracle_decode_pipeline.restype = ci
    lib.oracle_decode_pipeline.argtypes = [ci, ci, vp, vp, vp, vp, ci, ci, ci, vp, ci, ci, cd, ci, vp, vp]
    return lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


NEAR = 1e-3


def decode_block(H: SparseH, llr, max_iters: int, early_stop: bool = False,
                 lmax: float = LMAX, nthreads: int = 0, trace: bool = False, L_trace: bool = False,
                 near: float = NEAR):
    """Algorithm 1 in FP64 for every frame of llr [gamma, n] (float32).
    Returns dict(post, bits, iters, converged, min_abs, fragile[, syn_trace]
    [, L_trace]).

    min_abs: the smallest |L| of any decision made (all bits, every iteration
    up to the returned one).  fragile: the first iteration (up to the returned
    one) at which flipping decisions with |L| < near could change whether the
    syndrome is zero, else 0 -- where a decoder that rounds differently may
    stop at another iteration.  L_trace: [gamma, max_iters, n] unclipped L of
    every iteration (NaN after the returned one)."""
    y = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    if y.ndim != 2 or y.shape[1] != H.n:
        raise ValueError("llr must be [gamma, n]")
    g = y.shape[0]
    post = np.empty((g, H.n), dtype=np.float64)
    bits = np.empty((g, H.n), dtype=np.uint8)
    iters = np.empty(g, dtype=np.int32)
    conv = np.empty(g, dtype=np.uint8)
    mina = np.empty(g, dtype=np.float64)
    frag = np.empty(g, dtype=np.int32)
    syn = np.empty((g, max_iters), dtype=np.uint8) if trace else None
    Lt = np.full((g, max_iters, H.n), np.nan, dtype=np.float64) if L_trace else None
    rc = _lib().oracle_decode_block(H.n, H.m, _ptr(H.row_ptr), _ptr(H.col_idx), _ptr(y), g,
                                    int(max_iters), int(bool(early_stop)), float(lmax), int(nthreads),
                                    _ptr(post), _ptr(bits), _ptr(iters), _ptr(conv), _ptr(mina),
                                    _ptr(syn), float(near), _ptr(frag), _ptr(Lt))
    if rc != 0:
        raise ValueError("oracle_decode_block rejected its input")
    out = dict(post=post, bits=bits, iters=iters, converged=conv, min_abs=mina, fragile=frag)
    if trace:
        out["syn_trace"] = syn
    if L_trace:
        out["L_trace"] = Lt
    return out


def decode_window(H: SparseH, llr, W: int, K: int, lmax: float = LMAX, nthreads: int = 0):
    """Sliding-window decoding of a terminated convolutional code built by
    `unwrap_qc`.  Returns dict(post, bits)."""
    if H.layer_of_row is None:
        raise ValueError("H must come from unwrap_qc")
    y = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    if y.ndim != 2 or y.shape[1] != H.n:
        raise ValueError("llr must be [gamma, n]")
    g = y.shape[0]
    post = np.empty((g, H.n), dtype=np.float64)
    bits = np.empty((g, H.n), dtype=np.uint8)
    rc = _lib().oracle_decode_window(H.n, H.m, _ptr(H.row_ptr), _ptr(H.col_idx),
                                     _ptr(H.layer_of_row), _ptr(H.pos_of_col), H.nlayers, H.npos,
                                     _ptr(y), g, int(W), int(K), float(lmax), int(nthreads),
                                     _ptr(post), _ptr(bits))
    if rc != 0:
        raise ValueError("oracle_decode_window rejected its input")
    return dict(post=post, bits=bits)


def decode_pipeline(H: SparseH, llr, I: int, ms: int, lmax: float = LMAX, nthreads: int = 0):
    """Algorithm 2 with I processors on a terminated convolutional code built
    by `unwrap_qc` (syndrome-former memory ms).  Returns dict(post, bits)."""
    if H.layer_of_row is None:
        raise ValueError("H must come from unwrap_qc")
    y = np.ascontiguousarray(np.asarray(llr, dtype=np.float32))
    if y.ndim != 2 or y.shape[1] != H.n:
        raise ValueError("llr must be [gamma, n]")
    g = y.shape[0]
    post = np.empty((g, H.n), dtype=np.float64)
    bits = np.empty((g, H.n), dtype=np.uint8)
    rc = _lib().oracle_decode_pipeline(H.n, H.m, _ptr(H.row_ptr), _ptr(H.col_idx),
                                       _ptr(H.layer_of_row), _ptr(H.pos_of_col), H.nlayers, H.npos, int(ms),
                                       _ptr(y), g, int(I), float(lmax), int(nthreads), _ptr(post), _ptr(bits))
    if rc != 0:
        raise ValueError("oracle_decode_pipeline rejected its input")
    return dict(post=post, bits=bits)


# ----------------------------------------------------------------------------
# exact bitwise MAP by enumeration (tiny codes only)
# ----------------------------------------------------------------------------

def codewords(H) -> np.ndarray:
    """All codewords of the code with parity-check matrix H (dense), by brute
    force over all 2^n words (n <= 22)."""
    H = np.asarray(H, dtype=np.int64)
    m, n = H.shape
    if n > 22:
        raise ValueError("enumeration limited to n <= 22")
    words = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    ok = np.all((words @ H.T) % 2 == 0, axis=1)
    return words[ok]


def map_decode(H, llr) -> np.ndarray:
    """Bitwise MAP LLR: ln P(c_n = 0 | y) / P(c_n = 1 | y) over the codebook,
    with P(y | c) proportional to exp(sum_k (1 - 2 c_k) mu_k / 2)."""
    C = codewords(H)
    y = np.atleast_2d(np.asarray(llr, dtype=np.float64))
    out = np.empty_like(y)
    x = 1.0 - 2.0 * C                         # [ncw, n]
    for g in range(y.shape[0]):
        metric = x @ (y[g] / 2.0)            # log-likelihood up to a constant
        for v in range(y.shape[1]):
            z, o = metric[C[:, v] == 0], metric[C[:, v] == 1]
            lz = np.logaddexp.reduce(z) if len(z) else -np.inf
            lo = np.logaddexp.reduce(o) if len(o) else -np.inf
            out[g, v] = lz - lo
    return out
