"""Seeded synthetic inputs shared by the decoder tests, the benchmark and the
FP64 reference.

Everything here draws or prepares *inputs*: circulant shift tables, random
codewords, BPSK/AWGN channel LLRs.  None of the decoding arithmetic
(check-node, variable-node, hard decision, syndrome) lives here, so the
decoder under test and the reference decoder share nothing but their inputs.

Randomness is counter-based: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), keyed by a seed and
addressed by (frame, position, purpose), so the LLRs of frame g do not depend
on how many frames are drawn together.  Gaussian samples use the Box-Muller
transform.

Channel model (the paper's Sec. II-B): bit c maps to x = 1 - 2c, y = x + g with
g ~ N(0, sigma^2), and the channel LLR is mu = 2 y / sigma^2.  The paper gives
no Eb/N0 mapping; with unit symbol energy we take sigma^2 = 1 / (2 R Eb/N0)
using the design rate R.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

# purpose tags (third counter word) so independent draws never share counters
_TAG_SHIFT = 0x5348  # "SH"
_TAG_NOISE = 0x4E5A  # "NZ"
_TAG_INFO = 0x4946   # "IF"

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counters: np.ndarray, key) -> np.ndarray:
    """Philox-4x32 with 10 rounds.  counters: uint32 [N, 4]; key: two uint32.
    Returns uint32 [N, 4]."""
    c = np.asarray(counters, dtype=np.uint32)
    if c.ndim != 2 or c.shape[1] != 4:
        raise ValueError("counters must have shape [N, 4]")
    c0 = c[:, 0].astype(np.uint64)
    c1 = c[:, 1].astype(np.uint64)
    c2 = c[:, 2].astype(np.uint64)
    c3 = c[:, 3].astype(np.uint64)
    k0 = np.uint32(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint32(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def _uniform_open(words: np.ndarray) -> np.ndarray:
    """uint32 -> float64 uniform in the open interval (0, 1)."""
    return (words.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


# ----------------------------------------------------------------------------
# circulant shift tables
# ----------------------------------------------------------------------------

def closes_4cycle(shifts: np.ndarray, p: int, j: int, l: int, drawn) -> bool:
    """Fossorier's condition (IEEE Trans. IT 2004): entries (j1,l1),(j1,l2),
    (j2,l2),(j2,l1) of a QC base lift to a 4-cycle iff
    a[j1][l1] - a[j1][l2] + a[j2][l2] - a[j2][l1] == 0 (mod p).
    Checks the candidate at (j, l) against entries already in `drawn`."""
    a = shifts
    for j2 in range(a.shape[0]):
        if j2 == j or not drawn[j2][l] or a[j2, l] < 0:
            continue
        for l2 in range(a.shape[1]):
            if l2 == l or not drawn[j][l2] or not drawn[j2][l2]:
                continue
            if a[j, l2] < 0 or a[j2, l2] < 0:
                continue
            if (a[j, l] - a[j, l2] + a[j2, l2] - a[j2, l]) % p == 0:
                return True
    return False


def has_4cycle(shifts, p: int) -> bool:
    a = np.asarray(shifts, dtype=np.int64)
    J, L = a.shape
    for j1 in range(J):
        for j2 in range(j1 + 1, J):
            for l1 in range(L):
                for l2 in range(l1 + 1, L):
                    e = (a[j1, l1], a[j1, l2], a[j2, l2], a[j2, l1])
                    if min(e) < 0:
                        continue
                    if (e[0] - e[1] + e[2] - e[3]) % p == 0:
                        return True
    return False


def draw_qc_shifts(J: int, L: int, p: int, seed: int, max_attempts: int = 4096) -> np.ndarray:
    """Draw a J x L table of circulant shifts in [0, p) entry by entry in
    row-major order; an entry is redrawn while it closes a 4-cycle with the
    entries drawn before it.  Returns int32 [J, L]."""
    a = np.full((J, L), -1, dtype=np.int64)
    drawn = [[False] * L for _ in range(J)]
    key = _key(seed)
    for j in range(J):
        for l in range(L):
            for attempt in range(max_attempts):
                ctr = np.array([[j * L + l, attempt, _TAG_SHIFT, 0]], dtype=np.uint32)
                a[j, l] = int(philox4x32_10(ctr, key)[0, 0]) % p
                if not closes_4cycle(a, p, j, l, drawn):
                    break
            else:
                raise RuntimeError(f"no 4-cycle-free shift for entry ({j},{l}) at p={p}")
            drawn[j][l] = True
    return a.astype(np.int32)


# ----------------------------------------------------------------------------
# channel
# ----------------------------------------------------------------------------

def ebn0_to_sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def gaussian(seed: int, frame0: int, gamma: int, n: int, tag: int = _TAG_NOISE) -> np.ndarray:
    """Standard normal samples [gamma, n] in float64.  Sample (g, i) depends
    only on (seed, frame0 + g, i): block i // 4 of frame f uses the Philox
    counter (i // 4, f mod 2^32, tag, f >> 32) and its four words feed two
    Box-Muller pairs."""
    z = np.empty((gamma, n), dtype=np.float64)
    if gamma and n:
        _lib().synth_gaussian(int(seed) & 0xFFFFFFFFFFFFFFFF, int(frame0), int(gamma), int(n), int(tag),
                              z.ctypes.data)
    return z


def bpsk_awgn_llr(codewords, sigma2: float, seed: int, frame0: int = 0,
                  gamma: int | None = None, n: int | None = None) -> np.ndarray:
    """Channel LLRs mu = 2 y / sigma^2 as float32 [gamma, n], y = (1 - 2c) + sigma z.
    codewords: uint8 [gamma, n] of 0/1, or None for the all-zero codeword
    (then gamma and n must be given)."""
    if codewords is None:
        cw = None
    else:
        cw = np.ascontiguousarray(np.asarray(codewords, dtype=np.uint8))
        gamma, n = cw.shape
    out = np.empty((gamma, n), dtype=np.float32)
    if gamma and n:
        _lib().synth_llr(int(seed) & 0xFFFFFFFFFFFFFFFF, int(frame0), int(gamma), int(n), _TAG_NOISE,
                         cw.ctypes.data if cw is not None else None, float(sigma2), out.ctypes.data)
    return out


def random_bits(seed: int, frame0: int, gamma: int, k: int) -> np.ndarray:
    if gamma == 0 or k == 0:
        return np.zeros((gamma, k), dtype=np.uint8)
    nblk = (k + 127) // 128
    f = np.repeat(np.arange(frame0, frame0 + gamma, dtype=np.uint64), nblk)
    b = np.tile(np.arange(nblk, dtype=np.uint64), gamma)
    ctr = np.stack([b, f & np.uint64(0xFFFFFFFF), np.full_like(b, _TAG_INFO), f >> np.uint64(32)],
                   axis=1).astype(np.uint32)
    w = philox4x32_10(ctr, _key(seed)).reshape(gamma, nblk * 4)
    bits = np.unpackbits(w.view(np.uint8).reshape(gamma, -1), axis=1, bitorder="little")
    return bits[:, :k].copy()


# ----------------------------------------------------------------------------
# systematic encoder (GF(2) elimination in C)
# ----------------------------------------------------------------------------

def build_lib(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               os.path.join(_HERE, "synth.c"), "-o", _LIB_PATH, "-lm"])
    return _LIB_PATH


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build_lib(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gf2_qc_create.restype = ctypes.c_void_p
    lib.gf2_qc_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gf2_rank.restype = ctypes.c_int
    lib.gf2_rank.argtypes = [ctypes.c_void_p]
    lib.gf2_encode.restype = None
    lib.gf2_encode.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.gf2_destroy.restype = None
    lib.gf2_destroy.argtypes = [ctypes.c_void_p]
    u64, i64 = ctypes.c_uint64, ctypes.c_int64
    lib.synth_gaussian.restype = None
    lib.synth_gaussian.argtypes = [u64, i64, i64, i64, ctypes.c_uint32, ctypes.c_void_p]
    lib.synth_llr.restype = None
    lib.synth_llr.argtypes = [u64, i64, i64, i64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_double,
                              ctypes.c_void_p]
    lib.synth_philox_many.restype = None
    lib.synth_philox_many.argtypes = [ctypes.c_void_p, i64, u64, ctypes.c_void_p]
    return lib


def philox4x32_10_c(counters: np.ndarray, seed: int) -> np.ndarray:
    """The C implementation of philox4x32_10 (key = seed split into two words)."""
    c = np.ascontiguousarray(np.asarray(counters, dtype=np.uint32))
    out = np.empty_like(c)
    _lib().synth_philox_many(c.ctypes.data, c.shape[0], int(seed) & 0xFFFFFFFFFFFFFFFF, out.ctypes.data)
    return out


class QCEncoder:
    """Systematic encoder for the QC code lifted from `shifts` at size p."""

    def __init__(self, shifts, p: int):
        a = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32))
        self.J, self.L = a.shape
        self.p = int(p)
        self.n = self.L * self.p
        lib = _lib()
        self._h = lib.gf2_qc_create(a.ctypes.data, self.J, self.L, self.p)
        if not self._h:
            raise ValueError("invalid shift table")
        self.rank = lib.gf2_rank(self._h)
        self.k = self.n - self.rank

    def encode(self, info: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(np.asarray(info, dtype=np.uint8))
        if u.ndim != 2 or u.shape[1] != self.k:
            raise ValueError(f"info must be [count, {self.k}]")
        out = np.empty((u.shape[0], self.n), dtype=np.uint8)
        _lib().gf2_encode(self._h, u.ctypes.data, u.shape[0], out.ctypes.data)
        return out

    def random_codewords(self, gamma: int, seed: int, frame0: int = 0) -> np.ndarray:
        return self.encode(random_bits(seed, frame0, gamma, self.k))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib().gf2_destroy(h)
            except Exception:
                pass
            self._h = None


@lru_cache(maxsize=8)
def qc_encoder(shifts_key: tuple, J: int, L: int, p: int) -> QCEncoder:
    return QCEncoder(np.array(shifts_key, dtype=np.int32).reshape(J, L), p)


def encoder_for(shifts, p: int) -> QCEncoder:
    a = np.asarray(shifts, dtype=np.int32)
    return qc_encoder(tuple(int(x) for x in a.ravel()), a.shape[0], a.shape[1], int(p))


# ----------------------------------------------------------------------------
# named workloads (the shapes of the paper-scale experiments this package runs)
# ----------------------------------------------------------------------------

# Mixed batch for the multi-code plan: QC codes of rates 1/2, 2/3 and 5/6
# (3 x 6, 3 x 9, 3 x 18 bases), small to large circulants, 8 to 1024 frames
# per code, each at its own Eb/N0; shifts drawn with seed 50 + index.
MIXED_CODES = [
    dict(J=3, L=6, p=27, gamma=1024, ebn0_db=3.0),
    dict(J=3, L=6, p=81, gamma=256, ebn0_db=2.5),
    dict(J=3, L=6, p=2700, gamma=64, ebn0_db=1.75),
    dict(J=3, L=9, p=72, gamma=512, ebn0_db=3.0),
    dict(J=3, L=9, p=2400, gamma=32, ebn0_db=2.5),
    dict(J=3, L=18, p=36, gamma=128, ebn0_db=3.5),
    dict(J=3, L=18, p=3600, gamma=8, ebn0_db=3.5),
]


def mixed_shifts(i: int):
    c = MIXED_CODES[i]
    return draw_qc_shifts(c["J"], c["L"], c["p"], 50 + i)


WORKLOADS = {
    # (3,6)-regular QC code, p = 64: n = 384, m = 192; 64 frames, all-zero codeword, 2.0 dB
    "qc36_p64": dict(J=3, L=6, p=64, shift_seed=1, noise_seed=101, gamma=64, ebn0_db=2.0,
                     codeword="zero", max_iters=20, early_stop=1),
    # (3,6)-regular QC code, p = 3060: n = 18360, m = 9180, 55080 edges; 1024 frames
    "qc36_p3060": dict(J=3, L=6, p=3060, shift_seed=2, noise_seed=102, gamma=1024, ebn0_db=1.5,
                       codeword="random", max_iters=20, early_stop=0),
    # LDPC convolutional code unwrapped from the same 3x6 base at p = 512 (c = 1024),
    # 128 positions, terminated; 512 streams; window 6 with 10 iterations per
    # window, or the pipelined decoder with 20 processors
    "cc36_p512": dict(J=3, L=6, p=512, shift_seed=2, noise_seed=103, gamma=512, ebn0_db=1.5,
                      positions=128, window=6, iters_per_window=10, pipeline_iters=20),
}


def workload_inputs(name: str, gamma: int | None = None, ebn0_db: float | None = None,
                    frame0: int = 0, codeword: str | None = None):
    """Shifts, codewords (or None), LLRs and sigma^2 of a named workload."""
    w = dict(WORKLOADS[name])
    gamma = w["gamma"] if gamma is None else gamma
    ebn0 = w["ebn0_db"] if ebn0_db is None else ebn0_db
    cw_kind = w.get("codeword", "zero") if codeword is None else codeword
    shifts = draw_qc_shifts(w["J"], w["L"], w["p"], w["shift_seed"])
    rate = 1.0 - w["J"] / w["L"]
    sigma2 = ebn0_to_sigma2(ebn0, rate)
    if "positions" in w:
        n = w["positions"] * (w["L"] // math.gcd(w["J"], w["L"])) * w["p"]
    else:
        n = w["L"] * w["p"]
    if cw_kind == "random":
        cw = encoder_for(shifts, w["p"]).random_codewords(gamma, seed=w["noise_seed"] + 7, frame0=frame0)
        llr = bpsk_awgn_llr(cw, sigma2, w["noise_seed"], frame0=frame0)
    else:
        cw = None
        llr = bpsk_awgn_llr(None, sigma2, w["noise_seed"], frame0=frame0, gamma=gamma, n=n)
    return dict(spec=w, shifts=shifts, codewords=cw, llr=llr, sigma2=sigma2, gamma=gamma, n=n)
