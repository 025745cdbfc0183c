"""Seeded input generators: Philox known answers, 4-cycle rejection against a
brute-force girth check, the systematic encoder and the channel."""
import itertools

import numpy as np
import pytest

import synth
from conftest import read_golden


def test_philox_known_answers():
    # Known-answer vectors published with the Random123 library for
    # Philox-4x32-10 (counter, key) -> output.
    kat = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in kat:
        got = synth.philox4x32_10(np.array([ctr], dtype=np.uint32), key)[0]
        assert tuple(int(x) for x in got) == want


def _lifted_rows(shifts, p):
    """Explicit rows of the lifted matrix, built independently of the code
    under test (dense Kronecker-style assembly from the golden circulants'
    definition: row r of block (j,l) has its one at column (r + a) mod p)."""
    a = np.asarray(shifts)
    J, L = a.shape
    H = np.zeros((J * p, L * p), dtype=np.uint8)
    for j, l in itertools.product(range(J), range(L)):
        if a[j, l] >= 0:
            for r in range(p):
                H[j * p + r, l * p + (r + a[j, l]) % p] = 1
    return H


def _has_4cycle_bruteforce(H):
    # a 4-cycle exists iff two rows share at least two columns
    G = H.astype(np.int64) @ H.T.astype(np.int64)
    np.fill_diagonal(G, 0)
    return bool(np.any(G >= 2))


def test_circulant_convention_matches_golden():
    gold = read_golden("circulant_p4.txt")
    for key, rows in gold.items():
        a = int(key)
        H = _lifted_rows(np.array([[a]]), 4)
        assert H.tolist() == rows


@pytest.mark.parametrize("J,L,p", [(2, 3, 5), (2, 4, 7), (3, 4, 7), (3, 5, 6), (2, 3, 4)])
def test_fossorier_condition_matches_bruteforce(J, L, p):
    rng = np.random.default_rng(J * 100 + L * 10 + p)
    for _ in range(60):
        a = rng.integers(-1, p, size=(J, L))
        assert synth.has_4cycle(a, p) == _has_4cycle_bruteforce(_lifted_rows(a, p))


@pytest.mark.parametrize("J,L,p,seed", [(3, 6, 64, 1), (3, 6, 512, 2), (3, 6, 3060, 2), (3, 9, 72, 3)])
def test_drawn_shifts_are_4cycle_free(J, L, p, seed):
    a = synth.draw_qc_shifts(J, L, p, seed)
    assert a.shape == (J, L) and a.min() >= 0 and a.max() < p
    assert not synth.has_4cycle(a, p)
    assert np.array_equal(a, synth.draw_qc_shifts(J, L, p, seed))
    if p <= 72:
        assert not _has_4cycle_bruteforce(_lifted_rows(a, p))


@pytest.mark.parametrize("p", [16, 64])
def test_encoder_codewords_satisfy_parity(p):
    a = synth.draw_qc_shifts(3, 6, p, 1)
    enc = synth.QCEncoder(a, p)
    H = _lifted_rows(a, p).astype(np.int64)
    assert enc.k == enc.n - enc.rank and enc.k >= 6 * p - 3 * p
    cw = enc.random_codewords(32, seed=9)
    assert cw.shape == (32, 6 * p)
    assert not np.any((cw.astype(np.int64) @ H.T) % 2)
    # not all-zero, roughly balanced
    assert 0.3 < cw.mean() < 0.7


def test_encoder_large_code_parity():
    a = synth.draw_qc_shifts(3, 6, 3060, 2)
    enc = synth.encoder_for(a, 3060)
    assert enc.n == 18360 and enc.k >= 18360 - 9180
    cw = enc.random_codewords(4, seed=3)
    # sparse syndrome from the lifting definition
    J, L, p = 3, 6, 3060
    r = np.arange(p)
    for g in range(cw.shape[0]):
        for j in range(J):
            par = np.zeros(p, dtype=np.int64)
            for l in range(L):
                par ^= cw[g, l * p + (r + a[j, l]) % p]
            assert not par.any()


def test_gaussian_moments_and_frame_independence():
    z = synth.gaussian(5, 0, 64, 1000)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    z2 = synth.gaussian(5, 10, 3, 1000)
    assert np.array_equal(z[10:13], z2)
    llr = synth.bpsk_awgn_llr(None, 0.5, 7, gamma=8, n=100)
    assert llr.dtype == np.float32
    # all-zero codeword: mean 2/sigma^2, variance 4/sigma^2
    big = synth.bpsk_awgn_llr(None, 0.5, 7, gamma=64, n=2000).astype(np.float64)
    assert abs(big.mean() - 4.0) < 0.05 and abs(big.var() - 8.0) < 0.2


def test_sigma_mapping():
    # Eb/N0 = 0 dB at rate 1/2 -> sigma^2 = 1
    assert synth.ebn0_to_sigma2(0.0, 0.5) == pytest.approx(1.0)
    assert synth.ebn0_to_sigma2(2.0, 0.5) == pytest.approx(0.630957, rel=1e-5)


def test_c_gaussian_matches_numpy_philox_box_muller():
    seed, f0, gamma, n = 0xDEADBEEF12345, 7, 5, 37
    z = synth.gaussian(seed, f0, gamma, n)
    nblk = (n + 3) // 4
    for g in range(gamma):
        f = f0 + g
        ctr = np.array([[b, f & 0xFFFFFFFF, synth._TAG_NOISE, f >> 32] for b in range(nblk)], dtype=np.uint32)
        w = synth.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        u = (w.astype(np.float64) + 0.5) / 2.0 ** 32
        r0, r1 = np.sqrt(-2 * np.log(u[:, 0])), np.sqrt(-2 * np.log(u[:, 2]))
        want = np.stack([r0 * np.cos(2 * np.pi * u[:, 1]), r0 * np.sin(2 * np.pi * u[:, 1]),
                         r1 * np.cos(2 * np.pi * u[:, 3]), r1 * np.sin(2 * np.pi * u[:, 3])], 1).ravel()[:n]
        np.testing.assert_allclose(z[g], want, rtol=1e-12, atol=1e-12)
