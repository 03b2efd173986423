"""Seeded input generators (CPU): Philox4x32-10 against the published
known-answer vectors of its authors' reference implementation (Random123),
the derived uniform / normal draws, and the D + K family's structure."""
import numpy as np

from paper_2006_08498_amd import synth

KAT = [
    # counter (4 words), key (2 words) -> output (4 words)
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, out in KAT:
        got = synth.philox4x32_10(*[np.array([c]) for c in ctr], *key)
        assert tuple(int(g[0]) for g in got) == out


def test_uniform_and_normal_draws():
    i = np.arange(200000, dtype=np.uint64)
    u0, u1 = synth.uniform_pair(i, np.uint64(7), 3, seed=11)
    assert 0.0 <= u0.min() and u0.max() < 1.0 and 0.0 <= u1.min() and u1.max() < 1.0
    z0, z1 = synth.normal_pair(i, np.uint64(7), 3, seed=11)
    z = np.concatenate([z0, z1])
    # mean and variance of 4e5 standard normals: 6-sigma windows
    assert abs(z.mean()) < 6 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 6 * np.sqrt(2.0 / z.size)
    # different stream tag or seed -> different draws
    assert not np.array_equal(z0, synth.normal_pair(i, np.uint64(7), 4, seed=11)[0])
    assert not np.array_equal(z0, synth.normal_pair(i, np.uint64(7), 3, seed=12)[0])


def test_dk_structure_and_rows():
    N, seed, std, decay = 600, 5, 0.01, 40.0
    H = synth.dk_matrix(N, seed=seed, std=std, decay=decay)
    assert np.array_equal(H, H.conj().T)                       # Hermitian, bitwise
    d = synth.dk_diag(N, seed)
    assert 1.0 <= d.min() and d.max() < 6.0
    K = H - np.diag(d)
    far = np.abs(np.subtract.outer(np.arange(N), np.arange(N))) > 8 * decay
    assert np.abs(K[far]).max() < 10 * std * np.exp(-8)          # decays with |i - j|
    rows = [0, 1, 299, 599]
    assert np.array_equal(synth.dk_rows(rows, N, seed, std, decay), H[rows])
