"""Pins of the oracle's random numbers: Philox4x32-10 and the ]0,1] mapping.

The oracle's Philox is checked against rocRAND's host-callable Philox4x32-10 engine,
an independent published implementation (compiled here from its header), on many
counters and keys.  The float mapping is checked against its definition on the
bit patterns that decide it.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_ref(lines):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND reference")
    exe = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"spx_rocrand_ref_{os.getpid()}")
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, cwd=os.environ.get("TMPDIR", "/tmp"),
                   capture_output=True)
    try:
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    finally:
        os.remove(exe)
    return np.array([[int(v) for v in l.split()] for l in out.stdout.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand():
    rng = np.random.default_rng(1234)
    n = 4000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 29) - 1           # keep 4 * (c0 | c1 << 32) inside rocRAND's 64-bit offset
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # structured counters of the transport's keying: (particle, event, cfg<<8|cathode, sub)
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
               [9999999, 1 << 20, (63 << 8) | 3, 1], [2**32 - 1, 5, 2, 0], [7, 2**29 - 1, 2**32 - 1, 2**32 - 1]]
    key[:4] = [[0, 0], [1, 0], [0, 1], [2**32 - 1, 2**32 - 1]]
    lines = [" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key)]
    ref = _rocrand_ref(lines)
    ours = np.stack([oracle.philox(c, k)[0] for c, k in zip(ctr.astype(np.uint32), key.astype(np.uint32))])
    assert np.array_equal(ours.astype(np.uint64), ref)


def test_u01_mapping():
    # u = ((x >> 8) + 1) * 2^-24 lies in ]0, 1]: the paper's range for RN_1
    assert oracle.u01(0) == 2.0**-24
    assert oracle.u01(255) == 2.0**-24          # the low 8 bits are dropped
    assert oracle.u01(256) == 2.0 * 2.0**-24
    assert oracle.u01(0xFFFFFFFF) == 1.0
    assert oracle.u01(0x7FFFFFFF) == 0.5
    xs = np.random.default_rng(0).integers(0, 2**32, 2000, dtype=np.uint64)
    for x in xs:
        u = oracle.u01(int(x))
        assert 0.0 < u <= 1.0
        assert u * 2**24 == (int(x) >> 8) + 1


def test_philox_streams_uniform_and_distinct():
    # first words of consecutive particles: uniform (chi^2 over 64 cells) and no repeats
    ctr = np.array([[i, 1, 0, 0] for i in range(20000)], dtype=np.uint32)
    out = oracle.philox(ctr, [0, 0])
    w = out[:, 0].astype(np.float64) / 2**32
    h, _ = np.histogram(w, bins=64, range=(0, 1))
    chi2 = ((h - 20000 / 64) ** 2 / (20000 / 64)).sum()
    assert chi2 < 120          # dof 63: p ~ 1e-5
    assert len(np.unique(out[:, 0])) > 19990
    # event, config/cathode and sub words each change the block
    base = oracle.philox([5, 7, 3, 0], [0, 0])[0]
    for c in ([5, 8, 3, 0], [5, 7, 4, 0], [5, 7, 3, 1], [6, 7, 3, 0]):
        assert not np.array_equal(oracle.philox(c, [0, 0])[0], base)
    assert not np.array_equal(oracle.philox([5, 7, 3, 0], [1, 0])[0], base)


def _diff_u(n_pairs, seed=77, cfgcat=5):
    U = np.empty((2 * n_pairs, 3))
    for i in range(2 * n_pairs):
        # events 2..2n+1: pairs (2m, 2m+1) share a block; pid varies with the pair
        U[i] = oracle.diffusive_uniforms(seed, 1000 + i // 64, 2 + i, cfgcat)
    return U


def test_diffusive_uniforms_range_and_lattice():
    """RN of the diffusive walk lie on the 21-bit lattice (k + 1) 2^-21 of ]0,1]."""
    U = _diff_u(4096)
    k = U * 2**21 - 1
    assert np.all(U > 0) and np.all(U <= 1)
    assert np.array_equal(k, np.round(k)) and k.min() >= 0 and k.max() < 2**21


def test_diffusive_uniforms_uniform_and_independent():
    """Each RN is uniform (chi-square over 64 cells); the three RN of a step, the two steps
    sharing a Philox block, and consecutive steps from different blocks are uncorrelated --
    a shared or overlapping bit field between the halves of a block would show here."""
    n_pairs = 16384
    U = _diff_u(n_pairs)
    n = len(U)
    for j in range(3):
        h = np.bincount(np.minimum((U[:, j] * 64).astype(int), 63), minlength=64)
        chi2 = ((h - n / 64) ** 2 / (n / 64)).sum()
        assert chi2 < 63 + 5 * np.sqrt(2 * 63), (j, chi2)
    tol = 5.0 / np.sqrt(n_pairs)
    even, odd = U[0::2], U[1::2]
    for a in range(3):
        for b in range(3):
            assert abs(np.corrcoef(even[:, a], odd[:, b])[0, 1]) < tol, ("same block", a, b)
            assert abs(np.corrcoef(odd[:-1, a], even[1:, b])[0, 1]) < tol, ("next block", a, b)
            if a < b:
                assert abs(np.corrcoef(U[:, a], U[:, b])[0, 1]) < 5.0 / np.sqrt(n), ("same step", a, b)
    # low bits too: the parity of the 21-bit code is a fair coin in both halves
    k = np.round(U * 2**21 - 1).astype(np.int64)
    for half in (k[0::2], k[1::2]):
        for j in range(3):
            assert abs((half[:, j] & 1).mean() - 0.5) < 5 * 0.5 / np.sqrt(len(half))
