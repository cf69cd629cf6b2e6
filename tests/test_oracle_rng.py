"""Pins of the oracle's random numbers: Philox4x32-10 against the published
known-answer vectors and against rocRAND's independent implementation, and
the word -> uniform conversion against its definition's invariants."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(oracle_mod, row):
    ctr, key, out = row[0:4], row[4:6], row[6:10]
    assert oracle_mod.philox(ctr, key) == out


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.isdir("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    src = os.path.join(HERE, "golden", "rocrand_philox_ref.cpp")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-I/opt/rocm/include", "-O1",
                    "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(1, 0, 0), (1, 1, 0), (1, 0, 1), (0xdeadbeefcafef00d, 123456789, 77),
             (2**64 - 1, 2**40 + 5, 2**32 - 1)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2**63)) * 2 + 1, int(rng.integers(0, 2**61)),
                      int(rng.integers(0, 2**32))))
    text = "".join(f"{s} {k} {b}\n" for s, k, b in cases)
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (s, k, b), line in zip(cases, lines):
        ref = [int(x) for x in line.split()]
        ctr = [k & 0xFFFFFFFF, k >> 32, b, 0]
        key = [s & 0xFFFFFFFF, s >> 32]
        assert oracle_mod.philox(ctr, key) == ref, (s, k, b)


def test_uniform_conversion(oracle_mod):
    # u = ((x >> 8) | 1) * 2^-24: odd multiples of 2^-24 strictly inside (0, 1),
    # exactly representable in float32.
    for x in [0, 1, 255, 256, 0x7FFFFFFF, 0x80000000, 0xFFFFFF00, 0xFFFFFFFF]:
        u = oracle_mod.uniform(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        m = u * 2**24
        assert m == int(m) and int(m) % 2 == 1
        assert int(m) == ((x >> 8) | 1)
    assert oracle_mod.uniform(0) == 2.0**-24
    assert oracle_mod.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24


def test_uniform_is_uniform(oracle_mod):
    # Chi-square of 4e4 words from consecutive counters in 20 bins.
    words = []
    for k in range(10000):
        words += oracle_mod.philox([k, 0, 0, 0], [1, 0])
    u = np.array([oracle_mod.uniform(w) for w in words])
    counts, _ = np.histogram(u, bins=20, range=(0, 1))
    e = len(u) / 20
    chi2 = ((counts - e) ** 2 / e).sum()
    assert chi2 < 45.3  # 19 dof, p = 1e-3
