"""Pins of the oracle's random stream and seed-pair map (CPU only).

The generator is Philox4x32-10 (Salmon et al., SC'11); the hypotheses of
Alg. 1 draw their two seed indices from it.  Pins:
  * published known-answer vectors (tests/golden/philox4x32_10_kat.txt);
  * rocRAND's independent Philox4x32-10 on a grid of random blocks;
  * the index map is a monotone step function whose steps differ by at most one
    preimage (exact boundaries), never returns i == j, reaches every ordered
    pair, and draws pairs uniformly (chi-square) from the Philox stream.
"""
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
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            words = [int(w, 16) for w in line.split()]
            assert len(words) == 10
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle_mod.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_philox_matches_rocrand(oracle_mod, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND host build")
    exe = tmp_path / "xcheck"
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                    os.path.join(HERE, "rocrand_philox_xcheck.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    rng = np.random.default_rng(12345)
    blocks = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    # include structured counters like the estimator's (h, k, 0, 0)
    blocks[:100, 2:4] = 0
    blocks[:100, 0] = np.arange(100)
    text = "\n".join(" ".join(f"{int(w):08x}" for w in b) for b in blocks) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    assert len(lines) == len(blocks)
    for b, line in zip(blocks, lines):
        want = [int(w, 16) for w in line.split()]
        got = oracle_mod.philox4x32_10(b[0:4].astype(np.uint32), b[4:6].astype(np.uint32))
        assert [int(x) for x in got] == want


def test_draw_pair_uses_key_seed_and_counter_h_k(oracle_mod):
    # key = (low word of seed, high word of seed), counter = (h, k, 0, 0)
    seed = 0x0123456789ABCDEF
    for h, k, n in [(0, 0, 2), (5, 3, 17), (1023, 4095, 4096), (7, 1, 65536)]:
        u = oracle_mod.philox4x32_10([h, k, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle_mod.draw_pair(seed, h, k, n) == oracle_mod.map_pair(int(u[0]), int(u[1]), n)


@pytest.mark.parametrize("n", [2, 3, 5, 7, 12, 100, 4096, 65536, 2**31 - 1])
def test_map_pair_exact_step_boundaries(oracle_mod, n):
    # The first index is the multiply-shift map floor(u * n / 2^32): index a owns
    # the preimage [ceil(a 2^32 / n), ceil((a + 1) 2^32 / n)).  Check both sides
    # of a few boundaries with exact integer arithmetic.
    two32 = 1 << 32
    for a in sorted({0, 1, n // 2, n - 2, n - 1}):
        if a < 0 or a >= n:
            continue
        start = -(-a * two32 // n)
        end = -(-(a + 1) * two32 // n)
        assert oracle_mod.map_pair(start, 0, n)[0] == a
        assert oracle_mod.map_pair(end - 1, 0, n)[0] == a
        if start > 0:
            assert oracle_mod.map_pair(start - 1, 0, n)[0] == a - 1
    # preimage sizes differ by at most one
    sizes = {(-(-(a + 1) * two32 // n)) - (-(-a * two32 // n)) for a in range(min(n, 64))}
    assert max(sizes) - min(sizes) <= 1


@pytest.mark.parametrize("n", [2, 3, 4, 9, 16])
def test_map_pair_reaches_every_ordered_pair_and_never_repeats(oracle_mod, n):
    rng = np.random.default_rng(n)
    seen = set()
    for u0, u1 in rng.integers(0, 2**32, size=(20000, 2), dtype=np.uint64):
        i, j = oracle_mod.map_pair(int(u0), int(u1), n)
        assert 0 <= i < n and 0 <= j < n and i != j
        seen.add((i, j))
    assert seen == {(i, j) for i in range(n) for j in range(n) if i != j}
    # extremes of the second word
    for u0 in (0, 2**32 - 1):
        for u1 in (0, 2**32 - 1):
            i, j = oracle_mod.map_pair(u0, u1, n)
            assert i != j and 0 <= i < n and 0 <= j < n


def test_pairs_from_philox_are_uniform(oracle_mod):
    # 42 ordered pairs of a 7-point cluster, 84,000 draws over (h, k): chi-square
    # with 41 degrees of freedom stays below its 99.99th percentile (~ 85.0).
    n = 7
    counts = np.zeros((n, n))
    seed = 0xDEADBEEF
    for k in range(21):
        for h in range(4000):
            i, j = oracle_mod.draw_pair(seed, h, k, n)
            counts[i, j] += 1
    obs = counts[~np.eye(n, dtype=bool)]
    exp = obs.sum() / obs.size
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 85.0, chi2
