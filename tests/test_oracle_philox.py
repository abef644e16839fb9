"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al. SC11 2011) and of the
sample-to-counter layout: the published known-answer vectors, and PyTorch's independently written
header-only engine."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import binding as ob

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert ob.philox(ctr, key) == expect


@pytest.fixture(scope="module")
def torch_engine():
    try:
        import torch
    except Exception:  # pragma: no cover
        pytest.skip("torch not importable")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch Philox header missing")
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "tpr")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + inc, os.path.join(HERE, "torch_philox_ref.cpp"), "-o", exe],
                   check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_sample_words_match_torch_engine(torch_engine):
    """Word d of sample n of iteration it is stream word k = D*n + d: output k % 4 of the engine with subsequence
    uid | (epoch*64+it) << 32 and offset k // 4."""
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(64):
        seed = int(rng.integers(0, 2**63))
        uid = int(rng.integers(0, 2**32))
        epoch = int(rng.integers(0, 2**20))
        it = int(rng.integers(0, 64))
        n = int(rng.integers(0, 2**40))
        D = int(rng.choice([3, 6, 9, 12]))
        cases.append((seed, uid, epoch, it, n, D))
    lines = []
    for seed, uid, epoch, it, n, D in cases:
        sub = uid | (((epoch * 64 + it) & 0xFFFFFFFF) << 32)
        for d in range(D):
            lines.append("%d %d %d" % (seed, sub, (D * n + d) // 4))
    out = subprocess.run([torch_engine], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    k = 0
    for seed, uid, epoch, it, n, D in cases:
        words = []
        for d in range(D):
            words.append(int(out[k].split()[(D * n + d) % 4]))
            k += 1
        y = ob.uniforms(seed, uid, epoch, it, n, D)
        w_from_y = y * 2.0**32 - 0.5
        assert np.array_equal(w_from_y, np.array(words, dtype=np.float64))


def test_word_groups_fill_whole_blocks():
    """G = 4/gcd(D,4) consecutive samples from a multiple of G take the words of G*D/4 whole Philox blocks in order
    (blocks D*n0/4 ...), and the next sample starts the next block: no stream word is skipped or reused."""
    seed, uid, epoch, it = 5, 77, 1, 2
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for D in (3, 6, 9, 12):
        G = 4 // math.gcd(D, 4)
        n0 = 1000 * G
        got = np.concatenate([ob.uniforms(seed, uid, epoch, it, n0 + s, D) for s in range(2 * G)])
        b0 = n0 * D // 4
        words = []
        for b in range(b0, b0 + 2 * G * D // 4):
            words += list(ob.philox((b & 0xFFFFFFFF, b >> 32, uid, epoch * 64 + it), key))
        want = (np.array(words, dtype=np.float64) + 0.5) * 2.0**-32
        assert np.array_equal(got, want), D


def test_uniforms_open_interval():
    y = np.concatenate([ob.uniforms(0, 7, 0, 0, n, 12) for n in range(256)])
    assert y.min() > 0.0 and y.max() < 1.0
