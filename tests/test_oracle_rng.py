"""Pins for the oracle's random numbers (CPU only).

The paper only requires fresh, independent numbers per level (Sec. 5, after
eq. (eq:Yldef)); the generator is Philox4x32-10 (Salmon et al., SC'11) with
Box--Muller normals.  The oracle's Philox is pinned against an independent
implementation of the same published definition (rocRAND's), its uniforms and
normals against their distributions.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe,
                    os.path.join(HERE, "philox_rocrand_ref.cpp")], check=True,
                   capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(12345)
    cases = [np.zeros(6, np.uint32), np.full(6, 0xFFFFFFFF, np.uint32)]
    cases += list(rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).astype(np.uint32))
    # counters in the layout the sampler uses: small j, level, stream
    for j in range(4):
        for s in (0, 1, 2**32 - 1, 2**32 + 5):
            ctr = [j, s & 0xFFFFFFFF, 3 + 256 * (s >> 32), 1]
            cases.append(np.array(ctr + [1, 0], np.uint32))
    inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(w, 16) for w in line.split()]
        got = orc.philox(c[:4], c[4:])
        assert list(got) == ref, (c, got, ref)


def test_counter_layout(orc):
    # word 2 carries the level and the high path bits; word 3 the stream
    w = orc.path_words(seed=(7 << 32) | 3, level=5, s=(2 << 32) | 9, stream=1, nblocks=2)
    for j in range(2):
        ref = orc.philox([j, 9, 5 + 256 * 2, 1], [3, 7])
        assert list(w[4 * j:4 * j + 4]) == list(ref)


def test_uniform_map(orc):
    assert orc.u01(0) == 2.0 ** -25
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -25
    assert orc.u01(0x80000000) == 0.5 + 2.0 ** -25
    words = orc.path_words(1, 0, 0, 0, 50000)
    u = np.array([orc.u01(int(x)) for x in words[:100000]])
    assert u.min() > 0 and u.max() < 1
    counts, _ = np.histogram(u, bins=100, range=(0, 1))
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert stats.chi2.sf(chi2, 99) > 1e-4


def test_normals_distribution(orc):
    z = np.concatenate([orc.path_normals(1, 3, s, 0, 1, 64) for s in range(3000)])
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert abs(stats.skew(z)) < 4 * np.sqrt(6 / z.size)
    assert abs(stats.kurtosis(z)) < 4 * np.sqrt(24 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_normals_independent_across_steps_paths_levels(orc):
    Z = np.array([orc.path_normals(1, 2, s, 0, 1, 16) for s in range(4000)])
    # lag correlations along the path and across adjacent paths
    for lag in (1, 2, 3, 4):
        c = np.corrcoef(Z[:, :-lag].ravel(), Z[:, lag:].ravel())[0, 1]
        assert abs(c) < 5 / np.sqrt(Z[:, lag:].size)
    c = np.corrcoef(Z[:-1].ravel(), Z[1:].ravel())[0, 1]
    assert abs(c) < 5 / np.sqrt(Z[1:].size)
    # different levels use different numbers for the same path index
    Z3 = np.array([orc.path_normals(1, 3, s, 0, 1, 16) for s in range(4000)])
    c = np.corrcoef(Z.ravel(), Z3.ravel())[0, 1]
    assert abs(c) < 5 / np.sqrt(Z.size)


def test_normal_assignment_from_words(orc):
    w = orc.path_words(1, 2, 17, 0, 2)
    z1 = orc.path_normals(1, 2, 17, 0, 1, 8)
    z2 = orc.path_normals(1, 2, 17, 0, 2, 4)
    for j in range(2):
        a = orc.box_muller(w[4 * j], w[4 * j + 1])
        b = orc.box_muller(w[4 * j + 2], w[4 * j + 3])
        assert np.array_equal(z1[4 * j:4 * j + 4], np.array(a + b))
        assert np.array_equal(z2[4 * j:4 * j + 4], np.array(a + b))
    u = orc.path_uniforms(1, 2, 17, 1, 8)
    w1 = orc.path_words(1, 2, 17, 1, 2)
    assert np.array_equal(u, np.array([orc.u01(int(x)) for x in w1]))


def test_box_muller_is_polar_map(orc):
    # z0^2 + z1^2 = -2 ln u1 and atan2(z1, z0) = 2 pi u2 (mod 2 pi)
    rng = np.random.default_rng(3)
    for a, b in rng.integers(0, 2**32, size=(200, 2), dtype=np.uint64):
        z0, z1 = orc.box_muller(int(a), int(b))
        u1, u2 = orc.u01(int(a)), orc.u01(int(b))
        assert np.isclose(z0 * z0 + z1 * z1, -2 * np.log(u1), rtol=1e-12, atol=1e-14)
        ang = np.arctan2(z1, z0) % (2 * np.pi)
        assert np.isclose(ang, (2 * np.pi * u2) % (2 * np.pi), atol=1e-9) or \
            np.isclose(abs(ang - 2 * np.pi * u2), 2 * np.pi, atol=1e-9)


def test_short_paths_share_a_block(orc):
    # fewer than four numbers per path: q = 4/total paths read one block
    for dim, nsteps in [(1, 1), (1, 2), (2, 1)]:
        total = dim * nsteps
        q = 4 // total
        for s in (0, 1, 2, 3, 6, 2**33 + 5):
            w = orc.philox([0, (s // q) & 0xFFFFFFFF, 4 + 256 * ((s // q) >> 32), 0], [1, 0])
            zz = orc.box_muller(w[0], w[1]) + orc.box_muller(w[2], w[3])
            z = orc.path_normals(1, 4, s, 0, dim, nsteps)
            r = s % q
            assert np.array_equal(z, np.array(zz[r * total:(r + 1) * total]))
    # neighbouring paths get different numbers; the set of a block is all used
    zs = np.concatenate([orc.path_normals(1, 0, s, 0, 1, 1) for s in range(8)])
    assert len(set(zs)) == 8
    for nsteps in (1, 2):
        q = 4 // nsteps
        for s in (0, 3, 5):
            w = orc.philox([0, s // q, 2, 1], [1, 0])
            u = orc.path_uniforms(1, 2, s, 1, nsteps)
            r = s % q
            assert np.array_equal(u, np.array([orc.u01(int(x)) for x in w[r * nsteps:(r + 1) * nsteps]]))
