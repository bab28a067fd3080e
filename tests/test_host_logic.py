"""Host-side checks of the exact-arithmetic claims the kernels rely on (CPU).

1. Stage-1 rounding: floor(n / N) == (n * m) >> sh with sh = 31 + ceil(log2 N)
   and m = ceil(2^sh / N) < 2^32, for every 1 <= N <= 1225 and 0 <= n < 2^31.
   Proof: with e = m N - 2^sh in [0, N), n m / 2^sh = n / N + n e / (N 2^sh)
   and the second term is below 2^31 N / (N 2^(31 + lg)) = 2^-lg <= 1 / N, so
   it cannot carry n / N = k + j / N (j <= N - 1) past k + 1.  The test checks
   the bound m < 2^32 for every N and the identity at the extreme numerators.
2. Final division: with y = RN(1/N), q0 = RN(a y), r = RN(a - q0 N) (one
   fused multiply-add), q = RN(q0 + r y) equals RN(a / N) for every float
   0 <= a < 2^31 and every integer 1 <= N <= 1225.  The one-correction
   theorem for a faithful first quotient does not cover a q0 up to two ulps
   off, so the claim is checked exhaustively instead: tests/div_exhaustive.c
   enumerates every odd N and every 24-bit significand (5.1e9 cases, the
   host's fused multiply-add), and two exact scaling reductions (below) carry
   the result to every even N and every exponent.  A sampled exact-rational
   emulation stays as a second, independent check.
"""
import os
import subprocess
from fractions import Fraction

import numpy as np

NMAX = (2 * 17 + 1) ** 2


def magic(N):
    lg = 0 if N <= 1 else (N - 1).bit_length()
    sh = 31 + lg
    m = -(-(1 << sh) // N)
    return m, sh


def test_magic_division_exact():
    rng = np.random.default_rng(0)
    for N in range(1, NMAX + 1):
        m, sh = magic(N)
        assert m < (1 << 32)
        top = (1 << 31) - 1
        ns = [0, 1, N - 1, N, N + 1, top, top - 1, top - (top % N), top - (top % N) - 1]
        ns += [int(v) for v in rng.integers(0, 1 << 31, 40)]
        ns += [int(k) * N - 1 for k in rng.integers(1, top // N, 20)]
        for n in ns:
            if 0 <= n < (1 << 31):
                assert (n * m) >> sh == n // N, (N, n)


def test_magic_multiplier_from_double_quotient():
    """The record kernel computes m as the ceiling of the correctly rounded
    double quotient 2^sh / N (Python floats are IEEE doubles with correctly
    rounded division); it equals the exact integer ceiling for every N up to
    2^11."""
    import math
    for N in range(1, 2049):
        m, sh = magic(N)
        assert math.ceil(math.ldexp(1.0, sh) / N) == m, N


def rn32(x: Fraction) -> Fraction:
    """Round a rational to the nearest float32 (ties to even), normal range."""
    if x == 0:
        return Fraction(0)
    s = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    ulp = Fraction(2) ** (e - 23)
    q, r = divmod(x, ulp)
    q = int(q)
    if r * 2 > ulp or (r * 2 == ulp and q & 1):
        q += 1
    return s * q * ulp


def test_reciprocal_division_exact():
    rng = np.random.default_rng(1)
    Ns = list(range(1, 60)) + [int(v) for v in rng.integers(60, NMAX + 1, 120)] + [NMAX]
    for N in Ns:
        y = rn32(Fraction(1, N))
        samples = [int(v) for v in rng.integers(0, 1 << 31, 25)]
        samples += [int(v) for v in rng.integers(0, 1 << 24, 25)]
        samples += [int(k) * N + N // 2 for k in rng.integers(1, (1 << 30) // N, 10)]
        for s in samples:
            a = rn32(Fraction(s))          # (float)S, as both sides convert
            q0 = rn32(a * y)
            r = rn32(a - q0 * N)
            assert r == a - q0 * N          # the residual is exact
            q = rn32(q0 + r * y)
            assert q == rn32(a / N), (N, s)


def test_reciprocal_division_exhaustive(tmp_path):
    """Every odd N <= 1225 and every significand in [2^23, 2^24), on all host
    threads (a few seconds).  The program prints the number of cases."""
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "div_exhaustive.c")
    exe = str(tmp_path / "div_exhaustive")
    subprocess.check_call(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-std=c99", "-pthread",
                           "-o", exe, src, "-lm"])
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    r = subprocess.run([exe, str(NMAX), str(threads)], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout
    assert f"checks {613 * (1 << 23)} nmax {NMAX} fail 0" in r.stdout


def test_division_scaling_reductions():
    """The two reductions the exhaustive program relies on, checked with exact
    rationals on samples: the sequence for N = 2^k N' equals 2^-k times the
    sequence for N', and the sequence for m 2^e equals 2^e times the one
    for m."""
    rng = np.random.default_rng(5)

    def seq(a, N):
        y = rn32(Fraction(1, N))
        q0 = rn32(a * y)
        r = rn32(a - q0 * N)
        return rn32(q0 + r * y)

    for _ in range(300):
        Np = int(rng.integers(0, 612)) * 2 + 1
        k = int(rng.integers(0, 11))
        if Np << k > NMAX:
            continue
        m = int(rng.integers(1 << 23, 1 << 24))
        e = int(rng.integers(-23, 8))
        a = Fraction(m) * Fraction(2) ** e
        assert seq(a, Np << k) == seq(Fraction(m), Np) * Fraction(2) ** (e - k)


def test_bench_oracle_bands_equal_the_whole_frame(monkeypatch):
    """The all-cores CPU figure runs the oracle in row bands with a halo; the
    bands' rows must equal the whole-frame oracle result bit for bit (and a
    halo that is too short must not)."""
    import bench
    import oracle
    from paper_2203_02300_amd import synth
    p = synth.make_slanted_pair(160, 360, 24, 5, n_planes=4, dmin=2.0, dmax=22.0,
                                noise_sigma=2.0, occl_strip_frac=0.03)
    L, R = p["left"], p["right"]
    want_d, want_v, _, _ = oracle.match(L, R, 24)
    for nb, th in ((6, 3), (4, 2)):
        d, v, _, rows = bench.oracle_bands(L, R, 24, nb, th)
        assert np.array_equal(v, want_v)
        assert np.array_equal(d.view(np.uint32), want_d.view(np.uint32))
        assert 360 < rows <= 360 + 2 * bench.BAND_HALO * (nb - 1)
    monkeypatch.setattr(bench, "BAND_HALO", 4)
    d, v, _, _ = bench.oracle_bands(L, R, 24, 6, 3)
    assert not (np.array_equal(v, want_v) and np.array_equal(d.view(np.uint32), want_d.view(np.uint32)))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_committed_counter_summaries_match_the_kernel_sources():
    """The HBM-traffic and SQ/TA/TD summaries under profiles/ were taken from
    the aggregation kernel's current sources (bench.py reports them only
    then): a change to those sources needs a fresh profile."""
    import bench
    assert bench.measured_traffic() is not None
    busy = bench.measured_busy()
    assert busy is not None and 0.0 < busy["valu"] <= 1.0 and 0.0 < busy["td"] <= 1.0


def test_banded_oracle_of_the_gpu_tests_equals_the_whole_frame():
    """tests/gpu_util.oracle_banded (the reference of the whole-frame GPU
    parity tests) equals the whole-frame oracle bit for bit, with and without
    two Eq. 4 vote passes (whose halo grows by L1 rows per pass)."""
    import oracle
    from gpu_util import oracle_banded
    from paper_2203_02300_amd import synth
    p = synth.make_slanted_pair(150, 300, 20, 9, n_planes=4, dmin=2.0, dmax=18.0,
                                noise_sigma=2.0, occl_strip_frac=0.03)
    L, R = p["left"], p["right"]
    for kw in ({}, {"vote_iters": 2}):
        want = oracle.match(L, R, 20, **kw)
        got = oracle_banded(L, R, 20, nbands=5, threads=5, **kw)
        assert np.array_equal(got[1], want[1])
        assert np.array_equal(got[0].view(np.uint32), want[0].astype(np.float32).view(np.uint32))
        if not kw:
            assert np.array_equal(got[2], want[2]) and np.array_equal(got[3], want[3])
