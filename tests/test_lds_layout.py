"""Host checks of the LDS addressing the FFT stages rely on (no GPU).

The radix plans are read from the kernel header itself, so these checks follow
any change to the plan tables:
  * the padded LDS line accessors split a position p = a + k (a: the thread's
    part, k: the unrolled offset) as (a + a/16) + (k + k/16), which equals
    p + p/16 only when (a mod 16) + (k mod 16) < 16: every write (base + q Ns)
    and read (t + T e) of every exchanging stage of every plan must satisfy it
    (radices and lengths that are powers of two put a and k in disjoint bits;
    a table entry that is not would break it, e.g. N = 48 as 3 x 16);
  * the contiguous-axis passes synchronise their exchanges per wave, which
    needs every line of T = N / E threads to lie within one 64-lane wave;
  * the padded column tile (one spare row per 16 positions, pitch W) maps the
    N x W tile one to one into slots that fit the N (W + 1) slots allocated.
"""
import os
import re

import pytest

FFT_HPP = os.path.join(os.path.dirname(__file__), "..", "paper_2207_14222_amd", "csrc", "fft.hpp")


def read_plans(kind):
    """{N: (E, [radices])} for PassPlan or LinePlan as declared in fft.hpp."""
    src = open(FFT_HPP).read()
    pat = re.compile(r"template <> struct " + kind +
                     r"<(\d+)> \{ using P = Plan<([\d, ]+)>; static constexpr int E = (\d+); \};")
    plans = {int(n): (int(e), [int(r) for r in rs.split(",")]) for n, rs, e in pat.findall(src)}
    assert plans, kind
    return plans


def stage_accesses(N, E, radices):
    """(a, k) of every LDS write and read of the exchanging stages, in the
    decomposition the stage code passes to the accessor."""
    T = N // E
    out = []
    Ns = 1
    for R in radices:
        M = E // R
        if Ns * R != N:  # not the last stage: write, barrier, read back
            for t in range(T):
                for m in range(M):
                    j = t + m * T
                    base = (j // Ns) * Ns * R + (j & (Ns - 1))
                    out += [(base, q * Ns) for q in range(R)]
                out += [(t, T * e) for e in range(E)]
        Ns *= R
    return out


@pytest.mark.parametrize("kind", ["PassPlan", "LinePlan"])
def test_padded_position_split_is_exact(kind):
    for N, (E, radices) in read_plans(kind).items():
        assert N % E == 0 and all(E % r == 0 for r in radices), (kind, N)
        prod = 1
        for r in radices:
            prod *= r
        assert prod == N, (kind, N)
        acc = stage_accesses(N, E, radices)
        for a, k in acc:
            p = a + k
            assert 0 <= p < N
            assert (a + (a >> 4)) + (k + (k >> 4)) == p + (p >> 4), (kind, N, a, k)


def test_pass_lines_fit_one_wave():
    for N, (E, _) in read_plans("PassPlan").items():
        T = N // E
        assert T <= 64 and 64 % T == 0, N


@pytest.mark.parametrize("W", [4, 8, 16])
def test_padded_column_tile_fits_and_is_one_to_one(W):
    N = 1024
    slots = {(p + (p >> 4)) * W + c for p in range(N) for c in range(W)}
    assert len(slots) == N * W
    assert max(slots) < N * (W + 1)
