"""The library's inner-product arithmetic on the host, against exact rational
arithmetic (CPU).

The GPU carries every inner product as a triple (a, b, c) -- td_fma per term,
td_add to combine partial sums, td_round once at the end (device_common.hpp).
Those three functions also compile for the host; tests/td_host.cpp wraps them
in sums with several groupings and orders (the shapes of the device's
per-thread sums and tree reductions).  Every grouping must give the inner
product rounded once from its exact value, and td_round must round any triple
to nearest, ties to even, including half-way cases that a tiny third term
breaks.
"""
import ctypes
import fractions
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F = fractions.Fraction


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("td") / "libtd_host.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "--cuda-host-only", "-O2", "-std=c++17",
                           "-fPIC", "-shared", "-ffp-contract=off",
                           "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_2108_10591_amd", "csrc"),
                           "-x", "hip", os.path.join(ROOT, "tests", "td_host.cpp"), "-o", out])
    L = ctypes.CDLL(out)
    P = ctypes.c_void_p
    L.td_dot_grouped.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_int]
    L.td_dot_grouped.restype = ctypes.c_double
    L.td_round3.argtypes = [ctypes.c_double] * 3
    L.td_round3.restype = ctypes.c_double
    return L


def exact_dot(u, v):
    return float(sum(F(a) * F(b) for a, b in zip(u, v)))  # int / int: correctly rounded


def grouped(L, u, v, group, backward):
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return L.td_dot_grouped(u.size, u.ctypes.data, v.ctypes.data, group, backward)


def cases():
    rng = np.random.default_rng(17)
    out = []
    for n in (1, 5, 300, 4000):
        out.append((f"random n={n}", rng.standard_normal(n) * 2.0 ** rng.integers(-40, 40, n),
                    rng.standard_normal(n) * 2.0 ** rng.integers(-40, 40, n)))
    big = rng.standard_normal(300) * 1e18
    u = np.concatenate([big, big, rng.standard_normal(30)])
    v = np.concatenate([np.ones(300), -np.ones(300), rng.standard_normal(30) * 1e-12])
    p = rng.permutation(u.size)
    out.append(("cancellation to 1e-30", u[p], v[p]))
    # near-orthogonal pairs, as r0* and r_i late in a long solve
    for seed in range(4):
        r = np.random.default_rng(100 + seed)
        q = r.standard_normal(6000)
        z = r.standard_normal(6000)
        w = z - (q @ z) / (q @ q) * q
        w = w - (q @ w) / (q @ q) * q
        out.append((f"near-orthogonal {seed}", q, w))
    return out


@pytest.mark.parametrize("group,backward", [(1, 0), (7, 1), (64, 0), (256, 1), (1 << 30, 0),
                                            (1 << 30, 1)])
def test_grouped_sums_are_exactly_rounded(lib, group, backward):
    for name, u, v in cases():
        want = exact_dot(u, v)
        got = grouped(lib, u, v, group, backward)
        assert got == want, (name, group, backward, got, want)


def test_round3_half_way_cases(lib):
    h = 2.0 ** -53
    one_up = 1.0 + 2.0 ** -52
    for (a, b, c), want in [((1.0, h, 0.0), 1.0),                 # tie: to even
                            ((1.0, h, 2.0 ** -200), one_up),      # just above
                            ((1.0, h, -2.0 ** -200), 1.0),        # just below
                            ((one_up, h, 0.0), 1.0 + 2.0 ** -51),  # tie up to even
                            ((one_up, h, -2.0 ** -300), one_up),
                            ((2.0, -h, 0.0), 2.0),                # tie below a power of 2
                            ((2.0, -h, -2.0 ** -400), 2.0 - 2.0 ** -52),
                            ((0.0, 0.0, 0.0), 0.0),
                            ((1e300, -1e300, 1e-300), 1e-300)]:
        assert lib.td_round3(a, b, c) == want, (a, b, c)


def test_round3_random_triples(lib):
    """Triples in every magnitude relation, many placed at or next to half-way points."""
    rng = np.random.default_rng(23)
    for i in range(20000):
        a = rng.standard_normal() * 2.0 ** int(rng.integers(-30, 30))
        ulp = np.spacing(a)
        kind = i % 4
        if kind == 0:    # b near half a unit of a, c tiny either way
            b = ulp / 2 * rng.choice([-1.0, 1.0]) * (1 + rng.choice([0.0, 2.0 ** -50]))
            c = rng.choice([0.0, 1.0, -1.0]) * ulp * 2.0 ** -int(rng.integers(60, 200))
        elif kind == 1:  # unordered magnitudes
            b = rng.standard_normal() * 2.0 ** int(rng.integers(-60, 60))
            c = rng.standard_normal() * 2.0 ** int(rng.integers(-60, 60))
        elif kind == 2:  # cancellation between a and b
            b = -a * (1 + rng.standard_normal() * 2.0 ** -int(rng.integers(20, 52)))
            c = rng.standard_normal() * ulp * 2.0 ** -int(rng.integers(0, 80))
        else:            # b, c below a, as a triple accumulator leaves them
            b = rng.standard_normal() * ulp
            c = rng.standard_normal() * ulp * 2.0 ** -53
        want = float(F(a) + F(b) + F(c))
        got = lib.td_round3(a, b, c)
        assert got == want, (i, a, b, c, got, want)
