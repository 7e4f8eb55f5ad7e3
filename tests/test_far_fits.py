"""The fitted far-field tables in the generated constants header against SciPy's
exponentially scaled Bessel functions (no GPU): each piece of e^z sqrt(z) K_nu(z)
for z > 2 as a polynomial in the local variable of u = 4/z - 1 (this library's
evaluation of the kernels K0 and K1 of Sec. 2; the paper's series of App. C cover
small z), and K1 taken from the derivative of the K0 piece where the tile
kernels use it that way (the two pieces split at z = 6)."""
import os
import re

import numpy as np
import pytest
import scipy.special as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1908_07392_amd", "csrc", "constants.h")


def table(name):
    text = open(HEADER).read()
    m = re.search(r"static constexpr double " + name + r"\[(\d+)\] = \{(.*?)\};", text, re.S)
    vals = [float(x) for x in m.group(2).replace("\n", " ").split(",")]
    assert len(vals) == int(m.group(1))
    return np.array(vals)


def horner(c, v):
    p = np.zeros_like(v)
    for a in c[::-1]:
        p = p * v + a
    return p


def dhorner(c, v):
    return horner(np.arange(1, len(c)) * c[1:], v)


U6, U20 = 4.0 / 6 - 1, 4.0 / 20 - 1
PIECES = [  # name, nu, u range, with derivative
    ("KP0N", 0, (U6, 1.0), True), ("KP0F", 0, (-1.0, U6), True),
    ("KP0M", 0, (U20, U6), False), ("KP0X", 0, (-1.0, U20), False),
    ("KP1N", 1, (U6, 1.0), False), ("KP1F", 1, (-1.0, U6), False),
    ("KP1M", 1, (U20, U6), False), ("KP1X", 1, (-1.0, U20), False),
]


@pytest.mark.parametrize("name,nu,urange,der", PIECES)
def test_piece_matches_scaled_bessel(name, nu, urange, der):
    c = table(name)
    lo, hi = urange
    u = np.linspace(lo, hi, 2001)[1:] if lo == -1.0 else np.linspace(lo, hi, 2001)
    z = 4.0 / (u + 1.0)
    v = (2 * u - lo - hi) / (hi - lo)
    p = horner(c, v)
    ref = np.sqrt(z) * sp.kve(nu, z)
    assert np.max(np.abs(p / ref - 1)) < 4e-15, name
    if der:
        dp = dhorner(c, v) * 2 / (hi - lo)  # d/du
        k1 = p * (1 + 1 / (2 * z)) + 4 / z ** 2 * dp
        ref1 = np.sqrt(z) * sp.kve(1, z)
        assert np.max(np.abs(k1 / ref1 - 1)) < 4e-15, name


def test_pieces_join_at_the_breakpoints():
    """both sides of z = 6 and z = 20 give the same K0 (to rounding)"""
    def piece(name, lo, hi, z):
        u = 4.0 / z - 1
        return horner(table(name), np.array([(2 * u - lo - hi) / (hi - lo)]))[0]
    assert abs(piece("KP0N", U6, 1.0, 6.0) / piece("KP0M", U20, U6, 6.0) - 1) < 1e-15
    assert abs(piece("KP0M", U20, U6, 20.0) / piece("KP0X", -1.0, U20, 20.0) - 1) < 1e-15
    assert abs(piece("KP0F", -1.0, U6, 20.0) / piece("KP0X", -1.0, U20, 20.0) - 1) < 1e-15


def _fine_pieces():
    ulo, uhi = table("KQ_ULO"), table("KQ_UHI")
    out = []
    for k in range(len(ulo)):
        out.append((f"KQ0_{k}", 0, (ulo[k], uhi[k]), False))
        out.append((f"KQ1_{k}", 1, (ulo[k], uhi[k]), False))
    return out


@pytest.mark.parametrize("name,nu,urange,der", _fine_pieces())
def test_fine_piece_matches_scaled_bessel(name, nu, urange, der):
    """the fifteen fine pieces (eight single, seven spanning two neighbours) of the
    wave-classified far-field tiles, K0 and K1 each from a fit of its own"""
    test_piece_matches_scaled_bessel(name, nu, urange, der)


def table2d(name, rows, cols):
    text = open(HEADER).read()
    m = re.search(r"static constexpr float " + name + r"\[(\d+)\]\[(\d+)\] = \{(.*?)\};\n", text, re.S)
    assert (int(m.group(1)), int(m.group(2))) == (rows, cols)
    vals = [float(x.strip().rstrip("f")) for x in m.group(3).replace("{", " ").replace("}", " ").split(",") if x.strip()]
    return np.array(vals, dtype=np.float32).reshape(rows, cols)


@pytest.mark.parametrize("nu", [0, 1])
def test_fp32_fine_pieces_match_scaled_bessel(nu):
    """the FP32 fits of the fifteen fine pieces (mixed-precision far field),
    evaluated in float32 by Horner: within 1.2e-7 of e^z sqrt(z) K_nu(z)"""
    ulo, uhi = table("KQ_ULO"), table("KQ_UHI")
    c = table2d(f"KQF{nu}", 15, 6)
    for k in range(15):
        lo, hi = ulo[k], uhi[k]
        u = np.linspace(lo, hi, 801)[1:] if lo == -1.0 else np.linspace(lo, hi, 801)
        v = ((2 * u - lo - hi) / (hi - lo)).astype(np.float32)
        p = np.zeros_like(v)
        for a in c[k][::-1]:
            p = (p * v + a).astype(np.float32)
        z = 4.0 / (u + 1.0)
        ref = np.sqrt(z) * sp.kve(nu, z)
        assert np.max(np.abs(p.astype(np.float64) / ref - 1)) < 1.2e-7, (nu, k)


def test_fine_pieces_tile_the_axis():
    """single pieces k cover z in (B_k, B_k+1], the double pieces (B_s, B_s+2]"""
    b = table("KQ_B")
    ulo, uhi = table("KQ_ULO"), table("KQ_UHI")
    nb = len(b)
    zb = list(b) + [np.inf]
    for k in range(nb):
        assert abs(uhi[k] - (4 / zb[k] - 1)) < 1e-15 and abs(ulo[k] - (4 / zb[k + 1] - 1)) < 1e-15
    for s in range(nb - 1):
        assert abs(uhi[nb + s] - (4 / zb[s] - 1)) < 1e-15 and abs(ulo[nb + s] - (4 / zb[s + 2] - 1)) < 1e-15


YUKAWA = os.path.join(ROOT, "paper_1908_07392_amd", "csrc", "yukawa.h")


def yconst(name):
    m = re.search(r"constexpr double " + name + r" = ([-+0-9.eE]+);", open(YUKAWA).read())
    return float(m.group(1))


def test_exp_table_correctly_rounded():
    """2^(-j/64), j = 0..63, as the nearest doubles (Tang's table)."""
    import mpmath as mp
    mp.mp.dps = 40
    t = table("EXP2_NJ")
    assert len(t) == 64
    for j, v in enumerate(t):
        assert v == float(mp.mpf(2) ** (-mp.mpf(j) / 64)), j


def test_table_driven_exponential_matches_mpmath():
    """The kernels' e^{-z}: k = round(64 z log2 e) by the 1.5 2^52 shift,
    r = k ln2/64 - z in two fused steps, 2^{-(k >> 6)} 2^{-(k & 63)/64} times
    the degree-5 Taylor polynomial of e^r.  Emulated here with exactly rounded
    fused multiply-adds; within 3 ulp of e^{-z} from z = 0 to the underflow."""
    from fractions import Fraction
    import math
    import mpmath as mp
    mp.mp.dps = 40

    def fma(a, b, c):
        return float(Fraction(a) * Fraction(b) + Fraction(c))

    LOG2E, LN2_HI, LN2_LO = yconst("LOG2E"), yconst("LN2_HI"), yconst("LN2_LO")
    e2 = table("EXP2_NJ")
    expt = [1.0 / math.factorial(i) for i in range(6)]
    SHIFT = 6755399441055744.0
    rng = np.random.default_rng(3)
    zs = np.concatenate([np.linspace(0.0, 40.0, 1501), rng.uniform(0, 700, 500), [2.0, 3.0, 4.5, 7.0, 100.0, 0.0054]])
    worst = 0.0
    for z in zs:
        z = float(z)
        t = fma(z, 64.0 * LOG2E, SHIFT)
        kd = t - SHIFT
        r = fma(kd, LN2_HI / 64.0, -z)
        r = fma(kd, LN2_LO / 64.0, r)
        assert abs(r) <= math.log(2) / 128 * (1 + 1e-12)
        k = int(kd)
        p = expt[5]
        for c in expt[4::-1]:
            p = fma(p, r, c)
        v = math.ldexp(e2[k & 63] * p, -(k >> 6))
        ref = float(mp.exp(-mp.mpf(z)))
        if ref > 1e-300:
            worst = max(worst, abs(v - ref) / (ref * 2.0 ** -52))
    print(f"worst {worst:.2f} ulp")
    assert worst <= 3.0
