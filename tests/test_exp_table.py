"""The constants of the table-driven exp in csrc/gemv64.hip, checked on the CPU
against 60-digit decimal arithmetic: every (hi, lo) pair is 2^(j/64) rounded to
double and the rounded remainder, and the reduction constants are 64/ln2 and a
33-bit head of ln2/64 (so k * head is exact for |k| < 2^20) plus its tail."""
import math
import os
import re
from decimal import Decimal, getcontext

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2607_23354_amd", "csrc", "gemv64.hip")


def _source():
    return open(SRC).read()


def test_exp2_table_is_correctly_rounded():
    getcontext().prec = 60
    s = _source()
    body = s[s.index("kExp2Tab[128] = {"):]
    body = body[:body.index("};")]
    vals = [float.fromhex(v) for v in re.findall(r"-?0x[0-9a-f.]+p[+-]\d+", body)]
    assert len(vals) == 128
    for j in range(64):
        hi, lo = vals[2 * j], vals[2 * j + 1]
        exact = Decimal(2) ** (Decimal(j) / Decimal(64))
        assert hi == float(exact), j
        assert lo == float(exact - Decimal(hi)), j
        assert abs(Decimal(hi) + Decimal(lo) - exact) < Decimal(2) ** -104


def test_exp_reduction_constants():
    getcontext().prec = 60
    s = _source()
    body = s[s.index("__device__ __forceinline__ double exp_tab("):]
    body = body[:body.index("}")]
    c = [float.fromhex(v) for v in re.findall(r"0x[0-9a-f.]+p[+-]\d+", body)]
    inv, head, tail = c[0], c[1], c[2]
    ln2 = Decimal(2).ln()
    assert inv == float(Decimal(64) / ln2)
    m, _ = math.frexp(head)
    assert (m * 2 ** 33) == int(m * 2 ** 33)  # 33 significant bits
    assert abs(Decimal(head) + Decimal(tail) - ln2 / 64) < Decimal(2) ** -90
