#!/usr/bin/env python3
"""Print the constants of the table-driven exp in gemv64.hip.

T_j = 2^(j/64), j = 0..63, as a pair (hi, lo): hi the double nearest T_j, lo
the double nearest T_j - hi (so hi + lo carries about 106 bits); ln2/64 split
into a 33-bit head (k * head is exact for |k| < 2^20) and a tail.  Decimal
arithmetic at 60 digits; the output is C hex-float literals.
"""
from decimal import Decimal, getcontext
import math

getcontext().prec = 60
ln2 = Decimal(2).ln()
L = ln2 / 64
m, ex = math.frexp(float(L))
head = math.ldexp(math.floor(m * 2 ** 32) / 2 ** 32, ex)
tail = float(L - Decimal(head))
print(f"// 64/ln2 = {float(Decimal(64) / ln2).hex()}, ln2/64 head = {head.hex()}, tail = {tail.hex()}")
for j in range(64):
    v = Decimal(2) ** (Decimal(j) / Decimal(64))
    hi = float(v)
    lo = float(v - Decimal(hi))
    print(f"    {hi.hex()}, {lo.hex()},")
