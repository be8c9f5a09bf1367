"""CPU: the tables of the FP64 power in the edge kernels (csrc/pow_tables.inc) are what their
generator writes and what they claim to be -- C_j the double nearest 1 / (1 + (j + 1/2) / 128),
LH_j + LL_j = -ln C_j and TH_k + TL_k = 2^(k/128) as double-doubles -- checked against Python's
decimal logarithm and exponential at 50 digits, independently of the generator's code path."""
import math
import os
import re
import subprocess
import sys
from decimal import Decimal, getcontext

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2605_26975_amd", "csrc")


def _tables():
    text = open(os.path.join(CSRC, "pow_tables.inc")).read()
    vals = [float.fromhex(v) for v in re.findall(r"[-+]?0x[0-9a-fA-F.]+p[-+]?\d+", text)]
    assert len(vals) == 640
    return [vals[128 * i:128 * (i + 1)] for i in range(5)]


def test_generator_reproduces_the_committed_tables(tmp_path):
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_pow_tables.py")], cwd=tmp_path, check=True)
    assert (tmp_path / "pow_tables.inc").read_text() == open(os.path.join(CSRC, "pow_tables.inc")).read()


def test_table_values():
    getcontext().prec = 50
    C, LH, LL, TH, TL = _tables()
    ln2 = Decimal(2).ln()
    for j in range(128):
        c = 1 / (1 + (Decimal(j) + Decimal("0.5")) / 128)
        # nearest double: within half an ulp
        assert abs(Decimal(C[j]) - c) <= Decimal(math.ulp(C[j])) / 2
        # -ln C_j to double-double accuracy (|LL| below half an ulp of LH)
        exact = -Decimal(C[j]).ln()
        assert abs(Decimal(LH[j]) + Decimal(LL[j]) - exact) < Decimal(2) ** -100
        assert abs(LL[j]) <= math.ulp(LH[j]) / 2 if LH[j] != 0.0 else LL[j] == 0.0
    for k in range(128):
        exact = (Decimal(k) / 128 * ln2).exp()
        assert abs(Decimal(TH[k]) + Decimal(TL[k]) - exact) < Decimal(2) ** -100
        assert abs(TL[k]) <= math.ulp(TH[k]) / 2
    assert TH[0] == 1.0 and TL[0] == 0.0


def test_reduction_ranges():
    """The logarithm's reduction r = m C_j - 1 stays within 2^-8 for every m in [1, 2) of bin j, so
    the series of ln(1 + r) to r^8 leaves a truncation below 2^-67."""
    C = _tables()[0]
    for j in range(128):
        for m in (1 + j / 128, 1 + (j + 1) / 128 - 2.0 ** -52):
            r = m * C[j] - 1
            assert abs(r) <= 2.0 ** -8 * 1.0001
    assert (2.0 ** -8) ** 9 / 9 < 2.0 ** -67
