"""The tables of the table-driven binary64 exp and log (casim_math_tables.h)
against their definitions, recomputed here in 60-digit decimal arithmetic,
and against the generator that wrote them."""
import decimal
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2010_14823_amd", "csrc")
D = decimal.Decimal


def _tables():
    text = open(os.path.join(CSRC, "casim_math_tables.h")).read()
    hexnum = r"(-?0x[0-9a-fA-F.]+p[-+]?\d+)"
    consts = {m.group(1): float.fromhex(m.group(2))
              for m in re.finditer(r"constexpr double (\w+) = " + hexnum, text)}
    exp_block = text[text.index("kExp2Tab[kExpTab] = {"):]
    exp_block = exp_block[:exp_block.index("};")]
    exp2 = [float.fromhex(v) for v in re.findall(r"^\s+" + hexnum + ",", exp_block, re.M)]
    log_block = text[text.index("kLogTabData[kLogTab][3] = {"):]
    log_block = log_block[:log_block.index("};")]
    logt = [tuple(float.fromhex(v) for v in m)
            for m in re.findall(r"\{" + hexnum + ", " + hexnum + ", " + hexnum + r"\}", log_block)]
    return consts, exp2, logt


def test_exp_table_is_two_to_j_over_64_rounded_once():
    decimal.getcontext().prec = 60
    ln2 = D(2).ln()
    _, exp2, _ = _tables()
    assert len(exp2) == 64
    for j, v in enumerate(exp2):
        exact = (ln2 * j / 64).exp()
        assert v == float(exact), j
        # correctly rounded: within half an ulp
        assert abs(D(v) - exact) <= D(2) ** -53 * exact


def test_log_table_definition_and_exact_ends():
    decimal.getcontext().prec = 60
    consts, _, logt = _tables()
    hi2, lo2 = consts["kLn2Hi"], consts["kLn2Lo"]
    assert (D(hi2) * 2 ** 33) % 1 == 0                       # on the 2^-33 grid
    assert abs(D(hi2) + D(lo2) - D(2).ln()) <= D(2) ** -53 * abs(D(lo2))   # lo rounded once
    assert len(logt) == 129
    for j, (c, hi, lo) in zip(range(128, 257), logt):
        assert c == 256.0 / j
        assert (D(hi) * 2 ** 33) % 1 == 0
        target = -(D(c).ln())                                  # of the rounded c_j
        assert abs(D(hi) + D(lo) - target) <= D(2) ** -52 * max(abs(D(lo)), D(2) ** -80), j
    # ln(1) is exactly 0 (j = 256 and, via e = 1, j = 128): the high parts cancel
    assert logt[-1] == (1.0, 0.0, 0.0)
    assert logt[0] == (2.0, -hi2, -lo2)


def test_generator_reproduces_the_header(tmp_path):
    src = os.path.join(CSRC, "gen_math_tables.py")
    code = open(src).read().replace(
        'os.path.join(os.path.dirname(os.path.abspath(__file__)), "casim_math_tables.h")',
        repr(str(tmp_path / "t.h")))
    script = tmp_path / "gen.py"
    script.write_text(code)
    subprocess.run([sys.executable, str(script)], check=True, capture_output=True)
    assert (tmp_path / "t.h").read_text() == open(os.path.join(CSRC, "casim_math_tables.h")).read()
