"""The device's double-double powers (radii_dd.hpp, the radius ladder of
Sec. 2.1 formed without a host round trip) compiled for the host and held to
the correctly rounded power, computed here with 60-digit decimal arithmetic."""
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2203_14742_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "radii_dd.hpp"
#include <cstdio>
// "p x y": x^y;  "r x M": the ladder's base x^(1/M) and b^-1 .. b^-M from its log
int main() {
    cil::DDTables t;
    cil::dd_tables(t);
    char op;
    double x, y;
    while (std::scanf(" %c %la %la", &op, &x, &y) == 3) {
        if (op == 'p') {
            std::printf("%a\n", cil::pow_dd(x, y, t));
        } else {
            const int M = (int)y;
            cil::DD lb;
            const double b = cil::root_dd(x, M, t, &lb);
            std::printf("%a", b);
            for (int m = 1; m <= M; ++m) std::printf(" %a", cil::pow_dd_from_log(lb, -(double)m, t));
            std::printf("\n");
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("radii_dd")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I" + CSRC, "-x", "hip", str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


def correctly_rounded_pow(x: float, y: float) -> float:
    getcontext().prec = 60
    return float(str((Decimal(x).ln() * Decimal(y)).exp()))


def test_pow_dd_is_correctly_rounded(harness):
    g = np.random.default_rng(3)
    cases = []
    for _ in range(150):                        # b = (R_0 / R_M)^(1/M)
        cases.append((float(np.exp(g.uniform(0.0, 14.0))), 1.0 / int(g.integers(1, 65))))
    for _ in range(150):                        # b^-m
        cases.append((float(1.0 + g.uniform(0.0, 1.5)), float(-int(g.integers(1, 65)))))
    cases += [(1.0, 0.5), (2.0, -1.0), (4.0, 0.5), (1.2, -3.0), (float.fromhex("0x1.0000000000001p+0"), -64.0)]
    inp = "".join("p %s %s\n" % (float.hex(x), float.hex(y)) for x, y in cases)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout.split()
    got = [float.fromhex(v) for v in out]
    assert len(got) == len(cases)
    for (x, y), v in zip(cases, got):
        assert v == correctly_rounded_pow(x, y), (x, y)


def test_ladder_powers_are_correctly_rounded(harness):
    """The ladder's base b = x^(1/M) and the powers b^-m formed from log b
    (as the device forms the radii) are the correctly rounded ones."""
    g = np.random.default_rng(4)
    cases = [(float(np.exp(g.uniform(0.01, 12.0))), int(g.integers(1, 65))) for _ in range(40)]
    cases += [(1.0, 5), (float.fromhex("0x1.0000000000001p+0"), 64)]
    inp = "".join("r %s %s\n" % (float.hex(x), float.hex(float(M))) for x, M in cases)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout.splitlines()
    assert len(out) == len(cases)
    for (x, M), line in zip(cases, out):
        vals = [float.fromhex(v) for v in line.split()]
        b = vals[0]
        assert b == correctly_rounded_pow(x, 1.0 / M), (x, M)
        for m in range(1, M + 1):
            assert vals[m] == correctly_rounded_pow(b, -m), (x, M, m)
