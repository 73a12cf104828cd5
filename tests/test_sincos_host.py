"""The kernels' own sine/cosine (sincos_cw in the HIP sources, compiled here
for the host) against 60-digit values from Python's decimal module: the
accuracy the kernels' forcing terms rely on."""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_03931_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PI = Decimal("3.14159265358979323846264338327950288419716939937510582097494459230781640628620899862803")


def _ref(x: float):
    getcontext().prec = 60
    d = Decimal(x)
    k = (d / (PI / 2)).to_integral_value()
    r = d - k * (PI / 2)
    r2 = r * r
    s, term, n = Decimal(0), r, 1
    while abs(term) > Decimal(10) ** -58:
        s += term
        term = -term * r2 / ((n + 1) * (n + 2))
        n += 2
    c, term, n = Decimal(0), Decimal(1), 0
    while abs(term) > Decimal(10) ** -58:
        c += term
        term = -term * r2 / ((n + 1) * (n + 2))
        n += 2
    return [(s, c), (c, -s), (-s, -c), (-c, s)][int(k) % 4]


def _ulp(v: float) -> float:
    return math.ldexp(1.0, math.frexp(v)[1] - 53) if v != 0 else 5e-324


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("sincos")
    src = d / "t.hip"
    src.write_text("""
#include <cstdio>
#include "model_common.h"
int main() {
  double x;
  while (std::scanf("%la", &x) == 1) {
    double s, c;
    odeens::sincos_cw(x, s, c);
    std::printf("%a %a\\n", s, c);
  }
  return 0;
}
""")
    exe = d / "t"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def _run(exe, xs):
    out = subprocess.run([str(exe)], input="\n".join(float(x).hex() for x in xs), text=True,
                         capture_output=True, check=True).stdout.split()
    v = np.array([float.fromhex(t) for t in out]).reshape(-1, 2)
    return v[:, 0], v[:, 1]


def test_sincos_within_its_stated_bounds(prog):
    rng = np.random.default_rng(21)
    xs = list(rng.uniform(-7000, 7000, 600)) + list(rng.uniform(-1, 1, 200)) \
        + list(rng.uniform(-1e6, 1e6, 200))
    # next to the zeros of sin and cos: doubles adjacent to k*pi/2
    for k in rng.integers(1, 4000, 150):
        xs.append(float(np.nextafter(k * math.pi / 2, math.inf)))
    xs += [0.0, -0.0, 5e-310, 1e-20, math.pi / 4, 1e6]
    s, c = _run(prog, xs)
    rel, absol = [], []
    for x, sv, cv in zip(xs, s, c):
        rs, rc = _ref(x)
        for got, ref in ((sv, rs), (cv, rc)):
            err = abs(Decimal(got) - ref)
            absol.append(float(err))
            if abs(ref) > Decimal(2) ** -10:
                rel.append(float(err) / _ulp(float(ref)))
    rel = np.array(rel)
    assert rel.max() <= 0.75, rel.max()              # away from the zeros
    assert np.percentile(rel, 99) <= 0.6
    assert max(absol) <= 2.0 ** -53                     # everywhere, absolute


def test_large_arguments_use_the_library_and_symmetry(prog):
    xs = [2e6, -3.5e7, 1e15]
    s, c = _run(prog, xs)
    for x, sv, cv in zip(xs, s, c):
        assert sv == math.sin(x) and cv == math.cos(x)
    s1, c1 = _run(prog, [1.234, -1.234])
    assert s1[0] == -s1[1] and c1[0] == c1[1]
