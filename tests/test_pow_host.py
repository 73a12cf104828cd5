"""The kernels' own power function for positive bases (pow_pos in the HIP
sources, compiled here for the host) against 60-digit values from Python's
decimal module: the accuracy the Keller-Miksis gas-pressure term relies on."""
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


def _ulp(v: float) -> float:
    return math.ldexp(1.0, math.frexp(v)[1] - 53) if v != 0 else 5e-324


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("pow")
    src = d / "t.hip"
    src.write_text("""
#include <cstdio>
#include "model_common.h"
int main() {
  double x, c;
  while (std::scanf("%la %la", &x, &c) == 2) std::printf("%a\\n", odeens::pow_pos(x, c));
  return 0;
}
""")
    exe = d / "t"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def _run(exe, pairs):
    text = "\n".join(f"{float(x).hex()} {float(c).hex()}" for x, c in pairs)
    out = subprocess.run([str(exe)], input=text, text=True, capture_output=True,
                         check=True).stdout.split()
    return np.array([float.fromhex(t) for t in out])


def _ref(x: float, c: float) -> Decimal:
    getcontext().prec = 60
    return Decimal(x) ** Decimal(c)


def test_pow_within_one_ulp(prog):
    rng = np.random.default_rng(7)
    xs = list(10.0 ** rng.uniform(-3, 3, 1500)) + list(rng.uniform(0.5, 2.0, 500))
    cs = [4.2, 3.0 * 1.4, 1.4, 0.2] + list(rng.uniform(0.0, 8.0, 8))
    pairs = [(x, cs[i % len(cs)]) for i, x in enumerate(xs)]
    pairs += [(1.0, 4.2), (2.0, 3.0), (0.5, 4.2), (float(np.nextafter(1.0, 0.0)), 4.2),
              (float(np.nextafter(1.0, 2.0)), 4.2), (float.fromhex("0x1.6a09e667f3bcdp-1"), 4.2),
              (float.fromhex("0x1.6a09e667f3bcdp+0"), 4.2)]
    got = _run(prog, pairs)
    err = []
    for (x, c), g in zip(pairs, got):
        ref = _ref(x, c)
        err.append(float(abs(Decimal(g) - ref)) / _ulp(float(ref)))
    err = np.array(err)
    print(f"[pow_pos] ulp error: max {err.max():.3f} p99 {np.percentile(err, 99):.3f} "
          f"mean {err.mean():.3f}")
    assert err.max() <= 1.0
    assert np.percentile(err, 99) <= 0.75
    assert got[-7] == 1.0 and got[-6] == 8.0


def test_outside_the_fast_domain_uses_the_library(prog):
    pairs = [(0.0, 4.2), (-0.0, 3.0), (0.0, -2.0), (-2.0, 3.0), (-2.0, 2.0), (-2.0, 0.5),
             (math.inf, 2.0), (-math.inf, 3.0), (math.inf, -1.5), (math.nan, 2.0), (2.0, math.nan),
             (1.0, math.nan), (math.nan, 0.0), (0.5, math.inf), (2.0, -math.inf),
             (1e-300, 4.2), (1e300, 4.2), (1e-300, -4.2), (3.0, 700.0)]
    got = _run(prog, pairs)
    with np.errstate(all="ignore"):
        ref = np.power(np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]))
    for (x, c), g, r in zip(pairs, got, ref):
        assert (g == r and math.copysign(1, g) == math.copysign(1, r)) or \
            (math.isnan(g) and math.isnan(r)) or abs(g - r) <= 2 * _ulp(r), (x, c, g, r)
