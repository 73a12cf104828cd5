"""Build the CPU oracle shared libraries (test infrastructure only).

``python oracle/build.py`` compiles ``ode_oracle.c`` with gcc into

* ``liboracle.so``: binary64, no floating-point contraction -- the oracle;
* ``liboracle_fma.so``: the same source with every a*b+c contracted into a
  fused multiply-add.  It is a differently rounded but equally valid
  evaluation of the same definitions, used only to calibrate the parity bars
  (how far rounding alone moves a result, how many step decisions it flips);
  it is never the reference a result is compared with.

Both use OpenMP over systems.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ode_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")

COMMON = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra"]
VARIANTS = {
    LIB: ["-ffp-contract=off"],
    LIB_FMA: ["-ffp-contract=fast", "-mfma"],
}


def build(verbose: bool = False) -> str:
    for out, flags in VARIANTS.items():
        cmd = COMMON + flags + ["-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
