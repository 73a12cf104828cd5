"""Host-side checks of the C ABI (no GPU needed, no compute calls).

* the library loads and exports every function include/ode_ensemble.h
  declares;
* the synchronous validation paths that return before any HIP call;
* the ctypes structures have the C layout (sizes and offsets computed by a C
  compiler from the header itself);
* the oracle and the HIP path share no code, and the product never touches
  the oracle.
"""
import ctypes as C
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = glob.glob(os.path.join(ROOT, "include", "*.h"))


@pytest.fixture(scope="module")
def lib():
    from paper_1810_03931_amd import ensemble
    if not os.path.exists(ensemble.LIB_PATH):
        from paper_1810_03931_amd import build
        build.build()
    return ensemble.load_library()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(ode_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("ode_ensemble_create", "ode_ensemble_solve", "ode_ensemble_destroy",
              "ode_ensemble_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1810_03931_amd import ensemble
    out = subprocess.run(["nm", "-D", "--defined-only", ensemble.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for f in declared_functions():
        assert f in exported, f
        assert hasattr(lib, f)


def test_model_dims(lib):
    from paper_1810_03931_amd import ensemble as E
    assert E.model_dims("duffing") == (2, 5)
    assert E.model_dims("keller_miksis") == (2, 13)
    assert E.model_dims("relief_valve") == (3, 5)
    assert E.model_dims("ballistic") == (2, 1)
    assert E.model_dims("duffing_lyapunov") == (4, 5)
    ns, np_ = C.c_int32(), C.c_int32()
    assert lib.ode_ensemble_model_dims(99, C.byref(ns), C.byref(np_)) == E.EINVAL


@pytest.mark.parametrize("desc", [(99, 0, 0, 0), (1, 7, 0, 0), (1, 0, 5, 0), (1, 0, 0, 96),
                                  (1, 0, 0, 512), (1, 0, 0, 32), (1, 0, 0, 0, -1)])
def test_create_rejects_bad_descriptors_before_any_gpu_call(lib, desc):
    from paper_1810_03931_amd import ensemble as E
    d = E.Desc(*desc)
    h = C.c_void_p(123)
    rc = lib.ode_ensemble_create(C.byref(d), C.byref(h))
    assert rc in (E.EINVAL, E.ENOTSUP)
    assert h.value is None
    assert lib.ode_ensemble_last_error().decode()
    # the allocation-free solve checks the same descriptor before any HIP call
    a = E.SolveArgs()
    assert lib.ode_ensemble_solve_noalloc(C.byref(d), C.byref(a), None) in (E.EINVAL, E.ENOTSUP)


def test_null_arguments(lib):
    from paper_1810_03931_amd import ensemble as E
    assert lib.ode_ensemble_create(None, None) == E.EINVAL
    a = E.SolveArgs()
    assert lib.ode_ensemble_solve(None, C.byref(a), None) == E.EINVAL
    assert lib.ode_ensemble_solve_noalloc(None, C.byref(a), None) == E.EINVAL
    assert lib.ode_ensemble_solve_noalloc(C.byref(E.Desc(1, 0, 0, 0)), None, None) == E.EINVAL
    bad = E.SolveArgs()
    bad.n_systems, bad.ld = 5, 1  # ld < n_systems
    assert lib.ode_ensemble_solve_noalloc(C.byref(E.Desc(1, 0, 0, 0)), C.byref(bad), None) == E.EINVAL
    assert lib.ode_ensemble_solve_segments(None, C.byref(a), 1, 1.0, 1, None, None) == E.EINVAL
    r = E.TuneResult()
    assert lib.ode_ensemble_tune(None, C.byref(a), 1.0, None, C.byref(r)) == E.EINVAL
    n_pos = C.c_int64(0)
    assert lib.ode_ensemble_plan(None, C.byref(a), 0.02, 1.0, None, 0, C.byref(n_pos), None) == E.EINVAL
    assert lib.ode_plan_order(None, None, 0, 1, 1, None, 0, None) == E.EINVAL
    assert lib.ode_ensemble_query(None, None) == E.EINVAL
    lib.ode_ensemble_destroy(None)  # NULL is ignored


def test_struct_layout_matches_c(tmp_path):
    from paper_1810_03931_amd import ensemble as E
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "ode_ensemble.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ode_solve_args), sizeof(ode_event_spec),
         sizeof(ode_accessory_spec), sizeof(ode_ensemble_desc), sizeof(ode_ensemble_info),
         sizeof(ode_tune_result));
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", offsetof(ode_solve_args, tolerances),
         offsetof(ode_solve_args, rtol), offsetof(ode_solve_args, h0),
         offsetof(ode_solve_args, section_period), offsetof(ode_solve_args, max_steps),
         offsetof(ode_solve_args, events), offsetof(ode_solve_args, accessory_specs));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    sizes, offs = [list(map(int, l.split())) for l in
                   subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines()]
    assert sizes == [C.sizeof(E.SolveArgs), C.sizeof(E.EventSpec), C.sizeof(E.AccessorySpec),
                     C.sizeof(E.Desc), C.sizeof(E.Info), C.sizeof(E.TuneResult)]
    S = E.SolveArgs
    assert offs == [S.tolerances.offset, S.rtol.offset, S.h0.offset, S.section_period.offset, S.max_steps.offset,
                    S.events.offset, S.accessory_specs.offset]


def _sources(d, exts):
    for ext in exts:
        yield from glob.glob(os.path.join(ROOT, d, "**", "*" + ext), recursive=True)


def test_oracle_and_hip_path_share_no_code():
    for f in _sources("oracle", (".c", ".h", ".py")):
        text = open(f).read()
        assert "csrc" not in text and "ode_ensemble.h" not in text and \
            "paper_1810_03931_amd" not in text, f
    for f in _sources("paper_1810_03931_amd", (".hip", ".cpp", ".h", ".py")):
        text = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+oracle|oracle\.h|liboracle", text, re.M), f
