"""The C ABI library loads and exports what include/*.h declares (no GPU calls)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "inspirit.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(insp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2404_03226_amd import inspirit
    if not os.path.exists(inspirit.LIB_PATH):
        from paper_2404_03226_amd import build
        build.build()
    return inspirit.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "insp_build_dag" in names and "insp_schedule_batch" in names
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2404_03226_amd",
                                                                      "libinspirit.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(insp_[a-z_]+)\b", out))
    assert set(names) <= exported


def test_binding_names_cover_the_abi():
    from paper_2404_03226_amd import inspirit
    assert set(inspirit.EXPORTS) == set(declared_functions())


def test_struct_layouts_match_header():
    from paper_2404_03226_amd import inspirit
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "inspirit.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(insp_params), sizeof(insp_workers), sizeof(insp_trace_rec),
         offsetof(insp_params, max_events), offsetof(insp_trace_rec, popped));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = list(map(int, subprocess.check_output([exe]).split()))
    assert got[0] == C.sizeof(inspirit.Params)
    assert got[1] == C.sizeof(inspirit.Workers)
    assert got[2] == inspirit.TRACE_DTYPE.itemsize
    assert got[3] == inspirit.Params.max_events.offset
    assert got[4] == inspirit.TRACE_DTYPE.fields["popped"][1]


def test_error_path_without_gpu(lib):
    # argument checks that return before any device call
    from paper_2404_03226_amd import inspirit
    h = C.c_void_p()
    rc = lib.insp_build_dag(0, None, None, None, None, None, None, C.byref(h))
    assert rc == inspirit.E_INVAL
    assert b"n_dags" in lib.insp_last_error()
    assert lib.insp_sync_status(None, None) == inspirit.E_INVAL
    lib.insp_free_dag(None)


def test_cost_model_argument_checks_without_gpu(lib):
    # every insp_mlp_* entry point rejects a missing model before any device call
    from paper_2404_03226_amd import inspirit
    E = inspirit.E_INVAL
    assert lib.insp_mlp_create(None, None) == E
    assert lib.insp_mlp_grads(None, None, None, 32, None, None, None, None) == E
    assert lib.insp_mlp_train_step(None, None, None, 32, 1e-3, None, None) == E
    assert lib.insp_mlp_train(None, None, None, 1024, 32, 1, 1e-3, None, None) == E
    assert b"bad argument" in lib.insp_last_error()
    assert lib.insp_mlp_predict(None, None, 0, None, None, None) == E
    assert lib.insp_mlp_state(None, None, None, None, None, 1) == E
    lib.insp_mlp_free(None)


def test_missing_library_fails_loudly(tmp_path):
    from paper_2404_03226_amd import inspirit
    saved = inspirit._lib
    inspirit._lib = None
    try:
        with pytest.raises(ImportError):
            inspirit.load(str(tmp_path / "absent.so"))
    finally:
        inspirit._lib = saved
