"""The C-ABI library loads, exports every symbol include/refl.h declares, and
its struct layouts agree with the Python binding (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2605_24840_amd import refl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "refl.h")


def _declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:refl_status_t|const char\s*\*|int)\s*(refl_\w+)\s*\(", src, re.M)))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    assert set(names) == set(refl.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = refl.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", refl.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (refl_\w+)", out))
    assert set(_declared_functions()) <= exported
    # Nothing else leaks out under the refl_ prefix.
    assert exported == set(_declared_functions())


def test_debug_build_exports_the_same_symbols():
    """The bounds-checked build (-DREFL_DEBUG) is the same boundary: the
    same exported names, and refl_debug_build() tells the two apart (a call
    that touches no device)."""
    assert os.path.exists(refl.DEBUG_LIB_PATH), "build it with build(debug=True)"
    out = subprocess.run(["nm", "-D", "--defined-only", refl.DEBUG_LIB_PATH], capture_output=True,
                         text=True).stdout
    assert set(re.findall(r" T (refl_\w+)", out)) == set(_declared_functions())
    rel = ctypes.CDLL(refl.LIB_PATH)
    dbg = ctypes.CDLL(refl.DEBUG_LIB_PATH)
    assert rel.refl_debug_build() == 0 and dbg.refl_debug_build() == 1
    dbg.refl_status_string.restype = ctypes.c_char_p
    assert dbg.refl_status_string(refl.REFL_ERR_BOUNDS) == b"REFL_ERR_BOUNDS"


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "refl.h"\n'
        "int main(void){\n"
        'printf("%zu %zu\\n", sizeof(refl_params_t), sizeof(refl_info_t));\n'
        'printf("%zu %zu %zu\\n", offsetof(refl_params_t, seed), offsetof(refl_params_t, cg_tol),'
        " offsetof(refl_params_t, lanczos_steps));\n"
        'printf("%zu %zu %zu %zu\\n", offsetof(refl_info_t, s), offsetof(refl_info_t, dk_bound),'
        " offsetof(refl_info_t, ms_total), offsetof(refl_info_t, gamma));\n"
        'printf("%zu %zu %zu %zu\\n", offsetof(refl_params_t, check_symmetric), offsetof(refl_params_t, sym_tol),'
        " offsetof(refl_info_t, bulk_tile), offsetof(refl_info_t, bulk_words));\n"
        'printf("%zu\\n", offsetof(refl_params_t, words_max));\n'
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sp, si = map(int, lines[0].split())
    assert sp == ctypes.sizeof(refl.refl_params_t)
    assert si == ctypes.sizeof(refl.refl_info_t)
    o = list(map(int, lines[1].split()))
    assert o == [refl.refl_params_t.seed.offset, refl.refl_params_t.cg_tol.offset,
                 refl.refl_params_t.lanczos_steps.offset]
    o = list(map(int, lines[2].split()))
    assert o == [refl.refl_info_t.s.offset, refl.refl_info_t.dk_bound.offset, refl.refl_info_t.ms_total.offset,
                 refl.refl_info_t.gamma.offset]
    o = list(map(int, lines[3].split()))
    assert o == [refl.refl_params_t.check_symmetric.offset, refl.refl_params_t.sym_tol.offset,
                 refl.refl_info_t.bulk_tile.offset, refl.refl_info_t.bulk_words.offset]
    assert int(lines[4]) == refl.refl_params_t.words_max.offset


def _header_enum(name):
    """Enumerator -> value of the typedef enum ``name`` in include/refl.h."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef enum\s*\{([^{}]*)\}\s*" + name + r"\s*;", src)
    assert m, name
    body = m.group(1)
    out = {}
    for item in body.split(","):
        item = item.strip()
        if item:
            k, v = item.split("=")
            out[k.strip()] = int(v)
    return out


def test_enum_values_match_header_and_binding():
    """The binding's code tables equal the header's enumerators, and the
    status and scale codes are those of the boundary sketch (statuses
    0..8 in its order, REFL_ERR_NOT_FINITE added as 9 and the debug build's
    REFL_ERR_BOUNDS as 10; scales INF, FRO, LANCZOS, GIVEN = 0..3)."""
    st = _header_enum("refl_status_t")
    assert {v: k for k, v in st.items()} == refl.STATUS
    assert [st[n] for n in ("REFL_OK", "REFL_ERR_INVALID_ARG", "REFL_ERR_DEVICE", "REFL_ERR_NO_MEMORY",
                            "REFL_ERR_NOT_CONVERGED", "REFL_ERR_NOT_ADMISSIBLE", "REFL_ERR_NO_GAP",
                            "REFL_ERR_NOT_SYMMETRIC", "REFL_ERR_UNSUPPORTED",
                            "REFL_ERR_NOT_FINITE", "REFL_ERR_BOUNDS")] == list(range(11))
    sc = _header_enum("refl_scale_mode_t")
    assert sc == {"REFL_SCALE_INF": 0, "REFL_SCALE_FRO": 1, "REFL_SCALE_LANCZOS": 2, "REFL_SCALE_GIVEN": 3}
    assert {"REFL_SCALE_" + k.upper(): v for k, v in refl.SCALE.items()} == sc
    pr = _header_enum("refl_precision_t")
    assert {"REFL_PREC_" + k.upper(): v for k, v in refl.PRECISION.items()} == pr
    cg = _header_enum("refl_cg_prec_t")
    assert {"REFL_CG_" + k.upper(): v for k, v in refl.CG_PREC.items()} == cg
    gm = _header_enum("refl_grad_mode_t")
    assert {"REFL_GRAD_" + k.upper(): v for k, v in refl.GRAD_MODE.items()} == gm
    po = _header_enum("refl_policy_mode_t")
    assert {"REFL_POLICY_" + k.upper(): v for k, v in refl.POLICY.items()} == po


def test_params_default_and_status_strings():
    p = refl.refl_params_default()
    assert (p.k, p.tol, p.max_iter, p.fixed_steps, p.words, p.polish_sweeps) == (1, 1e-12, 100, 0, 2, 2)
    assert p.precision == refl.PRECISION["fp64"] and p.shift_mode == refl.SHIFT["given"]
    assert p.check_symmetric == 0 and p.sym_tol == 0.0 and p.scale_mode == refl.SCALE["inf"]
    for code, name in refl.STATUS.items():
        assert refl.refl_status_string(code) == name
    assert refl.refl_status_string(99) == "REFL_ERR_UNKNOWN"


def test_null_arguments_rejected_without_device():
    lib = refl.load()
    assert lib.refl_params_default(None) == 1
    assert lib.refl_create(None, 0, None) == 1
    assert lib.refl_destroy(None) == 1
    assert lib.refl_sign(None, 4, None, 4, None, None, 4, None) == 1
    assert lib.refl_sign_batched(None, 1, None, None, None, None, None, None, None, None) == 1
    assert lib.refl_sign_batched_workspace_size(None, 1, None, None, None) == 1
    assert refl.load().refl_last_error(None) == b"NULL handle"


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert refl.load().refl_create(ctypes.byref(h), 0, None) == 2


def test_policy_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "pol.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "refl.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(refl_policy_params_t), sizeof(refl_policy_info_t),'
        " offsetof(refl_policy_params_t, seed), offsetof(refl_policy_info_t, refreshed),"
        " offsetof(refl_policy_info_t, refreshes), offsetof(refl_policy_params_t, warm_start));\n"
        "return 0;}\n")
    exe = tmp_path / "pol"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    assert got == [ctypes.sizeof(refl.refl_policy_params_t), ctypes.sizeof(refl.refl_policy_info_t),
                   refl.refl_policy_params_t.seed.offset, refl.refl_policy_info_t.refreshed.offset,
                   refl.refl_policy_info_t.refreshes.offset, refl.refl_policy_params_t.warm_start.offset]
