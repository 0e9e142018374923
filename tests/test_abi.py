"""The C ABI without a GPU: the library loads, exports every entry point the header declares,
its argument checks answer before any device work, and the ctypes mirrors of the header's
structs have the C layout (checked against gcc's sizeof / offsetof)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1307_3692_amd as ldd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldd.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:const\s+)?\w+\**\s+\**(ldd_\w+)\(", text, re.M)))


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(ldd.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = ldd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ldd.SO_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if " T " in line}
    assert set(declared_functions()) <= exported


def test_status_strings():
    L = ldd.lib()
    names = [L.ldd_status_string(i).decode() for i in range(11)]
    assert names[0] == "ok" and names[ldd.ERR_PENDING] == "pending" and names[10] == "unknown status"
    assert len(set(names)) == 11


def test_argument_errors_answer_before_device_work():
    L = ldd.lib()
    assert L.ldd_decompose(None, None, 1.0, None, None, None, None, None) == ldd.ERR_INVALID_ARG
    assert b"NULL" in L.ldd_last_error()
    assert L.ldd_decompose_batch(-1, None, None, None, None, None, None, None, None, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_create(None, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_submit(None, None, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_poll(None, 1, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_wait(None, 1, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_cancel(None, 1) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_query(None, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_server_destroy(None) == ldd.ERR_INVALID_ARG
    assert L.ldd_tune(0, None, None, None, None, None, None, None, None, None, None, None) == ldd.ERR_INVALID_ARG
    # a graph descriptor with bad sizes is rejected from the descriptor alone
    g = ldd.Csr(-1, 0, None, None)
    assert L.ldd_decompose(ctypes.byref(g), None, 1.0, None, None, None, None, None) == ldd.ERR_INVALID_ARG


def test_workspace_bytes_grows_with_n():
    L = ldd.lib()
    a, b = L.ldd_workspace_bytes(1000, 16000), L.ldd_workspace_bytes(2000, 32000)
    # 32 B per vertex for the round engines, 16 more for the workgroup engines beside them
    assert 0 < a < b and b - a >= 1000 * 48


def test_host_shift_sampler_equals_the_input_generator():
    """ldd_make_shifts (the library's host sampler, a host function) gives byte for byte the
    shifts of the seeded input generator that every test and benchmark input comes from."""
    import numpy as np

    import inputs
    for n, beta, seed in ((0, 0.1, 1), (1, 0.05, 2), (4096, 0.1, 1), (100_003, 0.02, 77), (20_000, 2.5, 2**63 + 5)):
        assert np.array_equal(ldd.make_shifts(n, beta, seed), inputs.make_shifts(n, beta, seed)), (n, beta, seed)
    L = ldd.lib()
    out = np.empty(4, np.int64)
    assert L.ldd_make_shifts(4, 0.0, 1, out.ctypes.data) == ldd.ERR_INVALID_ARG
    assert L.ldd_make_shifts(4, float("inf"), 1, out.ctypes.data) == ldd.ERR_INVALID_ARG
    assert L.ldd_make_shifts(-1, 0.1, 1, out.ctypes.data) == ldd.ERR_INVALID_ARG
    assert L.ldd_make_shifts(4, 0.1, 1, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_make_shifts_device(4, -1.0, 1, None, None) == ldd.ERR_INVALID_ARG
    assert L.ldd_decompose_verified(None, 0.1, 1, None, None, None, None, None, None) == ldd.ERR_INVALID_ARG


def test_host_shift_variants_equal_the_input_generator():
    """ldd_make_shifts_variant (host) gives byte for byte the input generator's shift variants of
    Sec. 5's closing remarks (integer shifts with a permutation tie-break; shifts from
    permutation positions)."""
    import numpy as np

    import inputs
    for kind in (ldd.SHIFTS_EXP, ldd.SHIFTS_INT_PERM, ldd.SHIFTS_PERM_ORDER):
        for n, beta, seed in ((0, 0.1, 1), (1, 0.3, 2), (5000, 0.1, 3), (70_001, 0.02, 2**64 - 3)):
            a = ldd.make_shifts_variant(n, beta, seed, kind)
            b = inputs.make_shifts_variant(n, beta, seed, kind)
            assert np.array_equal(a, b), (kind, n, beta, seed)
    out = np.empty(4, np.int64)
    assert ldd.lib().ldd_make_shifts_variant(4, 0.1, 1, 3, out.ctypes.data) == ldd.ERR_INVALID_ARG


STRUCTS = {"ldd_csr": ldd.Csr, "ldd_options": ldd.Options, "ldd_stats": ldd.Stats,
           "ldd_server_config": ldd.ServerConfig, "ldd_request": ldd.Request, "ldd_result": ldd.Result,
           "ldd_server_info": ldd.ServerInfo, "ldd_tune_report": ldd.TuneReport,
           "ldd_verify_options": ldd.VerifyOptions, "ldd_verify_report": ldd.VerifyReport}


def test_ctypes_layouts_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ldd.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                             check=True).stdout.splitlines())
    for cname, cls in STRUCTS.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(cls, field).offset, f"{cname}.{field}"


@pytest.mark.parametrize("cname", sorted(STRUCTS))
def test_every_c_field_is_mirrored(cname):
    """The ctypes mirror lists the C struct's fields in order (names parsed from the header)."""
    text = open(HEADER).read()
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + r";", text)
    assert m, cname
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    names = re.findall(r"(\w+)(?:\[\d+\])?\s*;", body)
    assert names == [f for f, _ in STRUCTS[cname]._fields_]
