"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/bf.h declares, and rejects bad arguments before it
touches a device."""
import ctypes as C
import os
import re

import pytest

import paper_2002_03400_amd as bf

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "bf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z0-9_]+)\s*\(", text)) - {"bf_op_fn"})


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bf.LIB_PATH):
        pytest.skip("libbf.so not built")
    L = C.CDLL(bf.LIB_PATH)
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(bf.SIGNATURES)


def test_argument_errors_without_device():
    if not os.path.exists(bf.LIB_PATH):
        pytest.skip("libbf.so not built")
    lib = bf.lib()
    h = C.c_void_p()
    o = bf.bf_opts(2, 4, 0, 0, 0)
    # NULL callbacks, m <= 0, tol outside (0,1), leaf < 1
    assert lib.bf_construct(None, None, None, 10, 10, 1e-6, 4, C.byref(o), None, None,
                            C.byref(h)) == -1
    assert lib.bf_apply(None, 0, None, 1, 1, None, 1, None, None) == -1
    assert lib.bf_stats(None, None) == -1
    assert lib.bf_free(None, None) == -1
    assert lib.bf_strerror(-4) == b"rank cap exceeded or block too large"
    assert lib.bf_op_fio(7, None) == -1
    assert lib.bf_set_apply_precision(None, 1) == -1
    assert lib.bf_op_set_precision(None, 1) == -1
    # the autotuner switch and its counter touch no device
    assert lib.bf_autotune_entries(None) == -1
    n = C.c_int64(-1)
    assert lib.bf_set_autotune(0) == 0
    assert lib.bf_autotune_entries(C.byref(n)) == 0 and n.value >= 0
    assert lib.bf_set_autotune(1) == 0


def test_precision_enum_matches_header():
    text = open(HEADER).read()
    vals = dict((k, int(v)) for k, v in re.findall(r"(BF_PREC_[A-Z0-9]+)\s*=\s*(\d+)", text))
    assert vals == {"BF_PREC_FP64": 0, "BF_PREC_BF16X3": 1, "BF_PREC_FP32": 2}


def test_option_flags_match_header():
    """The bf_opts flag bits the binding passes are the header's."""
    text = open(HEADER).read()
    flags = dict((k, int(v)) for k, v in re.findall(r"(BF_OPT_[A-Z_]+)\s*=\s*(\d+)", text))
    assert flags == {"BF_OPT_CENTER_LEVEL": 1, "BF_OPT_SEQUENTIAL_LEAF": 2,
                     "BF_OPT_SEQUENTIAL_SWEEP": 4, "BF_OPT_ONE_STREAM": 8}
    for k, v in flags.items():
        assert getattr(bf, k) == v


def test_error_codes_match_header():
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"(BF_E[A-Z]+)\s*=\s*(-\d+)", text))
    assert codes == {"BF_EINVAL": -1, "BF_ENOMEM": -2, "BF_ECALLBACK": -3, "BF_ERANK": -4,
                     "BF_EHIP": -5, "BF_ENOTSUP": -6}


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the public structs have the C compiler's sizes
    and field offsets (a mismatch would pass garbage across the ABI)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"bf_opts": bf.bf_opts, "bf_info": bf.bf_info, "bf_operator": bf.bf_operator,
               "bf_kernel_stats": bf.bf_kernel_stats, "bf_server_opts": bf.bf_server_opts,
               "bf_request_info": bf.bf_request_info, "bf_alloc": bf.bf_alloc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bf.h"', "int main(void) {"]
    for name, py in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, py in structs.items():
        assert got[(name, "size")] == C.sizeof(py), name
        for fname, _ in py._fields_:
            assert got[(name, fname)] == getattr(py, fname).offset, (name, fname)


def test_allocator_without_functions_is_rejected():
    """A bf_alloc must carry both functions; the check comes before any device
    work (also for the request engine, whose options copy the allocator)."""
    if not os.path.exists(bf.LIB_PATH):
        pytest.skip("libbf.so not built")
    lib = bf.lib()
    half = bf.bf_alloc(None, bf.ALLOCFN(lambda c, n, s: None), bf.FREEFN())
    h = C.c_void_p()
    o = bf.bf_opts(2, 4, 0, 0, 0)
    cb = bf.OPFN(lambda *a: 0)
    assert lib.bf_construct(cb, cb, None, 10, 10, 1e-6, 4, C.byref(o), C.byref(half), None,
                            C.byref(h)) == -1
    assert not h.value
    so = bf.bf_server_opts(1, 0, 0, C.pointer(half))
    assert lib.bf_server_create(C.byref(so), C.byref(h)) == -1


def test_autotuner_table_round_trip(tmp_path):
    """The tuner's table is written and read back as text (one class per line:
    family, five class fields, choice) without a device; unknown families are
    ignored and a missing file is an error."""
    if not os.path.exists(bf.LIB_PATH):
        pytest.skip("libbf.so not built")
    lib = bf.lib()
    src = tmp_path / "in.tsv"
    src.write_text("# family  class fields (5)  choice\n"
                   "chain_rows 1 19 1024 64 0 20\n"
                   "cpqr_threads 0 64 64 1024 0 512\n"
                   "no_such_family 1 2 3 4 5 6\n")
    assert lib.bf_autotune_clear() == 0
    assert lib.bf_autotune_load(str(src).encode()) == 0
    n = C.c_int64(-1)
    assert lib.bf_autotune_entries(C.byref(n)) == 0 and n.value == 2
    out = tmp_path / "out.tsv"
    assert lib.bf_autotune_save(str(out).encode()) == 0
    lines = [l.split() for l in out.read_text().splitlines() if l and not l.startswith("#")]
    assert sorted(lines) == sorted([["chain_rows", "1", "19", "1024", "64", "0", "20"],
                                    ["cpqr_threads", "0", "64", "64", "1024", "0", "512"]])
    assert lib.bf_autotune_load(str(tmp_path / "missing.tsv").encode()) == -1
    assert lib.bf_autotune_clear() == 0
