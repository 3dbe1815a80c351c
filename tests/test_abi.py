"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/pmcmc.h, reports a missing device as PMC_ERR_HIP with a
message, and rejects invalid arguments before touching the device."""
import ctypes as C
import os

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pmcmc.h")


def _lib():
    from paper_2508_18413_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        from paper_2508_18413_amd import build
        build.build()
    return B, B.lib()


def test_exports_every_declared_symbol():
    B, L = _lib()
    names = B.exported_symbols(HEADER)
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_error_strings():
    B, L = _lib()
    assert b"libpmcmc" in L.pmc_version()
    assert isinstance(L.pmc_last_error(), bytes)


def test_null_arguments_are_rejected():
    B, L = _lib()
    assert L.pmc_create(None, 0, None) == B.PMC_ERR_INVALID
    assert b"NULL" in L.pmc_last_error()
    assert L.pmc_solve(None, None, None, None, 0, None) == B.PMC_ERR_INVALID
    assert L.pmc_sample_sequential(None, None, None) == B.PMC_ERR_INVALID
    assert L.pmc_linrec_diag(None, 0, 1, 1, None, None, None) == B.PMC_ERR_INVALID
    assert L.pmc_default_options(None, 0) == B.PMC_ERR_INVALID
    sz = C.c_size_t()
    assert L.pmc_workspace_size(None, None, None, C.byref(sz)) == B.PMC_ERR_INVALID
    # destroying NULL handles is a no-op
    assert L.pmc_destroy(None) == B.PMC_OK
    assert L.pmc_target_destroy(None) == B.PMC_OK


def test_default_options():
    B, L = _lib()
    o = B.pmc_options()
    assert L.pmc_default_options(C.byref(o), B.PMC_F32) == B.PMC_OK
    assert o.variant == B.PMC_QDEER_DIAG and o.atol == 5e-7 and o.damping == 1.0
    assert o.skip_converged_prefix == 1 and o.floor_stall == 16
    assert L.pmc_default_options(C.byref(o), B.PMC_F64) == B.PMC_OK
    assert o.atol == 1e-12


def test_no_device_is_reported_not_faked():
    """Without a GPU, creating a context fails loudly; with one it succeeds."""
    B, L = _lib()
    import torch
    h = C.c_void_p()
    st = L.pmc_create(C.byref(h), 0, None)
    if torch.cuda.is_available():
        assert st == B.PMC_OK
        L.pmc_destroy(h)
    else:
        assert st == B.PMC_ERR_HIP
        assert len(L.pmc_last_error()) > 0


def test_binding_has_no_fallback(monkeypatch):
    """The Python front end raises when the library is absent."""
    from paper_2508_18413_amd import _binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", os.path.join(ROOT, "does-not-exist.so"))
    with pytest.raises(RuntimeError):
        B.lib()


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures of the binding have the size and field offsets
    that a C compiler gives the header's structs (gcc on this host)."""
    import shutil
    import subprocess
    from paper_2508_18413_amd import _binding as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [B.pmc_target_desc, B.pmc_problem, B.pmc_options, B.pmc_result]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pmcmc.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in st._fields_:
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == C.sizeof(st), name
        for f in st._fields_:
            assert got[(name, f[0])] == getattr(st, f[0]).offset, (name, f[0])


def test_enum_values_match_header(tmp_path):
    """The binding's enum constants are the header's values (gcc on this host)."""
    import shutil
    import subprocess
    from paper_2508_18413_amd import _binding as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    names = [n for n in dir(B) if n.startswith(("PMC_PRODUCTS_", "PMC_GATE_", "PMC_SAMPLER_", "PMC_QDEER_"))
             and isinstance(getattr(B, n), int)]
    assert "PMC_PRODUCTS_REFINE" in names
    lines = ["#include <stdio.h>", '#include "pmcmc.h"', "int main(void) {"]
    lines += [f'  printf("{n} %d\\n", (int){n});' for n in names]
    lines += ["  return 0;", "}"]
    src = tmp_path / "enums.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "enums"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict((l.split()[0], int(l.split()[1])) for l in out if l)
    for n in names:
        assert got[n] == getattr(B, n), n
