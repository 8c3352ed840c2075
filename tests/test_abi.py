"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/sibfa_pol.h declares, and its host-only helpers work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sibfa_pol.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sibfa_[A-Za-z_]+)\s*\(", txt)))


def _lib():
    from paper_2201_00804_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsibfa_pol.so not built (run __graft_entry__.build())")
    return _lib, _lib.load()


def test_header_declares_the_path():
    names = _declared()
    for must in ("sibfa_set_system", "sibfa_set_multipoles", "sibfa_set_polarizabilities",
                 "sibfa_solve_induced", "sibfa_energy_forces", "sibfa_permanent_field",
                 "sibfa_apply_T"):
        assert must in names


def test_library_exports_every_declared_symbol():
    mod, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(mod.exported_names()) == _declared()


def test_default_params_and_footprint():
    mod, lib = _lib()
    p = mod.Params()
    lib.sibfa_default_params(ctypes.byref(p))
    assert p.order == 5 and p.thole_a == pytest.approx(0.28) and p.tol_debye == pytest.approx(1e-8)
    p.grid[0] = p.grid[1] = p.grid[2] = 96
    box = (ctypes.c_double * 3)(98.55, 98.55, 98.55)
    big = lib.sibfa_footprint_bytes(160000, 96000, box, ctypes.byref(p))
    small = lib.sibfa_footprint_bytes(1080, 648, box, ctypes.byref(p))
    assert big > small > 0
    # invalid arguments give 0
    assert lib.sibfa_footprint_bytes(0, 0, box, ctypes.byref(p)) == 0
    assert lib.sibfa_footprint_bytes(10, 11, box, ctypes.byref(p)) == 0
    # clusters: lists are all-pairs
    assert lib.sibfa_footprint_bytes(320, 192, None, ctypes.byref(p)) > 320 * 319 * 4


def test_struct_layout_matches_header(tmp_path):
    """The binding's structures against the header, as a C compiler lays
    them out (size and the offset of every field)."""
    import shutil
    import subprocess
    mod, _ = _lib()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"sibfa_params": mod.Params, "sibfa_stats": mod.Stats,
               "sibfa_md_stats": mod.MdStats, "sibfa_ct_params": mod.CtParams,
               "sibfa_profile": mod.Profile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sibfa_pol.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def _prototypes():
    """name -> number of parameters, from the header's declarations."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(sibfa_[A-Za-z_]+)\s*\(([^;{]*?)\)\s*;", txt, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else len(args.split(","))
    return out


def test_binding_argument_counts_match_header():
    from paper_2201_00804_amd import _lib
    protos = _prototypes()
    for name, _, args in _lib.SIGNATURES:
        assert name in protos, name
        assert len(args) == protos[name], (name, len(args), protos[name])
