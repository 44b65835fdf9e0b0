"""CPU-side checks of the C-ABI library: it loads and exports every symbol that
include/mcpt.h declares; host-side argument marshalling (no compute calls)."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcpt.h")
LIB = os.path.join(ROOT, "paper_1409_2700_amd", "libmcpt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcpt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mcpt_create", "mcpt_solve", "mcpt_energy", "mcpt_upload", "mcpt_run",
                     "mcpt_release", "mcpt_destroy", "mcpt_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcpt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcpt.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_1409_2700_amd import EXPORTS
    assert sorted(EXPORTS) == declared_functions()


def _c_layout(tmp_path):
    """Sizes and field offsets of the header's structs as a C compiler lays them out."""
    from paper_1409_2700_amd import mcpt as m
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcpt.h"', "int main(void) {"]
    for cname in ("mcpt_problem", "mcpt_options", "mcpt_summary", "mcpt_timing", "mcpt_serve_counters", "mcpt_tune_result",
                  "mcpt_singles_summary", "mcpt_lccd_integrals", "mcpt_fd_mode", "mcpt_fd_result",
                  "mcpt_dimer_integrals"):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(m, cname)._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_struct_layouts_match_header(tmp_path):
    from paper_1409_2700_amd import mcpt as m
    lay = _c_layout(tmp_path)
    for cname in ("mcpt_problem", "mcpt_options", "mcpt_summary", "mcpt_timing", "mcpt_serve_counters", "mcpt_tune_result",
                  "mcpt_singles_summary", "mcpt_lccd_integrals", "mcpt_fd_mode", "mcpt_fd_result",
                  "mcpt_dimer_integrals"):
        st = getattr(m, cname)
        assert ctypes.sizeof(st) == lay[(cname, "size")], cname
        for fname, _ in st._fields_:
            assert getattr(st, fname).offset == lay[(cname, fname)], (cname, fname)


def test_host_problem_marshalling():
    from paper_1409_2700_amd import HostProblem
    from synth import cubic_sites, make_lattice_problem
    p = make_lattice_problem(cubic_sites(2, 1, 1), None, sizes=[(2, 3), (1, 4)], workload=901)
    hp = HostProblem(p)
    assert hp.c.n_mono == 2 and hp.c.n_pair == 1
    assert hp.k.size == 2 * 2 * 3 * 3 + 1 * 1 * 4 * 4
    assert hp.v.size == 6 * 4
    assert hp.pairs.dtype == np.int32 and hp.pairs.shape == (1, 2)


def test_missing_library_fails_loudly(tmp_path):
    """With the HIP library absent the binding raises instead of computing anything."""
    code = ("import paper_1409_2700_amd as mc\n"
            "try:\n    mc.Context(0)\nexcept ImportError as e:\n    print('IMPORT-ERROR', e)\n")
    env = dict(os.environ, MCPT_LIBRARY=str(tmp_path / "absent" / "libmcpt.so"))
    out = subprocess.run([os.sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=120)
    assert "IMPORT-ERROR" in out.stdout, out.stdout + out.stderr


def test_no_cpu_fallback_in_product():
    """The product package never imports the oracle or computes the method on the host."""
    pkg = os.path.join(ROOT, "paper_1409_2700_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            text = open(os.path.join(pkg, name)).read()
            assert "oracle" not in text, name
            assert "einsum" not in text and "numpy.linalg" not in text, name
