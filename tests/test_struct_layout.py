"""The ctypes mirrors of the C structures agree with the headers: every field
offset and the structure size, as gcc lays them out, for the library's
chm.h and the oracle's chm_oracle.h (a mismatch would pass wrong values with
no error)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def layouts(header, structs, tmp_path):
    lines = [f'#include "{header}"', "#include <stddef.h>", "#include <stdio.h>", "int main(void) {"]
    for cname, py in structs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(header), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def check(header, structs, tmp_path):
    got = layouts(header, structs, tmp_path)
    for cname, py in structs:
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_library_structs_match_chm_h(tmp_path):
    from paper_2204_03575_amd import chm
    check(os.path.join(ROOT, "include", "chm.h"),
          [("chm_mesh_t", chm.chm_mesh_t), ("chm_params_t", chm.chm_params_t),
           ("chm_run_t", chm.chm_run_t), ("chm_stats_t", chm.chm_stats_t)], tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_structs_match_chm_oracle_h(tmp_path):
    from oracle import oracle as O
    check(os.path.join(ROOT, "oracle", "chm_oracle.h"),
          [("orc_params_t", O.orc_params_t), ("orc_stats_t", O.orc_stats_t)], tmp_path)
