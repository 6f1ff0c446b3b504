"""The boundary from plain C: include/katz.h compiles as C99 on its own, and a
C program linked against the built library runs the host-side calls
(communities, a host-only index build, info, the error path of a query on an
index without a device, a rebuild for another damping factor, free).  CPU only: no GPU compute is called."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1912_06525_amd")

_C_PROGRAM = r"""
#include <stdio.h>
#include "katz.h"

/* two triangles {0,1,2} and {3,4,5} joined by the edge 2-3 */
static const int32_t rp[7] = {0, 2, 4, 7, 10, 12, 14};
static const int32_t col[14] = {1, 2, 0, 2, 0, 1, 3, 2, 4, 5, 3, 5, 3, 4};

int main(void) {
  int32_t labels[6], passes = -1;
  int rc = katz_communities(6, 14, rp, col, NULL, 3, 10, labels, &passes);
  if (rc != KATZ_OK) { printf("communities %d %s\n", rc, katz_last_error()); return 1; }
  printf("labels %d %d %d %d %d %d passes %d\n", labels[0], labels[1], labels[2], labels[3], labels[4],
         labels[5], passes);
  katz_build_opts o;
  katz_build_opts_default(&o);
  o.device = -1;
  o.rank = 0;
  o.beta_frac = 0.5;
  o.labels = labels;
  katz_index* idx = NULL;
  rc = katz_index_build(6, 14, rp, col, NULL, &o, &idx);
  if (rc != KATZ_OK) { printf("build %d %s\n", rc, katz_last_error()); return 1; }
  katz_index_info_t info;
  if (katz_index_info(idx, &info) != KATZ_OK) return 1;
  printf("info n %d n1 %d n2 %d device %d c %.3f\n", info.n, info.n1, info.n2, info.device, info.c);
  double scores[6];
  int32_t q = 0;
  rc = katz_query(idx, &q, 1, NULL, scores, NULL, NULL);
  printf("query %d %s\n", rc == KATZ_EDEVICE, katz_last_error());
  o.beta_frac = 0.8;
  katz_index* idx2 = NULL;
  rc = katz_index_rebuild(idx, &o, &idx2);
  if (rc != KATZ_OK || katz_index_info(idx2, &info) != KATZ_OK) return 1;
  printf("rebuild n1 %d c %.3f\n", info.n1, info.c);
  katz_index_free(idx2);
  katz_index_free(idx);
  rc = katz_communities(6, 14, rp, col, NULL, 0, 10, labels, NULL);
  printf("bad cap %d\n", rc == KATZ_EINVAL);
  return 0;
}
"""


def test_header_is_c99():
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-x", "c",
                    os.path.join(ROOT, "include", "katz.h")], check=True)


def test_c_program_against_the_library(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc")
    lib = os.path.join(LIB_DIR, "libkatz_hip.so")
    if not os.path.exists(lib):
        pytest.skip("libkatz_hip.so is not built")
    src = tmp_path / "abi.c"
    src.write_text(_C_PROGRAM)
    exe = tmp_path / "abi"
    rocm_lib = "/opt/rocm/lib"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", LIB_DIR, "-l:libkatz_hip.so", "-Wl,-rpath," + LIB_DIR, "-Wl,-rpath," + rocm_lib,
                    "-Wl,-rpath-link," + rocm_lib, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout
    lines = out.strip().splitlines()
    assert lines[0].startswith("labels 0 0 0 1 1 1 passes "), out
    assert lines[1].startswith("info n 6 n1 ") and " device -1 c 0.500" in lines[1], out
    n1 = int(lines[1].split()[4])
    n2 = int(lines[1].split()[6])
    assert n1 + n2 == 6 and n2 >= 1, out
    assert lines[2].startswith("query 1 "), out
    assert lines[3] == "rebuild n1 %d c 0.800" % n1, out
    assert lines[4] == "bad cap 1", out


_STRUCTS = ["katz_build_opts", "katz_query_opts", "katz_query_stats", "katz_index_info_t", "katz_server_opts",
            "katz_server_info_t", "katz_kernel_stat"]


def test_binding_structs_match_the_header(tmp_path):
    """Every struct of the header has the same size and field offsets in the
    ctypes binding as the C compiler gives it (field names as in the
    header)."""
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc")
    K = pytest.importorskip("paper_1912_06525_amd")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "katz.h"', "int main(void) {"]
    for name in _STRUCTS:
        cls = getattr(K, name)
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, fname, name, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    import ctypes
    for name in _STRUCTS:
        cls = getattr(K, name)
        assert int(got["%s size" % name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got["%s.%s" % (name, fname)]) == getattr(cls, fname).offset, (name, fname)


def test_binding_constants_match_the_header():
    """Every enumerator the header defines (status codes, precisions, factor
    kinds, methods, orders, paths) has the same value in the binding."""
    import re
    K = pytest.importorskip("paper_1912_06525_amd")
    src = open(os.path.join(ROOT, "include", "katz.h")).read()
    found = re.findall(r"^\s*(KATZ_[A-Z0-9_]+)\s*=\s*(-?\d+)", src, re.M)
    assert len(found) >= 24, found
    for name, value in found:
        assert getattr(K, name) == int(value), name
