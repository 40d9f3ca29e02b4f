"""The C-ABI library: it loads, exports every function declared in
include/nep.h, and the binding's ctypes structures have the C layouts.
Runs without a GPU (no compute calls)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_1910_11712_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libnep.so not built")
    return C.CDLL(B.LIB_PATH)


def test_declared_symbols_nonempty():
    syms = B.declared_symbols()
    for name in ("nep_split_create", "nep_ciss_moments", "nep_extract", "nep_batch_create",
                 "nep_server_submit", "nep_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    missing = [s for s in B.declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_binding_loads_and_reports_version():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libnep.so not built")
    assert B.lib().nep_version().decode().startswith("libnep")


def test_last_error_after_bad_argument():
    """A host-side argument check fails with NEP_ERR_ARG and a message
    (no device work is started)."""
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libnep.so not built")
    L = B.lib()
    out = C.c_void_p()
    code = L.nep_split_create(0, 1, None, None, None, C.byref(out))
    assert code == B.NEP_ERR_ARG
    assert len(L.nep_last_error().decode()) > 0
    assert L.nep_server_destroy(None) == B.NEP_ERR_ARG


def test_tune_host_calls():
    """The tuner's switches and report are host-only: argument checks, and an
    empty report after the cache is cleared (no device work)."""
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libnep.so not built")
    L = B.lib()
    assert L.nep_tune_set(1, 0) == B.NEP_ERR_ARG
    assert L.nep_tune_set(1, 65) == B.NEP_ERR_ARG
    n, ch, ca = C.c_int(), C.c_int(), C.c_int()
    assert L.nep_tune_report(4, None, C.byref(n), C.byref(ch), C.byref(ca)) == B.NEP_ERR_ARG
    assert L.nep_tune_report(0, None, None, C.byref(ch), C.byref(ca)) == B.NEP_ERR_ARG
    B.nep_tune_set(True, 2)
    B.nep_tune_set(False, 3)
    B.nep_tune_clear()
    assert B.nep_tune_report() == {"candidates": [], "chosen": -1, "cached": False}


_LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "nep.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("nep_fn %zu\n", sizeof(nep_fn));
  P(nep_fn, alpha) P(nep_fn, beta) P(nep_fn, nnum) P(nep_fn, num) P(nep_fn, den) P(nep_fn, phi_k)
  P(nep_fn, comb_op) P(nep_fn, comb_a) P(nep_fn, comb_b)
  printf("nep_mat %zu\n", sizeof(nep_mat));
  P(nep_mat, data) P(nep_mat, ld) P(nep_mat, on_device)
  printf("nep_contour %zu\n", sizeof(nep_contour));
  P(nep_contour, c) P(nep_contour, rho) P(nep_contour, v)
  printf("nep_ciss_opts %zu\n", sizeof(nep_ciss_opts));
  P(nep_ciss_opts, max_refine) P(nep_ciss_opts, fp64_fallback) P(nep_ciss_opts, refine_tol) P(nep_ciss_opts, stream)
  printf("nep_ciss_stats %zu\n", sizeof(nep_ciss_stats));
  P(nep_ciss_stats, singular_node) P(nep_ciss_stats, bad_node) P(nep_ciss_stats, max_rel_residual)
  P(nep_ciss_stats, ms_total) P(nep_ciss_stats, ms_lu) P(nep_ciss_stats, min_abs_pivot)
  printf("nep_extract_opts %zu\n", sizeof(nep_extract_opts));
  P(nep_extract_opts, eta_tol) P(nep_extract_opts, max_eigs) P(nep_extract_opts, polish_its)
  printf("nep_server_opts %zu\n", sizeof(nep_server_opts));
  P(nep_server_opts, max_inflight) P(nep_server_opts, nstreams)
  printf("nep_query_info %zu\n", sizeof(nep_query_info));
  P(nep_query_info, n_inside) P(nep_query_info, reused) P(nep_query_info, t_submit) P(nep_query_info, t_done)
  printf("nep_tune_cand %zu\n", sizeof(nep_tune_cand));
  P(nep_tune_cand, paired) P(nep_tune_cand, small_min) P(nep_tune_cand, early_fork) P(nep_tune_cand, jb) P(nep_tune_cand, ms)
  return 0;
}
"""


def test_ctypes_layouts_match_header(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    ref = dict(l.rsplit(" ", 1) for l in lines if l.strip())
    structs = {"nep_fn": B.nep_fn, "nep_mat": B.nep_mat, "nep_contour": B.nep_contour,
               "nep_ciss_opts": B.nep_ciss_opts, "nep_ciss_stats": B.nep_ciss_stats,
               "nep_extract_opts": B.nep_extract_opts, "nep_server_opts": B.nep_server_opts,
               "nep_query_info": B.nep_query_info, "nep_tune_cand": B.nep_tune_cand}
    for key, val in ref.items():
        if "." in key:
            sname, field = key.split(".")
            assert getattr(structs[sname], field).offset == int(val), key
        else:
            assert C.sizeof(structs[key]) == int(val), key
