"""The host setup planner (host_plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only, no GPU) and run on the
problems the library is tested on, plus inputs it must reject.  Any
out-of-bounds access, use after free, leak, signed overflow or misaligned
access aborts the driver (halt_on_error); the plan it builds must equal the
one the library (built with hipcc) reports through the C ABI."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1710_03940_amd as L
from paper_1710_03940_amd import _lib
from workloads import tiny_problem, concat_problems, config_oseen
from workloads.convdiff import convection_diffusion7

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_03940_amd", "csrc")
HERE_SAN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:abort_on_error=0:exitcode=86",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("san") / "host_plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "host_plan.cpp"), os.path.join(HERE_SAN, "host_plan_driver.cpp"),
           "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _write_case(d, prm, A, part, nsub, Z, sys_off=None):
    A = sp.csr_matrix(A)
    A.sort_indices()
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "params.bin"), "wb") as fh:
        fh.write(bytes(prm))
    Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(A.shape[0], -1)
    nsys = 1 if sys_off is None else len(sys_off) - 1
    with open(os.path.join(d, "meta.txt"), "w") as fh:
        fh.write(f"{A.shape[0]} {nsub} {Z.shape[1]} {nsys}\n")
    A.indptr.astype(np.int64).tofile(os.path.join(d, "row_ptr.bin"))
    A.indices.astype(np.int32).tofile(os.path.join(d, "col.bin"))
    A.data.astype(np.float64).tofile(os.path.join(d, "val.bin"))
    np.asarray(part, dtype=np.int32).tofile(os.path.join(d, "part.bin"))
    Z.tofile(os.path.join(d, "Z.bin"))
    np.asarray(sys_off if sys_off is not None else [0, A.shape[0]], dtype=np.int64).tofile(
        os.path.join(d, "sys_off.bin"))


def _run(driver, d):
    env = dict(os.environ)
    env.update(SAN_ENV)
    r = subprocess.run([driver, d], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"driver exit {r.returncode}\n{r.stderr[-6000:]}"
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    return r.stdout.splitlines()


def _compare_with_library(lines, prm, A, part, nsub, Z, sys_off=None):
    p = L.dfamg_plan_create(prm, sp.csr_matrix(A), part, nsub, Z, sys_off)
    try:
        s_lines = [ln.split() for ln in lines if ln.startswith("S ")]
        assert len(s_lines) == nsub
        for f in s_lines:
            u, nl = int(f[1]), int(f[2])
            lib = L.dfamg_plan_levels(p, u)
            assert len(lib) == nl
            for l in range(nl):
                rows, nnz, pnnz, om = f[3 + 4 * l: 7 + 4 * l]
                assert (int(rows), int(nnz), int(pnnz)) == lib[l][:3], (u, l)
                assert abs(float(om) - lib[l][3]) <= 1e-12 * max(1.0, abs(lib[l][3])), (u, l)
        for ln in lines:
            if ln.startswith("E "):
                _, s, m, tot = ln.split()
                E = L.dfamg_plan_coarse_operator(p, int(s))
                assert E.shape[0] == int(m)
                assert abs(E.sum() - float(tot)) <= 1e-10 * max(1.0, np.abs(E).sum())
        lv = [ln for ln in lines if ln.startswith("L ")]
        assert lv and all("=" in ln for ln in lv)
    finally:
        L.dfamg_plan_destroy(p)


def _case(driver, tmp_path, name, A, part, nsub, Z, sys_off=None, **kw):
    prm = L.make_params(**kw)
    d = str(tmp_path / name)
    _write_case(d, prm, A, part, nsub, Z, sys_off)
    lines = _run(driver, d)
    assert not any(ln.startswith("ERR") for ln in lines), lines[:3]
    _compare_with_library(lines, prm, A, part, nsub, Z, sys_off)
    return lines


def test_sanitized_scalar_hierarchy(driver, tmp_path):
    P = tiny_problem(N=14, pieces=(2, 2, 1), deflation="linear", sigma=2.0, seed=4)
    _case(driver, tmp_path, "scalar", P.A, P.part, P.nsub, P.Z, coarse_enough=30)


def test_sanitized_jacobi_level_limit_and_nonsymmetric(driver, tmp_path):
    P = tiny_problem(N=12, pieces=(2, 1, 2), deflation="constant", seed=9)
    _case(driver, tmp_path, "jacobi", P.A, P.part, P.nsub, P.Z, coarse_enough=20, smoother="jacobi",
          max_levels=2)
    A = convection_diffusion7(12, peclet=8.0)
    _case(driver, tmp_path, "convdiff", A, P.part, P.nsub, P.Z, coarse_enough=20, solver="bicgstab")


def test_sanitized_batched_systems(driver, tmp_path):
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.0, seed=s)
             for n, pc, s in ((9, (1, 1, 2), 1), (13, (2, 2, 1), 2), (7, (1, 1, 1), 3))]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    _case(driver, tmp_path, "batched", A, part, nsub, Z, sys_off=off, coarse_enough=25)


@pytest.mark.parametrize("smoother", ["spai0", "block_spai0"])
def test_sanitized_point_block_hierarchy(driver, tmp_path, smoother):
    P = config_oseen(N=6, pieces=(2, 1, 1))
    _case(driver, tmp_path, "oseen_" + smoother, P.A, P.part, P.nsub, P.Z, block_size=4,
          solver="bicgstab", coarse_enough=60, smoother=smoother)


def test_sanitized_rejections(driver, tmp_path):
    # inputs the planner must reject through its error path, without a
    # sanitizer report on the way
    P = tiny_problem(N=6, pieces=(1, 1, 2), deflation="constant", seed=1)
    A = sp.csr_matrix(P.A)
    prm = L.make_params()
    cases = {}
    bad = np.array(P.part, dtype=np.int32)
    bad[5] = P.nsub
    cases["part_out_of_range"] = (A, bad, P.nsub, P.Z)
    B = A.copy()
    B.data[3] = np.nan
    cases["nan_value"] = (B, P.part, P.nsub, P.Z)
    C = A.copy()
    C.indices = C.indices.copy()
    C.indices[-1] = A.shape[0] + 3
    cases["column_out_of_range"] = (C, P.part, P.nsub, P.Z)
    empty = np.array(P.part, dtype=np.int32)
    empty[empty == 1] = 0
    cases["empty_subdomain"] = (A, empty, P.nsub, P.Z)
    for name, (M, part, nsub, Z) in cases.items():
        d = str(tmp_path / name)
        _write_case(d, prm, M, part, nsub, Z)
        lines = _run(driver, d)
        assert lines and lines[0].startswith(f"ERR {_lib.EINVAL} "), (name, lines[:2])
    # parameters out of range
    for kw in (dict(block_size=5), dict(npost=0), dict(max_levels=0), dict(coarse_enough=5000)):
        d = str(tmp_path / ("prm_" + "_".join(kw)))
        _write_case(d, L.make_params(**kw), A, P.part, P.nsub, P.Z)
        lines = _run(driver, d)
        assert lines and lines[0].startswith(f"ERR {_lib.EINVAL} "), (kw, lines[:2])
