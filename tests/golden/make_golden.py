"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the CPU oracle (oracle/) on the seeded inputs of
workloads/; nothing is taken from the GPU library.  Run from the repository
root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from workloads import (config_lognormal_poisson, config_small_poisson, config_batched,  # noqa: E402
                       config_oseen, config_oseen_schur)
from oracle import OracleSolver, OracleParams  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 2000
NSTRATUM = 64


def strata(P):
    """Stratified entries where a layout or tiling mistake would show first:
    for every subdomain its first and last NSTRATUM unknowns (ascending
    index, the first and last rows of its tiles) and up to NSTRATUM evenly
    spaced unknowns coupled to another subdomain."""
    part = np.asarray(P.part)
    A = P.A.tocsr()
    rows = np.repeat(np.arange(P.n), np.diff(A.indptr))
    coupled = np.zeros(P.n, dtype=bool)
    coupled[rows[part[rows] != part[A.indices]]] = True
    pick = []
    for s in range(P.nsub):
        r = np.flatnonzero(part == s)
        pick += [r[:NSTRATUM], r[-NSTRATUM:]]
        c = r[coupled[r]]
        if c.size:
            pick.append(c[np.linspace(0, c.size - 1, min(NSTRATUM, c.size)).astype(np.int64)])
    return np.unique(np.concatenate(pick))


def record(name, P, prm=None):
    t0 = time.time()
    S = OracleSolver(P.A, P.part, P.nsub, P.Z, prm)
    t1 = time.time()
    r = S.solve(P.b)
    t2 = time.time()
    idx = np.sort(np.random.default_rng(12345).choice(P.n, size=min(NSAMPLE, P.n), replace=False))
    out = {
        "workload": P.name, "n": int(P.n), "nnz": int(P.A.nnz), "nsub": int(P.nsub),
        "ndv": int(P.ndv), "rtol": 1e-8, "iters": int(r["iters"]),
        "params": dict(vars(S.prm)),
        "relres": float(r["relres"]), "relres_true": float(r["relres_true"]),
        "history": [float(h) for h in r["history"]],
        "x_norm": float(np.linalg.norm(r["x"])),
        "sample_index": [int(i) for i in idx],
        "sample_x": [float(v) for v in r["x"][idx]],
        "strata_index": [int(i) for i in strata(P)],
        "strata_x": [float(v) for v in r["x"][strata(P)]],
        "hierarchy_sub0": [list(map(float, lv)) for lv in S.hierarchy_summary()[0]],
        "oracle_setup_s": t1 - t0, "oracle_solve_s": t2 - t1,
        "source": "oracle/ (CPU FP64) via tests/golden/make_golden.py",
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(out, fh)
    print(name, out["iters"], out["relres_true"], f"setup {t1 - t0:.1f}s solve {t2 - t1:.1f}s")


BATCHED_SAMPLE_SYSTEMS = [2, 12, 19, 28, 31, 42, 44, 47]


def record_schur():
    """The 64^3 Oseen system (one backward-Euler step, dt = 0.1) with the
    Schur pressure-correction preconditioner inside FGMRES(50), rtol 1e-8."""
    from oracle.schur import schur_fgmres
    P, pmask, part_p, nsub, Zp = config_oseen_schur()
    t0 = time.time()
    r = schur_fgmres(P.A, P.b, pmask, part_p, nsub, Zp, rtol=1e-8, restart=50)
    t1 = time.time()
    idx = np.sort(np.random.default_rng(12345).choice(P.n, size=NSAMPLE, replace=False))
    out = {"workload": P.name + "_dt0.1_schur", "n": int(P.n), "nnz": int(P.A.nnz), "nsub": int(nsub), "ndv": 1,
           "rtol": 1e-8, "iters": int(r["iters"]), "restart": 50, "relres": float(r["relres"]),
           "relres_true": float(r["relres_true"]), "history": [float(h) for h in r["history"]],
           "x_norm": float(np.linalg.norm(r["x"])), "sample_index": [int(i) for i in idx],
           "sample_x": [float(v) for v in r["x"][idx]]}
    with open(os.path.join(HERE, "oseen64_boxes256_schur.json"), "w") as fh:
        json.dump(out, fh)
    print("oseen64_boxes256_schur", r["iters"], r["relres_true"], f"solve {t1 - t0:.1f}s", flush=True)


def record_batched():
    """Oracle solves of a subset of the 48 batched systems, one by one."""
    systems = {}
    for s, P in zip(BATCHED_SAMPLE_SYSTEMS, config_batched(systems=BATCHED_SAMPLE_SYSTEMS)):
        r = OracleSolver(P.A, P.part, P.nsub, P.Z).solve(P.b)
        idx = np.sort(np.random.default_rng(100 + s).choice(P.n, size=min(500, P.n), replace=False))
        systems[str(s)] = {"n": int(P.n), "nsub": int(P.nsub), "iters": int(r["iters"]),
                           "relres_true": float(r["relres_true"]),
                           "x_norm": float(np.linalg.norm(r["x"])),
                           "sample_index": [int(i) for i in idx],
                           "sample_x": [float(v) for v in r["x"][idx]],
                           "strata_index": [int(i) for i in strata(P)],
                           "strata_x": [float(v) for v in r["x"][strata(P)]]}
        print("batched system", s, P.n, r["iters"])
    with open(os.path.join(HERE, "batched48_sample.json"), "w") as fh:
        json.dump({"workload": "batched48_lognormal1_linear", "systems": systems,
                   "source": "oracle/ (CPU FP64) via tests/golden/make_golden.py"}, fh)


if __name__ == "__main__":
    which = sys.argv[1:] or ["small", "lognormal", "batched"]
    if "small" in which:
        record("poisson32_slabs8_constant", config_small_poisson())
    if "lognormal" in which:
        record("poisson150_lognormal2_boxes64_linear", config_lognormal_poisson())
    if "batched" in which:
        record_batched()
    if "lognormal_bicgstab2" in which:
        record("poisson150_lognormal2_boxes64_linear_bicgstab2", config_lognormal_poisson(),
               OracleParams(solver="bicgstabl", ell=2))
    if "lognormal_fgmres" in which:
        record("poisson150_lognormal2_boxes64_linear_fgmres30_fp32coarse", config_lognormal_poisson(),
               OracleParams(solver="fgmres", restart=30, coarse_solve="fp32"))
    if "lognormal_fgmres_cg" in which:
        record("poisson150_lognormal2_boxes64_linear_fgmres30_cgcoarse", config_lognormal_poisson(),
               OracleParams(solver="fgmres", restart=30, coarse_solve="cg", coarse_rtol=1e-2,
                            coarse_maxiter=100))
    if "oseen_schur" in which:
        record_schur()
    if "oseen_block" in which:
        record("oseen64_boxes256_field_blockspai0", config_oseen(),
               OracleParams(solver="bicgstab", block_size=4, smoother="block_spai0"))
    if "oseen" in which:
        record("oseen64_boxes256_field", config_oseen(),
               OracleParams(solver="bicgstab", block_size=4))
