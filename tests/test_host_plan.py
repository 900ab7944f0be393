"""CPU checks of the C-ABI library: exported symbols, host-side setup (the
same hierarchy, AZ and E as the oracle, built independently) and input
validation.  Nothing here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1710_03940_amd as L
from paper_1710_03940_amd import _lib
from workloads import tiny_problem, config_small_poisson, concat_problems, make_problem
from workloads.convdiff import convection_diffusion7
from workloads import config_oseen
from oracle import OracleSolver, OracleParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "dfamg.h")) as fh:
        text = fh.read()
    declared = set(re.findall(r"\b(dfamg_[a-z_]+)\s*\(", text))
    assert "dfamg_setup" in declared and "dfamg_solve" in declared
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [name for name in sorted(declared) if not hasattr(lib, name)]
    assert not missing, missing
    assert declared == set(_lib.EXPORTED)
    # the Python binding offers every entry point under the same name
    assert not [name for name in sorted(declared) if not callable(getattr(L, name, None))]


def test_params_default():
    p = L.make_params()
    assert p.solver == 0 and p.maxiter == 1000 and p.rtol == 1e-8
    assert p.coarse_enough == 500 and abs(p.eps_strong - 0.08) < 1e-15
    assert abs(p.jacobi_omega - 0.8) < 1e-15 and p.block_size == 1


def _significant(M, rel=1e-13):
    """Sparsity pattern without entries at rounding level: products in which
    the exact value cancels to zero leave a residue of about 1e-19 whose
    presence depends on the summation order."""
    M = sp.csr_matrix(M)
    keep = np.abs(M.data) > rel * np.abs(M.data).max()
    r = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    return set(zip(r[keep].tolist(), M.indices[keep].tolist()))


def _compare_hierarchy(P, prm_kw, oracle_kw, sys_row_off=None, exact_structure=True):
    plan = L.dfamg_plan_create(L.make_params(**prm_kw), P.A, P.part, P.nsub, P.Z,
                               sys_row_off=sys_row_off)
    try:
        ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**oracle_kw))
        summ = ora.hierarchy_summary()
        for s in range(P.nsub):
            lv = L.dfamg_plan_levels(plan, s)
            o = summ[s]
            if exact_structure:
                assert [x[:3] for x in lv] == [tuple(x[:3]) for x in o], (s, lv, o)
            else:
                assert [x[0] for x in lv] == [x[0] for x in o], (s, lv, o)
            for l in range(len(lv) - 1):
                assert lv[l][3] == pytest.approx(o[l][3], rel=1e-11)
                agg = L.dfamg_plan_aggregates(plan, s, l)
                assert np.array_equal(agg, ora.M.hierarchies[s].levels[l].agg)
                ptr, col, val, shape = L.dfamg_plan_level_matrix(plan, s, l, 1)
                Pm = sp.csr_matrix((val, col, ptr), shape=shape)
                ref = ora.M.hierarchies[s].levels[l].P
                assert abs(Pm - ref).max() <= 1e-12 * abs(ref).max()
                if not exact_structure:
                    assert _significant(Pm) == _significant(ref)
            ptr, col, val, shape = L.dfamg_plan_level_matrix(plan, s, len(lv) - 1, 0)
            Ac = sp.csr_matrix((val, col, ptr), shape=shape)
            ref = ora.M.hierarchies[s].levels[-1].A
            assert abs(Ac - ref).max() <= 1e-12 * abs(ref).max()
        if sys_row_off is None:
            E = L.dfamg_plan_coarse_operator(plan)
            assert np.abs(E - ora.defl.E).max() <= 1e-12 * np.abs(ora.defl.E).max()
    finally:
        L.dfamg_plan_destroy(plan)


def test_hierarchy_matches_oracle_small_poisson():
    _compare_hierarchy(config_small_poisson(), {}, {})


@pytest.mark.parametrize("N,pieces,defl,sigma,ce,smoother", [
    (12, (2, 2, 1), "linear", 2.0, 20, "spai0"),
    (14, (1, 3, 1), "constant", 1.0, 30, "jacobi"),
    (16, (2, 2, 2), "linear", 2.0, 15, "spai0"),
    (9, (3, 1, 1), "constant", 0.0, 500, "spai0"),
])
def test_hierarchy_matches_oracle(N, pieces, defl, sigma, ce, smoother):
    P = tiny_problem(N=N, pieces=pieces, deflation=defl, sigma=sigma, seed=N)
    _compare_hierarchy(P, dict(coarse_enough=ce, smoother=smoother),
                       dict(coarse_enough=ce, smoother=smoother))


def test_hierarchy_nonsymmetric_matches_oracle():
    base = tiny_problem(N=10, pieces=(2, 1, 1), seed=3)
    A = convection_diffusion7(10, peclet=2.0)
    P = base.__class__("cd", A, base.part, base.nsub, base.Z, base.b, base.x0)
    _compare_hierarchy(P, dict(coarse_enough=20, solver="bicgstab"),
                       dict(coarse_enough=20, solver="bicgstab"))


@pytest.mark.parametrize("N,pieces,ce", [(8, (2, 2, 1), 500), (10, (1, 2, 1), 60)])
def test_block_hierarchy_oseen_matches_oracle(N, pieces, ce):
    """Point-block (4x4) aggregation on the nonsymmetric Q1 Oseen operator,
    with the nonsymmetric per-field E."""
    P = config_oseen(N=N, pieces=pieces)
    kw = dict(coarse_enough=ce, solver="bicgstab", block_size=4)
    _compare_hierarchy(P, kw, kw, exact_structure=False)


@pytest.mark.parametrize("N,pieces,ce,smoother,bs", [
    (12, (2, 2, 1), 20, "spai0", 1),
    (14, (1, 3, 1), 30, "jacobi", 1),
    (8, (2, 1, 1), 60, "spai0", 4),
])
def test_fused_restriction_operator_matches_oracle_steps(N, pieces, ce, smoother, bs):
    """The solve applies pre-smoothing (zero guess), residual and restriction
    of a level as one operator B = R (I - A diag(m)); it must equal the
    oracle's three steps composed."""
    if bs == 4:
        P = config_oseen(N=N, pieces=pieces)
        kw = dict(coarse_enough=ce, smoother=smoother, solver="bicgstab", block_size=4)
    else:
        P = tiny_problem(N=N, pieces=pieces, deflation="linear", sigma=2.0, seed=N)
        kw = dict(coarse_enough=ce, smoother=smoother)
    plan = L.dfamg_plan_create(L.make_params(**kw), P.A, P.part, P.nsub, P.Z)
    try:
        ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**kw))
        checked = 0
        for s in range(P.nsub):
            levels = ora.M.hierarchies[s].levels
            for l in range(len(levels) - 1):
                lv = levels[l]
                ref = (lv.R @ (sp.eye(lv.A.shape[0]) - lv.A @ sp.diags(lv.m))).tocsr()
                ptr, col, val, shape = L.dfamg_plan_level_matrix(plan, s, l, 2)
                Bm = sp.csr_matrix((val, col, ptr), shape=shape)
                assert Bm.shape == ref.shape
                assert abs(Bm - ref).max() <= 1e-12 * abs(ref).max()
                # the reference applied to a vector, step by step
                f = np.random.default_rng(l).standard_normal(lv.A.shape[0])
                x = lv.m * f
                step = lv.R @ (f - lv.A @ x)
                assert np.linalg.norm(Bm @ f - step) <= 1e-12 * np.linalg.norm(step)
                checked += 1
        assert checked > 0
    finally:
        L.dfamg_plan_destroy(plan)


def test_batched_plan_hierarchies_match_standalone():
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.0, seed=n)
             for n, pc in [(9, (2, 1, 1)), (12, (2, 2, 1))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    plan = L.dfamg_plan_create(L.make_params(coarse_enough=30), A, part, nsub, Z, sys_row_off=off)
    try:
        s0 = 0
        for p in probs:
            ora = OracleSolver(p.A, p.part, p.nsub, p.Z, OracleParams(coarse_enough=30))
            for s in range(p.nsub):
                lv = L.dfamg_plan_levels(plan, s0 + s)
                assert [x[:3] for x in lv] == [tuple(x[:3]) for x in ora.hierarchy_summary()[s]]
            s0 += p.nsub
        E1 = L.dfamg_plan_coarse_operator(plan, 1)
        ora = OracleSolver(probs[1].A, probs[1].part, probs[1].nsub, probs[1].Z)
        assert np.abs(E1 - ora.defl.E).max() <= 1e-12 * np.abs(E1).max()
    finally:
        L.dfamg_plan_destroy(plan)


def test_permutation_invariance_of_E():
    # renumbering the subdomains permutes E symmetrically
    P = tiny_problem(N=8, pieces=(2, 2, 1), deflation="constant", sigma=1.0, seed=1)
    perm = np.array([2, 0, 3, 1])
    plan1 = L.dfamg_plan_create(L.make_params(), P.A, P.part, P.nsub, P.Z)
    plan2 = L.dfamg_plan_create(L.make_params(), P.A, perm[P.part].astype(np.int32), P.nsub, P.Z)
    E1 = L.dfamg_plan_coarse_operator(plan1)
    E2 = L.dfamg_plan_coarse_operator(plan2)
    L.dfamg_plan_destroy(plan1)
    L.dfamg_plan_destroy(plan2)
    assert np.allclose(E2[np.ix_(perm, perm)], E1, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# validation (host side, before any device work)
# --------------------------------------------------------------------------

def _expect(status, P, A=None, part=None, nsub=None, Z=None, **prm):
    with pytest.raises(L.DfamgError) as ei:
        plan = L.dfamg_plan_create(L.make_params(**prm), P.A if A is None else A,
                                   P.part if part is None else part,
                                   P.nsub if nsub is None else nsub, P.Z if Z is None else Z)
        L.dfamg_plan_destroy(plan)
    assert ei.value.status == status, str(ei.value)
    return str(ei.value)


def test_validation_errors():
    P = tiny_problem(N=6, pieces=(2, 1, 1), deflation="linear")
    _expect(_lib.EINVAL, P, nsub=3)                                   # empty subdomain
    bad = P.part.copy()
    bad[5] = 9
    _expect(_lib.EINVAL, P, part=bad)                                 # id out of range
    A = P.A.copy()
    A.data[3] = np.nan
    _expect(_lib.EINVAL, P, A=A)                                      # non-finite value
    A = P.A.copy()
    A.indices = A.indices.copy()
    A.indices[1] = A.indices[0]                                       # duplicate column
    _expect(_lib.EINVAL, P, A=A)
    A = P.A.copy()
    A.indices = A.indices.copy()
    A.indices[2] = P.n + 4                                            # column out of range
    with pytest.raises((L.DfamgError, ValueError)):
        plan = L.dfamg_plan_create(L.make_params(), A, P.part, P.nsub, P.Z)
        L.dfamg_plan_destroy(plan)
    Z = P.Z.copy()
    Z[0, 1] = np.inf
    _expect(_lib.EINVAL, P, Z=Z)
    _expect(_lib.EINVAL, P, maxiter=-1)
    _expect(_lib.EINVAL, P, solver=L.make_params().solver + 7)        # unknown solver
    _expect(_lib.EINVAL, P, solver=_lib.SOLVER_FGMRES, restart=0)
    _expect(_lib.EINVAL, P, spmv_format=_lib.FORMAT_COLUMN_TILED + 1)  # unknown layout family
    _expect(_lib.EINVAL, P, spmv_format=_lib.FORMAT_BSR4)              # BSR4 needs 4 x 4 blocks
    # at most 8 deflation vectors per subdomain
    assert "ndv" in _expect(_lib.EINVAL, P, Z=np.column_stack([P.Z, P.Z, P.Z[:, :1]]))
    _expect(_lib.EINVAL, P, spmv_format=-1)
    _expect(_lib.EINVAL, P, solver=_lib.SOLVER_FGMRES, restart=65)
    _expect(_lib.EINVAL, P, coarse_solve=2)
    # an inexact E only inside the flexible method: the projected solvers need
    # the exact coarse solve
    _expect(_lib.EINVAL, P, coarse_solve=_lib.COARSE_FP32)
    _expect(_lib.EINVAL, P, solver=_lib.SOLVER_BICGSTAB, coarse_solve=_lib.COARSE_FP32)
    _expect(_lib.EINVAL, P, coarse_solve=_lib.COARSE_CG)
    _expect(_lib.EINVAL, P, solver=_lib.SOLVER_FGMRES, coarse_solve=_lib.COARSE_CG, coarse_rtol=-1.0)
    _expect(_lib.EINVAL, P, solver=_lib.SOLVER_FGMRES, coarse_solve=_lib.COARSE_CG, coarse_maxiter=0)
    _expect(_lib.EINVAL, P, coarse_enough=0)
    _expect(_lib.EINVAL, P, max_levels=21)
    _expect(_lib.EINVAL, P, block_size=4)                             # 216 rows, 4 | 216 but
    # zero diagonal
    A = P.A.tolil()
    A[4, 4] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    _expect(_lib.EINVAL, P, A=A)


def test_degenerate_inputs_rejected():
    P = tiny_problem(N=6, pieces=(2, 1, 1), deflation="constant")
    _expect(_lib.EINVAL, P, solver=7)                                 # unknown solver
    empty = sp.csr_matrix((0, 0))
    empty.indptr = empty.indptr.astype(np.int64)
    empty.indices = empty.indices.astype(np.int32)
    with pytest.raises((L.DfamgError, ValueError)):
        plan = L.dfamg_plan_create(L.make_params(), empty, np.zeros(0, np.int32), 1, np.zeros((0, 1)))
        L.dfamg_plan_destroy(plan)


def test_rank_deficient_deflation_block_names_subdomain():
    P = make_problem("slab", (6, 6, 4), (1, 1, 4), deflation="linear")
    msg = _expect(_lib.ESINGULAR, P)
    assert "subdomain" in msg


def test_batched_rejects_coupled_systems():
    probs = [tiny_problem(N=5, pieces=(1, 1, 1)), tiny_problem(N=5, pieces=(1, 1, 1))]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    A = A.tolil()
    A[0, 130] = -0.1
    A = A.tocsr()
    with pytest.raises(L.DfamgError) as ei:
        L.dfamg_plan_create(L.make_params(), A, part, nsub, Z, sys_row_off=off)
    assert "couples two systems" in str(ei.value)


def test_setup_without_gpu_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    P = tiny_problem(N=5, pieces=(1, 1, 1))
    with pytest.raises(L.DfamgError) as ei:
        L.dfamg_setup(L.make_params(), P.A, P.part, P.nsub, P.Z)
    assert ei.value.status in (_lib.ENOGPU, _lib.EHIP)


def test_schur_setup_validation():
    """Rejected on the host before any device work."""
    from workloads import oseen_q1
    A, _ = oseen_q1(4)
    n = A.shape[0]
    pmask = (np.arange(n) % 4 == 3).astype(np.int32)
    part = np.zeros(64, dtype=np.int32)
    Z = np.ones((64, 1))
    for kw, mask in [(dict(solver=_lib.SOLVER_CG), pmask),           # needs FGMRES
                     (dict(solver=_lib.SOLVER_FGMRES), np.zeros(n, dtype=np.int32)),   # no pressure
                     (dict(solver=_lib.SOLVER_FGMRES), np.ones(n, dtype=np.int32))]:   # no velocity
        with pytest.raises(L.DfamgError) as ei:
            L.dfamg_setup_schur(L.make_params(**kw), A, mask, part, 1, Z)
        assert ei.value.status == _lib.EINVAL



@pytest.mark.parametrize("smoother", ["spai0", "block_spai0"])
def test_smoother_matrices_match_oracle(smoother):
    """The smoother of every level (diagonal SPAI-0, or the 4 x 4 blocks of
    block SPAI-0 on the Oseen point-block hierarchy) equals the oracle's."""
    from workloads import config_oseen
    from oracle import OracleSolver, OracleParams
    P = config_oseen(N=8, pieces=(2, 1, 1))
    kw = dict(block_size=4, coarse_enough=60)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="bicgstab", smoother=smoother, **kw))
    code = {"spai0": _lib.SMOOTHER_SPAI0, "block_spai0": _lib.SMOOTHER_BLOCK_SPAI0}[smoother]
    plan = L.dfamg_plan_create(L.make_params(solver=1, smoother=code, **kw), P.A, P.part, P.nsub, P.Z)
    try:
        checked = 0
        for s, H in enumerate(ref.M.hierarchies):
            for l, lvl in enumerate(H.levels[:-1]):
                ptr, col, val, shape = L.dfamg_plan_level_matrix(plan, s, l, 3)
                M = sp.csr_matrix((val, col, ptr), shape=shape).toarray()
                R = np.diag(lvl.m) if isinstance(lvl.m, np.ndarray) else lvl.m.toarray()
                assert np.allclose(M, R, rtol=1e-11, atol=1e-14 * np.abs(R).max())
                checked += 1
        assert checked >= 2
    finally:
        L.dfamg_plan_destroy(plan)


def test_header_constants_match_binding():
    # every enumerator of the C header has the same value in the binding (the
    # per-kernel span ids as the order of KERNEL_NAMES)
    import re
    import os
    from paper_1710_03940_amd import _lib
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "dfamg.h")).read()
    pairs = re.findall(r"\bDFAMG_([A-Z0-9_]+)\s*=\s*(-?\d+)", hdr)
    assert len(pairs) > 30
    for name, value in pairs:
        if name.startswith("KERNEL_"):
            span = name[len("KERNEL_"):].lower()
            if span == "count":
                assert int(value) == len(_lib.KERNEL_NAMES)
            else:
                assert _lib.KERNEL_NAMES[int(value)] == span, name
        else:
            assert getattr(_lib, name) == int(value), name


def test_cycle_options_validated_on_the_host():
    # flexible CG and the smoothing sweep counts: unsupported combinations
    # fail in the host validation, before any device is touched
    P = tiny_problem(N=6)
    for kw in (dict(flexible_cg=1, solver=_lib.SOLVER_BICGSTAB), dict(npre=5), dict(npost=0), dict(npre=-1),
               dict(flexible_cg=2), dict(npre=2, npost=2, smoother=_lib.SMOOTHER_BLOCK_SPAI0),
               dict(setup_device=2), dict(setup_device=1, smoother=_lib.SMOOTHER_BLOCK_SPAI0),
               dict(setup_device=1, block_size=2), dict(spmv_format=_lib.FORMAT_BSR4),
               dict(spmv_format=_lib.FORMAT_COLUMN_TILED + 1)):
        with pytest.raises(L.DfamgError) as ei:
            L.dfamg_setup(L.make_params(**kw), P.A, P.part, P.nsub, P.Z)
        assert ei.value.status == _lib.EINVAL, kw
    p = L.make_params()
    assert p.flexible_cg == 0 and p.npre == 1 and p.npost == 1 and p.setup_device == 0
