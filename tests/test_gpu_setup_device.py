"""Setup on the GPU (setup_device = 1): the smoothed-aggregation hierarchies
built by the device kernels against the host construction, and solves with
them against the oracle.

The device kernels reproduce the host's operations in the host's order, so
the bar is equality: aggregates (index work) bit for bit, and the level
operators A_l, P_l, B_l, the smoother diagonals and omega bit for bit too
(the host construction itself is pinned to the oracle on the CPU in
tests/test_host_plan.py); AZ, also formed on the device, is compared through
E = Z^T (AZ).
"""
import numpy as np
import pytest

from workloads import tiny_problem, config_small_poisson, config_lognormal_poisson, config_batched, \
    concat_problems, convection_diffusion7
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _plans(P, sys_row_off=None, **kw):
    import paper_1710_03940_amd as L
    ph = L.dfamg_plan_create(L.make_params(**kw), P.A, P.part, P.nsub, P.Z, sys_row_off)
    pd = L.dfamg_plan_create(L.make_params(setup_device=1, **kw), P.A, P.part, P.nsub, P.Z, sys_row_off)
    return L, ph, pd


def _compare(P, sys_row_off=None, subs=None, **kw):
    L, ph, pd = _plans(P, sys_row_off, **kw)
    try:
        nlev_total = 0
        for sub in (range(P.nsub) if subs is None else subs):
            lh, ld = L.dfamg_plan_levels(ph, sub), L.dfamg_plan_levels(pd, sub)
            assert lh == ld, (sub, lh, ld)      # rows, nnz(A), nnz(P) and omega per level, exactly
            nlev_total += len(lh)
            for lvl in range(len(lh)):
                last = lvl == len(lh) - 1
                if not last:
                    ah, ad = L.dfamg_plan_aggregates(ph, sub, lvl), L.dfamg_plan_aggregates(pd, sub, lvl)
                    assert np.array_equal(ah, ad), (sub, lvl)
                for which in ((0,) if last else (0, 1, 2, 3)):
                    mh = L.dfamg_plan_level_matrix(ph, sub, lvl, which)
                    md = L.dfamg_plan_level_matrix(pd, sub, lvl, which)
                    assert mh[3] == md[3], (sub, lvl, which)
                    for a, b in zip(mh[:3], md[:3]):
                        assert np.array_equal(a, b), (sub, lvl, which, np.abs(a - b).max() if a.size else 0)
        # E = Z^T (AZ) from the AZ each side built (on the device with
        # setup_device = 1): equal bit for bit as well
        nsys = 1 if sys_row_off is None else len(sys_row_off) - 1
        for sy in range(nsys):
            eh, ed = L.dfamg_plan_coarse_operator(ph, sy), L.dfamg_plan_coarse_operator(pd, sy)
            assert np.array_equal(eh, ed), (sy, np.abs(eh - ed).max())
        print(f"{P.name}: {nlev_total} subdomain levels and {nsys} coarse operators equal", flush=True)
    finally:
        L.dfamg_plan_destroy(ph)
        L.dfamg_plan_destroy(pd)


def test_setup_device_tiny_ragged():
    P = tiny_problem(N=20, pieces=(2, 2, 2), deflation="linear", sigma=2.0, seed=20)
    _compare(P, coarse_enough=40)


def test_setup_device_32_slabs():
    _compare(config_small_poisson(), coarse_enough=200)


def test_setup_device_damped_jacobi_and_level_limit():
    P = tiny_problem(N=18, pieces=(2, 1, 2), deflation="constant", sigma=1.0, seed=7)
    _compare(P, coarse_enough=20, smoother="jacobi", max_levels=3)


def test_setup_device_nonsymmetric_strength():
    # upwind convection: a_ij != a_ji, so the strong graph is directed
    base = tiny_problem(N=16, pieces=(2, 2, 1), deflation="constant", seed=3)
    A = convection_diffusion7(16, peclet=8.0)
    P = base.__class__("cd16", A, base.part, base.nsub, base.Z, base.b, base.x0)
    _compare(P, coarse_enough=30)


def test_setup_device_batched_systems():
    probs = config_batched(systems=[0, 5, 11, 30])
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    P = probs[0].__class__("batched4", A, part, nsub, Z, b, x0)
    _compare(P, sys_row_off=off)


def test_setup_device_full_150():
    # the 150^3 log-normal problem at full size, every subdomain
    _compare(config_lognormal_poisson())


def test_solve_with_device_setup_matches_oracle_and_host_setup():
    import paper_1710_03940_amd as L
    P = tiny_problem(N=22, pieces=(2, 2, 2), deflation="linear", sigma=2.0, seed=31)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=40)).solve(P.b)
    xs = []
    for dev in (0, 1):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=40, autotune=0, setup_device=dev)
        x = torch.zeros(P.n, dtype=torch.float64, device="cuda:0")
        out = S.solve(torch.tensor(P.b, device="cuda:0"), x)
        st = S.stats()
        S.close()
        assert st["setup_hierarchy_device"] == dev
        assert out["status"] == 0 and abs(out["iters"] - ref["iters"]) <= 2
        assert out["relres_true"] <= 1e-8
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])   # same hierarchy, same layouts: the same solve
    assert np.linalg.norm(xs[1] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
