"""GPU parity of the Schur pressure-correction solver (section
"Navier-Stokes problem") and of the SPAI-0 preconditioner against the
oracle on the stabilised Q1 Oseen operator."""
import numpy as np
import pytest

from workloads import oseen_q1, tiny_problem, convection_diffusion7
from workloads.partition import box_partition
from oracle import OracleSolver, OracleParams
from oracle.schur import schur_fgmres

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _oseen(N, pieces):
    A, _ = oseen_q1(N)
    n = A.shape[0]
    pmask = (np.arange(n) % 4 == 3).astype(np.int32)
    part_p, nsub = box_partition(N, N, N, *pieces)
    b = np.random.default_rng(N).uniform(-1.0, 1.0, n)
    return A, pmask, part_p, nsub, np.ones((N ** 3, 1)), b


def _gpu(A, pmask, part_p, nsub, Zp, b, **kw):
    import paper_1710_03940_amd as L
    S = L.SchurSolver(A, pmask, part_p, nsub, Zp, **kw)
    x = _t(np.zeros(A.shape[0]))
    out = S.solve(_t(b), x)
    out["x"] = x.cpu().numpy()
    S.close()
    return out


@pytest.mark.parametrize("N,pieces", [(12, (2, 2, 1)), (16, (2, 2, 2))])
def test_schur_fp64_parity(N, pieces):
    A, pmask, part_p, nsub, Zp, b = _oseen(N, pieces)
    print(f"case oseen{N} pieces {pieces}", flush=True)
    ref = schur_fgmres(A, b, pmask, part_p, nsub, Zp, rtol=1e-8)
    out = _gpu(A, pmask, part_p, nsub, Zp, b, rtol=1e-8)
    print(f"  gpu iters {out['iters']} status {out['status']} relres_true {out['relres_true']:.3e}"
          f" | oracle {ref['iters']} {ref['status']}", flush=True)
    assert ref["status"] == "ok" and out["status"] == 0
    assert abs(out["iters"] - ref["iters"]) <= 2
    assert out["relres_true"] <= 1e-8 * (1 + 1e-6)
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_schur_mixed_and_paper_tolerance():
    A, pmask, part_p, nsub, Zp, b = _oseen(16, (2, 2, 1))
    ref = schur_fgmres(A, b, pmask, part_p, nsub, Zp, rtol=1e-8)
    out = _gpu(A, pmask, part_p, nsub, Zp, b, rtol=1e-8, precision="mixed")
    print(f"mixed: gpu {out['iters']} oracle {ref['iters']}", flush=True)
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * (1 + 1e-6)
    assert out["iters"] <= int(np.floor(1.15 * ref["iters"])) + 1
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
    # the top-level tolerance of the paper's listing
    ref4 = schur_fgmres(A, b, pmask, part_p, nsub, Zp, rtol=1e-4)
    out4 = _gpu(A, pmask, part_p, nsub, Zp, b, rtol=1e-4)
    print(f"1e-4: gpu {out4['iters']} oracle {ref4['iters']}", flush=True)
    assert abs(out4["iters"] - ref4["iters"]) <= 2 and out4["relres_true"] <= 1e-4


def test_schur_handle_rejects_apply():
    import paper_1710_03940_amd as L
    A, pmask, part_p, nsub, Zp, b = _oseen(8, (1, 1, 1))
    S = L.SchurSolver(A, pmask, part_p, nsub, Zp)
    v = _t(np.zeros(A.shape[0]))
    with pytest.raises(L.DfamgError):
        S.apply(0, v, v)
    S.close()


@pytest.mark.parametrize("solver", ["fgmres", "bicgstab"])
def test_spai0_preconditioner_parity(solver):
    import paper_1710_03940_amd as L
    base = tiny_problem(N=10, pieces=(2, 1, 1), deflation="linear", seed=7)
    A = convection_diffusion7(10, peclet=2.0)
    ref = OracleSolver(A, base.part, base.nsub, base.Z,
                       OracleParams(solver=solver, precond="spai0")).solve(base.b)
    S = L.Solver(A, base.part, base.nsub, base.Z, solver=solver, precond="spai0")
    x = _t(np.zeros(A.shape[0]))
    out = S.solve(_t(base.b), x)
    S.close()
    print(f"spai0 {solver}: gpu {out['iters']} oracle {ref['iters']}", flush=True)
    assert ref["status"] == "ok" and out["status"] == 0
    assert abs(out["iters"] - ref["iters"]) <= 2
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_schur_without_pressure_deflation():
    """The pressure solves with the block AMG alone (no deflation vectors)."""
    A, pmask, part_p, nsub, Zp, b = _oseen(12, (2, 1, 1))
    Z0 = np.zeros((Zp.shape[0], 0))
    ref = schur_fgmres(A, b, pmask, part_p, nsub, Z0, rtol=1e-8)
    out = _gpu(A, pmask, part_p, nsub, Z0, b, rtol=1e-8)
    print(f"no deflation: gpu {out['iters']} oracle {ref['iters']}", flush=True)
    assert ref["status"] == "ok" and out["status"] == 0
    assert abs(out["iters"] - ref["iters"]) <= 2
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
