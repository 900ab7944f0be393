"""GPU parity of the block SPAI-0 smoother on the point-block (4 x 4) Oseen
hierarchy: one V-cycle against the oracle's, and whole BiCGStab and
BiCGStab(2) solves in FP64 and with the FP32 hierarchy."""
import numpy as np
import pytest

from workloads import config_oseen, config_small_poisson
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def test_block_smoother_vcycle_matches_oracle():
    import paper_1710_03940_amd as L
    for N, pieces in [(8, (2, 2, 1)), (12, (2, 1, 1))]:
        P = config_oseen(N=N, pieces=pieces)
        kw = dict(solver="bicgstab", block_size=4, smoother="block_spai0", coarse_enough=100)
        ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**kw))
        S = L.Solver(P.A, P.part, P.nsub, P.Z, **kw)
        v = np.random.default_rng(N).standard_normal(P.n)
        out = _t(np.zeros(P.n))
        S.apply(L._lib.OP_PRECOND, _t(v), out)
        S.close()
        ref = ora.apply_precond(v)
        print(f"oseen{N}: levels {len(ora.M.hierarchies[0].levels)}", flush=True)
        assert np.linalg.norm(out.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("solver,oracle_solver", [("bicgstab", "bicgstab"), ("bicgstab2", "bicgstabl")])
def test_block_smoother_solves_match_oracle(solver, oracle_solver):
    import paper_1710_03940_amd as L
    P = config_oseen(N=16, pieces=(2, 2, 1))
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z,
                       OracleParams(solver=oracle_solver, block_size=4, smoother="block_spai0")).solve(P.b)
    assert ref["status"] == "ok"
    for prec in ("fp64", "mixed"):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, solver=solver, block_size=4, smoother="block_spai0",
                     precision=prec)
        x = _t(np.zeros(P.n))
        out = S.solve(_t(P.b), x)
        S.close()
        print(f"{solver} {prec}: gpu {out['iters']} oracle {ref['iters']} relres {out['relres_true']:.2e}",
              flush=True)
        assert out["status"] == 0 and out["relres_true"] <= 1e-8 * (1 + 1e-6)
        if prec == "fp64":
            assert abs(out["iters"] - ref["iters"]) <= 2
        else:
            assert out["iters"] <= int(np.floor(1.15 * ref["iters"])) + 1
        assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_block_smoother_with_scalar_blocks_is_spai0():
    """Block size 1: block SPAI-0 is SPAI-0 (same iterations, same solution
    up to rounding)."""
    import paper_1710_03940_amd as L
    P = config_small_poisson()
    outs = []
    for sm in ("spai0", "block_spai0"):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, smoother=sm)
        x = _t(np.zeros(P.n))
        o = S.solve(_t(P.b), x)
        S.close()
        outs.append((o["iters"], x.cpu().numpy()))
    assert outs[0][0] == outs[1][0]
    assert np.linalg.norm(outs[0][1] - outs[1][1]) <= 1e-10 * np.linalg.norm(outs[0][1])


def test_block_smoother_batched_equals_standalone():
    import paper_1710_03940_amd as L
    from workloads import concat_problems
    probs = [config_oseen(N=n, pieces=pc) for n, pc in [(8, (2, 1, 1)), (10, (1, 2, 1))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    kw = dict(solver="bicgstab", block_size=4, smoother="block_spai0", coarse_enough=60, autotune=0)
    S = L.BatchedSolver(A, part, nsub, Z, off, **kw)
    xb = _t(np.zeros(A.shape[0]))
    outb = S.solve(_t(b), xb)
    S.close()
    xb = xb.cpu().numpy()
    for s, p in enumerate(probs):
        S1 = L.Solver(p.A, p.part, p.nsub, p.Z, **kw)
        x1 = _t(np.zeros(p.n))
        o1 = S1.solve(_t(p.b), x1)
        S1.close()
        assert int(outb["iters"][s]) == o1["iters"]
        assert np.array_equal(xb[off[s]:off[s + 1]], x1.cpu().numpy())
