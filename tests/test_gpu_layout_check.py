"""Every sparse layout the setup tuner times, checked against the first
candidate of the same operator (DFAMG_TUNE_VERIFY): each candidate is applied
once to the same varied input and its output must agree with the first
candidate's to rounding, or the setup fails.  The candidates cover SELL with
1, 2 and 4 rows per lane (natural and length-sorted rows, 16- and 32-bit
columns, staged or not), CSR with 1 to 64 lanes per row and tiles of 4 to
256 rows (unstaged, staged window, staged gather list), BSR4 and the
column-tiled restrictions, in FP64 and FP32, on the operators of a Poisson
hierarchy large enough for every candidate, of CSR-only hierarchies, of
batched systems and of a point-block Oseen hierarchy.  The chosen layouts
then solve to the tolerance."""
import os
import re

import numpy as np
import pytest

from workloads import make_problem, tiny_problem, concat_problems, config_oseen

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture
def verify_env():
    os.environ["DFAMG_TUNE_VERIFY"] = "1"
    yield
    del os.environ["DFAMG_TUNE_VERIFY"]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=torch.device("cuda:0"))


def _checks(err):
    """(checked candidates, the distinct layout names) from the tuner's log."""
    lines = re.findall(r"layout check (\S+) against (\S+): max difference", err)
    return len(lines), {a for a, _ in lines} | {b for _, b in lines}


def _solve(S, P):
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    S.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_candidate_agrees_large_poisson(verify_env, capfd, precision):
    # 82^3 in 2 x 2 x 2 boxes: level 0 has enough tiles for SELL with 2 and
    # (outer operator) 4 rows per lane, the restrictions are long enough for
    # column tiles, and the coarse levels small enough for the short CSR tiles
    import paper_1710_03940_amd as L
    P = make_problem("p82", (82, 82, 82), (2, 2, 2), deflation="linear", sigma=1.0, coef_seed=5,
                     rhs="uniform", rhs_seed=6)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, precision=precision, autotune=1, verbose=2)
    lay = S.stats()["layouts"]
    out = _solve(S, P)
    n, names = _checks(capfd.readouterr().err)
    print(precision, n, "candidates checked;", lay, flush=True)
    assert n >= 60, n
    assert any(nm.startswith("sell2") for nm in names) and any(nm.startswith("sell4") for nm in names), names
    assert any(nm.startswith("seg") for nm in names), names
    assert any("csr64/t4" in nm for nm in names) and any("/glist" in nm for nm in names), names
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.01


@pytest.mark.parametrize("fmt", ["csr", "csr_gather"])
def test_every_csr_candidate_agrees(verify_env, capfd, fmt):
    import paper_1710_03940_amd as L
    P = make_problem("p40", (40, 36, 33), (2, 2, 2), deflation="linear", sigma=2.0, coef_seed=7,
                     rhs="uniform", rhs_seed=8)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=60, spmv_format=fmt, autotune=1, verbose=2)
    out = _solve(S, P)
    n, names = _checks(capfd.readouterr().err)
    print(fmt, n, sorted(names), flush=True)
    assert n >= 10, n
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.01


def test_every_candidate_agrees_batched(verify_env, capfd):
    import paper_1710_03940_amd as L
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.5, seed=s)
             for n, pc, s in ((21, (2, 2, 1), 11), (17, (1, 2, 2), 12), (13, (1, 1, 1), 13))]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    S = L.BatchedSolver(A, part, nsub, Z, off, coarse_enough=30, autotune=1, verbose=2)
    x = _t(np.zeros(A.shape[0]))
    out = S.solve(_t(b), x)
    S.close()
    n, _ = _checks(capfd.readouterr().err)
    assert n >= 20, n
    assert np.all(np.asarray(out["status"]) == 0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_candidate_agrees_point_block(verify_env, capfd, precision):
    # 4 x 4 blocks: BSR4 joins the candidates of every operator
    import paper_1710_03940_amd as L
    P = config_oseen(N=12, pieces=(2, 2, 1))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, block_size=4, solver="bicgstab", coarse_enough=60,
                 precision=precision, autotune=1, verbose=2)
    out = _solve(S, P)
    n, names = _checks(capfd.readouterr().err)
    print(precision, n, sorted(names), flush=True)
    assert any(nm.startswith("bsr4") for nm in names), names
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.01
