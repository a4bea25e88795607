"""Several right-hand sides on one setup (lsq_solve_many) against the oracle.

The sample, M and the level sets depend on A only, so every column of B must
give what a setup with that column as b gives: the oracle's converged x for
that b, and, on the dense path (whose reductions run in a fixed order), the
very bytes of lsq_solve on the same setup.
"""
import copy
import ctypes as C

import numpy as np
import pytest

import oracle
from gpu_helpers import make_solver, rel
from workloads import gaussian_dense, make_config, sparse_rowscaled

pytestmark = pytest.mark.gpu


def _with_b(p, b):
    q = copy.copy(p)
    q.b = np.ascontiguousarray(b, dtype=np.float64)
    return q


def _columns(p, k, seed):
    rng = np.random.default_rng(seed)
    cols = [p.b]
    for j in range(1, k):
        cols.append(np.zeros(p.m) if j == 2 else rng.standard_normal(p.m))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("name", ["gaussian", "sparse", "sparse_ragged"])
def test_columns_match_the_oracle(name):
    import torch
    p = {"gaussian": lambda: make_config("gaussian", scale="small")[0],
         "sparse": lambda: make_config("sparse", scale="small")[0],
         "sparse_ragged": lambda: sparse_rowscaled(m=5003, n=131, k=7, seed=4)}[name]()
    sweeps = 2
    print("\n[case] solve_many", name, p.m, p.n, flush=True)
    s, dev = make_solver(p, C_=4.0, sweeps=sweeps, seed=0)
    Bh = _columns(p, 4, seed=11)
    X, infos = s.solve_many(torch.from_numpy(Bh).cuda())
    assert tuple(X.shape) == (p.n, 4) and len(infos) == 4
    Xh = X.cpu().numpy()
    # the zero column: no iteration, x = 0
    assert infos[2]["iters"] == 0 and not Xh[:, 2].any()
    for j in (0, 1, 3):
        xo, io = oracle.Oracle(_with_b(p, Bh[:, j]), C_=4.0, sweeps=sweeps, seed=0).solve(tol=1e-10)
        inf = infos[j]
        print("[%s col %d] gpu iters %d relres %.3g | oracle iters %d | x diff %.3g" % (
            name, j, inf["iters"], inf["relres_true"], io["iters"], rel(Xh[:, j], xo)), flush=True)
        assert inf["converged"] == 1 and inf["relres_true"] <= 1e-10
        assert abs(inf["iters"] - io["iters"]) <= 1
        if inf["iters"] == io["iters"]:
            assert rel(Xh[:, j], xo) <= 1e-9
    # the setup's own b is still the one lsq_solve uses afterwards
    x0, _ = s.solve()
    assert rel(x0.cpu().numpy(), Xh[:, 0]) <= 1e-12


def test_dense_columns_are_the_single_solves_bit_for_bit():
    import torch
    p = gaussian_dense(3001, 77, seed=9)
    s, dev = make_solver(p, C_=4.0, sweeps=1, seed=2)
    Bh = _columns(p, 3, seed=12)
    X, _ = s.solve_many(torch.from_numpy(Bh).cuda())
    x0, _ = s.solve()
    assert bool((X[:, 0] == x0).all())
    s2, _ = make_solver(_with_b(p, Bh[:, 1]), C_=4.0, sweeps=1, seed=2)
    x1, _ = s2.solve()
    assert bool((X[:, 1] == x1).all())


def test_argument_errors():
    import torch
    from paper_1806_02968_amd import LsqError
    from paper_1806_02968_amd.lsq import lib
    p = gaussian_dense(200, 9, seed=1)
    s, dev = make_solver(p)
    B = torch.zeros(p.m, 2, dtype=torch.float64, device="cuda")
    X = torch.zeros(2, p.n, dtype=torch.float64, device="cuda")
    L = lib()
    assert L.lsq_solve_many(s._ctx, 0, None, 0, None, 0, None) == 0
    assert L.lsq_solve_many(s._ctx, -1, None, 0, None, 0, None) == -1
    assert L.lsq_solve_many(s._ctx, 2, C.c_void_p(B.data_ptr()), p.m - 1, C.c_void_p(X.data_ptr()), p.n,
                            None) == -1
    assert L.lsq_solve_many(s._ctx, 2, C.c_void_p(B.data_ptr()), p.m, C.c_void_p(X.data_ptr()), p.n - 1,
                            None) == -1
    B[5, 1] = float("nan")
    with pytest.raises(LsqError) as e:
        s.solve_many(B)
    assert e.value.code == -3  # LSQ_ENONFINITE
    # nothing was solved: the setup still answers lsq_solve
    x, info = s.solve()
    assert info["converged"] == 1
