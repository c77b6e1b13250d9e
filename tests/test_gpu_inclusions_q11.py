"""The inclusion workload at full size: 2048 x 2048 cells, discs of a = 1e6 on
10% of the cells over the oscillatory product field, patch radius 4,
hierarchy + solve + adjoint, FP64-built hierarchy with FP32 subband
iterations and the FP64 outer iteration.

Gates: the solution against the oracle's direct solve within the larger of
1e-8 and ten times the distance between two FP64 direct solves of this
problem (tests/golden/inclusion_direct_noise.txt: the stiffness matrix is
too ill-conditioned for FP64 to fix more digits); the adjoint gradient of
J = |u|^2 / 2 against the oracle's (same factorization) within 1e-5.
"""
import os

import numpy as np
import pytest

import synthetic as S
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _noise(q):
    with open(os.path.join(HERE, "golden", "inclusion_direct_noise.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            if int(k) == q:
                return float(v)
    raise KeyError(q)


def _relerr(x, y):
    return float(np.linalg.norm(np.ravel(x) - np.ravel(y)) / np.linalg.norm(np.ravel(y)))


@pytest.mark.timeout(900)
def test_inclusion_workload_q11():
    import paper_1503_03467_amd as P
    q, nrhs = 11, 2
    print("CASE test=inclusion_workload q=11 a_incl=1e6 rho=4", flush=True)
    pr = S.inclusion_problem(q=q, nrhs=16, a_incl=1e6)
    dev = torch.device("cuda")
    a = torch.as_tensor(pr.a, device=dev)
    g = torch.as_tensor(pr.g[:nrhs], device=dev)
    H = P.Hierarchy(a, rho=4, precision="mixed-fp64-build", rtol=1e-8, max_rhs=nrhs, max_outer=6000,
                    inner="cheb-cg", inner_iters=16, inner_iters_coarse=8, window_tol=1000.0)
    u = H.solve(g)
    info = H.last_info
    print("solve", info, flush=True)
    ga, _, _ = H.adjoint(u[:1].contiguous(), u[:1].contiguous())
    print("adjoint", H.last_info, flush=True)
    u = u.cpu().numpy()
    ga = ga[0].cpu().numpy() if ga.dim() == 3 else ga.cpu().numpy()
    H.close()
    fe = fem.assemble(pr.a)
    ds = fem.DirectSolver(fe.A)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u_ref = ds.solve(b)
    gate = max(1e-8, 10.0 * _noise(q))
    err = _relerr(u[0][1:-1, 1:-1], u_ref)
    print("err vs direct", err, "gate", gate, flush=True)
    assert err < gate, err
    # adjoint of J = |u|^2 / 2: lambda = A^-1 u, dJ/dlog a_e = -a_e lambda_e^T K u_e
    lam = ds.solve(u_ref)
    ga_ref = fem.cell_energy_gradient(pr.a, fem.full_nodal(fe, u_ref), fem.full_nodal(fe, lam))
    gerr = _relerr(ga, ga_ref)
    print("gradient err", gerr, flush=True)
    assert gerr < 1e-5, gerr
