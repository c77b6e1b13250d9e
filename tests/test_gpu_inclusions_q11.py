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
def test_inclusion_workload_q11(capsys):
    import paper_1503_03467_amd as P
    q, nrhs = 11, 16

    def say(*a):
        with capsys.disabled():   # progress of the long steps reaches the log
            print(*a, flush=True)

    print("CASE test=inclusion_workload q=11 a_incl=1e6 rho=4", flush=True)
    pr = S.inclusion_problem(q=q, nrhs=16, a_incl=1e6)
    dev = torch.device("cuda")
    a = torch.as_tensor(pr.a, device=dev)
    g = torch.as_tensor(pr.g[:nrhs], device=dev)
    H = P.Hierarchy(a, rho=4, precision="mixed-fp64-build", rtol=1e-8, max_rhs=4, max_outer=6000,
                    inner="cheb-cg", inner_iters=8, inner_iters_coarse=16, window_tol=1000.0)
    say("built")
    parts = []
    for r0 in range(0, nrhs, 4):   # four calls of one 4-right-hand-side block each
        parts.append(H.solve(g[r0:r0 + 4].contiguous()))
        say("solved right-hand sides", r0, "to", r0 + 3, H.last_info)
    u = torch.cat(parts)
    ga, _, _ = H.adjoint(u[:1].contiguous(), u[:1].contiguous())
    say("adjoint", H.last_info)
    u = u.cpu().numpy()
    ga = ga[0].cpu().numpy() if ga.dim() == 3 else ga.cpu().numpy()
    H.close()
    fe = fem.assemble(pr.a)
    ds = fem.DirectSolver(fe.A)
    say("direct factorization done")
    gate = max(1e-8, 10.0 * _noise(q))
    for r in (0, nrhs - 1):
        u_ref = ds.solve(fem.load_cellwise(pr.g[r], fe.h))
        err = _relerr(u[r][1:-1, 1:-1], u_ref)
        say("rhs", r, "err vs direct", err, "gate", gate)
        assert err < gate, (r, err)
    u_ref = ds.solve(fem.load_cellwise(pr.g[0], fe.h))
    # adjoint of J = |u|^2 / 2: lambda = A^-1 u, dJ/dlog a_e = -a_e lambda_e^T K u_e
    lam = ds.solve(u_ref)
    ga_ref = fem.cell_energy_gradient(pr.a, fem.full_nodal(fe, u_ref), fem.full_nodal(fe, lam))
    gerr = _relerr(ga, ga_ref)
    print("gradient err", gerr, flush=True)
    assert gerr < 1e-5, gerr
