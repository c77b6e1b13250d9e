"""GPU hierarchy started from the level-q gamblets of the localized mass
inverse (Algorithm 2 with its own first lines; Definition 5.2), against the
FP64 CPU oracle, through the C ABI.

The oracle builds its localized hierarchy on A^(q) = Minv^T A Minv
(oracle.mass_inverse + oracle.gamblets); every level's A^(k), B^(k) and
R^(k-1,k) of the FP64 GPU hierarchy is compared at 1e-10 (as for the
nodal-basis hierarchy).  Solves: the preconditioner maps the nodal residual
r to g^(q) = Minv^T r and the level-q result v to Minv v, so the outer
iteration still solves the nodal finite-element system; results are held to
the direct solve at 1e-10 (FP64) and 1e-8 (mixed)."""
import numpy as np
import pytest

import synthetic as S
from oracle import fem
from oracle import gamblets as G
from oracle import mass_inverse as MI
from tests.gpu_layout import block_stencil_to_matrix, restriction_to_matrix, stencil_to_matrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _relerr(x, y):
    return float(np.linalg.norm(np.ravel(x) - np.ravel(y)) / max(np.linalg.norm(np.ravel(y)), 1e-300))


@pytest.mark.parametrize("q,rho,rho_q,sigma", [(4, 2, 2, 1.0), (5, 3, 1, 2.0), (5, 3, 3, 2.0), (5, 2, 4, 1.0), (3, 1, 1, 1.0)])
def test_hierarchy_levels_match_oracle_fp64(q, rho, rho_q, sigma):
    _case(test="mass_hierarchy", q=q, rho=rho, rho_q=rho_q, sigma=sigma)
    pr = S.rough_problem(q, sigma, 61)
    fe = fem.assemble(pr.a)
    tree = G.Tree(q)
    lq = MI.level_q_gamblets(fe, rho_q)
    ref = G.localized_hierarchy(lq.A, tree, rho)
    H = _P().Hierarchy(_dev(pr.a), rho=rho, precision="fp64", level_q_mass=rho_q)
    torch.cuda.synchronize()
    for k in range(q, 0, -1):
        lv = H.level(k)
        A_gpu = stencil_to_matrix(lv["A"].cpu().numpy(), q, k, tree.size(k))
        A_ref = ref.levels[k].A
        err = abs(A_gpu - A_ref).max() / abs(A_ref).max()
        print("level", k, "A err", err, flush=True)
        assert err < 1e-10, (k, "A", err)
        if k >= 2:
            B_gpu = block_stencil_to_matrix(lv["B"].cpu().numpy(), tree, k)
            B_ref = ref.levels[k].B
            err = abs(B_gpu - B_ref).max() / abs(B_ref).max()
            assert err < 1e-10, (k, "B", err)
            R_gpu = restriction_to_matrix(lv["R"].cpu().numpy(), lv["rho"], q, k, tree.size(k))
            R_ref = ref.levels[k].R
            err = abs(R_gpu - R_ref).max() / abs(R_ref).max()
            assert err < 1e-10, (k, "R", err)
    H.close()


@pytest.mark.parametrize("q,rho,rho_q,sigma,prec,tol", [
    (5, 2, 1, 1.0, "fp64", 1e-10), (6, 3, 3, 2.0, "fp64", 1e-10), (6, 3, 3, 2.0, "mixed", 1e-8),
    (7, 3, 2, 2.0, "mixed", 1e-8),
])
def test_solve_matches_direct(q, rho, rho_q, sigma, prec, tol):
    _case(test="mass_solve", q=q, rho=rho, rho_q=rho_q, sigma=sigma, prec=prec)
    pr = S.rough_problem(q, sigma, 62, nrhs=2)
    u_ref = fem.solve(pr.a, pr.g)
    H = _P().Hierarchy(_dev(pr.a), rho=rho, precision=prec, rtol=tol, max_rhs=2, level_q_mass=rho_q)
    u = H.solve(_dev(pr.g)).cpu().numpy()
    print("info", H.last_info, flush=True)
    for r in range(2):
        err = _relerr(u[r][1:-1, 1:-1], u_ref[r][1:-1, 1:-1])
        assert err < tol, (r, err, H.last_info)
    H.close()


@pytest.mark.timeout(300)
def test_full_size_q9_matches_direct():
    """The benchmark problem (512 x 512 cells, sigma = 2, rho = 3) with the
    level-q gamblets of the mass inverse (rho_q = 3): mixed path at 1e-8."""
    _case(test="mass_full_q9")
    pr = S.q9_rough_problem()
    u_ref = fem.solve(pr.a, pr.g)[0][1:-1, 1:-1]
    print("oracle done", flush=True)
    H = _P().Hierarchy(_dev(pr.a), rho=3, precision="mixed", rtol=1e-8, level_q_mass=3, max_outer=400)
    u = H.solve(_dev(pr.g[0])).cpu().numpy()
    err = _relerr(u[1:-1, 1:-1], u_ref)
    print("err", err, H.last_info, flush=True)
    assert err < 1e-8
    H.close()


def test_adjoint_gradient_matches_oracle():
    """The adjoint solve runs through the same preconditioner: dJ/dlog a and
    dJ/dg against the oracle's adjoint (mixed path, 1e-5)."""
    _case(test="mass_adjoint")
    pr = S.adjoint_problem(q=6, tag=64)
    u_obs = fem.solve(pr.extra["a_obs"], pr.g[0])
    _, _, ga_ref, gg_ref = fem.adjoint(pr.a, pr.g[0], u_obs[1:-1, 1:-1].ravel())
    H = _P().Hierarchy(_dev(pr.a), rho=3, precision="mixed", rtol=1e-8, level_q_mass=2, max_outer=400)
    u = H.solve(_dev(pr.g[0]))
    ga, gg, _ = H.adjoint(u, (u - _dev(u_obs)).contiguous())
    assert _relerr(ga.cpu().numpy(), ga_ref) < 1e-5
    assert _relerr(gg.cpu().numpy(), gg_ref) < 1e-5
    H.close()


def test_transform_rejects_mass_hierarchy():
    _case(test="mass_transform_rejected")
    pr = S.rough_problem(4, 1.0, 63)
    P = _P()
    H = P.Hierarchy(_dev(pr.a), rho=2, precision="fp64", level_q_mass=2)
    u = torch.zeros((17, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(P.GambletError):
        H.transform(u)
    H.close()
