"""The full batch workload through gbl_build_batched / gbl_solve_batched: 256
independent problems with q drawn from {6, 7, 8} (each with its own seeds,
sigma = 1), 64 N(0,1) right-hand sides each, solved as one block of 64.

Every problem's 64 solutions must equal, bit for bit, the same problem built
and solved on its own (same options), and a sample of problems and
right-hand sides must match the sparse direct solve at 1e-8 (the mixed-path
bound after the FP64 outer iteration).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


@pytest.mark.timeout(600)
def test_full_batch_equals_single_and_matches_direct():
    P = _P()
    probs = S.batch_problems(count=256, nrhs=64)
    print("CASE test=batch_full problems=256 rhs=64", flush=True)
    coeffs = [torch.as_tensor(p.a, device="cuda") for p in probs]
    srcs = [torch.as_tensor(p.g, device="cuda") for p in probs]
    hs = P.build_batched(coeffs, rho=3, precision="mixed", rtol=1e-8, max_rhs=64)
    us = P.solve_batched(hs, srcs)
    for h in hs:
        assert h.last_info.status == 0
        h.close()
    print("batched build and solve done", flush=True)
    for i, p in enumerate(probs):
        H = P.Hierarchy(coeffs[i], rho=3, precision="mixed", rtol=1e-8, max_rhs=64)
        u1 = H.solve(srcs[i])
        H.close()
        assert torch.equal(u1, us[i]), (i, p.q)
        if i % 64 == 0:
            print(f"problem {i} (q={p.q}) equals its single solve", flush=True)
    # direct solves on a sample: the first problem of each depth, three right-hand sides
    seen = set()
    for i, p in enumerate(probs):
        if p.q in seen:
            continue
        seen.add(p.q)
        rr = [0, 31, 63]
        u_ref = fem.solve(p.a, p.g[rr])
        u = us[i][rr].cpu().numpy()
        for j in range(len(rr)):
            a, b = u[j][1:-1, 1:-1], u_ref[j][1:-1, 1:-1]
            err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
            print(f"problem {i} q={p.q} rhs {rr[j]} rel err {err:.2e}", flush=True)
            assert err < 1e-8
