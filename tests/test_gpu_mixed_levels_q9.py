"""Mixed-precision hierarchy intermediates at the benchmark size (512 x 512
cells, sigma = 2, rho = 3): every level's A^(k), R^(k-1,k) and B^(k) of the
FP32 build against the FP64 build of the same problem (itself held to the
oracle at 1e-10 on q <= 6).  Bound 1e-3 relative to each array's largest
entry: FP32 unit roundoff 6e-8 times the scaled patch condition numbers (up
to ~1e3), compounded through the FP32 Galerkin products of the levels above
(the bound of the small-size mixed-path tests)."""
import numpy as np
import pytest

import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mixed_levels_match_fp64_at_benchmark_size():
    import paper_1503_03467_amd as P
    print("CASE test=mixed_levels_q9", flush=True)
    pr = S.q9_rough_problem()
    a = torch.as_tensor(pr.a, device="cuda")
    Hm = P.Hierarchy(a, rho=3, precision="mixed")
    Hd = P.Hierarchy(a, rho=3, precision="fp64")
    worst = {}
    for k in range(pr.q, 0, -1):
        lm, ld = Hm.level(k), Hd.level(k)
        names = ["A"] + (["R", "B"] if k >= 2 else [])
        for nm in names:
            xm = lm[nm].double()
            xd = ld[nm]
            err = float((xm - xd).abs().max() / xd.abs().max())
            worst[(k, nm)] = err
            assert err < 1e-3, (k, nm, err)
    print("largest relative differences", {f"{k}{nm}": f"{e:.1e}" for (k, nm), e in worst.items()}, flush=True)
    Hm.close()
    Hd.close()
