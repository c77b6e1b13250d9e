"""The allocation-free compression entry point against the workspace one.

gbl_compress_noalloc keeps its selection state in a fixed device array of the
library instead of a hierarchy workspace; its output must equal gbl_compress's
bit for bit (selection work), on two calls in a row, the second on a smaller
vector, so that what the first call left in the shared array cannot leak into
the second.
"""
import numpy as np
import pytest
import torch

import paper_1503_03467_amd as P
import synthetic as S

pytestmark = pytest.mark.gpu


def _coefficients(count: int, seed: int) -> np.ndarray:
    """Magnitudes over many binades, with repeated values and zeros (ties at the threshold)."""
    gen = np.random.default_rng([71, seed])
    c = gen.standard_normal(count) * np.exp(gen.uniform(-30.0, 30.0, count))
    c[gen.choice(count, count // 16, replace=False)] = 0.0
    rep = gen.choice(count, count // 8, replace=False)
    c[rep] = np.sign(c[rep]) * 1.25
    return c


@pytest.mark.parametrize("first_q,second_q", [(7, 5), (8, 6)])
def test_noalloc_compression_matches_workspace_compression(first_q, second_q):
    dev = torch.device("cuda:0")
    for q, keep_frac, seed in ((first_q, 0.01, 1), (second_q, 0.25, 2)):
        pr = S.rough_problem(q, 1.0, S.TAG_BATCH, problem=90 + q)
        H = P.Hierarchy(torch.as_tensor(pr.a, device=dev), rho=3, precision="mixed")
        count = H.transform_size()
        c = torch.as_tensor(_coefficients(count, seed + q), device=dev)
        keep = max(1, int(keep_frac * count))
        ref = c.clone()
        thr_ref = H.compress(ref, keep)
        out = c.clone()
        thr = P.compress_noalloc(out, keep)
        torch.cuda.synchronize()
        H.close()
        assert thr == thr_ref, (q, thr, thr_ref)
        assert torch.equal(out, ref), q
        kept = int((out != 0).sum())
        assert kept >= keep - int((c == 0).sum()), (kept, keep)


def test_noalloc_compression_edge_keeps():
    dev = torch.device("cuda:0")
    c = torch.as_tensor(_coefficients(4096, 9), device=dev)
    out = c.clone()
    assert P.compress_noalloc(out, 0) == float("inf")
    assert int((out != 0).sum()) == 0
    out = c.clone()
    assert P.compress_noalloc(out, 4096) == 0.0
    assert torch.equal(out, c)
    # a call after the edge cases still selects exactly
    out = c.clone()
    thr = P.compress_noalloc(out, 1)
    mags = torch.abs(c)
    assert thr == float(mags.max())
    assert torch.equal(out, torch.where(mags >= thr, c, torch.zeros_like(c)))
